"""ctypes binding of the C ABI in ``include/gs.h`` -- argument marshalling only.

Every function here has the name of the C entry point it calls, takes torch
CUDA tensors (or plain device pointers) and passes their data pointers and the
current HIP stream.  No computation happens in Python.  Loading fails loudly if
``libgs_hip.so`` is missing: there is no fallback.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgs_hip.so")

GS_OK = 0
GS_ERR_CAPACITY = -2
GS_ERR = {-1: "GS_ERR_INVALID_ARG", -2: "GS_ERR_CAPACITY", -3: "GS_ERR_HIP",
          -4: "GS_ERR_UNSUPPORTED"}
GS_FLAG_ISECT_OVERFLOW = 1
GS_FLAG_NONFINITE = 2
GS_FLAG_SCAN_STALLED = 4
GS_FLAG_COUNT_BOUND = 8
GS_MAX_VIEWS = 64
GS_RECORD_FLOATS = 12
GS_GRAD2D_FLOATS = 9
GS_ADAM_MAX_GROUPS = 16

c_vp = ctypes.c_void_p


class gs_capacity(ctypes.Structure):
    _fields_ = [("max_pairs", ctypes.c_int64), ("max_isect", ctypes.c_int64),
                ("max_tiles", ctypes.c_int64), ("max_views", ctypes.c_int32),
                ("max_cams", ctypes.c_int32)]


class gs_settings(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("near_plane", ctypes.c_float), ("eps2d", ctypes.c_float),
                ("fov_pad", ctypes.c_float), ("alpha_min", ctypes.c_float),
                ("alpha_max", ctypes.c_float), ("t_min", ctypes.c_float),
                ("grad_accumulate", ctypes.c_int32), ("tile_order", ctypes.c_int32),
                ("eval_stats", ctypes.c_int32), ("lazy_lists", ctypes.c_int32)]


class gs_gaussians(ctypes.Structure):
    _fields_ = [("means", c_vp), ("log_scales", c_vp), ("quats", c_vp),
                ("opacity_logit", c_vp), ("sh", c_vp), ("N", ctypes.c_int32),
                ("sh_degree", ctypes.c_int32)]


class gs_gaussians_grad(ctypes.Structure):
    _fields_ = [("means", c_vp), ("log_scales", c_vp), ("quats", c_vp),
                ("opacity_logit", c_vp), ("sh", c_vp)]


class gs_cameras(ctypes.Structure):
    _fields_ = [("viewmat", c_vp), ("intr", c_vp), ("wh", c_vp), ("V", ctypes.c_int32),
                ("index", c_vp)]


class gs_diag(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("n_isect", ctypes.c_int64),
                ("n_isect_needed", ctypes.c_int64), ("n_masked_obs", ctypes.c_int64),
                ("n_visible", ctypes.c_int64)]


class gs_adam_group(ctypes.Structure):
    _fields_ = [("param", c_vp), ("grad", c_vp), ("exp_avg", c_vp), ("exp_avg_sq", c_vp),
                ("n", ctypes.c_int64), ("lr", ctypes.c_float)]


class gs_gaussian_adam(ctypes.Structure):
    _fields_ = [("params", c_vp * 5), ("exp_avg", c_vp * 5), ("exp_avg_sq", c_vp * 5),
                ("lr", ctypes.c_float * 5)]


EXPORTS = [
    "gs_strerror", "gs_default_settings", "gs_ctx_create", "gs_ctx_destroy", "gs_ctx_status",
    "gs_ctx_reset_status", "gs_ctx_buffers", "gs_ctx_tile_stats", "gs_project", "gs_bin_sort", "gs_render_fwd",
    "gs_render_bwd", "gs_raster_bwd", "gs_project_bwd", "gs_l1_loss_grad", "track_reproj_fwd_bwd", "gs_pose_compose",
    "gs_pose_compose_bwd", "gs_adam_step", "gs_project_bwd_adam", "track_point_index",
    "gs_step_advance", "gs_ctx_generation", "track_reproj_fwd_bwd_noalloc", "gs_photo_loss_grad",
    "gs_init_gaussians", "gs_ba_create", "gs_ba_destroy", "gs_ba_lm_step", "gs_mcmc_relocate",
    "gs_mcmc_noise",
]

_lib = None


class GsError(RuntimeError):
    def __init__(self, name, code):
        super().__init__(f"{name} returned {GS_ERR.get(code, code)}")
        self.code = code


def load():
    """Load libgs_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2603_04847_amd.build "
                          "(there is no non-HIP fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.gs_strerror.restype = ctypes.c_char_p
    lib.gs_strerror.argtypes = [ctypes.c_int]
    lib.gs_default_settings.restype = None
    lib.gs_default_settings.argtypes = [ctypes.POINTER(gs_settings)]
    for name in EXPORTS[2:]:
        getattr(lib, name).restype = ctypes.c_int
    lib.gs_ctx_create.argtypes = [ctypes.POINTER(c_vp), ctypes.POINTER(gs_capacity)]
    lib.gs_ctx_destroy.argtypes = [c_vp]
    lib.gs_ctx_status.argtypes = [c_vp, ctypes.POINTER(gs_diag)]
    lib.gs_ctx_reset_status.argtypes = [c_vp, c_vp]
    lib.gs_ctx_buffers.argtypes = [c_vp, ctypes.POINTER(c_vp), ctypes.POINTER(c_vp),
                                   ctypes.POINTER(c_vp), ctypes.POINTER(ctypes.c_int64)]
    lib.gs_ctx_tile_stats.argtypes = [c_vp, ctypes.POINTER(c_vp), ctypes.POINTER(c_vp),
                                      ctypes.POINTER(c_vp), ctypes.POINTER(c_vp),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
    lib.gs_project.argtypes = [c_vp, ctypes.POINTER(gs_gaussians), ctypes.POINTER(gs_cameras),
                               ctypes.POINTER(gs_settings), c_vp]
    lib.gs_bin_sort.argtypes = [c_vp, ctypes.POINTER(gs_cameras), ctypes.c_int32,
                                ctypes.POINTER(gs_settings), c_vp, c_vp]
    lib.gs_render_fwd.argtypes = [c_vp, ctypes.POINTER(gs_cameras), ctypes.POINTER(gs_settings),
                                  c_vp, c_vp, c_vp, c_vp, c_vp]
    lib.gs_render_bwd.argtypes = [c_vp, ctypes.POINTER(gs_gaussians), ctypes.POINTER(gs_cameras),
                                  ctypes.POINTER(gs_settings), c_vp, c_vp, c_vp, c_vp,
                                  ctypes.POINTER(gs_gaussians_grad), c_vp, c_vp]
    lib.gs_raster_bwd.argtypes = [c_vp, ctypes.POINTER(gs_cameras), ctypes.POINTER(gs_settings),
                                  c_vp, c_vp, c_vp, c_vp, c_vp]
    lib.gs_project_bwd.argtypes = [c_vp, ctypes.POINTER(gs_gaussians), ctypes.POINTER(gs_cameras),
                                   ctypes.POINTER(gs_settings), ctypes.POINTER(gs_gaussians_grad),
                                   c_vp, c_vp]
    lib.gs_l1_loss_grad.argtypes = [c_vp, ctypes.POINTER(gs_cameras), c_vp, c_vp, c_vp, c_vp, c_vp]
    lib.track_reproj_fwd_bwd.argtypes = [
        c_vp, c_vp, ctypes.c_int32, c_vp, c_vp, ctypes.c_int32, c_vp, c_vp, c_vp, ctypes.c_int32,
        ctypes.c_float, ctypes.c_float, ctypes.c_float, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
        c_vp, c_vp, c_vp, c_vp]
    lib.gs_mcmc_relocate.argtypes = [c_vp, ctypes.POINTER(gs_gaussian_adam), ctypes.c_int32,
                                     ctypes.c_int32, c_vp, ctypes.c_float, c_vp, c_vp, c_vp]
    lib.gs_mcmc_noise.argtypes = [c_vp, c_vp, c_vp, c_vp, ctypes.c_int32, c_vp, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_float, c_vp]
    lib.gs_ba_create.argtypes = [ctypes.POINTER(c_vp), ctypes.c_int64, ctypes.c_int32]
    lib.gs_ba_destroy.argtypes = [c_vp]
    lib.gs_ba_lm_step.argtypes = [c_vp, c_vp, ctypes.c_int32, c_vp, c_vp, ctypes.c_int32, c_vp, c_vp,
                                  c_vp, ctypes.c_int32, c_vp, c_vp, c_vp, c_vp, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_float, ctypes.c_int32, ctypes.c_float, c_vp,
                                  c_vp, c_vp, c_vp]
    lib.gs_init_gaussians.argtypes = [c_vp, c_vp, c_vp, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_float, ctypes.c_int32, c_vp, c_vp, c_vp, c_vp,
                                      c_vp, c_vp]
    lib.gs_photo_loss_grad.argtypes = [c_vp, ctypes.POINTER(gs_cameras), c_vp, c_vp, ctypes.c_float,
                                       c_vp, c_vp, c_vp]
    lib.track_reproj_fwd_bwd_noalloc.argtypes = [
        c_vp, ctypes.c_int32, c_vp, c_vp, ctypes.c_int32, c_vp, c_vp, c_vp, ctypes.c_int32,
        ctypes.c_float, ctypes.c_float, ctypes.c_float, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
        c_vp, c_vp]
    lib.track_point_index.argtypes = [c_vp, c_vp, ctypes.c_int32, ctypes.c_int32, c_vp, c_vp, c_vp,
                                      c_vp, c_vp, c_vp, c_vp]
    lib.gs_pose_compose.argtypes = [ctypes.c_int32, c_vp, c_vp, c_vp, c_vp]
    lib.gs_pose_compose_bwd.argtypes = [ctypes.c_int32, c_vp, c_vp, c_vp, c_vp]
    lib.gs_adam_step.argtypes = [ctypes.POINTER(gs_adam_group), ctypes.c_int32, ctypes.c_int32,
                                 c_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, c_vp]
    lib.gs_project_bwd_adam.argtypes = [c_vp, ctypes.POINTER(gs_gaussians), ctypes.POINTER(gs_cameras),
                                        ctypes.POINTER(gs_settings), ctypes.POINTER(gs_gaussian_adam),
                                        ctypes.c_int32, c_vp, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, c_vp, c_vp]
    lib.gs_step_advance.argtypes = [c_vp, c_vp]
    lib.gs_ctx_generation.argtypes = [c_vp, ctypes.POINTER(ctypes.c_int64)]
    _lib = lib
    return lib


_hip = None


def hip_runtime():
    """The HIP runtime library this process already uses (the one libgs_hip.so
    resolved), so raw device pointers from the context stay valid."""
    global _hip
    if _hip is None:
        load()
        path = None
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64.so" in line:
                    path = line.split()[-1]
                    break
        if path is None:
            raise RuntimeError("HIP runtime not loaded")
        _hip = ctypes.CDLL(path)
        _hip.hipMemcpy.argtypes = [c_vp, c_vp, ctypes.c_size_t, ctypes.c_int]
        _hip.hipDeviceSynchronize.restype = ctypes.c_int
    return _hip


def copy_to_host(ptr, count, dtype):
    """Synchronise the device and copy `count` elements at device address `ptr`."""
    import numpy as np
    out = np.empty(count, dtype)
    if count == 0:
        return out
    h = hip_runtime()
    if h.hipDeviceSynchronize() != 0 or h.hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2) != 0:
        raise RuntimeError("hipMemcpy failed")
    return out


def _check(name, rc):
    if rc != GS_OK:
        raise GsError(name, rc)


def _ptr(t):
    """Device pointer of a tensor (or an int address, or None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_contiguous():
        raise ValueError("tensors passed to the C ABI must be contiguous")
    return t.data_ptr()


def _stream(stream=None):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def default_settings(**over):
    s = gs_settings()
    load().gs_default_settings(ctypes.byref(s))
    for k, v in over.items():
        setattr(s, k, v)
    return s


def make_gaussians(means, log_scales, quats, opacity_logit, sh, sh_degree):
    return gs_gaussians(_ptr(means), _ptr(log_scales), _ptr(quats), _ptr(opacity_logit), _ptr(sh),
                        int(means.shape[1]), int(sh_degree))


def make_grads(means, log_scales, quats, opacity_logit, sh):
    return gs_gaussians_grad(_ptr(means), _ptr(log_scales), _ptr(quats), _ptr(opacity_logit),
                             _ptr(sh))


class Cameras:
    """Camera arguments: device viewmat [rows,12], intr [rows,4]; host wh [V,2]
    int32; optional host index [V] (camera row of each view of the call)."""

    def __init__(self, viewmat, intr, wh, index=None):
        import numpy as np
        self.viewmat = viewmat
        self.intr = intr
        self.wh = np.ascontiguousarray(np.asarray(wh, dtype=np.int32).reshape(-1, 2))
        self.V = self.wh.shape[0]
        self.index = None if index is None else np.ascontiguousarray(index, dtype=np.int32)
        self._c = gs_cameras(_ptr(viewmat), _ptr(intr), self.wh.ctypes.data_as(c_vp), self.V,
                             None if self.index is None else self.index.ctypes.data_as(c_vp))

    @property
    def struct(self):
        return self._c

    @property
    def n_pixels(self):
        return int((self.wh[:, 0].astype("int64") * self.wh[:, 1]).sum())


class Context:
    """A gs_ctx: the workspace, allocated once."""

    def __init__(self, max_pairs, max_isect, max_tiles, max_views=GS_MAX_VIEWS, max_cams=1):
        lib = load()
        self.cap = gs_capacity(int(max_pairs), int(max_isect), int(max_tiles), int(max_views),
                               int(max_cams))
        h = c_vp()
        _check("gs_ctx_create", lib.gs_ctx_create(ctypes.byref(h), ctypes.byref(self.cap)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load().gs_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def status(self):
        d = gs_diag()
        _check("gs_ctx_status", load().gs_ctx_status(self.handle, ctypes.byref(d)))
        return dict(flags=d.flags, n_isect=d.n_isect, n_isect_needed=d.n_isect_needed,
                    n_masked_obs=d.n_masked_obs, n_visible=d.n_visible)

    def generation(self):
        """gs_bin_sort calls enqueued on this context so far."""
        g = ctypes.c_int64()
        _check("gs_ctx_generation", load().gs_ctx_generation(self.handle, ctypes.byref(g)))
        return g.value

    def reset_status(self, stream=None):
        _check("gs_ctx_reset_status", load().gs_ctx_reset_status(self.handle, _stream(stream)))

    def buffers(self):
        """Device addresses of the records, the tile lists and their ranges, and
        the tile count of the last gs_bin_sort."""
        rec, ids, rng = c_vp(), c_vp(), c_vp()
        nt = ctypes.c_int64()
        _check("gs_ctx_buffers", load().gs_ctx_buffers(self.handle, ctypes.byref(rec),
                                                       ctypes.byref(ids), ctypes.byref(rng),
                                                       ctypes.byref(nt)))
        return dict(records=rec.value, isect_ids=ids.value, tile_ranges=rng.value,
                    n_tiles=nt.value)


def gs_ctx_tile_stats(ctx):
    """Device addresses of the per-tile contributor, entry and evaluation
    counts and the tile order, and the tile count of the last gs_bin_sort."""
    a, b, c, d = c_vp(), c_vp(), c_vp(), c_vp()
    o = ctypes.c_int32()
    nt = ctypes.c_int64()
    _check("gs_ctx_tile_stats", load().gs_ctx_tile_stats(ctx.handle, ctypes.byref(a),
                                                         ctypes.byref(b), ctypes.byref(c),
                                                         ctypes.byref(d), ctypes.byref(o),
                                                         ctypes.byref(nt)))
    return dict(tile_contrib=a.value, tile_entries=b.value, tile_evals=c.value,
                tile_order=d.value, ordered=bool(o.value), n_tiles=nt.value)


def gs_project(ctx, gaussians, cams, settings, stream=None):
    _check("gs_project", load().gs_project(ctx.handle, ctypes.byref(gaussians),
                                           ctypes.byref(cams.struct), ctypes.byref(settings),
                                           _stream(stream)))


def gs_bin_sort(ctx, cams, N, settings, records=None, stream=None):
    _check("gs_bin_sort", load().gs_bin_sort(ctx.handle, ctypes.byref(cams.struct), int(N),
                                             ctypes.byref(settings), _ptr(records),
                                             _stream(stream)))


def gs_render_fwd(ctx, cams, settings, bg, rgb, T_final, last, stream=None):
    _check("gs_render_fwd", load().gs_render_fwd(ctx.handle, ctypes.byref(cams.struct),
                                                 ctypes.byref(settings), _ptr(bg), _ptr(rgb),
                                                 _ptr(T_final), _ptr(last), _stream(stream)))


def gs_render_bwd(ctx, gaussians, cams, settings, bg, T_final, last, v_rgb, grads, v_twist,
                  stream=None):
    _check("gs_render_bwd", load().gs_render_bwd(
        ctx.handle, ctypes.byref(gaussians), ctypes.byref(cams.struct), ctypes.byref(settings),
        _ptr(bg), _ptr(T_final), _ptr(last), _ptr(v_rgb), ctypes.byref(grads), _ptr(v_twist),
        _stream(stream)))


def gs_raster_bwd(ctx, cams, settings, bg, T_final, last, v_rgb, stream=None):
    _check("gs_raster_bwd", load().gs_raster_bwd(ctx.handle, ctypes.byref(cams.struct),
                                                 ctypes.byref(settings), _ptr(bg), _ptr(T_final),
                                                 _ptr(last), _ptr(v_rgb), _stream(stream)))


def gs_project_bwd(ctx, gaussians, cams, settings, grads, v_twist, stream=None):
    _check("gs_project_bwd", load().gs_project_bwd(ctx.handle, ctypes.byref(gaussians),
                                                   ctypes.byref(cams.struct),
                                                   ctypes.byref(settings), ctypes.byref(grads),
                                                   _ptr(v_twist), _stream(stream)))


def gs_l1_loss_grad(ctx, cams, rgb, target, v_rgb, loss, stream=None):
    _check("gs_l1_loss_grad", load().gs_l1_loss_grad(ctx.handle, ctypes.byref(cams.struct),
                                                     _ptr(rgb), _ptr(target), _ptr(v_rgb),
                                                     _ptr(loss), _stream(stream)))


def gs_mcmc_relocate(ctx, params, exp_avg, exp_avg_sq, sh_degree, u, dead_opacity=0.005,
                     src=None, n_relocated=None, stream=None):
    """params / exp_avg / exp_avg_sq: the five planar Gaussian tensors (means,
    log_scales, quats, opacity_logit, sh) and their moments, updated in place;
    u: [N] uniforms in [0, 1) (device)."""
    a = gs_gaussian_adam()
    for q in range(5):
        a.params[q] = _ptr(params[q])
        a.exp_avg[q] = _ptr(exp_avg[q])
        a.exp_avg_sq[q] = _ptr(exp_avg_sq[q])
        a.lr[q] = 0.0
    _check("gs_mcmc_relocate", load().gs_mcmc_relocate(
        ctx.handle, ctypes.byref(a), int(params[3].shape[0]), int(sh_degree), _ptr(u),
        float(dead_opacity), _ptr(src), _ptr(n_relocated), _stream(stream)))


def gs_mcmc_noise(means, log_scales, quats, opacity_logit, eta, scale, k=100.0, t=0.005,
                  stream=None):
    _check("gs_mcmc_noise", load().gs_mcmc_noise(
        _ptr(means), _ptr(log_scales), _ptr(quats), _ptr(opacity_logit), int(means.shape[1]),
        _ptr(eta), float(scale), float(k), float(t), _stream(stream)))


class BundleAdjuster:
    """A gs_ba workspace (one Levenberg-Marquardt step of bundle adjustment)."""

    def __init__(self, max_points, max_cams):
        h = c_vp()
        _check("gs_ba_create", load().gs_ba_create(ctypes.byref(h), int(max_points), int(max_cams)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load().gs_ba_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gs_ba_lm_step(ba, X, viewmat, intr, obs_cam, obs_pt, obs_xy, pt_index, delta, lm_lambda,
                  near_plane, max_iter, tol, d_twist, d_X, stats=None, stream=None):
    """pt_index: from track_point_index, with or without the point-major
    copies (with them the passes over the points read them in order)."""
    pt_off, pt_obs, pm_cam, pm_xy = _index_parts(pt_index)
    _check("gs_ba_lm_step", load().gs_ba_lm_step(
        ba.handle, _ptr(X), int(X.shape[0]), _ptr(viewmat), _ptr(intr), int(viewmat.shape[0]),
        _ptr(obs_cam), _ptr(obs_pt), _ptr(obs_xy), int(obs_cam.shape[0]), _ptr(pt_off),
        _ptr(pt_obs), _ptr(pm_cam), _ptr(pm_xy), float(delta), float(lm_lambda), float(near_plane),
        int(max_iter), float(tol), _ptr(d_twist), _ptr(d_X), _ptr(stats), _stream(stream)))


def gs_init_gaussians(ctx, points, rgb, sh_degree=3, k=4, opacity=0.1, out=None, stream=None):
    """Gaussians from points [n,3] and colours [n,3] (device tensors); returns
    the dict of planar parameter tensors (or fills `out`)."""
    import torch
    n = int(points.shape[0])
    K = (int(sh_degree) + 1) ** 2
    if out is None:
        f = lambda *shape: torch.empty(shape, device=points.device, dtype=torch.float32)
        out = dict(means=f(3, n), log_scales=f(3, n), quats=f(4, n), opacity_logit=f(n),
                   sh=f(K, 3, n))
    _check("gs_init_gaussians", load().gs_init_gaussians(
        ctx.handle, _ptr(points), _ptr(rgb), n, int(k), float(opacity), int(sh_degree),
        _ptr(out["means"]), _ptr(out["log_scales"]), _ptr(out["quats"]),
        _ptr(out["opacity_logit"]), _ptr(out["sh"]), _stream(stream)))
    return out


def gs_photo_loss_grad(ctx, cams, rgb, target, lambda_ssim, v_rgb, loss, stream=None):
    _check("gs_photo_loss_grad", load().gs_photo_loss_grad(
        ctx.handle, ctypes.byref(cams.struct), _ptr(rgb), _ptr(target), float(lambda_ssim),
        _ptr(v_rgb), _ptr(loss), _stream(stream)))


def track_reproj_fwd_bwd(ctx, X, viewmat, intr, obs_cam, obs_pt, obs_xy, delta, lam, near_plane,
                         loss, v_X, v_twist, residual=None, J_pose=None, J_X=None, pt_index=None,
                         stream=None):
    """pt_index: from track_point_index, (pt_off, pt_obs) or (pt_off, pt_obs,
    pm_cam, pm_xy) with the point-major copies; or None."""
    pt_off, pt_obs, pm_cam, pm_xy = _index_parts(pt_index)
    _check("track_reproj_fwd_bwd", load().track_reproj_fwd_bwd(
        ctx.handle, _ptr(X), int(X.shape[0]), _ptr(viewmat), _ptr(intr), int(viewmat.shape[0]),
        _ptr(obs_cam), _ptr(obs_pt), _ptr(obs_xy), int(obs_cam.shape[0]), float(delta),
        float(lam), float(near_plane), _ptr(residual), _ptr(loss), _ptr(v_X), _ptr(v_twist),
        _ptr(J_pose), _ptr(J_X), _ptr(pt_off), _ptr(pt_obs), _ptr(pm_cam), _ptr(pm_xy),
        _stream(stream)))


def _index_parts(pt_index):
    if pt_index is None:
        return None, None, None, None
    if len(pt_index) == 2:
        return pt_index[0], pt_index[1], None, None
    return tuple(pt_index)


def track_reproj_fwd_bwd_noalloc(X, viewmat, intr, obs_cam, obs_pt, obs_xy, delta, lam,
                                 near_plane, loss, v_X, v_twist, residual=None, J_pose=None,
                                 J_X=None, pt_index=None, stream=None):
    """track_reproj_fwd_bwd without a context (the library allocates nothing);
    point-major copies in pt_index are not used."""
    pt_off, pt_obs = _index_parts(pt_index)[:2]
    _check("track_reproj_fwd_bwd_noalloc", load().track_reproj_fwd_bwd_noalloc(
        _ptr(X), int(X.shape[0]), _ptr(viewmat), _ptr(intr), int(viewmat.shape[0]),
        _ptr(obs_cam), _ptr(obs_pt), _ptr(obs_xy), int(obs_cam.shape[0]), float(delta),
        float(lam), float(near_plane), _ptr(residual), _ptr(loss), _ptr(v_X), _ptr(v_twist),
        _ptr(J_pose), _ptr(J_X), _ptr(pt_off), _ptr(pt_obs), _stream(stream)))


def track_point_index(ctx, obs_pt, n_points, obs_cam=None, obs_xy=None, stream=None):
    """The point-major index of the observations (pt_off [Pt + 1], pt_obs [M],
    int32 device tensors) for track_reproj_fwd_bwd's pt_index; with obs_cam and
    obs_xy also their point-major copies (pm_cam [M], pm_xy [M, 2]), returned
    as a 4-tuple."""
    import torch
    M = int(obs_pt.shape[0])
    pt_off = torch.empty(int(n_points) + 1, dtype=torch.int32, device=obs_pt.device)
    pt_obs = torch.empty(max(M, 1), dtype=torch.int32, device=obs_pt.device)
    pm_cam = pm_xy = None
    if obs_cam is not None:
        pm_cam = torch.empty(max(M, 1), dtype=torch.int32, device=obs_pt.device)
        pm_xy = torch.empty((max(M, 1), 2), dtype=torch.float32, device=obs_pt.device)
    _check("track_point_index", load().track_point_index(
        ctx.handle, _ptr(obs_pt), M, int(n_points), _ptr(pt_off), _ptr(pt_obs), _ptr(obs_cam),
        _ptr(obs_xy), _ptr(pm_cam), _ptr(pm_xy), _stream(stream)))
    return (pt_off, pt_obs) if obs_cam is None else (pt_off, pt_obs, pm_cam, pm_xy)


def gs_pose_compose(twist, base, out, stream=None):
    _check("gs_pose_compose", load().gs_pose_compose(int(twist.shape[0]), _ptr(twist), _ptr(base),
                                                     _ptr(out), _stream(stream)))


def gs_pose_compose_bwd(twist, g, out, stream=None):
    _check("gs_pose_compose_bwd", load().gs_pose_compose_bwd(int(twist.shape[0]), _ptr(twist),
                                                             _ptr(g), _ptr(out), _stream(stream)))


def gs_project_bwd_adam(ctx, gaussians, cams, settings, params, exp_avg, exp_avg_sq, lrs, step,
                        v_twist, beta1=0.9, beta2=0.999, eps=1e-15, step_dev=None, stream=None):
    """params / exp_avg / exp_avg_sq: the five Gaussian tensors (means,
    log_scales, quats, opacity_logit, sh) and their moments; lrs: five rates;
    step_dev: an int32 device tensor holding the step number (then `step` is
    ignored)."""
    a = gs_gaussian_adam()
    for q in range(5):
        a.params[q] = _ptr(params[q])
        a.exp_avg[q] = _ptr(exp_avg[q])
        a.exp_avg_sq[q] = _ptr(exp_avg_sq[q])
        a.lr[q] = float(lrs[q])
    _check("gs_project_bwd_adam", load().gs_project_bwd_adam(
        ctx.handle, ctypes.byref(gaussians), ctypes.byref(cams.struct), ctypes.byref(settings),
        ctypes.byref(a), int(step), _ptr(step_dev), float(beta1), float(beta2), float(eps),
        _ptr(v_twist), _stream(stream)))


def gs_adam_step(groups, step, beta1=0.9, beta2=0.999, eps=1e-15, step_dev=None, stream=None):
    """groups: list of (param, grad, exp_avg, exp_avg_sq, lr) tensors/floats;
    step_dev: an int32 device tensor holding the step number (then `step` is
    ignored)."""
    arr = (gs_adam_group * len(groups))()
    for i, (p, g, m, v, lr) in enumerate(groups):
        arr[i] = gs_adam_group(_ptr(p), _ptr(g), _ptr(m), _ptr(v), int(p.numel()), float(lr))
    _check("gs_adam_step", load().gs_adam_step(arr, len(groups), int(step), _ptr(step_dev),
                                               float(beta1), float(beta2), float(eps),
                                               _stream(stream)))


def gs_step_advance(step_dev, stream=None):
    """step_dev (int32 device tensor) += 1 on the device."""
    _check("gs_step_advance", load().gs_step_advance(_ptr(step_dev), _stream(stream)))
