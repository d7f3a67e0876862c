"""FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow definitions of what the splatting hot path computes (see
``oracle.c`` for the formulas and the passages of GloSplat they follow).  Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the product path never does.  It shares
no code with the HIP library.

``build()`` compiles ``oracle.c`` with gcc into ``liboracle.so`` next to it.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Default settings (see oracle.h): near, eps2d, frustum pad, alpha_min,
# alpha_max, T_min, and the ambiguity bands used by the parity rule.
CFG_DEFAULT = dict(near=0.01, eps2d=0.3, pad=0.3, alpha_min=1.0 / 255.0,
                   alpha_max=0.99, t_min=1e-4, band_pos=2.4e-7, band_t=2e-4,
                   band_sig=2e-5, band_mid=1e-12)
_CFG_ORDER = ["near", "eps2d", "pad", "alpha_min", "alpha_max", "t_min",
              "band_pos", "band_t", "band_sig", "band_mid"]

_lib = None


def build_sanitized(path):
    """The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (every report fatal) into `path`; loaded instead of the plain build when
    the ORACLE_LIB environment variable names it (with libasan preloaded)."""
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-Wall", "-Wno-unknown-pragmas",
                           "-o", path, _SRC, "-lm"])
    return path


def build(force=True):
    """Compile the oracle (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        alt = os.environ.get("ORACLE_LIB")
        if alt:
            _lib = ctypes.CDLL(alt)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            _lib = ctypes.CDLL(_LIB)
        _lib.or_bin_sort.restype = ctypes.c_longlong
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def cfg_array(**over):
    c = dict(CFG_DEFAULT)
    c.update(over)
    return np.array([c[k] for k in _CFG_ORDER], dtype=np.float64)


def num_threads():
    return _load().or_num_threads()


def set_num_threads(n):
    """Threads of the oracle's parallel loops from now on (timing runs)."""
    _load().or_set_num_threads(int(n))


def project(scene, viewmat=None, intr=None, wh=None, **cfg):
    """Per-(view, Gaussian) projection.  Returns a dict of [V*N, ...] arrays."""
    lib = _load()
    viewmat = _f64(scene["viewmat"] if viewmat is None else viewmat)
    intr = _f64(scene["intr"] if intr is None else intr)
    wh = _i32(scene["wh"] if wh is None else wh)
    N = scene["means"].shape[1]
    V = viewmat.shape[0]
    VN = V * N
    out = dict(valid=np.zeros(VN, np.int32), depth=np.zeros(VN), mean2d=np.zeros((VN, 2)),
               cov2d=np.zeros((VN, 3)), conic=np.zeros((VN, 3)), opacity=np.zeros(VN),
               rgb=np.zeros((VN, 3)), ext=np.zeros((VN, 2)))
    rc = lib.or_project(
        ctypes.c_int(N), ctypes.c_int(int(scene["sh_degree"])),
        _p(_f64(scene["means"])), _p(_f64(scene["log_scales"])), _p(_f64(scene["quats"])),
        _p(_f64(scene["opacity_logit"])), _p(_f64(scene["sh"])),
        ctypes.c_int(V), _p(viewmat), _p(intr), _p(wh), _p(cfg_array(**cfg)),
        _p(out["valid"]), _p(out["depth"]), _p(out["mean2d"]), _p(out["cov2d"]),
        _p(out["conic"]), _p(out["opacity"]), _p(out["rgb"]), _p(out["ext"]))
    if rc != 0:
        raise ValueError("or_project failed")
    return out


def render(proj, wh, bg=None, pix=None, v_rgb=None, **cfg):
    """Brute-force compositing.  Returns a dict with rgb [n,3], T [n],
    ncontrib [n], ngate [n], nclamp [n], ambiguous [n] and v2d [V*N,9] (None
    without v_rgb)."""
    lib = _load()
    wh = _i32(wh)
    V = wh.shape[0]
    VN = proj["valid"].shape[0]
    N = VN // V
    P = int(np.sum(wh[:, 0].astype(np.int64) * wh[:, 1]))
    if pix is not None:
        pix = np.ascontiguousarray(pix, dtype=np.int64)
        n = pix.shape[0]
    else:
        n = P
    rgb = np.zeros((n, 3))
    T = np.zeros(n)
    nc = np.zeros(n, np.int32)
    ng = np.zeros(n, np.int32)
    ncl = np.zeros(n, np.int32)
    amb = np.zeros(n, np.int32)
    v2d = np.zeros((VN, 9)) if v_rgb is not None else None
    bga = None if bg is None else _f64(bg)
    rc = lib.or_render(
        ctypes.c_int(V), _p(wh), ctypes.c_int(N), _p(_i32(proj["valid"])), _p(_f64(proj["depth"])),
        _p(_f64(proj["mean2d"])), _p(_f64(proj["conic"])), _p(_f64(proj["opacity"])),
        _p(_f64(proj["rgb"])), _p(bga), _p(cfg_array(**cfg)),
        ctypes.c_longlong(n), _p(pix), _p(rgb), _p(T), _p(nc), _p(ng), _p(ncl), _p(amb),
        _p(None if v_rgb is None else _f64(v_rgb)), _p(v2d))
    if rc != 0:
        raise ValueError("or_render failed")
    return dict(rgb=rgb, T=T, ncontrib=nc, ngate=ng, nclamp=ncl, ambiguous=amb.astype(bool),
                v2d=v2d)


def project_bwd(scene, v2d, viewmat=None, intr=None, wh=None, **cfg):
    """Chain the per-pair 2D gradients to the parameters and view twists."""
    lib = _load()
    viewmat = _f64(scene["viewmat"] if viewmat is None else viewmat)
    intr = _f64(scene["intr"] if intr is None else intr)
    wh = _i32(scene["wh"] if wh is None else wh)
    N = scene["means"].shape[1]
    V = viewmat.shape[0]
    K = (int(scene["sh_degree"]) + 1) ** 2
    g = dict(means=np.zeros((3, N)), log_scales=np.zeros((3, N)), quats=np.zeros((4, N)),
             opacity_logit=np.zeros(N), sh=np.zeros((K, 3, N)), twist=np.zeros((V, 6)))
    rc = lib.or_project_bwd(
        ctypes.c_int(N), ctypes.c_int(int(scene["sh_degree"])),
        _p(_f64(scene["means"])), _p(_f64(scene["log_scales"])), _p(_f64(scene["quats"])),
        _p(_f64(scene["opacity_logit"])), _p(_f64(scene["sh"])),
        ctypes.c_int(V), _p(viewmat), _p(intr), _p(wh), _p(cfg_array(**cfg)), _p(_f64(v2d)),
        _p(g["means"]), _p(g["log_scales"]), _p(g["quats"]), _p(g["opacity_logit"]),
        _p(g["sh"]), _p(g["twist"]))
    if rc != 0:
        raise ValueError("or_project_bwd failed")
    return g


def render_fwd_bwd(scene, v_rgb=None, pix=None, bg=None, viewmat=None, **cfg):
    """Projection + compositing (+ backward when v_rgb is given)."""
    proj = project(scene, viewmat=viewmat, **cfg)
    out = render(proj, scene["wh"], bg=bg, pix=pix, v_rgb=v_rgb, **cfg)
    out["proj"] = proj
    if v_rgb is not None:
        out["grads"] = project_bwd(scene, out["v2d"], viewmat=viewmat, **cfg)
    return out


def track(X, viewmat, intr, obs_cam, obs_pt, obs_xy, delta=1.0, lam=1e-4, near=0.01,
          jacobians=True):
    lib = _load()
    X = _f64(X)
    viewmat = _f64(viewmat)
    Pt = X.shape[0]
    ncam = viewmat.shape[0]
    M = obs_cam.shape[0]
    out = dict(residual=np.zeros((M, 2)), loss=np.zeros(1), v_X=np.zeros((Pt, 3)),
               v_twist=np.zeros((ncam, 6)), masked=np.zeros(M, np.int32))
    if jacobians:
        out["J_pose"] = np.zeros((M, 2, 6))
        out["J_X"] = np.zeros((M, 2, 3))
    rc = lib.or_track(
        ctypes.c_int(Pt), _p(X), ctypes.c_int(ncam), _p(viewmat), _p(_f64(intr)),
        ctypes.c_int(M), _p(_i32(obs_cam)), _p(_i32(obs_pt)), _p(_f64(obs_xy)),
        ctypes.c_double(delta), ctypes.c_double(lam), ctypes.c_double(near),
        _p(out["residual"]), _p(out["loss"]), _p(out["v_X"]), _p(out["v_twist"]),
        _p(out.get("J_pose")), _p(out.get("J_X")), _p(out["masked"]))
    if rc != 0:
        raise ValueError("or_track failed")
    out["loss"] = float(out["loss"][0])
    return out


def se3_exp_compose(xi, base):
    lib = _load()
    xi = _f64(xi).reshape(-1, 6)
    base = _f64(base).reshape(-1, 12)
    out = np.zeros_like(base)
    lib.or_se3_exp_compose(ctypes.c_int(xi.shape[0]), _p(xi), _p(base), _p(out))
    return out


def se3_jl_transpose(xi, g):
    lib = _load()
    xi = _f64(xi).reshape(-1, 6)
    g = _f64(g).reshape(-1, 6)
    out = np.zeros_like(g)
    lib.or_se3_jl_transpose(ctypes.c_int(xi.shape[0]), _p(xi), _p(g), _p(out))
    return out


def adam(p, g, m, v, lr, beta1=0.9, beta2=0.999, eps=1e-15, step=1):
    """In-place Adam on float64 arrays."""
    lib = _load()
    for a in (p, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib.or_adam(ctypes.c_longlong(p.size), _p(p), _p(g), _p(m), _p(v), ctypes.c_double(lr),
                ctypes.c_double(beta1), ctypes.c_double(beta2), ctypes.c_double(eps),
                ctypes.c_int(step))


def sh_basis(deg, d, grad=False):
    lib = _load()
    K = (deg + 1) ** 2
    d = _f64(d)
    Y = np.zeros(K)
    dY = np.zeros((K, 3)) if grad else None
    lib.or_sh_basis(ctypes.c_int(deg), _p(d), _p(Y), _p(dY))
    return (Y, dY) if grad else Y


def l1(rgb, target, wh):
    """Photometric L1 term and its image gradient: (loss, v_rgb [P,3])."""
    lib = _load()
    wh = _i32(wh)
    rgb, target = _f64(rgb), _f64(target)
    v = np.zeros(rgb.shape)
    loss = np.zeros(1)
    if lib.or_l1(ctypes.c_int(wh.shape[0]), _p(wh), _p(rgb), _p(target), _p(loss), _p(v)) != 0:
        raise ValueError("or_l1 failed")
    return float(loss[0]), v


# SSIM window and constants (Wang et al. 2004 defaults for data in [0, 1])
SSIM_WIN, SSIM_SIGMA, SSIM_C1, SSIM_C2 = 11, 1.5, 0.01 ** 2, 0.03 ** 2


def ssim(rgb, target, wh, grad=True, ssim_map=False, win=SSIM_WIN, sigma=SSIM_SIGMA,
         c1=SSIM_C1, c2=SSIM_C2):
    """Mean SSIM over views (each the mean over its pixels and channels).
    Returns (ssim, v_rgb [P,3] or None, map [P,3] or None)."""
    lib = _load()
    wh = _i32(wh)
    rgb, target = _f64(rgb), _f64(target)
    v = np.zeros(rgb.shape) if grad else None
    m = np.zeros(rgb.shape) if ssim_map else None
    s = np.zeros(1)
    rc = lib.or_ssim(ctypes.c_int(wh.shape[0]), _p(wh), _p(rgb), _p(target), ctypes.c_int(win),
                     ctypes.c_double(sigma), ctypes.c_double(c1), ctypes.c_double(c2), _p(s),
                     _p(m), _p(v))
    if rc != 0:
        raise ValueError("or_ssim failed")
    return float(s[0]), v, m


def photo_loss(rgb, target, wh, lam=0.2):
    """L_photo = (1 - lam) L1 + lam (1 - SSIM) and its image gradient."""
    l, vl = l1(rgb, target, wh)
    s, vs, _ = ssim(rgb, target, wh)
    return (1 - lam) * l + lam * (1 - s), (1 - lam) * vl - lam * vs


def knn_mean_dist(points, k=4, queries=None):
    """Mean distance of each point (or of the points `queries` index) to its k
    nearest other points (brute force)."""
    lib = _load()
    pts = _f64(points).reshape(-1, 3)
    q = None if queries is None else np.ascontiguousarray(queries, dtype=np.int64)
    nq = pts.shape[0] if q is None else q.shape[0]
    out = np.zeros(nq)
    if lib.or_knn_mean_dist(ctypes.c_longlong(pts.shape[0]), _p(pts), ctypes.c_int(k),
                            ctypes.c_longlong(nq), _p(q), _p(out)) != 0:
        raise ValueError("or_knn_mean_dist failed")
    return out


def init_gaussians(points, rgb, sh_degree=3, k=4, opacity=0.1, s_min=1e-7):
    """Gaussians from SfM points (planar layout, float64)."""
    lib = _load()
    pts = _f64(points).reshape(-1, 3)
    n = pts.shape[0]
    K = (sh_degree + 1) ** 2
    out = dict(means=np.zeros((3, n)), log_scales=np.zeros((3, n)), quats=np.zeros((4, n)),
               opacity_logit=np.zeros(n), sh=np.zeros((K, 3, n)))
    rc = lib.or_init_gaussians(ctypes.c_longlong(n), _p(pts), _p(_f64(rgb).reshape(-1, 3)),
                               ctypes.c_int(k), ctypes.c_double(opacity), ctypes.c_double(s_min),
                               ctypes.c_int(sh_degree), _p(out["means"]), _p(out["log_scales"]),
                               _p(out["quats"]), _p(out["opacity_logit"]), _p(out["sh"]))
    if rc != 0:
        raise ValueError("or_init_gaussians failed")
    return out


def ba_normal(X, viewmat, intr, obs_cam, obs_pt, obs_xy, delta=1.0, near=0.01):
    """Dense Gauss-Newton normal equations of the Huber BA cost: (H, g, cost,
    masked), unknowns ordered cameras (6 each) then points (3 each)."""
    lib = _load()
    X = _f64(X).reshape(-1, 3)
    viewmat = _f64(viewmat).reshape(-1, 12)
    n = 6 * viewmat.shape[0] + 3 * X.shape[0]
    H = np.zeros((n, n))
    g = np.zeros(n)
    cost = np.zeros(1)
    m = lib.or_ba_normal(ctypes.c_int(X.shape[0]), _p(X), ctypes.c_int(viewmat.shape[0]), _p(viewmat),
                         _p(_f64(intr)), ctypes.c_int(len(obs_cam)), _p(_i32(obs_cam)), _p(_i32(obs_pt)),
                         _p(_f64(obs_xy)), ctypes.c_double(delta), ctypes.c_double(near), _p(H),
                         _p(g), _p(cost))
    if m < 0:
        raise ValueError("or_ba_normal failed")
    return H, g, float(cost[0]), m


def ba_step(X, viewmat, intr, obs_cam, obs_pt, obs_xy, delta=1.0, lm_lambda=1e-3, near=0.01):
    """One LM step: d solves (H + lambda diag(H)) d = -g over the unknowns with a
    non-zero diagonal (the others stay 0).  Returns (d_twist [ncam,6],
    d_X [Pt,3], cost).  The solve is LAPACK's (numpy)."""
    H, g, cost, _ = ba_normal(X, viewmat, intr, obs_cam, obs_pt, obs_xy, delta, near)
    A = H + lm_lambda * np.diag(np.diag(H))
    live = np.diag(H) > 0
    d = np.zeros_like(g)
    d[live] = np.linalg.solve(A[np.ix_(live, live)], -g[live])
    nc = np.asarray(viewmat).reshape(-1, 12).shape[0]
    return d[:6 * nc].reshape(nc, 6), d[6 * nc:].reshape(-1, 3), cost


def ba_normal_residual(X, viewmat, intr, obs_cam, obs_pt, obs_xy, d_twist, d_X, delta=1.0,
                       lm_lambda=1e-3, near=0.01):
    """(H + lambda diag(H)) d + g for d = (d_twist, d_X), per observation (any
    size); returns (cameras part [ncam,6], points part [Pt,3])."""
    lib = _load()
    X = _f64(X).reshape(-1, 3)
    viewmat = _f64(viewmat).reshape(-1, 12)
    nc = viewmat.shape[0]
    d = np.concatenate([_f64(d_twist).reshape(-1), _f64(d_X).reshape(-1)])
    out = np.zeros_like(d)
    rc = lib.or_ba_normal_residual(ctypes.c_int(X.shape[0]), _p(X), ctypes.c_int(nc), _p(viewmat),
                                   _p(_f64(intr)), ctypes.c_int(len(obs_cam)), _p(_i32(obs_cam)),
                                   _p(_i32(obs_pt)), _p(_f64(obs_xy)), ctypes.c_double(delta),
                                   ctypes.c_double(near), ctypes.c_double(lm_lambda), _p(d), _p(out))
    if rc != 0:
        raise ValueError("or_ba_normal_residual failed")
    return out[:6 * nc].reshape(nc, 6), out[6 * nc:].reshape(-1, 3)


def mcmc_relocate(g, moments, u, sh_degree, t_dead=0.005):
    """MCMC relocation on float64 copies: g = dict of the five planar arrays,
    moments = (exp_avg dict, exp_avg_sq dict) in the same layout, u [N].
    Returns (new g, new moments, src [N], n_relocated)."""
    lib = _load()
    keys = ("means", "log_scales", "quats", "opacity_logit", "sh")
    G = {k: np.array(g[k], dtype=np.float64, copy=True, order="C") for k in keys}
    M1 = {k: np.array(moments[0][k], dtype=np.float64, copy=True, order="C") for k in keys}
    M2 = {k: np.array(moments[1][k], dtype=np.float64, copy=True, order="C") for k in keys}
    N = G["opacity_logit"].shape[0]
    src = np.zeros(N, np.int64)
    nrel = ctypes.c_longlong()
    arr1 = (ctypes.c_void_p * 5)(*[M1[k].ctypes.data for k in keys])
    arr2 = (ctypes.c_void_p * 5)(*[M2[k].ctypes.data for k in keys])
    rc = lib.or_mcmc_relocate(ctypes.c_longlong(N), ctypes.c_int(sh_degree), _p(G["means"]),
                              _p(G["log_scales"]), _p(G["quats"]), _p(G["opacity_logit"]),
                              _p(G["sh"]), arr1, arr2, _p(_f64(u)), ctypes.c_double(t_dead),
                              _p(src), ctypes.byref(nrel))
    if rc != 0:
        raise ValueError("or_mcmc_relocate failed")
    return G, (M1, M2), src, int(nrel.value)


def mcmc_noise(g, eta, scale, k=100.0, t=0.005):
    """Means after the MCMC noise step (float64 copy)."""
    lib = _load()
    means = np.array(g["means"], dtype=np.float64, copy=True, order="C")
    N = means.shape[1]
    lib.or_mcmc_noise(ctypes.c_longlong(N), _p(means), _p(_f64(g["log_scales"])),
                      _p(_f64(g["quats"])), _p(_f64(g["opacity_logit"])), _p(_f64(eta)),
                      ctypes.c_double(scale), ctypes.c_double(k), ctypes.c_double(t))
    return means


def bin_sort(wh, tile, valid, mean2d, conic, opacity, depth, alpha_min=1.0 / 255.0,
             margin=0.0, with_masks=False):
    """Tile lists ordered by (float32 depth bits, pair index).  Returns
    (ranges [T_total,2] int64, ids [I] int32) and, with_masks, the quadrant
    masks [I] int32."""
    lib = _load()
    wh = _i32(wh)
    V = wh.shape[0]
    VN = valid.shape[0]
    N = VN // V
    tw, th = tile
    T_total = int(sum(((w + tw - 1) // tw) * ((h + th - 1) // th) for w, h in wh))
    ranges = np.zeros((T_total, 2), np.int64)
    args = [ctypes.c_int(V), _p(wh), ctypes.c_int(tw), ctypes.c_int(th), ctypes.c_int(N),
            _p(_i32(valid)), _p(_f32(mean2d)), _p(_f32(conic)), _p(_f32(opacity)),
            _p(_f32(depth)), ctypes.c_double(alpha_min), ctypes.c_double(margin)]
    n = lib.or_bin_sort(*args, ctypes.c_longlong(0), _p(ranges), None, None)
    need = -n if n < 0 else n
    ids = np.zeros(max(need, 1), np.int32)
    masks = np.zeros(max(need, 1), np.int32)
    n = lib.or_bin_sort(*args, ctypes.c_longlong(need), _p(ranges), _p(ids), _p(masks))
    if with_masks:
        return ranges, ids[:need], masks[:need]
    return ranges, ids[:need]
