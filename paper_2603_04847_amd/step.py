"""One joint pose-appearance step (GloSplat Algorithm 1, one iteration) through
the C ABI, without Python-side arithmetic:

  a1  compose every pose T_i = Exp(dT_i) T_i^(0)           gs_pose_compose
  a2  project the Gaussians into the sampled views          gs_project
  a3+a4 bin and key-sort the tile intersections             gs_bin_sort
  a5  front-to-back composite                               gs_render_fwd
  a6  photometric loss (1 - l) L1 + l (1 - SSIM), l = 0.2,  gs_photo_loss_grad
      and its image gradient (l = 0: L1 alone,               (gs_l1_loss_grad)
      gs_l1_loss_grad)
  a7  raster backward (2D gradients)                        gs_raster_bwd
  a8  chain to Gaussian parameters + per-view twists        gs_project_bwd
  a9  track reprojection Huber loss, grads to X and twists  track_reproj_fwd_bwd
      (the same twist buffer: poses get both gradients)
  a1' twist gradient through the composition                gs_pose_compose_bwd
  a10 Adam on Gaussians, poses and track points             gs_adam_step
      (in `run`, the Gaussians' Adam step is taken inside the projection
      backward, gs_project_bwd_adam, so their gradients never reach memory)

Learning rates follow Sec. 3.3 "Implementation" and the pose rate of Sec. 3.3;
the track-point rate (not given in the paper) is the position rate.
"""

from __future__ import annotations

import numpy as np
import torch

from . import _lib as L

PARAM_KEYS = ("means", "log_scales", "quats", "opacity_logit", "sh")


def learning_rates(extent):
    return dict(means=1.6e-4 * extent, log_scales=5e-3, quats=1e-3, opacity_logit=5e-2,
                sh=2.5e-3, twist=1e-5, X=1.6e-4 * extent)


class JointStep:
    """State and buffers of the joint step; `run(b)` executes one iteration on
    batch b (views batches[b]); every buffer is allocated up front so a run
    can be captured in a HIP graph."""

    def __init__(self, scene, batches, targets, device="cuda", settings=None, max_isect=None,
                 lam=1e-4, delta=1.0, extent=None, lambda_ssim=0.2, lazy_lists=True,
                 overlap_track=True):
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device, torch.float32)
        self.sh_degree = int(scene["sh_degree"])
        self.params = {k: f(scene[k]) for k in PARAM_KEYS}
        self.N = self.params["means"].shape[1]
        self.base = f(scene["viewmat"])
        self.intr = f(scene["intr"])
        self.wh_all = np.asarray(scene["wh"], np.int32)
        self.n_cams = self.base.shape[0]
        self.twist = torch.zeros((self.n_cams, 6), device=device)
        self.viewmat = torch.empty_like(self.base)
        self.X = f(scene["X"])
        self.obs_cam = torch.from_numpy(scene["obs_cam"]).to(device, torch.int32)
        self.obs_pt = torch.from_numpy(scene["obs_pt"]).to(device, torch.int32)
        self.obs_xy = f(scene["obs_xy"])
        self.batches = [np.asarray(b, np.int32) for b in batches]
        self.targets = [f(t) for t in targets]
        self.settings = settings if settings is not None else L.default_settings()
        # the step never reads the tile lists itself: by default the forward
        # writes only the part of each list it reads (gs_settings.lazy_lists)
        self.lazy_lists = bool(lazy_lists)
        # without a timer, the track term runs on a second stream beside the
        # projection, binning and raster (it shares none of their buffers; it
        # joins before the projection backward adds its twist rows).  Timed
        # calls run in order, one at a time.
        self.overlap_track = bool(overlap_track)
        self._side = torch.cuda.Stream(device=device) if overlap_track else None
        self.lam, self.delta = lam, delta
        self.lambda_ssim = float(lambda_ssim)
        if extent is None:
            c = np.stack([-(np.asarray(scene["viewmat"][i]).reshape(3, 4)[:, :3].T
                            @ np.asarray(scene["viewmat"][i]).reshape(3, 4)[:, 3])
                          for i in range(self.n_cams)])
            extent = 1.1 * float(np.max(np.linalg.norm(c - c.mean(0), axis=1)))
        self.lr = learning_rates(extent)
        Vb = max(len(b) for b in self.batches)
        P = max(int(sum(int(self.wh_all[v, 0]) * int(self.wh_all[v, 1]) for v in b))
                for b in self.batches)
        tiles = max(int(sum(((self.wh_all[v, 0] + 15) // 16) * ((self.wh_all[v, 1] + 15) // 16)
                            for v in b)) for b in self.batches)
        tiles = max(tiles, 4 * tiles)  # room for the smallest tile shape
        self._cap = dict(max_pairs=Vb * self.N, max_tiles=tiles, max_views=Vb,
                         max_cams=self.n_cams)
        self.ctx = L.Context(max_isect=max_isect or 32 * P, **self._cap)
        # the observations' point-major index and copies (fixed for the scene):
        # the track term is then one in-order pass over the points without
        # atomics; a context too small to build it keeps the atomic path
        try:
            self.pt_index = L.track_point_index(self.ctx, self.obs_pt, int(self.X.shape[0]),
                                                self.obs_cam, self.obs_xy)
        except L.GsError as e:
            if e.code != L.GS_ERR_CAPACITY:
                raise
            self.pt_index = None
        self.rgb = torch.empty((P, 3), device=device)
        self.T = torch.empty((P,), device=device)
        self.last = torch.empty((P,), device=device, dtype=torch.int32)
        self.v_rgb = torch.empty((P, 3), device=device)
        # the per-step accumulators (the point gradient, this step's twist
        # gradient, the losses) share one buffer, so one fill clears them all;
        # v_X leads, 16-byte aligned for the vector Adam path
        n_tw, n_x = self.twist.numel(), self.X.numel()
        o_tw = (n_x + 3) // 4 * 4
        self._acc = torch.zeros(o_tw + n_tw + 2, device=device)
        self.v_X = self._acc[:n_x].view_as(self.X)
        self.v_tw_cur = self._acc[o_tw:o_tw + n_tw].view_as(self.twist)
        self.loss = self._acc[o_tw + n_tw:]
        self.grads = {k: torch.empty_like(v) for k, v in self.params.items()}
        self.v_tw = torch.zeros_like(self.twist)
        self.m = {k: torch.zeros_like(v) for k, v in self._opt_params().items()}
        self.v = {k: torch.zeros_like(v) for k, v in self._opt_params().items()}
        self.step_count = 0
        # the Adam step number on the device: `run` advances it in a kernel and
        # the Adam kernels read it, so a captured step replays as successive
        # steps (1 / (1 - beta^t) changes every replay)
        self.d_step = torch.zeros(1, device=device, dtype=torch.int32)
        self.cams = [L.Cameras(self.viewmat, self.intr, self.wh_all[b], index=b) for b in self.batches]
        self.g = L.make_gaussians(*(self.params[k] for k in PARAM_KEYS), self.sh_degree)
        self.gg = L.make_grads(*(self.grads[k] for k in PARAM_KEYS))

    def set_capacity(self, max_isect):
        """Re-create the context with room for `max_isect` tile intersections."""
        self.ctx.close()
        self.ctx = L.Context(max_isect=int(max_isect), **self._cap)

    def _opt_params(self):
        d = dict(self.params)
        d["twist"] = self.twist
        d["X"] = self.X
        return d

    def _opt_grads(self):
        d = dict(self.grads)
        d["twist"] = self.v_tw
        d["X"] = self.v_X
        return d

    def forward_backward(self, b, timer=None, adam_step=None, step_dev=None):
        """a1-a9 and the twist chain, for batch b.  `timer(name)` brackets calls.
        With `adam_step` (the Adam step number t, or 0 with `step_dev` the
        device counter holding it), the projection backward also takes the
        Gaussians' Adam step and self.grads is left untouched."""
        t = timer or (lambda name: _Null())
        cams = self.cams[b]
        P = cams.n_pixels
        s = self.settings
        s.lazy_lists = int(self.lazy_lists)
        with t("pose_compose"):
            L.gs_pose_compose(self.twist, self.base, self.viewmat)
        side = self._side if (self.overlap_track and timer is None) else None
        if side is not None:
            self._acc.zero_()  # v_X, v_tw_cur, loss
            main = torch.cuda.current_stream()
            side.wait_stream(main)
            with torch.cuda.stream(side):
                L.track_reproj_fwd_bwd(self.ctx, self.X, self.viewmat, self.intr, self.obs_cam,
                                       self.obs_pt, self.obs_xy, self.delta, self.lam, 0.01,
                                       self.loss[1:2], self.v_X, self.v_tw_cur, pt_index=self.pt_index,
                                       stream=side)
        with t("project"):
            L.gs_project(self.ctx, self.g, cams, s)
        with t("bin_sort"):
            L.gs_bin_sort(self.ctx, cams, self.N, s)
        with t("render_fwd"):
            L.gs_render_fwd(self.ctx, cams, s, None, self.rgb, self.T, self.last)
        if side is None:
            self._acc.zero_()  # v_X, v_tw_cur, loss
        if self.lambda_ssim > 0:
            with t("photo"):
                L.gs_photo_loss_grad(self.ctx, cams, self.rgb, self.targets[b], self.lambda_ssim,
                                     self.v_rgb, self.loss[0:1])
        else:
            with t("l1"):
                L.gs_l1_loss_grad(self.ctx, cams, self.rgb, self.targets[b], self.v_rgb,
                                  self.loss[0:1])
        with t("raster_bwd"):
            L.gs_raster_bwd(self.ctx, cams, s, None, self.T, self.last, self.v_rgb)
        if side is not None:
            torch.cuda.current_stream().wait_stream(side)
        if adam_step is None and step_dev is None:
            with t("project_bwd"):
                L.gs_project_bwd(self.ctx, self.g, cams, s, self.gg, self.v_tw_cur)
        else:
            with t("project_bwd_adam"):
                L.gs_project_bwd_adam(self.ctx, self.g, cams, s,
                                      [self.params[k] for k in PARAM_KEYS],
                                      [self.m[k] for k in PARAM_KEYS],
                                      [self.v[k] for k in PARAM_KEYS],
                                      [self.lr[k] for k in PARAM_KEYS], adam_step, self.v_tw_cur,
                                      step_dev=step_dev)
        if side is None:
            with t("track"):
                L.track_reproj_fwd_bwd(self.ctx, self.X, self.viewmat, self.intr, self.obs_cam,
                                       self.obs_pt, self.obs_xy, self.delta, self.lam, 0.01,
                                       self.loss[1:2], self.v_X, self.v_tw_cur, pt_index=self.pt_index)
        with t("pose_compose_bwd"):
            L.gs_pose_compose_bwd(self.twist, self.v_tw_cur, self.v_tw)
        del P

    def save_state(self, path):
        """Checkpoint to an .npz file: every optimised array (the Gaussians,
        the camera twists, the track points), its two Adam moments, the base
        poses and both step counters (host and device).  Plain arrays only,
        nothing pickled."""
        arrs = {}
        for k, v in self._opt_params().items():
            arrs["param/" + k] = v.detach().cpu().numpy()
            arrs["m/" + k] = self.m[k].cpu().numpy()
            arrs["v/" + k] = self.v[k].cpu().numpy()
        arrs["base_viewmat"] = self.base.cpu().numpy()
        arrs["sh_degree"] = np.array([self.sh_degree], np.int64)
        arrs["step"] = np.array([self.step_count, int(self.d_step.item())], np.int64)
        np.savez(path, **arrs)

    def load_state(self, path):
        """Restore a checkpoint written by save_state into this step's arrays,
        in place (captured graphs keep pointing at them).  Shapes must match."""
        with np.load(path, allow_pickle=False) as z:
            if int(z["sh_degree"][0]) != self.sh_degree:
                raise ValueError("checkpoint has another SH degree")
            for k, v in self._opt_params().items():
                for name, dst in (("param/", v), ("m/", self.m[k]), ("v/", self.v[k])):
                    a = z[name + k]
                    if tuple(a.shape) != tuple(dst.shape):
                        raise ValueError(f"checkpoint {name}{k} has shape {a.shape}, not {tuple(dst.shape)}")
                    dst.copy_(torch.from_numpy(a))
            self.base.copy_(torch.from_numpy(z["base_viewmat"]))
            host, dev = (int(x) for x in z["step"])
        self.d_step.fill_(dev)
        self.step_count = host

    def set_step(self, n):
        """Set the device step counter (the next `run` takes step n + 1)."""
        self.d_step.fill_(int(n))
        self.step_count = int(n)

    def adam(self, timer=None, step=None, keys=None, step_dev=None):
        """Adam on the groups `keys` (default: all) from their gradients, at
        step `step`, or at the step the device counter `step_dev` holds."""
        t = timer or (lambda name: _Null())
        if step is None and step_dev is None:
            self.step_count += 1
            step = self.step_count
        p, g = self._opt_params(), self._opt_grads()
        groups = [(p[k], g[k], self.m[k], self.v[k], self.lr[k]) for k in (keys or p)]
        with t("adam"):
            L.gs_adam_step(groups, step or 0, step_dev=step_dev)

    def run(self, b, timer=None, step=None):
        """One iteration: forward, backward with the Gaussians' Adam step fused
        into the projection backward, then Adam on the twists and track points.
        Without `step` the device counter is advanced first and every Adam
        kernel reads it (the form a captured graph replays); with `step` that
        step number is used and the counter is left alone."""
        if step is None:
            L.gs_step_advance(self.d_step)
            self.step_count += 1
            self.forward_backward(b, timer, adam_step=0, step_dev=self.d_step)
            self.adam(timer, keys=("twist", "X"), step_dev=self.d_step)
        else:
            self.forward_backward(b, timer, adam_step=step)
            self.adam(timer, step, keys=("twist", "X"))


class _Null:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False
