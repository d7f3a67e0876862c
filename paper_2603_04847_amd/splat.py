"""Orchestration of the C-ABI calls for one rendering pass, and the autograd
Functions wrapping them.

Everything here marshals arguments: the arithmetic of every step runs in the
HIP kernels of ``libgs_hip.so``.  torch is used for device memory and streams.

* ``Splatter`` -- project + bin/sort + forward composite, and the backward,
  for one batch of views (GloSplat Algorithm 1, render step and backward).
* ``RasterizeGaussians`` -- torch.autograd.Function: (Gaussian parameters,
  per-view twist dT, base poses T0) -> images; the pose is composed as
  Exp(dT) T0 inside the kernels (Algorithm 1, pose adjustment).
* ``TrackReprojection`` -- torch.autograd.Function: (track points X, twist,
  base poses) -> lambda * sum Huber(|pi(X) - x|^2) (Sec. 3.3 eq. L_BA^joint).
  Both Functions return d/d twist, so autograd adds the photometric and the
  reprojection gradients of each pose (the dual gradient flow of Algorithm 1).
"""

from __future__ import annotations

import numpy as np
import torch

from . import _lib as L

PARAM_KEYS = ("means", "log_scales", "quats", "opacity_logit", "sh")


def _dev(t, dtype=torch.float32):
    return t.contiguous() if t.dtype == dtype else t.to(dtype).contiguous()


class Splatter:
    """One rendering pass over a batch of views through the C ABI."""

    def __init__(self, ctx: L.Context, settings=None, bg=None):
        self.ctx = ctx
        # without settings of the caller's, the tile lists are left to the
        # forward (gs_settings.lazy_lists): nothing here reads them
        self.settings = settings if settings is not None else L.default_settings(lazy_lists=1)
        self.bg = bg

    def forward(self, params, sh_degree, viewmat, intr, wh, stream=None):
        """params: dict of device tensors (planar layouts); viewmat [V,12], intr [V,4]
        device; wh [V,2] host.  Returns (rgb [P,3], T_final [P], last [P], cams)."""
        cams = L.Cameras(_dev(viewmat), _dev(intr), wh)
        g = L.make_gaussians(*(params[k] for k in PARAM_KEYS), sh_degree)
        dev = viewmat.device
        P = cams.n_pixels
        rgb = torch.empty((P, 3), device=dev, dtype=torch.float32)
        T = torch.empty((P,), device=dev, dtype=torch.float32)
        last = torch.empty((P,), device=dev, dtype=torch.int32)
        L.gs_project(self.ctx, g, cams, self.settings, stream)
        L.gs_bin_sort(self.ctx, cams, g.N, self.settings, None, stream)
        L.gs_render_fwd(self.ctx, cams, self.settings, self.bg, rgb, T, last, stream)
        return rgb, T, last, cams

    def rebin(self, params, sh_degree, cams, stream=None):
        """Project and bin again (the records and lists a later forward on the
        same context replaced); deterministic, so they equal the forward's."""
        g = L.make_gaussians(*(params[k] for k in PARAM_KEYS), sh_degree)
        L.gs_project(self.ctx, g, cams, self.settings, stream)
        L.gs_bin_sort(self.ctx, cams, g.N, self.settings, None, stream)

    def backward(self, params, sh_degree, cams, T, last, v_rgb, v_twist=None, grads=None,
                 stream=None):
        """Gradients of the last forward.  Returns (grads dict, v_twist [V,6]);
        v_twist accumulates into a given buffer."""
        g = L.make_gaussians(*(params[k] for k in PARAM_KEYS), sh_degree)
        if grads is None:
            grads = {k: torch.empty_like(params[k]) for k in PARAM_KEYS}
        if v_twist is None:
            v_twist = torch.zeros((cams.V, 6), device=T.device, dtype=torch.float32)
        gg = L.make_grads(*(grads[k] for k in PARAM_KEYS))
        L.gs_render_bwd(self.ctx, g, cams, self.settings, self.bg, T, last, _dev(v_rgb), gg,
                        v_twist, stream)
        return grads, v_twist


class RasterizeGaussians(torch.autograd.Function):
    """Images of the batch; gradients to the Gaussian parameters and to the twist."""

    @staticmethod
    def forward(actx, means, log_scales, quats, opacity_logit, sh, twist, base_viewmat, intr,
                wh, sh_degree, splatter):
        params = dict(means=_dev(means), log_scales=_dev(log_scales), quats=_dev(quats),
                      opacity_logit=_dev(opacity_logit), sh=_dev(sh))
        tw = _dev(twist)
        viewmat = torch.empty_like(_dev(base_viewmat))
        L.gs_pose_compose(tw, _dev(base_viewmat), viewmat)
        rgb, T, last, cams = splatter.forward(params, sh_degree, viewmat, intr, wh)
        actx.splatter = splatter
        actx.sh_degree = sh_degree
        actx.cams = cams
        actx.keep = (viewmat, _dev(intr))
        # the lists this forward built; a later forward on the context replaces them
        actx.generation = splatter.ctx.generation()
        actx.save_for_backward(tw, T, last, *(params[k] for k in PARAM_KEYS))
        actx.mark_non_differentiable(T, last)
        return rgb, T, last

    @staticmethod
    def backward(actx, v_rgb, _vT, _vlast):
        tw, T, last, *pv = actx.saved_tensors
        params = dict(zip(PARAM_KEYS, pv))
        if actx.splatter.ctx.generation() != actx.generation:
            actx.splatter.rebin(params, actx.sh_degree, actx.cams)
        grads, v_tw_cur = actx.splatter.backward(params, actx.sh_degree, actx.cams, T, last,
                                                 v_rgb.contiguous())
        actx.generation = actx.splatter.ctx.generation()
        v_tw = torch.empty_like(tw)
        L.gs_pose_compose_bwd(tw, v_tw_cur, v_tw)
        return (grads["means"], grads["log_scales"], grads["quats"], grads["opacity_logit"],
                grads["sh"], v_tw, None, None, None, None, None)


class TrackReprojection(torch.autograd.Function):
    """lambda * sum_obs Huber(|pi_i(X_k) - x|^2; delta) with gradients to X and twist."""

    @staticmethod
    def forward(actx, X, twist, base_viewmat, intr, obs_cam, obs_pt, obs_xy, delta, lam, ctx,
                near_plane=0.01):
        tw = _dev(twist)
        viewmat = torch.empty_like(_dev(base_viewmat))
        L.gs_pose_compose(tw, _dev(base_viewmat), viewmat)
        loss = torch.zeros((1,), device=X.device, dtype=torch.float32)
        v_X = torch.zeros_like(_dev(X))
        v_tw_cur = torch.zeros_like(tw)
        L.track_reproj_fwd_bwd(ctx, _dev(X), viewmat, _dev(intr), obs_cam, obs_pt, _dev(obs_xy),
                               delta, lam, near_plane, loss, v_X, v_tw_cur)
        v_tw = torch.empty_like(tw)
        L.gs_pose_compose_bwd(tw, v_tw_cur, v_tw)
        actx.save_for_backward(v_X, v_tw)
        return loss[0]

    @staticmethod
    def backward(actx, g):
        v_X, v_tw = actx.saved_tensors
        return v_X * g, v_tw * g, None, None, None, None, None, None, None, None, None


def rasterize(params, sh_degree, twist, base_viewmat, intr, wh, splatter):
    return RasterizeGaussians.apply(params["means"], params["log_scales"], params["quats"],
                                    params["opacity_logit"], params["sh"], twist, base_viewmat,
                                    intr, np.asarray(wh, np.int32), sh_degree, splatter)[0]


def track_loss(X, twist, base_viewmat, intr, obs_cam, obs_pt, obs_xy, ctx, delta=1.0, lam=1e-4):
    return TrackReprojection.apply(X, twist, base_viewmat, intr, obs_cam, obs_pt, obs_xy, delta,
                                   lam, ctx)
