"""MI355X-native hot path of GloSplat's joint pose-appearance step.

A C-ABI HIP library (``libgs_hip.so``, declared in ``include/gs.h``) does the
work: EWA projection, tile binning and key sort, front-to-back compositing and
its backward to the Gaussian parameters and per-view SE(3) twists, the track
reprojection term, the L1 term, pose composition and Adam.  This package is
the Python binding (``_lib``: same names as the C entry points) and the
autograd wrappers (``splat``).
"""

from . import _lib
from ._lib import (BundleAdjuster, Cameras, Context, GsError, default_settings, gs_adam_step, gs_bin_sort,
                   gs_l1_loss_grad, gs_pose_compose, gs_pose_compose_bwd, gs_project,
                   gs_project_bwd, gs_project_bwd_adam, gs_raster_bwd, gs_render_bwd, gs_render_fwd,
                   gs_ba_lm_step, gs_init_gaussians, gs_mcmc_noise, gs_mcmc_relocate,
                   gs_photo_loss_grad, gs_step_advance, load, track_point_index,
                   track_reproj_fwd_bwd)

__all__ = [
    "Cameras", "Context", "GsError", "default_settings", "load", "gs_project", "gs_bin_sort",
    "gs_render_fwd", "gs_render_bwd", "gs_raster_bwd", "gs_project_bwd", "gs_l1_loss_grad", "track_reproj_fwd_bwd",
    "gs_pose_compose", "gs_pose_compose_bwd", "gs_adam_step", "gs_project_bwd_adam", "track_point_index",
    "gs_step_advance", "gs_photo_loss_grad", "gs_init_gaussians", "BundleAdjuster",
    "gs_ba_lm_step", "gs_mcmc_relocate", "gs_mcmc_noise",
]
