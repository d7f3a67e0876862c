"""Seeded synthetic scenes for the splatting hot path.

This module only draws inputs.  It holds none of the renderer's arithmetic:
no covariance, no EWA projection, no spherical harmonics, no compositing and
no gradients.  The one piece of geometry it carries is a pinhole placement
(``_pixel_of`` and its vectorised form in ``make_tracks``) used to put
synthetic feature observations where a camera would see a track point; both the oracle and the HIP path then read the same
observation arrays, so neither depends on it for its own correctness.

Every array is drawn with numpy's PCG64 generator, in float64, and cast to
float32 at the end.  Layouts are the ones the C ABI takes:

* ``means [3,N]``, ``log_scales [3,N]``, ``quats [4,N]`` (w,x,y,z),
  ``opacity_logit [N]``, ``sh [K,3,N]`` with K = (deg+1)^2 -- planar (SoA).
* ``viewmat [V,12]``: world-to-camera [R|t], 3x4 row-major; camera axes are
  x right, y down, z forward.  ``intr [V,4]`` = fx, fy, cx, cy.
  ``wh [V,2]`` int32 = width, height.
* ``target [sum_v W_v*H_v, 3]``: views packed view-major, pixels row-major,
  RGB interleaved.
* ``X [Pt,3]``: track points (kept separate from the Gaussian means).
* ``obs_cam [M]`` int32, ``obs_pt [M]`` int32, ``obs_xy [M,2]``: feature
  observations, sorted by camera then by track.

The named configurations C1..C5 follow the five workloads of the benchmark
description (tiny single view, paper-scale single view, batched uneven views,
full joint step, large scene); sizes are the workload sizes, seeds 1..5.
"""

from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation

__all__ = [
    "make_config",
    "frustum_scene",
    "blob_scene",
    "sphere_cameras",
    "make_tracks",
    "synthetic_records",
    "view_targets",
    "batch_views",
    "C3_RESOLUTIONS",
]

# Per-view resolutions of the batched uneven-view workload.
C3_RESOLUTIONS = [
    (640, 480), (800, 600), (960, 720), (1024, 768),
    (1237, 822), (1280, 960), (1440, 960), (1600, 1066),
]

# Focal length per unit image width that gives the 256 px / fx=300 field of view.
FX_PER_W = 300.0 / 256.0


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _sh_dc_uniform_rgb(rng, n):
    """Degree-0 coefficient whose colour 0.5 + Y00*c is uniform on [0,1].

    Y00 = 1/(2 sqrt(pi)), so c uniform on [-sqrt(pi), sqrt(pi)] gives that.
    Stated as a distribution so no basis function is evaluated here.
    """
    b = np.sqrt(np.pi)
    return rng.uniform(-b, b, size=(3, n))


def _gaussian_params(rng, n, sh_degree, log_scale_mu, log_scale_sd, sh_sd=None,
                     unit_quats=True):
    K = (sh_degree + 1) ** 2
    log_scales = rng.normal(log_scale_mu, log_scale_sd, size=(3, n))
    q = rng.normal(0.0, 1.0, size=(4, n))
    if unit_quats:
        q = q / np.linalg.norm(q, axis=0, keepdims=True)
    logit = rng.normal(0.0, 1.0, size=n)
    sh = np.zeros((K, 3, n))
    if sh_sd is None:
        sh[0] = _sh_dc_uniform_rgb(rng, n)
    else:
        sh[:] = rng.normal(0.0, sh_sd, size=(K, 3, n))
    return log_scales, q, logit, sh


def _look_at(center, target, up):
    """World-to-camera [R|t] for a camera at `center` looking at `target`."""
    f = target - center
    f = f / np.linalg.norm(f)
    r = np.cross(f, up)
    r = r / np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f], axis=0)
    t = -R @ center
    return R, t


def _pack_viewmat(R, t):
    return np.concatenate([R, t[:, None]], axis=1).reshape(12)


def _pixel_of(R, t, fx, fy, cx, cy, X):
    """Pinhole placement of world points X [n,3]; returns (uv [n,2], depth [n])."""
    Xc = X @ R.T + t
    z = Xc[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        uv = np.stack([fx * Xc[:, 0] / z + cx, fy * Xc[:, 1] / z + cy], axis=1)
    return uv, z


def _frustum_points(rng, n, W, H, fx, fy, cx, cy, zmin, zmax):
    """Points uniform in the volume of the image frustum between two depths."""
    u = rng.uniform(size=n)
    z = (zmin ** 3 + (zmax ** 3 - zmin ** 3) * u) ** (1.0 / 3.0)
    px = rng.uniform(0.0, W, size=n)
    py = rng.uniform(0.0, H, size=n)
    x = (px - cx) / fx * z
    y = (py - cy) / fy * z
    return np.stack([x, y, z], axis=1)


def frustum_scene(seed, W, H, fx, fy, N, sh_degree, log_scale_mu, log_scale_sd,
                  sh_sd=None, zmin=2.0, zmax=6.0, unit_quats=True,
                  random_world=True, n_tracks=0, track_cams=5, obs_per_track=3,
                  track_offset=0.25):
    """One camera looking into a frustum of Gaussians (configs C1, C2).

    The scene is built in camera-0 coordinates and moved into the world by a
    random rigid transform so the view matrix is not the identity.  With
    ``n_tracks`` > 0 it adds track points drawn from the same frustum, each
    seen by ``obs_per_track`` of ``track_cams`` cameras: camera 0 and cameras
    shifted by ``track_offset`` along +-x and +-y aimed at the frustum centre.
    """
    rng = _rng(seed)
    cx, cy = W / 2.0, H / 2.0
    Pc = _frustum_points(rng, N, W, H, fx, fy, cx, cy, zmin, zmax)
    log_scales, q, logit, sh = _gaussian_params(
        rng, N, sh_degree, log_scale_mu, log_scale_sd, sh_sd, unit_quats)
    if random_world:
        Rw = Rotation.random(random_state=rng).as_matrix()
        tw = rng.normal(0.0, 1.0, size=3)
    else:
        Rw, tw = np.eye(3), np.zeros(3)
    # camera-0 frame -> world: X_w = Rw^T (X_c - tw), so Rw X_w + tw = X_c
    means = (Pc - tw) @ Rw
    views = [(Rw, tw)]
    if n_tracks > 0:
        centre_c = np.array([0.0, 0.0, (zmin + zmax) / 2.0])
        offs = [np.array(o) * track_offset for o in
                ([1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0])][: track_cams - 1]
        for o in offs:
            Rl, tl = _look_at(o, centre_c, np.array([0.0, -1.0, 0.0]))
            # compose camera-k (in camera-0 coords) with the world transform
            views.append((Rl @ Rw, Rl @ tw + tl))
    V = len(views)
    viewmat = np.stack([_pack_viewmat(R, t) for R, t in views])
    intr = np.tile(np.array([fx, fy, cx, cy]), (V, 1))
    wh = np.tile(np.array([W, H], dtype=np.int32), (V, 1))
    target = rng.uniform(0.0, 1.0, size=(W * H, 3))
    out = dict(
        means=_f32(means.T), log_scales=_f32(log_scales), quats=_f32(q),
        opacity_logit=_f32(logit), sh=_f32(sh), sh_degree=sh_degree,
        viewmat=_f32(viewmat[:1]), intr=_f32(intr[:1]), wh=wh[:1].copy(),
        target=_f32(target),
    )
    if n_tracks > 0:
        out.update(_frustum_tracks(rng, n_tracks, W, H, fx, fy, cx, cy, zmin, zmax,
                                   Rw, tw, views, obs_per_track))
        out["track_viewmat"] = _f32(viewmat)
        out["track_intr"] = _f32(intr)
        out["track_wh"] = wh.copy()
    return out


def _frustum_tracks(rng, n, W, H, fx, fy, cx, cy, zmin, zmax, Rw, tw, views, k):
    Xs, cams, pts, xys = [], [], [], []
    pid = 0
    while pid < n:
        Pc = _frustum_points(rng, 1, W, H, fx, fy, cx, cy, zmin, zmax)
        Xw = (Pc - tw) @ Rw
        ok = []
        for ci, (R, t) in enumerate(views):
            uv, z = _pixel_of(R, t, fx, fy, cx, cy, Xw)
            if z[0] > 0.01 and 0 <= uv[0, 0] < W and 0 <= uv[0, 1] < H:
                ok.append((ci, uv[0]))
        if len(ok) < k:
            continue
        pick = rng.choice(len(ok), size=k, replace=False)
        for j in sorted(pick):
            ci, uv = ok[j]
            cams.append(ci)
            pts.append(pid)
            xys.append(uv + rng.normal(0.0, 1.0, size=2))
        Xs.append(Xw[0])
        pid += 1
    return _sorted_obs(np.array(Xs), np.array(cams), np.array(pts), np.array(xys))


def _sorted_obs(X, cams, pts, xys):
    order = np.lexsort((pts, cams))
    return dict(
        X=_f32(X),
        obs_cam=np.ascontiguousarray(cams[order], dtype=np.int32),
        obs_pt=np.ascontiguousarray(pts[order], dtype=np.int32),
        obs_xy=_f32(xys[order]),
    )


def sphere_cameras(rng, resolutions, radius=4.0):
    """Cameras uniform on a sphere around the origin, looking at it (up +z)."""
    vms, intr, wh = [], [], []
    for (W, H) in resolutions:
        while True:
            c = rng.normal(size=3)
            c = radius * c / np.linalg.norm(c)
            if abs(c[2]) / radius < 0.95:     # avoid a view direction parallel to up
                break
        R, t = _look_at(c, np.zeros(3), np.array([0.0, 0.0, 1.0]))
        vms.append(_pack_viewmat(R, t))
        fx = FX_PER_W * W
        intr.append([fx, fx, W / 2.0, H / 2.0])
        wh.append([W, H])
    return _f32(np.stack(vms)), _f32(np.array(intr)), np.array(wh, dtype=np.int32)


def _blob_points(rng, n, n_blobs=50, ball_r=1.5, sig_lo=0.02, sig_hi=0.4, dirichlet=0.3):
    d = rng.normal(size=(n_blobs, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    centres = d * (ball_r * rng.uniform(size=(n_blobs, 1)) ** (1.0 / 3.0))
    sig = np.exp(rng.uniform(np.log(sig_lo), np.log(sig_hi), size=n_blobs))
    w = rng.dirichlet(np.full(n_blobs, dirichlet))
    comp = rng.choice(n_blobs, size=n, p=w)
    return centres[comp] + sig[comp, None] * rng.normal(size=(n, 3))


def blob_scene(seed, resolutions, N, sh_degree=3, log_scale_mu=-4.0, log_scale_sd=0.7,
               sh_sd=0.1, n_blobs=50, make_target=True, dirichlet=0.3):
    """Cameras on a sphere of radius 4 around a mixture of isotropic blobs of
    Gaussians (configs C3, C4, C5).  Blob weights are Dirichlet(`dirichlet`)
    (0.3 unless given), so the per-tile load is very uneven."""
    rng = _rng(seed)
    viewmat, intr, wh = sphere_cameras(rng, resolutions)
    means = _blob_points(rng, N, n_blobs, dirichlet=dirichlet)
    log_scales, q, logit, sh = _gaussian_params(rng, N, sh_degree, log_scale_mu,
                                                log_scale_sd, sh_sd)
    P = int(sum(w * h for w, h in resolutions))
    target = (rng.uniform(0.0, 1.0, size=(P, 3)).astype(np.float32)
              if make_target else None)
    return dict(
        means=_f32(means.T), log_scales=_f32(log_scales), quats=_f32(q),
        opacity_logit=_f32(logit), sh=_f32(sh), sh_degree=sh_degree,
        viewmat=viewmat, intr=intr, wh=wh, target=target, _rng=rng,
    )


def make_tracks(rng, n_tracks, viewmat, intr, wh, max_len, n_cand=None, n_blobs=50,
                points=None, chunk=4096):
    """Track points seen by 2 + Geom(0.3) cameras (capped at ``max_len``).

    Each point is observed by cameras in whose image it falls, chosen uniformly
    among all cameras (or among ``n_cand`` random candidate cameras for large
    camera sets); points seen by fewer than two cameras are dropped.
    Observations get N(0, 1 px) noise per axis.
    """
    V = viewmat.shape[0]
    X = points if points is not None else _blob_points(rng, n_tracks, n_blobs)
    L = np.minimum(max_len, 1 + rng.geometric(0.3, size=n_tracks))
    M3 = viewmat.astype(np.float64).reshape(V, 3, 4)
    Rall, tall = M3[:, :, :3], M3[:, :, 3]
    fi = intr.astype(np.float64)
    cams, pts, xys = [], [], []
    keep = np.zeros(n_tracks, dtype=bool)
    for s in range(0, n_tracks, chunk):
        e = min(n_tracks, s + chunk)
        n = e - s
        if n_cand is None:
            cand = np.broadcast_to(np.arange(V), (n, V))
            dup = np.zeros(cand.shape, dtype=bool)
        else:
            cand = np.sort(rng.integers(0, V, size=(n, n_cand)), axis=1)
            dup = np.zeros(cand.shape, dtype=bool)
            dup[:, 1:] = cand[:, 1:] == cand[:, :-1]
        Xc = np.einsum("ncij,nj->nci", Rall[cand], X[s:e]) + tall[cand]
        z = Xc[..., 2]
        with np.errstate(divide="ignore", invalid="ignore"):
            u = fi[cand, 0] * Xc[..., 0] / z + fi[cand, 2]
            v = fi[cand, 1] * Xc[..., 1] / z + fi[cand, 3]
        W = wh[cand, 0]
        H = wh[cand, 1]
        vis = (z > 0.01) & (u >= 0) & (u < W) & (v >= 0) & (v < H) & ~dup
        key = rng.uniform(size=vis.shape)
        key[~vis] = 2.0
        order = np.argsort(key, axis=1)
        nvis = vis.sum(axis=1)
        k = np.minimum(L[s:e], nvis)
        ok = nvis >= 2
        rank = np.arange(cand.shape[1])[None, :]
        sel = (rank < k[:, None]) & ok[:, None]
        rows, cols = np.nonzero(sel)
        j = order[rows, cols]
        cams.append(cand[rows, j])
        pts.append(s + rows)
        xys.append(np.stack([u[rows, j], v[rows, j]], axis=1))
        keep[s:e] = ok
    cams = np.concatenate(cams)
    pts = np.concatenate(pts)
    xys = np.concatenate(xys) + rng.normal(0.0, 1.0, size=(len(cams), 2))
    new_id = np.cumsum(keep) - 1          # renumber the kept tracks densely
    return _sorted_obs(X[keep], cams, new_id[pts], xys)


def perturb_poses(rng, viewmat, rho_sd=0.005, phi_sd=0.002):
    """Initial poses: each true pose moved by a small random rotation (axis-angle
    N(0, phi_sd^2) per axis) and translation N(0, rho_sd^2) per axis."""
    out = viewmat.astype(np.float64).copy()
    for i in range(viewmat.shape[0]):
        M = out[i].reshape(3, 4)
        Rd = Rotation.from_rotvec(rng.normal(0.0, phi_sd, size=3)).as_matrix()
        R = Rd @ M[:, :3]
        t = Rd @ M[:, 3] + rng.normal(0.0, rho_sd, size=3)
        out[i] = np.concatenate([R, t[:, None]], axis=1).reshape(12)
    return _f32(out)


def synthetic_records(seed, V, wh, N, tile=(16, 16), depth_ties=True):
    """Projected-splat records for testing the bin/sort step on its own.

    Every splat is either tiny (its support stays inside the tile quadrant
    -- a tile_w/2 x tile_h/2 block -- holding its centre, which is kept at least
    1 px away from the quadrant's pixel-centre edges) or huge (it covers the
    whole image), so which tiles and quadrants a splat meets is never a
    near-tie.  Depths are drawn from a small set of values when ``depth_ties``
    so equal depths occur often.

    Returns float arrays laid out as the projected record (mean2d [V*N,2],
    conic [V*N,3], opacity [V*N], depth [V*N], rgb [V*N,3]) and ``valid``.
    """
    rng = _rng(seed)
    tw, th = tile
    qw, qh = tw // 2, th // 2
    VN = V * N
    mean2d = np.zeros((VN, 2))
    conic = np.zeros((VN, 3))
    opac = rng.uniform(0.05, 0.95, size=VN)
    valid = rng.uniform(size=VN) > 0.1
    kind = rng.uniform(size=VN)
    for v in range(V):
        W, H = wh[v]
        gx, gy = (W + qw - 1) // qw, (H + qh - 1) // qh     # quadrant grid
        sl = slice(v * N, (v + 1) * N)
        qx = rng.integers(0, gx, size=N)
        qy = rng.integers(0, gy, size=N)
        x0 = qx * qw + 0.5
        x1 = np.minimum(qx * qw + qw, W) - 0.5
        y0 = qy * qh + 0.5
        y1 = np.minimum(qy * qh + qh, H) - 0.5
        fx = rng.uniform(size=N)
        fy = rng.uniform(size=N)
        mx = np.where(x1 - x0 > 2, x0 + 1 + fx * (x1 - x0 - 2), 0.5 * (x0 + x1))
        my = np.where(y1 - y0 > 2, y0 + 1 + fy * (y1 - y0 - 2), 0.5 * (y0 + y1))
        mean2d[sl, 0] = mx
        mean2d[sl, 1] = my
    big = kind[:] > 0.97
    # tiny: variance 1e-3 px^2 -> support radius < 0.2 px; big: variance 1e8 px^2
    var = np.where(big, 1e8, 1e-3)
    conic[:, 0] = 1.0 / var
    conic[:, 1] = 0.0
    conic[:, 2] = 1.0 / var
    if depth_ties:
        depth = rng.choice(np.linspace(0.5, 9.5, 37), size=VN)
    else:
        depth = rng.uniform(0.5, 9.5, size=VN)
    rgb = rng.uniform(size=(VN, 3))
    return dict(mean2d=_f32(mean2d), conic=_f32(conic), opacity=_f32(opac),
                depth=_f32(depth), rgb=_f32(rgb), valid=valid.astype(np.int32))


def view_targets(seed, wh, views):
    """Target images U[0,1] for a subset of views, each drawn from its own
    stream (seed, view) so a batch never needs every view's image at once."""
    out = []
    for v in views:
        W, H = (int(x) for x in wh[v])
        out.append(_rng([seed, int(v)]).uniform(0.0, 1.0, size=(W * H, 3)))
    return _f32(np.concatenate(out))


def batch_views(seed, n_views, batch, steps):
    """Per-step view batches (without replacement inside a step)."""
    rng = _rng([seed, 7919])
    return [np.sort(rng.choice(n_views, size=batch, replace=False)) for _ in range(steps)]


C3_DIRICHLET = 0.05


def make_config(name, seed=None):
    """The five named workloads.  Returns the scene dict (see module doc)."""
    name = name.upper()
    if name == "C1":
        return frustum_scene(1 if seed is None else seed, 256, 256, 300.0, 300.0,
                             10_000, 0, -3.0, 0.5, n_tracks=500)
    if name == "C2":
        W, H = 1237, 822
        return frustum_scene(2 if seed is None else seed, W, H, FX_PER_W * W,
                             FX_PER_W * W, 1_000_000, 3, -4.0, 0.7, sh_sd=0.1)
    if name == "C3":
        # Dirichlet(0.05) blob weights: the recipe lowers the concentration from
        # 0.3 until the largest per-tile splat count is at least 100 times the
        # median (0.3 gives about 42, 0.1 about 110, 0.05 about 140)
        s = blob_scene(3 if seed is None else seed, C3_RESOLUTIONS, 3_000_000,
                       dirichlet=C3_DIRICHLET)
        s.pop("_rng")
        return s
    if name == "C4":
        s = blob_scene(4 if seed is None else seed, [(1237, 822)] * 150, 1_000_000,
                       make_target=False)
        rng = s.pop("_rng")
        s.update(make_tracks(rng, 100_000, s["viewmat"], s["intr"], s["wh"], 12))
        s["viewmat_true"] = s["viewmat"]
        s["viewmat"] = perturb_poses(rng, s["viewmat"])
        return s
    if name == "C5":
        s = blob_scene(5 if seed is None else seed, [(1600, 1066)] * 1000, 5_000_000,
                       make_target=False)
        rng = s.pop("_rng")
        s.update(make_tracks(rng, 1_500_000, s["viewmat"], s["intr"], s["wh"], 30,
                             n_cand=64))
        s["viewmat"] = perturb_poses(rng, s["viewmat"])
        return s
    raise ValueError(f"unknown config {name}")
