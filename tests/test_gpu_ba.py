"""One Levenberg-Marquardt step of bundle adjustment (Sec. 3.2 "Bundle
Adjustment", eq. L_BA^SfM) through the C ABI against the FP64 oracle, which
forms the dense normal equations and solves them with LAPACK: a small problem
with inliers, outliers, a masked observation, a camera and a point without
observations; repeated steps converging on exact observations; and the
normal-equation residual of the step at the full sizes (150 cameras / 425k
observations and 1000 cameras / 6.5M observations)."""

import numpy as np
import pytest

import oracle
import scenegen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_04847_amd as P
    P.load()
    return P


def _t(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def _close(a, b, what, rtol=1e-4):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    err = np.max(np.abs(a - b))
    assert err <= rtol * np.max(np.abs(b)), f"{what}: {err:.3e} vs {rtol * np.max(np.abs(b)):.3e}"


def _step(gs, X, vm, intr, cam, pt, xy, lm_lambda, max_iter=500, tol=1e-12, copies=True):
    """One step; with `copies` the index carries the point-major copies of
    the cameras and pixels (the passes over the points read those)."""
    Pt, C = X.shape[0], vm.shape[0]
    ctx = gs.Context(max_pairs=Pt + 1, max_isect=1 << 10, max_tiles=16, max_views=1, max_cams=C)
    obs_pt, obs_cam, obs_xy = _t(pt, torch.int32), _t(cam, torch.int32), _t(xy)
    index = (gs.track_point_index(ctx, obs_pt, Pt, obs_cam, obs_xy) if copies
             else gs.track_point_index(ctx, obs_pt, Pt))
    ba = gs.BundleAdjuster(Pt, C)
    dtw = torch.empty((C, 6), device="cuda")
    dX = torch.empty((Pt, 3), device="cuda")
    stats = torch.zeros(5, device="cuda")
    gs.gs_ba_lm_step(ba, _t(X), _t(vm), _t(intr), obs_cam, obs_pt, obs_xy, index, 1.0,
                     lm_lambda, 0.01, max_iter, tol, dtw, dX, stats)
    torch.cuda.synchronize()
    return dtw.cpu().numpy(), dX.cpu().numpy(), stats.cpu().numpy()


def _problem():
    """The tiny workload's tracks (5 cameras, 500 points, 3 observations each,
    N(0, 1 px) noise: inliers and Huber outliers), made harder: poses and
    points perturbed, one point behind camera 0, a sixth camera and an extra
    point with no observation."""
    sc = scenegen.make_config("C1")
    rng = np.random.default_rng(7)
    X = sc["X"].astype(np.float64) + rng.normal(0, 0.01, sc["X"].shape)
    vm = sc["track_viewmat"].astype(np.float64).copy()
    vm[:, [3, 7, 11]] += rng.normal(0, 0.01, (vm.shape[0], 3))
    M3 = vm[0].reshape(3, 4)
    X[0] = M3[:, :3].T @ (np.array([0.1, 0.2, -3.0]) - M3[:, 3])     # behind camera 0
    X = np.concatenate([X, [[0.3, 0.2, 4.0]]])                          # no observation
    vm = np.concatenate([vm, vm[:1]])                                   # camera 5: none
    intr = np.concatenate([sc["track_intr"], sc["track_intr"][:1]])
    return (X.astype(np.float32), vm.astype(np.float32), intr.astype(np.float32), sc["obs_cam"],
            sc["obs_pt"], sc["obs_xy"])


@pytest.mark.parametrize("copies", [False, True])
@pytest.mark.parametrize("lm_lambda", [1e-3, 1.0])
def test_ba_step_matches_oracle(gs, lm_lambda, copies):
    X, vm, intr, cam, pt, xy = _problem()
    dtw, dX, stats = _step(gs, X, vm, intr, cam, pt, xy, lm_lambda, copies=copies)
    otw, oX, cost = oracle.ba_step(X, vm, intr, cam, pt, xy, lm_lambda=lm_lambda)
    print(f"[ba] lambda {lm_lambda}: {int(stats[0])} PCG iterations, residual {stats[1]:.2e}", flush=True)
    assert stats[1] <= 1e-8 and stats[4] == 0
    assert stats[3] > 0                                                 # the masked observations
    assert abs(stats[2] - cost) <= 1e-5 * cost
    _close(dtw, otw, "d_twist")
    _close(dX, oX, "d_X")
    assert np.all(dtw[5] == 0) and np.all(dX[-1] == 0)                  # held fixed


def test_ba_steps_converge_on_exact_observations(gs):
    """Observations made exact at the true poses and points; from perturbed
    ones, five steps (applied with the pose composition) bring the robust cost
    down by more than six orders of magnitude."""
    sc = scenegen.make_config("C1")
    X0 = sc["X"].astype(np.float64)
    vm0 = sc["track_viewmat"].astype(np.float64)
    intr = sc["track_intr"]
    cam, pt = sc["obs_cam"], sc["obs_pt"]
    xy = np.zeros((len(cam), 2))
    for o in range(len(cam)):
        M3 = vm0[cam[o]].reshape(3, 4)
        p = M3[:, :3] @ X0[pt[o]] + M3[:, 3]
        f = intr[cam[o]]
        xy[o] = [f[0] * p[0] / p[2] + f[2], f[1] * p[1] / p[2] + f[3]]
    rng = np.random.default_rng(3)
    X = _t(X0 + rng.normal(0, 0.003, X0.shape))
    base = _t(vm0)
    tw = _t(rng.normal(0, 0.002, (vm0.shape[0], 6)))
    vm = torch.empty_like(base)
    gs.gs_pose_compose(tw, base, vm)
    C, Pt = vm0.shape[0], X0.shape[0]
    ctx = gs.Context(max_pairs=Pt + 1, max_isect=1 << 10, max_tiles=16, max_views=1, max_cams=C)
    obs_pt = _t(pt, torch.int32)
    index = gs.track_point_index(ctx, obs_pt, Pt)
    ba = gs.BundleAdjuster(Pt, C)
    dtw = torch.empty((C, 6), device="cuda")
    dX = torch.empty((Pt, 3), device="cuda")
    stats = torch.zeros(5, device="cuda")
    costs = []
    for it in range(6):
        gs.gs_ba_lm_step(ba, X, vm, _t(intr), _t(cam, torch.int32), obs_pt, _t(xy), index, 1.0, 1e-4,
                         0.01, 300, 1e-10, dtw, dX, stats)
        torch.cuda.synchronize()
        costs.append(float(stats[2].item()))
        nv = torch.empty_like(vm)
        gs.gs_pose_compose(dtw, vm, nv)
        vm = nv
        X = X + dX
    print(f"[ba] costs {costs}", flush=True)
    assert costs[-1] < 1e-6 * costs[0]


def _full_size(gs, name, lm_lambda=1e-2):
    sc = scenegen.make_config(name)
    X, vm, intr = sc["X"], sc["viewmat"], sc["intr"]
    cam, pt, xy = sc["obs_cam"], sc["obs_pt"], sc["obs_xy"]
    dtw, dX, stats = _step(gs, X, vm, intr, cam, pt, xy, lm_lambda, max_iter=300, tol=1e-9)
    print(f"[ba] {name}: {int(stats[0])} PCG iterations, residual {stats[1]:.2e}", flush=True)
    H_g = oracle.ba_normal_residual(X, vm, intr, cam, pt, xy, np.zeros_like(dtw), np.zeros_like(dX),
                                    lm_lambda=lm_lambda)
    g = np.concatenate([H_g[0].reshape(-1), H_g[1].reshape(-1)])
    rc, rp = oracle.ba_normal_residual(X, vm, intr, cam, pt, xy, dtw, dX, lm_lambda=lm_lambda)
    res = np.concatenate([rc.reshape(-1), rp.reshape(-1)])
    # the step solves the damped normal equations: what is left of the
    # gradient is a small fraction of it (float32 outputs, PCG tolerance)
    print(f"[ba] {name}: |(H + l D) d + g| / |g| = {np.linalg.norm(res) / np.linalg.norm(g):.2e}")
    assert np.linalg.norm(res) <= 1e-4 * np.linalg.norm(g)
    assert stats[4] == 0


def test_ba_step_full_size_joint_step_scene(gs):
    _full_size(gs, "C4")


def test_ba_step_full_size_large_scene(gs):
    _full_size(gs, "C5")
