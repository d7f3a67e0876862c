"""track_reproj_fwd_bwd_noalloc (no context, accumulators in a fixed device
array of the library) against track_reproj_fwd_bwd through the C ABI, and
both against the oracle: two calls in a row, the second with fewer cameras,
points and observations, so any state the first left in the fixed array would
show."""

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


def _close(a, b, rtol, what):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    err = np.max(np.abs(a - b)) if a.size else 0.0
    assert err <= rtol * max(np.max(np.abs(b)) if b.size else 0.0, 1e-30), (what, err)


def _inputs(case):
    sc = scenegen.make_config("C1")
    X = sc["X"].astype(np.float32)
    vm, intr = sc["track_viewmat"], sc["track_intr"]
    cam, pt, xy = sc["obs_cam"], sc["obs_pt"], sc["obs_xy"]
    if case == 1:
        # fewer cameras (3 of 5), points and observations, still sorted by camera
        keep = (cam < 3) & (pt < 300)
        cam, pt, xy = cam[keep], pt[keep], xy[keep]
        X, vm, intr = X[:300], vm[:3], intr[:3]
    return X, vm, intr, cam, pt, xy


def _run(gs, fn, X, vm, intr, cam, pt, xy, index, ctx=None):
    M = len(cam)
    out = dict(loss=torch.zeros(1, device="cuda"), v_X=torch.zeros((X.shape[0], 3), device="cuda"),
               v_tw=torch.zeros((vm.shape[0], 6), device="cuda"),
               res=torch.empty((M, 2), device="cuda"), Jp=torch.empty((M, 12), device="cuda"),
               Jx=torch.empty((M, 6), device="cuda"))
    args = (_t(X), _t(vm), _t(intr), _t(cam, torch.int32), _t(pt, torch.int32), _t(xy), 1.0, 1e-4,
            0.01, out["loss"], out["v_X"], out["v_tw"])
    kw = dict(residual=out["res"], J_pose=out["Jp"], J_X=out["Jx"], pt_index=index)
    if ctx is None:
        fn(*args, **kw)
    else:
        fn(ctx, *args, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("indexed", [False, True])
def test_noalloc_track_matches_the_context_entry_point(gs, indexed):
    ctx = gs.Context(max_pairs=1000, max_isect=1 << 16, max_tiles=16, max_views=1, max_cams=8)
    for case in (0, 1):
        X, vm, intr, cam, pt, xy = _inputs(case)
        print(f"[noalloc] case {case}: {len(cam)} observations, {vm.shape[0]} cameras, "
              f"{X.shape[0]} points, indexed={indexed}", flush=True)
        index = gs.track_point_index(ctx, _t(pt, torch.int32), X.shape[0]) if indexed else None
        a = _run(gs, gs._lib.track_reproj_fwd_bwd_noalloc, X, vm, intr, cam, pt, xy, index)
        b = _run(gs, gs.track_reproj_fwd_bwd, X, vm, intr, cam, pt, xy, index, ctx=ctx)
        # the same kernels: per-observation outputs are identical, sums agree
        # up to the order of their atomic additions
        for k in ("res", "Jp", "Jx"):
            assert np.array_equal(a[k], b[k]), (case, k)
        for k in ("loss", "v_X", "v_tw"):
            _close(a[k], b[k], 1e-6, (case, k))
        o = oracle.track(X, vm, intr, cam, pt, xy, delta=1.0, lam=1e-4)
        assert abs(a["loss"][0] - o["loss"]) <= 1e-4 * o["loss"]
        _close(a["v_X"], o["v_X"], 1e-4, (case, "v_X vs oracle"))
        for v in range(vm.shape[0]):
            _close(a["v_tw"][v], o["v_twist"][v], 1e-4, (case, f"twist {v} vs oracle"))


def test_noalloc_track_rejects_too_many_cameras(gs):
    import paper_2603_04847_amd._lib as L
    lim = 4096
    X = torch.zeros((1, 3), device="cuda")
    vm = torch.zeros((lim + 1, 12), device="cuda")
    intr = torch.ones((lim + 1, 4), device="cuda")
    e0 = torch.zeros(1, dtype=torch.int32, device="cuda")
    xy = torch.zeros((1, 2), device="cuda")
    loss = torch.zeros(1, device="cuda")
    with pytest.raises(L.GsError) as e:
        L.track_reproj_fwd_bwd_noalloc(X, vm, intr, e0, e0, xy, 1.0, 1e-4, 0.01, loss,
                                       torch.zeros((1, 3), device="cuda"),
                                       torch.zeros((lim + 1, 6), device="cuda"))
    assert e.value.code == L.GS_ERR_CAPACITY
