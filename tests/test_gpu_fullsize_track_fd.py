"""Full-size checks of the joint step's geometric half and of its gradients:

* the track term at the full sizes (150 cameras / 425k observations, 1000
  cameras / 6.5M observations) against the FP64 oracle, on the atomic and on
  the point-indexed paths;
* central finite differences in FP64 (the oracle's loss) against the
  autograd gradients of the whole joint loss, L_photo (L1 + SSIM, lambda 0.2)
  of a 64 x 64 sub-crop of view 0 of the 150-camera scene with 20 of its
  Gaussians, plus lambda_BA times the Huber track loss of 10 of its points
  (Sec. 3.3, total objective), to the Gaussians, the track points and the
  pose twists."""

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


def _t(a, dtype=torch.float32, grad=False):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype).requires_grad_(grad)


def _close(a, b, what, rtol=1e-4):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    err = np.max(np.abs(a - b))
    assert err <= rtol * np.max(np.abs(b)), f"{what}: {err:.3e} vs {rtol * np.max(np.abs(b)):.3e}"


@pytest.mark.parametrize("name", ["C4", "C5"])
def test_track_term_full_size(gs, name):
    sc = scenegen.make_config(name)
    X, vm, intr = sc["X"], sc["viewmat"], sc["intr"]
    cam, pt, xy = sc["obs_cam"], sc["obs_pt"], sc["obs_xy"]
    Pt, C, M = X.shape[0], vm.shape[0], len(cam)
    print(f"[track] {name}: {M} observations, {C} cameras, {Pt} points", flush=True)
    o = oracle.track(X, vm, intr, cam, pt, xy, delta=1.0, lam=1e-4, jacobians=False)
    ctx = gs.Context(max_pairs=Pt + 1, max_isect=1 << 10, max_tiles=16, max_views=1, max_cams=C)
    obs_pt, obs_cam, obs_xy = _t(pt, torch.int32), _t(cam, torch.int32), _t(xy)
    index = gs.track_point_index(ctx, obs_pt, Pt)
    index_pm = gs.track_point_index(ctx, obs_pt, Pt, obs_cam, obs_xy)
    for what, pi in (("atomic", None), ("indexed", index), ("point-major", index_pm)):
        loss = torch.zeros(1, device="cuda")
        v_X = torch.zeros((Pt, 3), device="cuda")
        v_tw = torch.zeros((C, 6), device="cuda")
        # the point-major pass runs when no residual is asked for
        res = torch.empty((M, 2), device="cuda") if what != "point-major" else None
        ctx.reset_status()
        gs.track_reproj_fwd_bwd(ctx, _t(X), _t(vm), _t(intr), obs_cam, obs_pt, obs_xy, 1.0,
                                1e-4, 0.01, loss, v_X, v_tw, residual=res, pt_index=pi)
        torch.cuda.synchronize()
        assert ctx.status()["n_masked_obs"] == int(o["masked"].sum())
        if res is not None:
            _close(res.cpu().numpy(), o["residual"], f"{what} residual")
        assert abs(loss.item() - o["loss"]) <= 1e-4 * o["loss"], what
        _close(v_X.cpu().numpy(), o["v_X"], f"{what} v_X")
        tw = v_tw.cpu().numpy()
        for v in range(C):
            if np.any(o["v_twist"][v]):
                _close(tw[v], o["v_twist"][v], f"{what} twist {v}")


def _subcrop():
    """64 x 64 window at the centre of view 0, the 20 Gaussians projecting
    nearest its centre, and 10 track points seen in view 0 with all their
    observations."""
    sc = scenegen.make_config("C4")
    W, H = (int(x) for x in sc["wh"][0])
    x0, y0 = W // 2 - 32, H // 2 - 32
    intr = sc["intr"][0].astype(np.float64).copy()
    intr[2] -= x0
    intr[3] -= y0
    one = dict(sc, viewmat=sc["viewmat"][:1], intr=intr[None].astype(np.float32),
               wh=np.array([[64, 64]], np.int32))
    pr = oracle.project(one)
    m = pr["mean2d"]
    d = np.hypot(m[:, 0] - 32, m[:, 1] - 32)
    d[~pr["valid"].astype(bool)] = np.inf
    sel = np.argsort(d)[:20]
    crop = dict(one)
    for k in ("means", "log_scales", "quats", "sh"):
        crop[k] = np.ascontiguousarray(sc[k][..., sel])
    crop["opacity_logit"] = np.ascontiguousarray(sc["opacity_logit"][sel])
    tgt = scenegen.view_targets(4, sc["wh"], [0]).reshape(H, W, 3)[y0:y0 + 64, x0:x0 + 64].reshape(-1, 3)
    crop["target"] = np.ascontiguousarray(tgt)
    seen = np.unique(sc["obs_pt"][sc["obs_cam"] == 0])[:10]
    keep = np.isin(sc["obs_pt"], seen)
    remap = {int(p): i for i, p in enumerate(seen)}
    obs_pt = np.array([remap[int(p)] for p in sc["obs_pt"][keep]], np.int32)
    tracks = dict(X=sc["X"][seen].astype(np.float32), cam=sc["obs_cam"][keep], pt=obs_pt,
                  xy=sc["obs_xy"][keep], viewmat=sc["viewmat"], intr=sc["intr"])
    return crop, tracks


def _oracle_loss(crop, tracks, viewmat0, viewmat_all, X, lam_ba=1e-4):
    c = dict(crop, viewmat=viewmat0[None])
    out = oracle.render_fwd_bwd(c)
    lp, _ = oracle.photo_loss(out["rgb"], crop["target"], crop["wh"], lam=0.2)
    t = oracle.track(X, viewmat_all, tracks["intr"], tracks["cam"], tracks["pt"], tracks["xy"],
                     delta=1.0, lam=lam_ba, jacobians=False)
    state = (out["ncontrib"].copy(), out["ngate"].copy(), out["nclamp"].copy(),
             np.sign(out["rgb"] - crop["target"]))
    return lp + t["loss"], state


def _left(viewmat12, xi):
    import scipy.linalg
    r, f = xi[:3], xi[3:]
    A = np.array([[0, -f[2], f[1], r[0]], [f[2], 0, -f[0], r[1]], [-f[1], f[0], 0, r[2]], [0, 0, 0, 0]])
    T = np.eye(4)
    T[:3] = np.asarray(viewmat12, np.float64).reshape(3, 4)
    return (scipy.linalg.expm(A) @ T)[:3].reshape(12)


def test_joint_loss_gradients_against_fp64_finite_differences_on_a_subcrop(gs):
    from paper_2603_04847_amd.splat import Splatter, rasterize, track_loss
    crop, tracks = _subcrop()
    C = tracks["viewmat"].shape[0]
    # GPU: autograd through both Functions; the photometric gradient from the
    # library's loss kernel
    params = {k: _t(crop[k], grad=True) for k in ("means", "log_scales", "quats", "opacity_logit", "sh")}
    tw = _t(np.zeros((C, 6), np.float32), grad=True)
    X = _t(tracks["X"], grad=True)
    ctx = gs.Context(max_pairs=64, max_isect=1 << 16, max_tiles=64, max_views=1, max_cams=C)
    sp = Splatter(ctx)
    img = rasterize(params, 3, tw[0:1], _t(crop["viewmat"]), _t(crop["intr"]), crop["wh"], sp)
    cams = gs.Cameras(_t(crop["viewmat"]), _t(crop["intr"]), crop["wh"])
    v_img = torch.empty_like(img)
    lph = torch.zeros(1, device="cuda")
    gs.gs_photo_loss_grad(ctx, cams, img.detach().contiguous(), _t(crop["target"]), 0.2, v_img, lph)
    lt = track_loss(X, tw, _t(tracks["viewmat"]), _t(tracks["intr"]), _t(tracks["cam"], torch.int32),
                    _t(tracks["pt"], torch.int32), _t(tracks["xy"]), ctx)
    torch.autograd.backward([img, lt], [v_img, torch.ones((), device="cuda")])
    torch.cuda.synchronize()
    # oracle, FP64 central differences of the same loss
    vm0 = crop["viewmat"][0].astype(np.float64)
    vma = tracks["viewmat"].astype(np.float64)
    Xo = tracks["X"].astype(np.float64)
    base = {k: crop[k].astype(np.float64) for k in params}
    L0, st0 = _oracle_loss(dict(crop, **base), tracks, vm0, vma, Xo)
    assert abs(L0 - (lph.item() + lt.item())) <= 1e-4 * L0

    def fd(perturb, h):
        # central difference where neither side moves a gate, the stop, a clamp
        # or an L1 sign; else one-sided on the side that keeps the base state
        # (the base may sit on such a boundary); else unusable
        Lp, sp_ = perturb(h)
        Lm, sm_ = perturb(-h)
        okp = all(np.array_equal(a, b) for a, b in zip(st0, sp_))
        okm = all(np.array_equal(a, b) for a, b in zip(st0, sm_))
        if okp and okm:
            return (Lp - Lm) / (2 * h), True
        if okp:
            return (Lp - L0) / h, True
        if okm:
            return (L0 - Lm) / h, True
        return 0.0, False

    checked = 0
    for k in params:
        flat = base[k].reshape(-1)
        got = params[k].grad.cpu().numpy().reshape(-1)
        want, ok = np.zeros_like(flat), np.zeros(flat.shape, bool)
        # SH: the degree-0 and degree-1 bands (the higher ones chain the same way)
        n = flat.size if k != "sh" else 4 * 3 * base[k].shape[2]
        for i in range(n):
            h = 1e-6 * max(1.0, abs(flat[i]))

            def pert(d, i=i):
                b2 = {kk: v.copy() for kk, v in base.items()}
                b2[k].reshape(-1)[i] += d
                return _oracle_loss(dict(crop, **b2), tracks, vm0, vma, Xo)
            want[i], ok[i] = fd(pert, h)
        ok[n:] = False
        # a parameter whose +h and -h both move a gate, the stop or an L1 sign is skipped
        assert ok[:n].mean() >= 0.9, k
        _close(got[ok], want[ok], f"d L / d {k}")
        checked += int(ok.sum())
    gX = X.grad.cpu().numpy().reshape(-1)
    wX = np.zeros_like(gX)
    for i in range(gX.size):
        def pert(d, i=i):
            X2 = Xo.copy().reshape(-1)
            X2[i] += d
            return _oracle_loss(dict(crop, **base), tracks, vm0, vma, X2.reshape(-1, 3))
        wX[i], _ = fd(pert, 1e-6)
    _close(gX, wX, "d L / d X")
    gtw = tw.grad.cpu().numpy()
    lt_of = lambda vm_all: oracle.track(Xo, vm_all, tracks["intr"], tracks["cam"], tracks["pt"],
                                        tracks["xy"], delta=1.0, lam=1e-4, jacobians=False)["loss"]
    for v in sorted(set(np.unique(tracks["cam"]).tolist()) | {0}):
        want = np.zeros(6)
        for e in range(6):
            def pert(d, e=e, v=v):
                xi = np.zeros(6)
                xi[e] = d
                vma2 = vma.copy()
                vma2[v] = _left(vma[v], xi)
                if v == 0:  # the rendered view: photometric and track terms
                    return _oracle_loss(dict(crop, **base), tracks, vma2[0], vma2, Xo)
                return lt_of(vma2), st0  # the other cameras: the track term only
            want[e], ok_ = fd(pert, 1e-6)
            assert ok_, (v, e)
        _close(gtw[v], want, f"d L / d twist {v}")
    print(f"[fd] {checked} Gaussian parameters, {gX.size} point coordinates, twists of "
          f"{len(np.unique(tracks['cam']))} cameras checked")
