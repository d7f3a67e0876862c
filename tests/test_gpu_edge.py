"""Degenerate inputs on the HIP path: no Gaussians, no splat that survives
culling, no track observation.  Front-to-back compositing of an empty list
(the rasterization of Sec. 3.3 and Algorithm 1, a sum over no terms) leaves
the transmittance at 1 and the pixel at the background, and the track loss of
Sec. 3.3 over no observation is 0, so these results are exact."""

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


def _scene(N, seed=31):
    # ragged views: 203 = 12*16 + 11, 150 = 9*16 + 6; 70 x 45 is under 5 x 3 tiles
    s = scenegen.frustum_scene(seed, 203, 150, 238.0, 238.0, max(N, 1), 3, -3.3, 0.6, sh_sd=0.2,
                               unit_quats=False)
    s2 = scenegen.frustum_scene(seed + 1, 70, 45, 82.0, 82.0, 1, 3, -3.3, 0.6, sh_sd=0.2,
                                unit_quats=False)
    s["viewmat"] = np.concatenate([s["viewmat"], s2["viewmat"]])
    s["intr"] = np.concatenate([s["intr"], s2["intr"]])
    s["wh"] = np.concatenate([s["wh"], s2["wh"]])
    if N == 0:
        for k in ("means", "log_scales", "quats", "opacity_logit", "sh"):
            s[k] = s[k][..., :0]
    return s


def _run(gs, s, bg):
    from paper_2603_04847_amd.splat import Splatter
    N = s["means"].shape[1]
    V = s["viewmat"].shape[0]
    ctx = gs.Context(max_pairs=max(V * N, 1), max_isect=1 << 16, max_tiles=4096, max_views=V, max_cams=V)
    sp = Splatter(ctx, gs.default_settings(), _t(bg))
    params = {k: _t(s[k]) for k in ("means", "log_scales", "quats", "opacity_logit", "sh")}
    rgb, T, last, cams = sp.forward(params, 3, _t(s["viewmat"]), _t(s["intr"]), s["wh"])
    v_rgb = _t(np.random.default_rng(3).normal(size=(cams.n_pixels, 3)))
    grads, v_tw = sp.backward(params, 3, cams, T, last, v_rgb)
    torch.cuda.synchronize()
    st = ctx.status()
    return st, rgb.cpu().numpy(), T.cpu().numpy(), last.cpu().numpy(), grads, v_tw.cpu().numpy()


def _assert_background(s, bg, st, rgb, T, last, v_tw):
    P = int(sum(int(w) * int(h) for w, h in s["wh"]))
    assert st["flags"] == 0 and st["n_isect"] == 0
    assert rgb.shape == (P, 3) and np.array_equal(rgb, np.broadcast_to(bg.astype(np.float32), (P, 3)))
    assert np.array_equal(T, np.ones(P, np.float32))
    assert np.array_equal(last, np.zeros(P, np.int32))
    assert np.array_equal(v_tw, np.zeros_like(v_tw))


def test_no_gaussians_renders_background(gs):
    s = _scene(0)
    bg = np.array([0.25, 0.5, 0.75])
    st, rgb, T, last, grads, v_tw = _run(gs, s, bg)
    _assert_background(s, bg, st, rgb, T, last, v_tw)
    assert all(g.numel() == 0 for g in grads.values())


def test_all_splats_culled_renders_background_with_zero_gradients(gs):
    """Every opacity far below the alpha gate: no splat is binned, the image is
    the background, every gradient is exactly zero; the oracle culls them too."""
    s = _scene(400)
    s["opacity_logit"][:] = -40.0
    bg = np.array([0.1, 0.6, 0.3])
    st, rgb, T, last, grads, v_tw = _run(gs, s, bg)
    _assert_background(s, bg, st, rgb, T, last, v_tw)
    for k, g in grads.items():
        assert not torch.any(g != 0).item(), k
    # the oracle reaches the same image on the first view
    s1 = dict(s, viewmat=s["viewmat"][:1], intr=s["intr"][:1], wh=s["wh"][:1])
    o = oracle.render_fwd_bwd(s1, bg=bg)
    assert np.allclose(o["rgb"], bg, rtol=0, atol=0)


def test_track_without_observations(gs):
    """No observation: zero loss and zero gradients, on the atomic and the
    point-indexed paths; the index of no observations is all zeros."""
    sc = scenegen.make_config("C1")
    X = sc["X"]
    Pt = X.shape[0]
    vm, intr = sc["track_viewmat"], sc["track_intr"]
    C = vm.shape[0]
    ctx = gs.Context(max_pairs=Pt, max_isect=1 << 16, max_tiles=16, max_views=1, max_cams=C)
    obs_cam = torch.zeros(0, dtype=torch.int32, device="cuda")
    obs_pt = torch.zeros(0, dtype=torch.int32, device="cuda")
    obs_xy = torch.zeros((0, 2), device="cuda")
    index = gs.track_point_index(ctx, obs_pt, Pt)
    index_pm = gs.track_point_index(ctx, obs_pt, Pt, obs_cam, obs_xy)
    torch.cuda.synchronize()
    assert not torch.any(index[0] != 0).item()
    for pi in (None, index, index_pm):
        loss = torch.zeros(1, device="cuda")
        v_X = torch.zeros((Pt, 3), device="cuda")
        v_tw = torch.zeros((C, 6), device="cuda")
        ctx.reset_status()
        gs.track_reproj_fwd_bwd(ctx, _t(X), _t(vm), _t(intr), obs_cam, obs_pt, obs_xy, 1.0, 1e-4, 0.01,
                                loss, v_X, v_tw, pt_index=pi)
        torch.cuda.synchronize()
        assert loss.item() == 0.0
        assert not torch.any(v_X != 0).item() and not torch.any(v_tw != 0).item()
        assert ctx.status()["n_masked_obs"] == 0


def test_nonfinite_parameters_are_culled_and_flagged(gs):
    """Gaussians with a NaN or infinite parameter (a mean, a log-scale, a
    quaternion, an opacity logit, an SH coefficient) raise GS_FLAG_NONFINITE
    and drop out: the image and every other gradient equal the oracle's for
    the scene without them, and their own gradients are exactly zero."""
    from paper_2603_04847_amd.splat import Splatter
    s = _scene(600, seed=41)
    s1 = dict(s, viewmat=s["viewmat"][:1], intr=s["intr"][:1], wh=s["wh"][:1])
    bad = np.array([3, 50, 77, 140, 201, 333, 420, 599])
    s1 = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in s1.items()}
    s1["means"][0, bad[0]] = np.nan
    s1["means"][2, bad[1]] = np.inf
    s1["log_scales"][1, bad[2]] = np.inf
    s1["log_scales"][0, bad[3]] = -np.inf
    s1["quats"][2, bad[4]] = np.nan
    s1["opacity_logit"][bad[5]] = np.nan
    s1["sh"][0, 1, bad[6]] = np.inf
    s1["sh"][9, 2, bad[7]] = np.nan
    keep = np.setdiff1d(np.arange(600), bad)
    good = dict(s1)
    for k in ("means", "log_scales", "quats", "sh"):
        good[k] = s1[k][..., keep]
    good["opacity_logit"] = s1["opacity_logit"][keep]
    N = 600
    ctx = gs.Context(max_pairs=N, max_isect=1 << 18, max_tiles=4096, max_views=1)
    sp = Splatter(ctx)
    params = {k: _t(s1[k]) for k in ("means", "log_scales", "quats", "opacity_logit", "sh")}
    rgb, T, last, cams = sp.forward(params, 3, _t(s1["viewmat"]), _t(s1["intr"]), s1["wh"])
    torch.cuda.synchronize()
    assert ctx.status()["flags"] & gs._lib.GS_FLAG_NONFINITE
    o = oracle.render_fwd_bwd(good)
    ok = ~o["ambiguous"]
    g = rgb.cpu().numpy()
    assert np.all(np.isfinite(g))
    assert np.max(np.abs(g[ok] - o["rgb"][ok])) <= 1e-4
    w = np.random.default_rng(2).normal(size=(cams.n_pixels, 3))
    w[o["ambiguous"]] = 0.0
    grads, v_tw = sp.backward(params, 3, cams, T, last, _t(w))
    og = oracle.render_fwd_bwd(good, v_rgb=w)["grads"]
    for k in ("means", "log_scales", "quats", "opacity_logit", "sh"):
        a = grads[k].cpu().numpy()
        assert not np.any(a[..., bad]), k
        err = np.max(np.abs(a[..., keep] - og[k]))
        assert err <= 1e-4 * np.max(np.abs(og[k])), (k, err)
    tw = v_tw.cpu().numpy()[0]
    assert np.max(np.abs(tw - og["twist"][0])) <= 1e-4 * np.max(np.abs(og["twist"][0]))


def test_render_bwd_checks_everything_before_enqueueing(gs):
    """A backward rejected by an argument check (a missing gradient array)
    enqueues nothing: the next, valid backward finds no stale 2D gradients."""
    from paper_2603_04847_amd.splat import Splatter
    import paper_2603_04847_amd._lib as L
    s = _scene(500, seed=43)
    s1 = dict(s, viewmat=s["viewmat"][:1], intr=s["intr"][:1], wh=s["wh"][:1])
    ctx = gs.Context(max_pairs=500, max_isect=1 << 18, max_tiles=4096, max_views=1)
    sp = Splatter(ctx)
    params = {k: _t(s1[k]) for k in ("means", "log_scales", "quats", "opacity_logit", "sh")}
    rgb, T, last, cams = sp.forward(params, 3, _t(s1["viewmat"]), _t(s1["intr"]), s1["wh"])
    v_rgb = _t(np.random.default_rng(4).normal(size=(cams.n_pixels, 3)))
    ref, ref_tw = sp.backward(params, 3, cams, T, last, v_rgb)
    ref = {k: v.clone() for k, v in ref.items()}
    g = L.make_gaussians(*(params[k] for k in ("means", "log_scales", "quats", "opacity_logit", "sh")), 3)
    gr = {k: torch.empty_like(v) for k, v in params.items()}
    bad = L.make_grads(gr["means"], gr["log_scales"], None, gr["opacity_logit"], gr["sh"])
    v_tw = torch.zeros((1, 6), device="cuda")
    with pytest.raises(gs.GsError) as e:
        L.gs_render_bwd(ctx, g, cams, sp.settings, None, T, last, v_rgb, bad, v_tw)
    assert e.value.code == -1
    again, tw2 = sp.backward(params, 3, cams, T, last, v_rgb)
    torch.cuda.synchronize()
    for k in ref:
        a, b = again[k].cpu().numpy(), ref[k].cpu().numpy()
        assert np.max(np.abs(a - b)) <= 1e-5 * (np.max(np.abs(b)) + 1e-30), k
    assert not torch.any(v_tw != 0).item()


def test_entry_counts_past_the_packed_count_field(gs):
    """The depth sort carries each pair's block-entry count in the bits above
    its pair index; past 2^25 pairs that leaves 6 bits, and larger counts are
    read back from the per-pair array.  48 splats of unit scale, each meeting
    far more than 63 blocks of a 1024 x 768 view, render the same image with
    and without 2^25 - 47 culled Gaussians after them (the pair indices of the
    48 do not change), and their gradients agree to float-atomic rounding."""
    from paper_2603_04847_amd.splat import Splatter
    s = scenegen.frustum_scene(47, 1024, 768, 600.0, 600.0, 48, 0, 0.0, 0.0, sh_sd=0.3)
    keys = ("means", "log_scales", "quats", "opacity_logit", "sh")
    small = {k: _t(s[k]) for k in keys}
    n_big = (1 << 25) + 1
    pad = n_big - 48
    big = {
        "means": torch.cat([small["means"], torch.zeros((3, pad), device="cuda")], 1),
        "log_scales": torch.cat([small["log_scales"], torch.full((3, pad), -5.0, device="cuda")], 1),
        "quats": torch.cat([small["quats"], torch.tensor([[1.0], [0.0], [0.0], [0.0]], device="cuda").expand(4, pad)], 1),
        "opacity_logit": torch.cat([small["opacity_logit"], torch.full((pad,), -40.0, device="cuda")]),
        "sh": torch.cat([small["sh"], torch.zeros((1, 3, pad), device="cuda")], 2),
    }
    big = {k: v.contiguous() for k, v in big.items()}
    vm, intr = _t(s["viewmat"]), _t(s["intr"])
    v_rgb = _t(np.random.default_rng(5).normal(size=(1024 * 768, 3)))
    out = []
    for params, n in ((small, 48), (big, n_big)):
        print(f"[entry counts] N = {n}", flush=True)
        ctx = gs.Context(max_pairs=n, max_isect=1 << 20, max_tiles=4096, max_views=1)
        sp = Splatter(ctx)
        rgb, T, last, cams = sp.forward(params, 0, vm, intr, s["wh"])
        grads, v_tw = sp.backward(params, 0, cams, T, last, v_rgb)
        torch.cuda.synchronize()
        st = ctx.status()
        assert st["flags"] == 0, st
        out.append((rgb.cpu().numpy(), T.cpu().numpy(), last.cpu().numpy(),
                    {k: g[..., :48].cpu().numpy() for k, g in grads.items()}, v_tw.cpu().numpy(),
                    st["n_isect"]))
        del ctx, sp, grads
    (r0, T0, l0, g0, tw0, i0), (r1, T1, l1, g1, tw1, i1) = out
    # tile entries past 48 x 63 x 16: some splat meets more than 63 blocks of
    # 16 tiles, so its count took the escape
    assert i0 == i1 and i0 > 48 * 63 * 16
    assert np.array_equal(r0, r1) and np.array_equal(T0, T1) and np.array_equal(l0, l1)
    for k in keys:
        assert np.max(np.abs(g0[k] - g1[k])) <= 1e-5 * (np.max(np.abs(g0[k])) + 1e-30), k
    assert np.max(np.abs(tw0 - tw1)) <= 1e-5 * np.max(np.abs(tw0))
