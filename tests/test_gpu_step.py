"""GPU tests of the autograd wrappers and of the joint step (Algorithm 1, one
iteration) replayed as a captured HIP graph.

Gradients of the autograd Functions are compared with the oracle composed with
the SE(3) left Jacobian: d L / d dT = J_l(dT)^T g, g the left-twist gradient at
the composed pose Exp(dT) T0.
"""

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
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)
    return t.requires_grad_(grad)


def _close(a, b, what, rtol=1e-4):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    err = np.max(np.abs(a - b))
    assert err <= rtol * np.max(np.abs(b)), f"{what}: {err:.3e} vs {rtol * np.max(np.abs(b)):.3e}"


def _scene():
    return scenegen.frustum_scene(77, 120, 90, 140.0, 140.0, 1500, 3, -3.0, 0.5, sh_sd=0.2,
                                  n_tracks=80)


def test_rasterize_autograd_with_pose_twist(gs):
    from paper_2603_04847_amd.splat import Splatter, rasterize
    sc = _scene()
    N = sc["means"].shape[1]
    twist = np.array([[0.01, -0.02, 0.015, 0.004, -0.003, 0.002]], np.float32)
    params = {k: _t(sc[k], grad=True) for k in ("means", "log_scales", "quats", "opacity_logit", "sh")}
    tw = _t(twist, grad=True)
    ctx = gs.Context(max_pairs=N, max_isect=2_000_000, max_tiles=1000, max_views=1)
    sp = Splatter(ctx)
    img = rasterize(params, 3, tw, _t(sc["viewmat"]), _t(sc["intr"]), sc["wh"], sp)
    # the oracle renders at the composed pose
    vm = oracle.se3_exp_compose(twist.astype(np.float64), sc["viewmat"].astype(np.float64))
    o = oracle.render_fwd_bwd(sc, viewmat=vm)
    w = np.random.default_rng(0).normal(size=img.shape)
    w[o["ambiguous"]] = 0
    (img * _t(w)).sum().backward()
    og = oracle.render_fwd_bwd(sc, v_rgb=w, viewmat=vm)["grads"]
    for k in ("means", "log_scales", "quats", "opacity_logit", "sh"):
        _close(params[k].grad.cpu().numpy(), og[k], k)
    want = oracle.se3_jl_transpose(twist.astype(np.float64), og["twist"])
    _close(tw.grad.cpu().numpy(), want, "twist")


def test_track_autograd_and_dual_gradient_flow(gs):
    from paper_2603_04847_amd.splat import Splatter, rasterize, track_loss
    sc = _scene()
    N = sc["means"].shape[1]
    V = sc["track_viewmat"].shape[0]
    rng = np.random.default_rng(1)
    twist = (rng.normal(size=(V, 6)) * 0.003).astype(np.float32)
    tw = _t(twist, grad=True)
    X = _t(sc["X"], grad=True)
    ctx = gs.Context(max_pairs=N, max_isect=2_000_000, max_tiles=1000, max_views=1, max_cams=V)
    lt = track_loss(X, tw, _t(sc["track_viewmat"]), _t(sc["track_intr"]),
                    _t(sc["obs_cam"], torch.int32), _t(sc["obs_pt"], torch.int32), _t(sc["obs_xy"]),
                    ctx, delta=1.0, lam=1e-4)
    # photometric term on camera 0 (same twist row 0)
    params = {k: _t(sc[k]) for k in ("means", "log_scales", "quats", "opacity_logit", "sh")}
    sp = Splatter(ctx)
    img = rasterize(params, 3, tw[0:1], _t(sc["viewmat"]), _t(sc["intr"]), sc["wh"], sp)
    vm_all = oracle.se3_exp_compose(twist.astype(np.float64), sc["track_viewmat"].astype(np.float64))
    o = oracle.render_fwd_bwd(sc, viewmat=vm_all[:1])
    w = rng.normal(size=img.shape)
    w[o["ambiguous"]] = 0
    (lt + (img * _t(w)).sum()).backward()
    ot = oracle.track(sc["X"], vm_all, sc["track_intr"], sc["obs_cam"], sc["obs_pt"], sc["obs_xy"],
                      delta=1.0, lam=1e-4)
    assert abs(lt.item() - ot["loss"]) <= 1e-4 * ot["loss"]
    _close(X.grad.cpu().numpy(), ot["v_X"], "X")
    g_photo = oracle.render_fwd_bwd(sc, v_rgb=w, viewmat=vm_all[:1])["grads"]["twist"]
    g = ot["v_twist"].copy()
    g[0] += g_photo[0]            # camera 0 receives both gradients
    want = oracle.se3_jl_transpose(twist.astype(np.float64), g)
    for v in range(V):
        _close(tw.grad.cpu().numpy()[v], want[v], f"twist {v}")


def test_joint_step_graph_replays_match_eager(gs):
    from paper_2603_04847_amd.step import JointStep
    sc = scenegen.blob_scene(5, [(160, 120)] * 6, 20000, sh_degree=3)
    rng = sc.pop("_rng")
    sc.update(scenegen.make_tracks(rng, 3000, sc["viewmat"], sc["intr"], sc["wh"], 12))
    batches = [np.array([0, 2, 5]), np.array([1, 3, 4])]
    targets = [scenegen.view_targets(5, sc["wh"], b) for b in batches]
    st = JointStep(sc, batches, targets, max_isect=4_000_000)
    keys = list(st._opt_params().keys())

    def snapshot():
        return {k: v.detach().clone() for k, v in st._opt_params().items()}, \
            {k: v.clone() for k, v in st.m.items()}, {k: v.clone() for k, v in st.v.items()}

    def restore(s):
        p, m, v = s
        for k in keys:
            st._opt_params()[k].copy_(p[k])
            st.m[k].copy_(m[k])
            st.v[k].copy_(v[k])

    st.run(0, step=1)  # warm up (also allocates nothing new)
    torch.cuda.synchronize()
    s0 = snapshot()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        st.run(1, step=1)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    restore(s0)
    with torch.cuda.graph(g):
        st.run(1, step=1)
    torch.cuda.synchronize()
    for rep in range(3):
        restore(s0)
        st.run(1, step=1)                       # eager reference
        torch.cuda.synchronize()
        ref = {k: v.detach().clone() for k, v in st._opt_params().items()}
        loss_ref = st.loss.clone()
        restore(s0)
        st.run(0, step=1)                       # unrelated eager work between replays
        torch.cuda.synchronize()
        restore(s0)
        g.replay()
        torch.cuda.synchronize()
        assert st.ctx.status()["flags"] == 0
        for k in keys:
            a = st._opt_params()[k].cpu().numpy()
            b = ref[k].cpu().numpy()
            # Adam's first step moves each parameter by lr * g/(|g|+eps): the
            # order of float atomics can flip only near-zero gradients
            diff = np.abs(a - b)
            assert np.mean(diff > 1e-6 * (1 + np.abs(b))) < 1e-3, (rep, k)
        assert torch.allclose(st.loss, loss_ref, rtol=1e-5), rep


def test_fused_gaussian_adam_matches_separate_adam(gs):
    """gs_project_bwd_adam (the Gaussians' Adam step taken inside the
    projection backward) against gs_project_bwd followed by gs_adam_step, over
    two consecutive iterations (the second uses the moments of the first)."""
    from paper_2603_04847_amd.step import JointStep
    sc = scenegen.blob_scene(6, [(150, 110)] * 4, 12000, sh_degree=3)
    rng = sc.pop("_rng")
    sc.update(scenegen.make_tracks(rng, 2000, sc["viewmat"], sc["intr"], sc["wh"], 10))
    batches = [np.array([0, 3]), np.array([1, 2])]
    targets = [scenegen.view_targets(6, sc["wh"], b) for b in batches]
    st = JointStep(sc, batches, targets, max_isect=3_000_000)
    keys = list(st._opt_params().keys())
    p0 = {k: v.detach().clone() for k, v in st._opt_params().items()}

    def reset():
        for k in keys:
            st._opt_params()[k].copy_(p0[k])
            st.m[k].zero_()
            st.v[k].zero_()

    reset()
    for step in (1, 2):
        st.forward_backward(step - 1)
        st.adam(step=step)
    torch.cuda.synchronize()
    ref = {k: (st._opt_params()[k].cpu().numpy(), st.m[k].cpu().numpy(), st.v[k].cpu().numpy())
           for k in keys}
    reset()
    for step in (1, 2):
        st.run(step - 1, step=step)
    torch.cuda.synchronize()
    assert st.ctx.status()["flags"] == 0
    for k in keys:
        got = (st._opt_params()[k].cpu().numpy(), st.m[k].cpu().numpy(), st.v[k].cpu().numpy())
        for what, a, b in zip(("param", "exp_avg", "exp_avg_sq"), got, ref[k]):
            # float atomics in the raster backward may round a 2D gradient
            # differently between runs; Adam's first steps magnify that only
            # for near-zero gradients
            diff = np.abs(a - b)
            assert np.mean(diff > 1e-5 * (1e-3 + np.abs(b))) < 2e-3, (k, what)
        assert not np.array_equal(st._opt_params()[k].cpu().numpy(), p0[k].cpu().numpy()), k


def test_graph_replays_take_successive_adam_steps(gs):
    """A step captured once replays as successive iterations: the Adam step
    number lives on the device and each replay advances it, so two replays
    equal eager steps 1 and 2 (bias corrections 1 / (1 - beta^t) of t = 1, 2)."""
    from paper_2603_04847_amd.step import JointStep
    sc = scenegen.blob_scene(7, [(150, 110)] * 4, 12000, sh_degree=3)
    rng = sc.pop("_rng")
    sc.update(scenegen.make_tracks(rng, 2000, sc["viewmat"], sc["intr"], sc["wh"], 10))
    batches = [np.array([0, 3]), np.array([1, 2])]
    targets = [scenegen.view_targets(7, sc["wh"], b) for b in batches]
    st = JointStep(sc, batches, targets, max_isect=3_000_000)
    keys = list(st._opt_params().keys())
    p0 = {k: v.detach().clone() for k, v in st._opt_params().items()}

    def reset():
        for k in keys:
            st._opt_params()[k].copy_(p0[k])
            st.m[k].zero_()
            st.v[k].zero_()
        st.set_step(0)

    reset()
    st.run(0, step=1)
    st.run(1, step=2)
    torch.cuda.synchronize()
    ref = {k: v.detach().cpu().numpy().copy() for k, v in st._opt_params().items()}
    # capture one graph per batch (warm-up on a side stream first)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        st.run(0)
        st.run(1)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graphs = []
    for b in (0, 1):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            st.run(b)
        graphs.append(g)
    torch.cuda.synchronize()
    for rep in range(2):
        reset()
        torch.cuda.synchronize()
        graphs[0].replay()
        graphs[1].replay()
        torch.cuda.synchronize()
        assert int(st.d_step.item()) == 2
        for k in keys:
            a = st._opt_params()[k].cpu().numpy()
            diff = np.abs(a - ref[k])
            assert np.mean(diff > 1e-5 * (1e-3 + np.abs(ref[k]))) < 2e-3, (rep, k)
    # replaying step 2 with the bias of step 1 would move the parameters
    # differently: the same two replays from a counter at 5 (steps 6, 7) differ
    reset()
    st.set_step(5)
    graphs[0].replay()
    graphs[1].replay()
    torch.cuda.synchronize()
    moved = [np.mean(np.abs(st._opt_params()[k].cpu().numpy() - ref[k]) > 1e-6 * (1 + np.abs(ref[k])))
             for k in ("means", "log_scales")]
    assert max(moved) > 0.05


def test_two_forwards_then_backward(gs):
    """Two rasterize calls on one Splatter before one backward (gradient
    accumulation over two batches): the first call's backward re-projects and
    re-bins because the second replaced its lists; both gradients land."""
    from paper_2603_04847_amd.splat import Splatter, rasterize
    sc = scenegen.blob_scene(9, [(120, 90), (100, 80)], 5000, sh_degree=2)
    sc.pop("_rng")
    N = sc["means"].shape[1]
    params = {k: _t(sc[k], grad=True) for k in ("means", "log_scales", "quats", "opacity_logit", "sh")}
    tw = _t(np.zeros((2, 6), np.float32), grad=True)
    ctx = gs.Context(max_pairs=N, max_isect=2_000_000, max_tiles=2000, max_views=1)
    sp = Splatter(ctx)
    vm, intr = _t(sc["viewmat"]), _t(sc["intr"])
    img0 = rasterize(params, 2, tw[0:1], vm[0:1], intr[0:1], sc["wh"][0:1], sp)
    img1 = rasterize(params, 2, tw[1:2], vm[1:2], intr[1:2], sc["wh"][1:2], sp)
    s0 = dict(sc, viewmat=sc["viewmat"][:1], intr=sc["intr"][:1], wh=sc["wh"][:1])
    s1 = dict(sc, viewmat=sc["viewmat"][1:], intr=sc["intr"][1:], wh=sc["wh"][1:])
    o0, o1 = oracle.render_fwd_bwd(s0), oracle.render_fwd_bwd(s1)
    rng = np.random.default_rng(5)
    w0 = rng.normal(size=img0.shape)
    w1 = rng.normal(size=img1.shape)
    w0[o0["ambiguous"]] = 0
    w1[o1["ambiguous"]] = 0
    ((img0 * _t(w0)).sum() + (img1 * _t(w1)).sum()).backward()
    g0 = oracle.render_fwd_bwd(s0, v_rgb=w0)["grads"]
    g1 = oracle.render_fwd_bwd(s1, v_rgb=w1)["grads"]
    for k in ("means", "log_scales", "quats", "opacity_logit", "sh"):
        _close(params[k].grad.cpu().numpy(), g0[k] + g1[k], k)
    want = np.concatenate([g0["twist"], g1["twist"]])  # J_l(0) = I
    _close(tw.grad.cpu().numpy(), want, "twist")


def test_checkpoint_round_trip(gs, tmp_path):
    """save_state / load_state: two steps, a checkpoint, a third step; then
    the checkpoint loaded back into a step perturbed by two more steps and the
    third step taken again from it: the same parameters, moments and step
    counters (to the atomics' summation-order rounding)."""
    from paper_2603_04847_amd.step import JointStep
    sc = scenegen.blob_scene(9, [(150, 110)] * 4, 8000, sh_degree=3)
    rng = sc.pop("_rng")
    sc.update(scenegen.make_tracks(rng, 1500, sc["viewmat"], sc["intr"], sc["wh"], 10))
    batches = [np.array([0, 3]), np.array([1, 2])]
    targets = [scenegen.view_targets(9, sc["wh"], b) for b in batches]
    st = JointStep(sc, batches, targets, max_isect=3_000_000)
    st.run(0)
    st.run(1)
    f = tmp_path / "state.npz"
    st.save_state(str(f))
    st.run(0)
    torch.cuda.synchronize()
    want = {k: (v.detach().cpu().numpy().copy(), st.m[k].cpu().numpy().copy(), st.v[k].cpu().numpy().copy())
            for k, v in st._opt_params().items()}
    st.run(1)
    st.run(0)
    st.load_state(str(f))
    assert st.step_count == 2 and int(st.d_step.item()) == 2
    st.run(0)
    torch.cuda.synchronize()
    assert st.step_count == 3 and int(st.d_step.item()) == 3
    for k, v in st._opt_params().items():
        for got, ref, what in ((v.detach().cpu().numpy(), want[k][0], "param"),
                               (st.m[k].cpu().numpy(), want[k][1], "m"),
                               (st.v[k].cpu().numpy(), want[k][2], "v")):
            bad = np.abs(got - ref) > 1e-5 * (1e-3 + np.abs(ref))
            assert np.mean(bad) < 2e-3, (k, what)
    with np.load(str(f), allow_pickle=False) as z:
        assert set(z["step"].tolist()) == {2}
        assert z["param/sh"].shape == tuple(st.params["sh"].shape)


def test_track_on_a_second_stream_matches_in_line(gs):
    """The joint step with the track term on its own stream (the default: it
    joins before the projection backward adds its twist rows) against the
    same step with every call in line."""
    from paper_2603_04847_amd.step import JointStep
    sc = scenegen.blob_scene(9, [(150, 110)] * 4, 12000, sh_degree=3)
    rng = sc.pop("_rng")
    sc.update(scenegen.make_tracks(rng, 2000, sc["viewmat"], sc["intr"], sc["wh"], 10))
    batches = [np.array([0, 3]), np.array([1, 2])]
    targets = [scenegen.view_targets(9, sc["wh"], b) for b in batches]
    st = JointStep(sc, batches, targets, max_isect=3_000_000)
    assert st.overlap_track
    outs = []
    for overlap in (True, False):
        st.overlap_track = overlap
        st.forward_backward(1)
        torch.cuda.synchronize()
        outs.append(dict(v_X=st.v_X.cpu().numpy().copy(), v_tw=st.v_tw.cpu().numpy().copy(),
                         loss=st.loss.cpu().numpy().copy(),
                         **{k: v.cpu().numpy().copy() for k, v in st.grads.items()}))
    a, b = outs
    # the track term's sums run in a fixed order: its gradient is the same bit for bit
    assert np.array_equal(a["v_X"], b["v_X"])
    assert a["loss"][1] == b["loss"][1]
    for k in a:
        _close(a[k], b[k], f"{k} (second stream vs in line)", rtol=1e-5)
