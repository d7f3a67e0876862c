"""The photometric loss (1 - lambda) L1 + lambda (1 - SSIM) and its image
gradient (Sec. 3.3 eq. L_photo, lambda = 0.2) through the C ABI against the
FP64 oracle: ragged views (one smaller than the 11 x 11 window), the L1-only
and SSIM-only ends of lambda, exact ties, and a full-size batch of rendered
views."""

import numpy as np
import pytest

import oracle
import scenegen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

RTOL = 1e-4


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_04847_amd as P
    P.load()
    return P


def _t(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def _close(a, b, what, rtol=RTOL):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    err = np.max(np.abs(a - b))
    assert err <= rtol * np.max(np.abs(b)), f"{what}: {err:.3e} vs {rtol * np.max(np.abs(b)):.3e}"


def _photo(gs, wh, x, y, lam):
    P = int((wh[:, 0].astype(np.int64) * wh[:, 1]).sum())
    ctx = gs.Context(max_pairs=1, max_isect=1, max_tiles=16, max_views=wh.shape[0])
    cams = gs.Cameras(_t(np.zeros((wh.shape[0], 12))), _t(np.zeros((wh.shape[0], 4))), wh)
    v = torch.empty((P, 3), device="cuda")
    loss = torch.zeros(1, device="cuda")
    gs.gs_photo_loss_grad(ctx, cams, _t(x), _t(y), lam, v, loss)
    torch.cuda.synchronize()
    return loss.item(), v.cpu().numpy()


@pytest.mark.parametrize("lam", [0.2, 1.0, 0.0])
def test_photo_loss_matches_oracle_on_ragged_views(gs, lam):
    # 203 x 150 (ragged against 32 x 32 tiles), 70 x 45, and 9 x 6 (smaller
    # than the window); smooth content plus noise, a few exact ties
    rng = np.random.default_rng(3)
    wh = np.array([[203, 150], [70, 45], [9, 6]], np.int32)
    P = int((wh[:, 0] * wh[:, 1]).sum())
    u = np.concatenate([np.tile(np.arange(w), h) for w, h in wh]).astype(float)
    base = 0.5 + 0.3 * np.sin(u[:, None] * np.array([0.05, 0.08, 0.11]))
    x = np.clip(base + rng.normal(0, 0.05, (P, 3)), 0, 1).astype(np.float32)
    y = np.clip(base + rng.normal(0, 0.05, (P, 3)), 0, 1).astype(np.float32)
    y[:40] = x[:40]
    loss, v = _photo(gs, wh, x, y, lam)
    want_l, want_v = oracle.photo_loss(x, y, wh, lam=lam)
    assert abs(loss - want_l) <= RTOL * abs(want_l), (loss, want_l)
    _close(v, want_v, f"v_rgb lambda={lam}")


def test_ssim_of_identical_images(gs):
    rng = np.random.default_rng(4)
    wh = np.array([[64, 40]], np.int32)
    x = rng.uniform(size=(64 * 40, 3)).astype(np.float32)
    loss, v = _photo(gs, wh, x, x, 1.0)
    assert abs(loss) <= 1e-6                 # 1 - SSIM(x, x) = 0
    # zero up to rounding: against the gradient's natural scale (~10 per pixel
    # and channel before the 1 / (3 P) weight)
    assert np.max(np.abs(v)) <= 1e-4 * 10 / (3 * 64 * 40)


def test_photo_loss_full_size_rendered_batch(gs):
    """A batch of the joint step at full size: 4 rendered views of 1237 x 822
    against their targets, lambda = 0.2."""
    from paper_2603_04847_amd.step import JointStep
    sc = scenegen.make_config("C4")
    b = scenegen.batch_views(4, sc["viewmat"].shape[0], 4, 1)
    tg = [scenegen.view_targets(4, sc["wh"], bb) for bb in b]
    st = JointStep(sc, b, tg, max_isect=120_000_000, lambda_ssim=0.2)
    st.forward_backward(0)
    torch.cuda.synchronize()
    rgb = st.rgb.cpu().numpy()
    wh = st.wh_all[b[0]]
    loss, v = _photo(gs, wh, rgb, tg[0], 0.2)
    want_l, want_v = oracle.photo_loss(rgb, tg[0], wh, lam=0.2)
    assert abs(loss - want_l) <= RTOL * abs(want_l), (loss, want_l)
    _close(v, want_v, "v_rgb full size")
