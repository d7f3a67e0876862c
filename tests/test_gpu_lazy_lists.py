"""Lazy tile lists (gs_settings.lazy_lists = 1): the forward draws each tile's
list from its block's list and writes the part it reads.  Against the full
lists of the same scene:

* image, final transmittance and last-contributor positions bit for bit, and
  the same per-tile workload counts, for every tile shape and launch order,
  over ragged views;
* the tile lists the lazy forward wrote equal the full ones over every entry
  the forward read;
* the backward after the lazy forward, and a backward run straight after a
  lazy bin step (which writes the lists in full first), give the gradients of
  the full lists (up to the order of float atomics)."""

import numpy as np
import pytest

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


@pytest.fixture(scope="module")
def scene():
    s = scenegen.blob_scene(23, [(203, 150), (96, 64), (130, 77)], 15000, sh_degree=2)
    s.pop("_rng")
    return s


def _t(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def _close(a, b, rtol, what):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    err = np.max(np.abs(a - b)) if a.size else 0.0
    assert err <= rtol * max(np.max(np.abs(b)), 1e-30), f"{what}: {err:.3e}"


KEYS = ("means", "log_scales", "quats", "opacity_logit", "sh")


def _run(gs, sc, tile, order, lazy, forward=True):
    """Project, bin, (forward), backward on a fresh context; returns the
    outputs, the per-tile counts of the counting forward and the lists."""
    from paper_2603_04847_amd import _lib as L
    V, N = sc["viewmat"].shape[0], sc["means"].shape[1]
    ctx = gs.Context(max_pairs=V * N, max_isect=4_000_000, max_tiles=200_000, max_views=V)
    params = {k: _t(sc[k]) for k in KEYS}
    g = L.make_gaussians(*(params[k] for k in KEYS), sc["sh_degree"])
    cams = L.Cameras(_t(sc["viewmat"]), _t(sc["intr"]), sc["wh"])
    s = gs.default_settings(tile_w=tile[0], tile_h=tile[1], tile_order=order, eval_stats=1,
                            lazy_lists=int(lazy))
    P = cams.n_pixels
    rgb = torch.empty((P, 3), device="cuda")
    T = torch.empty((P,), device="cuda")
    last = torch.empty((P,), device="cuda", dtype=torch.int32)
    L.gs_project(ctx, g, cams, s)
    L.gs_bin_sort(ctx, cams, N, s)
    out = {}
    if forward:
        L.gs_render_fwd(ctx, cams, s, None, rgb, T, last)
        torch.cuda.synchronize()
        ts = L.gs_ctx_tile_stats(ctx)
        nt = ts["n_tiles"]
        for k in ("tile_entries", "tile_contrib", "tile_evals"):
            out[k] = L.copy_to_host(ts[k], nt, np.int32).copy()
        b = ctx.buffers()
        out["ranges"] = L.copy_to_host(b["tile_ranges"], 2 * nt, np.int32).reshape(nt, 2).copy()
        n = int(out["ranges"][:, 1].max()) if nt else 0
        out["ids"] = L.copy_to_host(b["isect_ids"], n, np.int32).view(np.uint32).copy()
        out["rgb"], out["T"], out["last"] = rgb.cpu().numpy(), T.cpu().numpy(), last.cpu().numpy()
    return ctx, g, cams, s, params, out


def _backward(gs, ctx, g, cams, s, params, T, last, w):
    from paper_2603_04847_amd import _lib as L
    grads = {k: torch.empty_like(params[k]) for k in KEYS}
    v_tw = torch.zeros((cams.V, 6), device="cuda")
    L.gs_render_bwd(ctx, g, cams, s, None, T, last, w, L.make_grads(*(grads[k] for k in KEYS)), v_tw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in grads.items()}, v_tw.cpu().numpy()


@pytest.mark.parametrize("order", [0, 1, 2])
@pytest.mark.parametrize("tile", [(16, 16), (16, 8), (8, 8), (32, 16)])
def test_lazy_lists_render_bitwise_and_lists_agree(gs, scene, tile, order):
    print(f"[lazy] tile {tile} order {order}", flush=True)
    # (the Gaussian structs hold raw pointers: every run's tensors stay referenced)
    ctx_f, g_f, cams, s_f, params, full = _run(gs, scene, tile, order, lazy=False)
    ctx_l, g_l, cams_l, s_l, params_l, lazy = _run(gs, scene, tile, order, lazy=True)
    for k in ("rgb", "T", "last", "tile_entries", "tile_contrib", "tile_evals"):
        assert np.array_equal(full[k], lazy[k]), k
    assert np.array_equal(full["ranges"], lazy["ranges"])
    # every entry the forward read is in the lazily written lists
    r = full["ranges"]
    read = np.zeros(full["ids"].shape, bool)
    for t in np.nonzero(full["tile_entries"])[0]:
        read[r[t, 0]:r[t, 0] + full["tile_entries"][t]] = True
    assert read.sum() == full["tile_entries"].sum() > 0
    assert np.array_equal(full["ids"][read], lazy["ids"][read])
    # the backward reads no further than the lists hold
    w = _t(np.random.default_rng(5).normal(size=(cams.n_pixels, 3)))
    T, last = _t(full["T"]), _t(full["last"], torch.int32)
    gf, tf = _backward(gs, ctx_f, g_f, cams, s_f, params, T, last, w)
    gl, tl = _backward(gs, ctx_l, g_l, cams_l, s_l, params_l, T, last, w)
    for k in gf:
        _close(gl[k], gf[k], 1e-5, k)
    _close(tl, tf, 1e-5, "twist")
    ctx_f.close()
    ctx_l.close()


def test_backward_straight_after_a_lazy_bin_step(gs, scene):
    """No forward between the lazy bin step and the backward: the backward
    writes the lists in full first, and its gradients are those of the full
    lists (T_final and last taken from a forward on another context)."""
    tile = (16, 16)
    ctx_f, g_f, cams, s_f, params, full = _run(gs, scene, tile, 0, lazy=False)
    ctx_l, g_l, cams_l, s_l, params_l, _ = _run(gs, scene, tile, 0, lazy=True, forward=False)
    w = _t(np.random.default_rng(6).normal(size=(cams.n_pixels, 3)))
    T, last = _t(full["T"]), _t(full["last"], torch.int32)
    gf, tf = _backward(gs, ctx_f, g_f, cams, s_f, params, T, last, w)
    gl, tl = _backward(gs, ctx_l, g_l, cams_l, s_l, params_l, T, last, w)
    for k in gf:
        _close(gl[k], gf[k], 1e-5, k)
    _close(tl, tf, 1e-5, "twist")
    # and the lists are now complete
    from paper_2603_04847_amd import _lib as L
    b = ctx_l.buffers()
    n = int(full["ranges"][:, 1].max())
    ids = L.copy_to_host(b["isect_ids"], n, np.int32).view(np.uint32)
    assert np.array_equal(ids, full["ids"])
    ctx_f.close()
    ctx_l.close()
