"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Rule for floating point: per tensor group, max|gpu - oracle| <= 1e-4 * max|oracle|
(images: 1e-4 * max(max|oracle|, 1)), over pixels the oracle does not flag as
ambiguous (a gate, clamp, stop or depth-order decision within float32 error of
its threshold).  Integer and index results are compared bit-exactly.
"""

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


def _params(scene):
    return {k: _t(scene[k]) for k in ("means", "log_scales", "quats", "opacity_logit", "sh")}


def _ctx(gs, scene, max_isect=4_000_000, views=None, max_cams=8):
    N = scene["means"].shape[1]
    V = scene["viewmat"].shape[0] if views is None else views
    return gs.Context(max_pairs=V * N, max_isect=max_isect, max_tiles=200_000, max_views=max(V, 1),
                      max_cams=max_cams)


def _render(gs, scene, ctx=None, settings=None, bg=None):
    from paper_2603_04847_amd.splat import Splatter
    ctx = ctx or _ctx(gs, scene)
    sp = Splatter(ctx, settings or gs.default_settings(), bg)
    params = _params(scene)
    rgb, T, last, cams = sp.forward(params, scene["sh_degree"], _t(scene["viewmat"]),
                                    _t(scene["intr"]), scene["wh"])
    torch.cuda.synchronize()
    return sp, params, rgb, T, last, cams, ctx


def _close(a, b, scale=None, rtol=RTOL, what=""):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    s = np.max(np.abs(b)) if scale is None else scale
    err = np.max(np.abs(a - b)) if a.size else 0.0
    assert err <= rtol * max(s, 1e-30), f"{what}: max err {err:.3e} vs tol {rtol * s:.3e}"


def _parity_scene(seed=101, W=203, H=150, N=3000, deg=3):
    # ragged: 203 = 12*16 + 11, 150 = 9*16 + 6
    return scenegen.frustum_scene(seed, W, H, 1.1719 * W, 1.1719 * W, N, deg, -3.3, 0.6,
                                  sh_sd=0.2, unit_quats=False)


# ------------------------------------------------------------------ projection

def test_project_matches_oracle(gs):
    sc = _parity_scene()
    sp, params, rgb, T, last, cams, ctx = _render(gs, sc)
    N = sc["means"].shape[1]
    rec_host = gs._lib.copy_to_host(ctx.buffers()["records"], N * 12, np.float32).reshape(N, 12)
    pr = oracle.project(sc)
    valid = pr["valid"].astype(bool)
    gvalid = rec_host[:, 3] > 0
    assert np.array_equal(valid, gvalid)
    _close(rec_host[valid, 0:2], pr["mean2d"][valid], what="mean2d")
    _close(rec_host[valid, 2], pr["depth"][valid], what="depth")
    _close(rec_host[valid, 3], pr["opacity"][valid], what="opacity")
    _close(rec_host[valid, 4:7], pr["conic"][valid], what="conic")
    _close(rec_host[valid][:, [7, 8, 9]], pr["rgb"][valid], what="rgb")


# ------------------------------------------------------------------ bin / sort

@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 16)])
def test_bin_sort_bit_exact_on_synthetic_records(gs, tile):
    wh = np.array([[203, 150], [64, 48], [130, 77]], np.int32)
    N = 700
    r = scenegen.synthetic_records(7, 3, wh, N, tile=tile)
    rec = np.zeros((3 * N, 12), np.float32)
    rec[:, 0:2] = r["mean2d"]
    rec[:, 2] = r["depth"]
    rec[:, 3] = np.where(r["valid"] > 0, r["opacity"], 0.0)
    rec[:, 4:7] = r["conic"]
    rec[:, 7:10] = r["rgb"]
    ctx = gs.Context(max_pairs=3 * N, max_isect=2_000_000, max_tiles=100_000, max_views=3)
    s = gs.default_settings(tile_w=tile[0], tile_h=tile[1])
    cams = gs.Cameras(_t(np.zeros((3, 12))), _t(np.zeros((3, 4))), wh)
    drec = _t(rec)
    gs.gs_bin_sort(ctx, cams, N, s, drec)
    st = ctx.status()
    assert st["flags"] == 0
    ranges_o, ids_o, masks_o = oracle.bin_sort(wh, tile, r["valid"], r["mean2d"], r["conic"],
                                               r["opacity"], r["depth"], with_masks=True)
    assert st["n_isect"] == len(ids_o)
    b = ctx.buffers()
    T = b["n_tiles"]
    assert T == ranges_o.shape[0]
    ranges = _read_i32(b["tile_ranges"], 2 * T).reshape(T, 2)
    ent = _read_i32(b["isect_ids"], len(ids_o)).view(np.uint32)
    assert np.array_equal(ranges, ranges_o.astype(np.int32))
    # an entry is the pair index (low 28 bits) and the quadrant mask (top 4)
    assert np.array_equal(ent & 0x0FFFFFFF, ids_o.astype(np.uint32))
    assert np.array_equal(ent >> 28, masks_o.astype(np.uint32))


def test_bin_sort_bit_exact_past_2048_blocks(gs):
    """8x8 tiles on a 2048x1536 view and a 640x480 one: 3072 + 300 blocks of
    4x4 tiles, so the block ids take 12 bits and the block-key sort runs as
    two 6-bit passes instead of its single 11-bit pass; lists stay
    bit-exact."""
    wh = np.array([[2048, 1536], [640, 480]], np.int32)
    N = 500
    r = scenegen.synthetic_records(17, 2, wh, N, tile=(8, 8))
    rec = np.zeros((2 * N, 12), np.float32)
    rec[:, 0:2] = r["mean2d"]
    rec[:, 2] = r["depth"]
    rec[:, 3] = np.where(r["valid"] > 0, r["opacity"], 0.0)
    rec[:, 4:7] = r["conic"]
    rec[:, 7:10] = r["rgb"]
    ctx = gs.Context(max_pairs=2 * N, max_isect=2_000_000, max_tiles=200_000, max_views=2)
    s = gs.default_settings(tile_w=8, tile_h=8)
    cams = gs.Cameras(_t(np.zeros((2, 12))), _t(np.zeros((2, 4))), wh)
    gs.gs_bin_sort(ctx, cams, N, s, _t(rec))
    st = ctx.status()
    assert st["flags"] == 0
    ranges_o, ids_o, masks_o = oracle.bin_sort(wh, (8, 8), r["valid"], r["mean2d"], r["conic"],
                                               r["opacity"], r["depth"], with_masks=True)
    assert st["n_isect"] == len(ids_o)
    b = ctx.buffers()
    T = b["n_tiles"]
    assert T == ranges_o.shape[0]
    ranges = _read_i32(b["tile_ranges"], 2 * T).reshape(T, 2)
    ent = _read_i32(b["isect_ids"], len(ids_o)).view(np.uint32)
    assert np.array_equal(ranges, ranges_o.astype(np.int32))
    assert np.array_equal(ent & 0x0FFFFFFF, ids_o.astype(np.uint32))
    assert np.array_equal(ent >> 28, masks_o.astype(np.uint32))


def test_bin_sort_bit_exact_with_many_scan_tiles(gs):
    """A large capacity makes the capacity-sized scans (chunk counts, block-key
    digit counts) span hundreds of 4096-item tiles, so the single-pass scans
    walk back over more than one 64-tile window; lists stay bit-exact."""
    wh = np.array([[1237, 822], [640, 480]], np.int32)
    N = 12000
    r = scenegen.synthetic_records(11, 2, wh, N, tile=(16, 16))
    rec = np.zeros((2 * N, 12), np.float32)
    rec[:, 0:2] = r["mean2d"]
    rec[:, 2] = r["depth"]
    rec[:, 3] = np.where(r["valid"] > 0, r["opacity"], 0.0)
    rec[:, 4:7] = r["conic"]
    rec[:, 7:10] = r["rgb"]
    ctx = gs.Context(max_pairs=2 * N, max_isect=40_000_000, max_tiles=100_000, max_views=2)
    s = gs.default_settings(tile_w=16, tile_h=16)
    cams = gs.Cameras(_t(np.zeros((2, 12))), _t(np.zeros((2, 4))), wh)
    drec = _t(rec)
    ranges_o, ids_o, masks_o = oracle.bin_sort(wh, (16, 16), r["valid"], r["mean2d"], r["conic"],
                                               r["opacity"], r["depth"], with_masks=True)
    for rep in range(2):  # the second call finds the scan workspace as the first left it
        gs.gs_bin_sort(ctx, cams, N, s, drec)
        st = ctx.status()
        assert st["flags"] == 0
        assert st["n_isect"] == len(ids_o)
        b = ctx.buffers()
        T = b["n_tiles"]
        ranges = _read_i32(b["tile_ranges"], 2 * T).reshape(T, 2)
        ent = _read_i32(b["isect_ids"], len(ids_o)).view(np.uint32)
        assert np.array_equal(ranges, ranges_o.astype(np.int32)), rep
        assert np.array_equal(ent & 0x0FFFFFFF, ids_o.astype(np.uint32)), rep
        assert np.array_equal(ent >> 28, masks_o.astype(np.uint32)), rep


@pytest.mark.parametrize("view", [(256, 192), (1040, 144)])
def test_bin_sort_bit_exact_with_wide_splats(gs, view):
    """Most splats cover the whole view, so a 256-entry chunk of a block list
    holds more tile entries than the expansion stages in LDS (2048): those
    chunks take the direct-store path, the rest the staged one; lists stay
    bit-exact.  The 1040-px view is 17 block columns wide (the last one
    ragged), so the emit pass builds a whole-view splat's masks in five runs
    of four block columns."""
    wh = np.array([view], np.int32)
    N = 2000
    r = scenegen.synthetic_records(13, 1, wh, N, tile=(16, 16))
    huge = np.random.default_rng(5).uniform(size=N) < 0.6
    r["conic"][huge] = np.array([1e-8, 0.0, 1e-8], np.float32)  # support far beyond the view
    rec = np.zeros((N, 12), np.float32)
    rec[:, 0:2] = r["mean2d"]
    rec[:, 2] = r["depth"]
    rec[:, 3] = np.where(r["valid"] > 0, r["opacity"], 0.0)
    rec[:, 4:7] = r["conic"]
    rec[:, 7:10] = r["rgb"]
    ctx = gs.Context(max_pairs=N, max_isect=2_000_000, max_tiles=10_000, max_views=1)
    s = gs.default_settings(tile_w=16, tile_h=16)
    cams = gs.Cameras(_t(np.zeros((1, 12))), _t(np.zeros((1, 4))), wh)
    gs.gs_bin_sort(ctx, cams, N, s, _t(rec))
    st = ctx.status()
    assert st["flags"] == 0
    ranges_o, ids_o, masks_o = oracle.bin_sort(wh, (16, 16), r["valid"], r["mean2d"], r["conic"],
                                               r["opacity"], r["depth"], with_masks=True)
    # a block list of ~1200 whole-view splats: 16 tile entries per block entry
    assert len(ids_o) > 150_000
    assert st["n_isect"] == len(ids_o)
    b = ctx.buffers()
    T = b["n_tiles"]
    ranges = _read_i32(b["tile_ranges"], 2 * T).reshape(T, 2)
    ent = _read_i32(b["isect_ids"], len(ids_o)).view(np.uint32)
    assert np.array_equal(ranges, ranges_o.astype(np.int32))
    assert np.array_equal(ent & 0x0FFFFFFF, ids_o.astype(np.uint32))
    assert np.array_equal(ent >> 28, masks_o.astype(np.uint32))


def _read_i32(ptr, n):
    import paper_2603_04847_amd._lib as L
    return L.copy_to_host(ptr, n, np.int32)


def test_bin_sort_real_scene_lists(gs):
    # Membership: every (tile, splat) the exact float64 test keeps with some
    # room to spare is listed; nothing listed is far outside.  Order: each
    # list is strictly ascending in (float32 depth bits of the GPU's own
    # record, pair index), bit for bit.
    sc = _parity_scene(seed=5, N=1500)
    sp, params, rgb, T, last, cams, ctx = _render(gs, sc)
    st = ctx.status()
    b = ctx.buffers()
    nt = b["n_tiles"]
    N = sc["means"].shape[1]
    ranges = _read_i32(b["tile_ranges"], 2 * nt).reshape(nt, 2)
    ids = (_read_i32(b["isect_ids"], st["n_isect"]).view(np.uint32) & 0x0FFFFFFF).astype(np.int64)
    rec = gs._lib.copy_to_host(b["records"], N * 12, np.float32).reshape(N, 12)
    dbits = rec[:, 2].copy().view(np.uint32).astype(np.int64)
    pr = oracle.project(sc)
    inner_r, inner = oracle.bin_sort(sc["wh"], (16, 16), pr["valid"], pr["mean2d"], pr["conic"],
                                     pr["opacity"], pr["depth"].astype(np.float32), margin=-0.05)
    outer_r, outer = oracle.bin_sort(sc["wh"], (16, 16), pr["valid"], pr["mean2d"], pr["conic"],
                                     pr["opacity"], pr["depth"].astype(np.float32), margin=0.05)
    n_ties = 0
    for t in range(nt):
        g = ids[ranges[t, 0]:ranges[t, 1]]
        gi = set(inner[inner_r[t, 0]:inner_r[t, 1]].tolist())
        go = set(outer[outer_r[t, 0]:outer_r[t, 1]].tolist())
        assert gi <= set(g.tolist()) <= go, t
        key = dbits[g] * (1 << 32) + g        # (depth bits, pair) as one integer
        assert np.all(np.diff(key) > 0), t
        n_ties += int(np.sum(np.diff(dbits[g]) == 0))
        # the GPU's float32 depth is the rounding of the FP64 depth
        np.testing.assert_allclose(rec[g, 2], pr["depth"][g], rtol=6e-8)


# ------------------------------------------------------------------ forward

@pytest.mark.parametrize("name", ["parity", "C1"])
def test_render_fwd_matches_oracle(gs, name):
    sc = _parity_scene() if name == "parity" else scenegen.make_config("C1")
    sp, params, rgb, T, last, cams, ctx = _render(gs, sc)
    o = oracle.render_fwd_bwd(sc)
    amb = o["ambiguous"]
    assert amb.mean() < 0.02, amb.mean()
    ok = ~amb
    g = rgb.cpu().numpy()
    _close(g[ok], o["rgb"][ok], scale=max(1.0, np.abs(o["rgb"]).max()), what="rgb")
    _close(T.cpu().numpy()[ok], o["T"][ok], scale=1.0, what="T_final")


def test_render_with_clamped_opacities_matches_oracle(gs):
    """A quarter of the Gaussians above the 0.99 opacity clamp (logits 6..9)
    and large enough that ~4% of the pixels see a clamped alpha: image and every
    gradient group against the oracle (clamped hits pass no opacity or
    geometry gradient)."""
    sc = _parity_scene(seed=23, N=1500)
    rng = np.random.default_rng(23)
    hi = rng.choice(1500, 375, replace=False)
    sc["opacity_logit"][hi] = rng.uniform(6.0, 9.0, size=375).astype(np.float32)
    sc["log_scales"][:, hi] += np.float32(2.0)
    o = oracle.render_fwd_bwd(sc)
    assert o["nclamp"].sum() > 800, o["nclamp"].sum()
    assert o["ambiguous"].mean() < 0.02
    sp, params, rgb, T, last, cams, ctx = _render(gs, sc)
    ok = ~o["ambiguous"]
    _close(rgb.cpu().numpy()[ok], o["rgb"][ok], scale=1.0, what="rgb")
    _close(T.cpu().numpy()[ok], o["T"][ok], scale=1.0, what="T_final")
    w = np.random.default_rng(1).normal(size=(cams.n_pixels, 3))
    w[o["ambiguous"]] = 0.0
    grads, v_tw = sp.backward(params, sc["sh_degree"], cams, T, last, _t(w))
    og = oracle.render_fwd_bwd(sc, v_rgb=w)["grads"]
    for k in ("means", "log_scales", "quats", "opacity_logit", "sh"):
        _close(grads[k].cpu().numpy(), og[k], what=k)
    _close(v_tw.cpu().numpy()[0], og["twist"][0], what="twist")


def test_render_fwd_bitwise_independent_of_tile_shape(gs):
    sc = _parity_scene(seed=9)
    outs = []
    for tw, th in [(16, 16), (16, 8), (8, 8), (32, 16)]:
        s = gs.default_settings(tile_w=tw, tile_h=th)
        outs.append(_render(gs, sc, settings=s)[2].cpu().numpy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def _length_bucket(n):
    """Launch weight of a tile list of length n: 16 buckets per octave."""
    n = np.asarray(n, np.int64)
    out = np.zeros(n.shape, np.int64)
    for i, v in np.ndenumerate(n):
        if v > 0:
            msb = int(v).bit_length() - 1
            frac = (v >> (msb - 4)) & 15 if msb >= 4 else (v << (4 - msb)) & 15
            out[i] = 1 + 16 * msb + frac
    return out


def test_length_bucket_is_monotone():
    b = _length_bucket(np.arange(0, 5000))
    assert np.all(np.diff(b) >= 0) and b[0] == 0 and b[1] == 1 and b[2] == 17


def test_tile_order_and_contributor_counts(gs):
    # Launching the tiles heaviest-first changes nothing in the image; the
    # per-tile contributor counts equal the oracle's per-pixel counts summed
    # over tiles free of ambiguous pixels; the entry and evaluation counts
    # agree with the lists and with `last`.
    sc = _parity_scene(seed=14)
    a = _render(gs, sc)
    ctx = _ctx(gs, sc)
    r = _render(gs, sc, ctx=ctx, settings=gs.default_settings(tile_order=1, eval_stats=1))
    assert np.array_equal(a[2].cpu().numpy(), r[2].cpu().numpy())
    st = gs._lib.gs_ctx_tile_stats(ctx)
    assert st["ordered"]
    nt = st["n_tiles"]
    order = gs._lib.copy_to_host(st["tile_order"], nt, np.uint32)
    assert np.array_equal(np.sort(order), np.arange(nt))
    bufs = ctx.buffers()
    ranges = _read_i32(bufs["tile_ranges"], 2 * nt).reshape(nt, 2)
    lens = ranges[:, 1] - ranges[:, 0]
    assert np.all(np.diff(_length_bucket(lens[order])) <= 0)
    W, H = sc["wh"][0]
    gx = (W + 15) // 16
    contrib = gs._lib.copy_to_host(st["tile_contrib"], nt, np.int32)
    o = oracle.render_fwd_bwd(sc)
    nc = o["ncontrib"].reshape(H, W)
    amb = o["ambiguous"].reshape(H, W)
    checked = 0
    for t in range(nt):
        ty, tx = divmod(t, gx)
        blk = (slice(ty * 16, ty * 16 + 16), slice(tx * 16, tx * 16 + 16))
        if amb[blk].any():
            continue
        assert contrib[t] == nc[blk].sum(), t
        checked += 1
    assert checked > nt // 2
    # entries read per tile: no more than the tile's list
    ent = gs._lib.copy_to_host(st["tile_entries"], nt, np.int32)
    assert np.all(ent <= lens)
    # evaluations per tile: over its pixels, the entries covering the pixel's
    # quadrant up to the pixel's last contributor
    last = r[4].cpu().numpy().reshape(H, W)
    ids = _read_i32(bufs["isect_ids"], int(ranges[:, 1].max())).view(np.uint32)
    ev = gs._lib.copy_to_host(st["tile_evals"], nt, np.int32)
    for t in range(nt):
        ty, tx = divmod(t, gx)
        m4 = ids[ranges[t, 0]:ranges[t, 1]] >> 28
        want = 0
        for y in range(ty * 16, min(ty * 16 + 16, H)):
            for x in range(tx * 16, min(tx * 16 + 16, W)):
                q = ((x % 16) >= 8) + 2 * ((y % 16) >= 8)
                want += int(((m4[:last[y, x]] >> q) & 1).sum())
        assert ev[t] == want, t


@pytest.mark.parametrize("tile", [(16, 16), (16, 8), (8, 8), (32, 16)])
def test_xcd_launch_order_changes_nothing(gs, tile):
    """The XCD-grouped launch order (tiles walked by 4x4 blocks, a block per
    XCD) gives the image, transmittance and contributor indices of the natural
    order bit for bit, and the same gradients (up to the order of float
    atomics), over ragged views."""
    s = scenegen.blob_scene(17, [(203, 150), (96, 64), (130, 77)], 15000, sh_degree=2)
    s.pop("_rng")
    outs = []
    for order in (0, 2):
        st = gs.default_settings(tile_w=tile[0], tile_h=tile[1], tile_order=order)
        sp, params, rgb, T, last, cams, ctx = _render(gs, s, settings=st)
        w = _t(np.random.default_rng(2).normal(size=(cams.n_pixels, 3)))
        grads, v_tw = sp.backward(params, 2, cams, T, last, w)
        torch.cuda.synchronize()
        outs.append((rgb.cpu().numpy(), T.cpu().numpy(), last.cpu().numpy(),
                     {k: v.cpu().numpy() for k, v in grads.items()}, v_tw.cpu().numpy()))
    a, b = outs
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    for k in a[3]:
        _close(b[3][k], a[3][k], rtol=1e-5, what=k)
    _close(b[4], a[4], rtol=1e-5, what="twist")


def test_batched_views_bitwise_equal_per_view(gs):
    s = scenegen.blob_scene(11, [(160, 120), (203, 150), (96, 64)], 20000, sh_degree=3)
    s.pop("_rng")
    batched = _render(gs, s)[2].cpu().numpy()
    per = []
    ctx = _ctx(gs, s)
    for v in range(3):
        sv = dict(s, viewmat=s["viewmat"][v:v + 1], intr=s["intr"][v:v + 1], wh=s["wh"][v:v + 1])
        per.append(_render(gs, sv, ctx=ctx)[2].cpu().numpy())
    assert np.array_equal(batched, np.concatenate(per))


def test_background_colour(gs):
    sc = _parity_scene(seed=12, N=500)
    bg = _t(np.array([0.2, 0.5, 0.9]))
    sp, params, rgb, T, last, cams, ctx = _render(gs, sc, bg=bg)
    o = oracle.render_fwd_bwd(sc, bg=np.array([0.2, 0.5, 0.9]))
    ok = ~o["ambiguous"]
    _close(rgb.cpu().numpy()[ok], o["rgb"][ok], scale=1.0, what="rgb with bg")


# ------------------------------------------------------------------ backward

def _backward_case(gs, sc, bg=None, seed=0):
    sp, params, rgb, T, last, cams, ctx = _render(gs, sc, bg=None if bg is None else _t(bg))
    P = cams.n_pixels
    o = oracle.render_fwd_bwd(sc, bg=bg)
    w = np.random.default_rng(seed).normal(size=(P, 3))
    w[o["ambiguous"]] = 0.0
    grads, v_tw = sp.backward(params, sc["sh_degree"], cams, T, last, _t(w))
    torch.cuda.synchronize()
    og = oracle.render_fwd_bwd(sc, v_rgb=w, bg=bg)["grads"]
    return grads, v_tw, og


@pytest.mark.parametrize("name", ["parity", "C1"])
def test_render_bwd_matches_oracle(gs, name):
    sc = _parity_scene(seed=21) if name == "parity" else scenegen.make_config("C1")
    grads, v_tw, og = _backward_case(gs, sc)
    K = (sc["sh_degree"] + 1) ** 2
    for k in ("means", "log_scales", "quats", "opacity_logit"):
        _close(grads[k].cpu().numpy(), og[k], what=k)
    sh = grads["sh"].cpu().numpy()
    for l in range(sc["sh_degree"] + 1):
        band = slice(l * l, (l + 1) * (l + 1))
        _close(sh[band], og["sh"][band], what=f"sh band {l}")
    assert K == sh.shape[0]
    tw = v_tw.cpu().numpy()
    for v in range(tw.shape[0]):
        _close(tw[v], og["twist"][v], what=f"twist view {v}")


def _full_size_check(gs, sub, tile, order, npix, max_isect, seed, min_frac=0.97, lazy=0):
    """Sampled pixels and gradients of one full-size batch against the oracle:
    colour and transmittance of `npix` random pixels against the oracle's
    per-pixel definition, and the backward with an image gradient that is
    non-zero only at those pixels, so the oracle's gradients of every Gaussian
    parameter and of each view's twist come from them alone.  At least
    `min_frac` of the sampled pixels must be free of ambiguity (a gate, clamp,
    stop or depth-rounding decision within float32 error of its threshold).
    `lazy` = 1 leaves the tile lists to the forward (gs_settings.lazy_lists)."""
    from paper_2603_04847_amd.splat import Splatter
    V = sub["viewmat"].shape[0]
    N = sub["means"].shape[1]
    T_max = int(sum(((w + tile[0] - 1) // tile[0]) * ((h + tile[1] - 1) // tile[1]) for w, h in sub["wh"]))
    ctx = gs.Context(max_pairs=V * N, max_isect=max_isect, max_tiles=T_max, max_views=V)
    sp = Splatter(ctx, gs.default_settings(tile_w=tile[0], tile_h=tile[1], tile_order=order,
                                           lazy_lists=lazy))
    params = _params(sub)
    rgb, T, last, cams = sp.forward(params, 3, _t(sub["viewmat"]), _t(sub["intr"]), sub["wh"])
    torch.cuda.synchronize()
    assert ctx.status()["flags"] == 0
    P = cams.n_pixels
    rng = np.random.default_rng(seed)
    pix = np.sort(rng.choice(P, size=npix, replace=False))
    w = rng.normal(size=(pix.size, 3))
    pr = oracle.project(sub)
    o = oracle.render(pr, sub["wh"], pix=pix, v_rgb=w)
    ok = ~o["ambiguous"].astype(bool)
    print(f"[full-size] {ok.sum()}/{npix} sampled pixels unambiguous", flush=True)
    assert ok.mean() >= min_frac, ok.mean()
    g_rgb = rgb.cpu().numpy()[pix]
    g_T = T.cpu().numpy()[pix]
    _close(g_rgb[ok], o["rgb"][ok], scale=max(np.max(np.abs(o["rgb"][ok])), 1.0), what="rgb")
    _close(g_T[ok], o["T"][ok], scale=1.0, what="T_final")
    # backward: the image gradient at the sampled, non-ambiguous pixels only
    w[~ok] = 0.0
    o = oracle.render(pr, sub["wh"], pix=pix, v_rgb=w)
    og = oracle.project_bwd(sub, o["v2d"])
    v_img = np.zeros((P, 3))
    v_img[pix] = w
    grads, v_tw = sp.backward(params, 3, cams, T, last, _t(v_img))
    torch.cuda.synchronize()
    for k in ("means", "log_scales", "quats", "opacity_logit"):
        _close(grads[k].cpu().numpy(), og[k], what=k)
    sh = grads["sh"].cpu().numpy()
    for l in range(4):
        band = slice(l * l, (l + 1) * (l + 1))
        _close(sh[band], og["sh"][band], what=f"sh band {l}")
    tw = v_tw.cpu().numpy()
    for v in range(V):
        _close(tw[v], og["twist"][v], what=f"twist view {v}")
    return ctx


def test_full_size_batch_sampled_pixels_and_gradients(gs):
    """The joint step's batch at full size (4 views of 1237x822, 1M Gaussians,
    SH degree 3), in the configuration the benchmark times (16x16 tiles,
    heaviest tile first, lazy tile lists)."""
    sc = scenegen.make_config("C4")
    b = scenegen.batch_views(4, sc["viewmat"].shape[0], 4, 1)[0]
    sub = dict(sc, viewmat=sc["viewmat"][b], intr=sc["intr"][b], wh=sc["wh"][b])
    _full_size_check(gs, sub, (16, 16), 1, 400, 120_000_000, 12, lazy=1)


def test_full_size_single_view_sampled(gs):
    """The single-view workload at full size (1237x822, 1M Gaussians, SH
    degree 3) at 16x16 tiles, heaviest first."""
    sc = scenegen.make_config("C2")
    _full_size_check(gs, sc, (16, 16), 1, 400, 150_000_000, 15)


def test_full_size_uneven_views_sampled(gs):
    """The batched uneven-view workload at full size: 8 views from 640x480 to
    1600x1066 around 3M clustered Gaussians (SH degree 3), one call."""
    sc = scenegen.make_config("C3")
    ctx = _full_size_check(gs, sc, (16, 16), 1, 300, 400_000_000, 13)
    # the workload's stated load imbalance, on the exact tile lists: the
    # longest list is at least 100 times the median non-empty one
    b = ctx.buffers()
    nt = b["n_tiles"]
    ranges = _read_i32(b["tile_ranges"], 2 * nt).reshape(nt, 2)
    lens = (ranges[:, 1] - ranges[:, 0]).astype(np.int64)
    nz = lens[lens > 0]
    print(f"[C3] tile lists: max {nz.max()}, median {np.median(nz):.0f}", flush=True)
    assert nz.max() >= 100 * np.median(nz)


def test_full_size_large_scene_sampled(gs):
    """The large-scene batch at full size (4 views of 1600x1066, 5M Gaussians,
    SH degree 3) in the configuration its benchmark picks (32x16 tiles, the
    XCD launch order, lazy tile lists)."""
    sc = scenegen.make_config("C5")
    b = scenegen.batch_views(5, sc["viewmat"].shape[0], 4, 1)[0]
    sub = dict(sc, viewmat=sc["viewmat"][b], intr=sc["intr"][b], wh=sc["wh"][b])
    _full_size_check(gs, sub, (32, 16), 2, 300, 400_000_000, 14, lazy=1)


def test_render_bwd_batched_views(gs):
    s = scenegen.blob_scene(31, [(128, 96), (203, 150)], 6000, sh_degree=2)
    s.pop("_rng")
    grads, v_tw, og = _backward_case(gs, s, bg=np.array([0.1, 0.3, 0.2]), seed=3)
    for k in ("means", "log_scales", "quats", "opacity_logit", "sh"):
        _close(grads[k].cpu().numpy(), og[k], what=k)
    _close(v_tw.cpu().numpy()[0], og["twist"][0], what="twist 0")
    _close(v_tw.cpu().numpy()[1], og["twist"][1], what="twist 1")


# ------------------------------------------------------------------ L1, track, pose, Adam

def test_l1_loss_grad(gs):
    rng = np.random.default_rng(4)
    wh = np.array([[40, 30], [17, 9]], np.int32)
    P = int((wh[:, 0] * wh[:, 1]).sum())
    a = rng.uniform(size=(P, 3)).astype(np.float32)
    b = rng.uniform(size=(P, 3)).astype(np.float32)
    b[:10] = a[:10]  # exact ties: sign(0) = 0
    ctx = gs.Context(max_pairs=1, max_isect=1, max_tiles=16, max_views=2)
    cams = gs.Cameras(_t(np.zeros((2, 12))), _t(np.zeros((2, 4))), wh)
    v = torch.empty((P, 3), device="cuda")
    loss = torch.zeros(1, device="cuda")
    gs.gs_l1_loss_grad(ctx, cams, _t(a), _t(b), v, loss)
    want_l, want_v = oracle.l1(a, b, wh)
    # the sign is decided exactly on both sides (float32 subtraction keeps it)
    assert np.array_equal(np.sign(v.cpu().numpy()), np.sign(want_v))
    _close(v.cpu().numpy(), want_v, what="v_rgb")
    assert abs(loss.item() - want_l) <= RTOL * want_l


def test_track_matches_oracle(gs):
    sc = scenegen.make_config("C1")
    X = sc["X"].copy()
    vm, intr = sc["track_viewmat"], sc["track_intr"]
    # one point pushed behind camera 0 -> its observations there are masked
    M3 = vm[0].reshape(3, 4).astype(np.float64)
    X[0] = M3[:, :3].T @ (np.array([0.1, 0.2, -3.0]) - M3[:, 3])
    ctx = gs.Context(max_pairs=1, max_isect=1, max_tiles=16, max_views=1, max_cams=8)
    o = oracle.track(X, vm, intr, sc["obs_cam"], sc["obs_pt"], sc["obs_xy"], delta=1.0, lam=1e-4)
    M = len(sc["obs_cam"])
    loss = torch.zeros(1, device="cuda")
    v_X = torch.zeros((X.shape[0], 3), device="cuda")
    v_tw = torch.zeros((5, 6), device="cuda")
    res = torch.empty((M, 2), device="cuda")
    Jp = torch.empty((M, 12), device="cuda")
    Jx = torch.empty((M, 6), device="cuda")
    ctx.reset_status()
    gs.track_reproj_fwd_bwd(ctx, _t(X), _t(vm), _t(intr), _t(sc["obs_cam"], torch.int32),
                            _t(sc["obs_pt"], torch.int32), _t(sc["obs_xy"]), 1.0, 1e-4, 0.01,
                            loss, v_X, v_tw, residual=res, J_pose=Jp, J_X=Jx)
    st = ctx.status()
    assert st["n_masked_obs"] == int(o["masked"].sum()) > 0
    _close(res.cpu().numpy(), o["residual"], what="residual")
    assert abs(loss.item() - o["loss"]) <= RTOL * o["loss"]
    _close(v_X.cpu().numpy(), o["v_X"], what="v_X")
    for v in range(5):
        _close(v_tw.cpu().numpy()[v], o["v_twist"][v], what=f"twist {v}")
    _close(Jp.cpu().numpy().reshape(M, 2, 6), o["J_pose"], what="J_pose")
    _close(Jx.cpu().numpy().reshape(M, 2, 3), o["J_X"], what="J_X")


def test_track_point_index_is_a_stable_csr(gs):
    """The point-major index equals a stable sort of the observations by point
    (each point's observations ascending); out-of-range points are left out."""
    rng = np.random.default_rng(21)
    Pt, M = 5000, 40000
    obs_pt = rng.integers(-3, Pt + 3, size=M).astype(np.int32)
    ctx = gs.Context(max_pairs=Pt, max_isect=1 << 16, max_tiles=16, max_views=1, max_cams=8)
    cam = rng.integers(0, 8, size=M).astype(np.int32)
    xy = rng.uniform(0, 500, size=(M, 2)).astype(np.float32)
    pt_off, pt_obs, pm_cam, pm_xy = gs.track_point_index(ctx, _t(obs_pt, torch.int32), Pt,
                                                         _t(cam, torch.int32), _t(xy))
    torch.cuda.synchronize()
    ok = (obs_pt >= 0) & (obs_pt < Pt)
    n = int(ok.sum())
    order = np.argsort(np.where(ok, obs_pt, Pt), kind="stable")[:n]
    counts = np.bincount(obs_pt[ok], minlength=Pt)
    off_ref = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    assert np.array_equal(pt_off.cpu().numpy(), off_ref)
    assert np.array_equal(pt_obs.cpu().numpy()[:n], order.astype(np.int32))
    # the point-major copies of the cameras and pixels, bit for bit
    assert np.array_equal(pm_cam.cpu().numpy()[:n], cam[order])
    assert np.array_equal(pm_xy.cpu().numpy()[:n], xy[order])


def test_track_with_point_index_matches_oracle(gs):
    """With the point-major index the point gradients are summed per point (no
    atomics); they match the oracle and the atomic path, the rest is unchanged."""
    sc = scenegen.make_config("C1")
    X = sc["X"].copy()
    vm, intr = sc["track_viewmat"], sc["track_intr"]
    M3 = vm[0].reshape(3, 4).astype(np.float64)
    X[0] = M3[:, :3].T @ (np.array([0.1, 0.2, -3.0]) - M3[:, 3])  # masked in camera 0
    ctx = gs.Context(max_pairs=X.shape[0], max_isect=1 << 16, max_tiles=16, max_views=1, max_cams=8)
    o = oracle.track(X, vm, intr, sc["obs_cam"], sc["obs_pt"], sc["obs_xy"], delta=1.0, lam=1e-4)
    obs_pt = _t(sc["obs_pt"], torch.int32)
    obs_cam, obs_xy = _t(sc["obs_cam"], torch.int32), _t(sc["obs_xy"])
    index = gs.track_point_index(ctx, obs_pt, X.shape[0])
    index_pm = gs.track_point_index(ctx, obs_pt, X.shape[0], obs_cam, obs_xy)
    out = {}
    for name, pi in (("atomic", None), ("indexed", index), ("point-major", index_pm)):
        loss = torch.zeros(1, device="cuda")
        v_X = torch.zeros((X.shape[0], 3), device="cuda")
        v_tw = torch.zeros((5, 6), device="cuda")
        # the point-major pass writes no residual (asking for one selects the
        # other paths)
        res = torch.empty((len(sc["obs_cam"]), 2), device="cuda") if name != "point-major" else None
        ctx.reset_status()
        gs.track_reproj_fwd_bwd(ctx, _t(X), _t(vm), _t(intr), obs_cam, obs_pt, obs_xy, 1.0, 1e-4, 0.01,
                                loss, v_X, v_tw, residual=res, pt_index=pi)
        torch.cuda.synchronize()
        assert ctx.status()["n_masked_obs"] == int(o["masked"].sum()) > 0, name
        out[name] = (loss.item(), v_X.cpu().numpy(), v_tw.cpu().numpy(),
                     res.cpu().numpy() if res is not None else None)
    la, vXa, twa, ra = out["atomic"]
    li, vXi, twi, ri = out["indexed"]
    _close(vXi, o["v_X"], what="v_X indexed")
    _close(vXi, vXa, what="v_X indexed vs atomic")
    assert np.array_equal(ri, ra) and np.array_equal(twi, twa) and li == la
    lp, vXp, twp, _ = out["point-major"]
    _close(vXp, o["v_X"], what="v_X point-major")
    for v in range(5):
        _close(twp[v], o["v_twist"][v], what=f"twist {v} point-major")
    assert abs(lp - o["loss"]) <= RTOL * o["loss"]


def test_track_point_major_past_the_camera_limit(gs):
    """More cameras than the point-major pass holds in LDS: the call takes
    the indexed path and the results still match the oracle."""
    sc = scenegen.make_config("C1")
    X = sc["X"]
    C = 2100                                             # > GS_TRACK_PM_MAX_CAMS
    vm = np.concatenate([sc["track_viewmat"]] * (C // 5 + 1))[:C]
    intr = np.concatenate([sc["track_intr"]] * (C // 5 + 1))[:C]
    rng = np.random.default_rng(3)
    cam = (sc["obs_cam"] + 5 * rng.integers(0, C // 5, size=len(sc["obs_cam"]))).astype(np.int32)
    ctx = gs.Context(max_pairs=X.shape[0], max_isect=1 << 16, max_tiles=16, max_views=1, max_cams=C)
    o = oracle.track(X, vm, intr, cam, sc["obs_pt"], sc["obs_xy"], delta=1.0, lam=1e-4, jacobians=False)
    obs_pt, obs_cam, obs_xy = _t(sc["obs_pt"], torch.int32), _t(cam, torch.int32), _t(sc["obs_xy"])
    index_pm = gs.track_point_index(ctx, obs_pt, X.shape[0], obs_cam, obs_xy)
    loss = torch.zeros(1, device="cuda")
    v_X = torch.zeros((X.shape[0], 3), device="cuda")
    v_tw = torch.zeros((C, 6), device="cuda")
    gs.track_reproj_fwd_bwd(ctx, _t(X), _t(vm), _t(intr), obs_cam, obs_pt, obs_xy, 1.0, 1e-4, 0.01,
                            loss, v_X, v_tw, pt_index=index_pm)
    torch.cuda.synchronize()
    _close(v_X.cpu().numpy(), o["v_X"], what="v_X")
    _close(v_tw.cpu().numpy(), o["v_twist"], what="twists")
    assert abs(loss.item() - o["loss"]) <= RTOL * o["loss"]


def test_pose_compose_and_backward(gs):
    rng = np.random.default_rng(8)
    V = 7
    xi = rng.normal(size=(V, 6)) * np.array([0.01, 0.01, 0.01, 0.003, 0.003, 0.003])
    xi[0] *= 0
    xi[1] *= 100          # a large twist takes the closed-form branch
    from scipy.spatial.transform import Rotation
    base = np.stack([np.concatenate([Rotation.random(random_state=i).as_matrix(),
                                     rng.normal(size=(3, 1))], 1).reshape(12) for i in range(V)])
    out = torch.empty((V, 12), device="cuda")
    gs.gs_pose_compose(_t(xi), _t(base), out)
    want = oracle.se3_exp_compose(xi.astype(np.float32), base.astype(np.float32))
    _close(out.cpu().numpy(), want, what="Exp(xi) T0")
    g = rng.normal(size=(V, 6))
    outg = torch.empty((V, 6), device="cuda")
    gs.gs_pose_compose_bwd(_t(xi), _t(g), outg)
    wantg = oracle.se3_jl_transpose(xi.astype(np.float32), g.astype(np.float32))
    _close(outg.cpu().numpy(), wantg, what="J_l^T g")


def test_adam_matches_oracle(gs):
    rng = np.random.default_rng(9)
    sizes = [1000, 37, 5000]
    lrs = [1e-3, 5e-2, 2.5e-3]
    ps = [rng.normal(size=n) for n in sizes]
    dev = [[_t(p), None, torch.zeros(len(p), device="cuda"), torch.zeros(len(p), device="cuda")]
           for p in ps]
    ref = [[p.astype(np.float32).astype(np.float64), np.zeros(len(p)), np.zeros(len(p))] for p in ps]
    for step in range(1, 4):
        gr = [rng.normal(size=n).astype(np.float32) for n in sizes]
        groups = []
        for q in range(3):
            dev[q][1] = _t(gr[q])
            groups.append((dev[q][0], dev[q][1], dev[q][2], dev[q][3], lrs[q]))
            oracle.adam(ref[q][0], gr[q].astype(np.float64), ref[q][1], ref[q][2], lrs[q],
                        eps=1e-8, step=step)
        gs.gs_adam_step(groups, step, eps=1e-8)
    for q in range(3):
        d = dev[q][0].cpu().numpy() - ref[q][0]
        assert np.max(np.abs(d)) <= 1e-6 + 1e-5 * lrs[q] * 3


# ------------------------------------------------------------------ error paths

@pytest.mark.parametrize("lazy", [0, 1])
def test_capacity_overflow_is_flagged(gs, lazy):
    """An overflowed bin step is flagged and leaves every list empty: the
    image is the background, and a backward over it adds nothing (with full
    and with lazy lists)."""
    sc = _parity_scene(seed=40, N=800)
    ctx = _ctx(gs, sc, max_isect=100)
    sp, params, rgb, T, last, cams, _ = _render(gs, sc, ctx=ctx, settings=gs.default_settings(lazy_lists=lazy))
    st = ctx.status()
    assert st["flags"] & 1
    assert st["n_isect_needed"] > 100 and st["n_isect"] == 0
    assert torch.all(T == 1.0) and torch.all(last == 0) and torch.all(rgb == 0.0)
    grads, v_tw = sp.backward(params, sc["sh_degree"], cams, T, last, torch.ones_like(rgb))
    torch.cuda.synchronize()
    for k in grads:
        assert torch.all(grads[k] == 0.0), k
    assert torch.all(v_tw == 0.0)


def test_host_argument_errors(gs):
    sc = _parity_scene(seed=41, N=100)
    ctx = _ctx(gs, sc)
    with pytest.raises(gs.GsError) as e:
        _render(gs, sc, ctx=ctx, settings=gs.default_settings(tile_w=12))
    assert e.value.code == -4
    big = dict(sc, means=np.zeros((3, 10**6), np.float32))
    with pytest.raises(gs.GsError) as e:
        sp, *_ = _render(gs, dict(sc, means=sc["means"]), ctx=gs.Context(10, 10, 10, 1))
    assert e.value.code == -2
    del big
