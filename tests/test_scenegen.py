"""The seeded workload generators: reproducible, and the uneven-view scene
(8 views from 640x480 to 1600x1066 around 3M clustered Gaussians) meets its
stated load imbalance, per-tile splat counts varying by at least 100x.  CPU
only; the per-tile counts come from the oracle's projection: each splat counts
in every tile its alpha >= 1/255 bounding box reaches (an upper bound of the
tile-list length; the GPU tests check the exact lists)."""

import numpy as np

import oracle
import scenegen


def test_generators_reproduce_bit_for_bit():
    a, b = scenegen.make_config("C1"), scenegen.make_config("C1")
    for k in ("means", "log_scales", "quats", "opacity_logit", "sh", "viewmat", "intr", "X",
              "obs_cam", "obs_pt", "obs_xy", "target"):
        assert np.array_equal(a[k], b[k]), k
    c = scenegen.make_config("C1", seed=2)
    assert not np.array_equal(a["means"], c["means"])


def per_tile_bbox_counts(sc, tile=16):
    pr = oracle.project(sc)
    V, N = sc["wh"].shape[0], sc["means"].shape[1]
    out = []
    for v in range(V):
        W, H = sc["wh"][v]
        gx, gy = (W + tile - 1) // tile, (H + tile - 1) // tile
        sl = slice(v * N, (v + 1) * N)
        ok = pr["valid"][sl].astype(bool)
        m, e = pr["mean2d"][sl][ok], pr["ext"][sl][ok]
        # tiles whose pixel-centre span meets [m - e, m + e]
        x0 = np.clip(np.floor((m[:, 0] - e[:, 0] - 0.5) / tile), 0, gx)
        x1 = np.clip(np.floor((m[:, 0] + e[:, 0] - 0.5) / tile), -1, gx - 1)
        y0 = np.clip(np.floor((m[:, 1] - e[:, 1] - 0.5) / tile), 0, gy)
        y1 = np.clip(np.floor((m[:, 1] + e[:, 1] - 0.5) / tile), -1, gy - 1)
        keep = (x0 <= x1) & (y0 <= y1)
        x0, x1, y0, y1 = (a[keep].astype(int) for a in (x0, x1, y0, y1))
        D = np.zeros((gy + 1, gx + 1), np.int64)
        np.add.at(D, (y0, x0), 1)
        np.add.at(D, (y0, x1 + 1), -1)
        np.add.at(D, (y1 + 1, x0), -1)
        np.add.at(D, (y1 + 1, x1 + 1), 1)
        out.append(D.cumsum(0).cumsum(1)[:gy, :gx].ravel())
    return np.concatenate(out)


def test_uneven_view_scene_load_imbalance():
    sc = scenegen.make_config("C3")
    assert sc["means"].shape[1] == 3_000_000 and sc["wh"].shape[0] == 8
    c = per_tile_bbox_counts(sc)
    nz = c[c > 0]
    ratio = nz.max() / np.median(nz)
    print(f"C3 per-tile counts: max {nz.max()}, median {np.median(nz):.0f}, ratio {ratio:.1f}")
    assert ratio >= 100, ratio
