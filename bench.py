#!/usr/bin/env python
"""Throughput of the joint pose-appearance step on one MI355X.

Metric: forward+backward megapixels per second with pose gradients.  The
default workload is the large scene: 1000 cameras at 1600x1066, 5M Gaussians
(SH degree 3), 1.5M tracks (6.5M observations), 4 views per step; every step
runs pose composition, projection, bin/sort, compositing, the photometric loss
(L1 + SSIM, lambda 0.2), raster and projection backward, track reprojection
over all observations, the twist chain and Adam.  The joint step of 150
cameras at 1237x822 and 1M Gaussians is timed too and reported under
`extra_workloads`.  Inputs are seeded synthetic scenes resident in HBM before
the timed region.

The timed steps are replayed from captured HIP graphs (one per batch of
views, every kernel of the step); the same steps run eagerly, call by call,
are reported beside them and give the per-call breakdown.

Also reported: a per-call breakdown (HIP events on the launch stream), the
roofline of the dominant kernel, the batched-vs-per-view comparison on the
8-view uneven-resolution scene (3M Gaussians), and the FP64 oracle timed on a
bounded sample of the same workload on the host cores.

  python bench.py [--steps K] [--warmup W] [--workload C5|C4|C2|C3] [--lambda-ssim L]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

WORKLOADS = {
    "C2": "single view 1237x822, 1M Gaussians SH3, 16x16 tiles",
    "C3": "8 views 640x480..1600x1066 on a sphere around 3M blob Gaussians SH3",
    "C4": "joint step: 150 cameras 1237x822, 1M Gaussians SH3, 100k tracks, 4 views/step",
    "C5": "large scene: 1000 cameras 1600x1066, 5M Gaussians SH3, 1.5M tracks, 4 views/step",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class EventTimer:
    """HIP events around named calls on the current stream; mean ms per name."""

    def __init__(self, torch):
        self.torch = torch
        self.ev = {}
        self.on = True

    def __call__(self, name):
        timer = self

        class _Ctx:
            def __enter__(self_):
                if timer.on:
                    self_.a = timer.torch.cuda.Event(enable_timing=True)
                    self_.a.record()
                return self_

            def __exit__(self_, *exc):
                if timer.on:
                    b = timer.torch.cuda.Event(enable_timing=True)
                    b.record()
                    timer.ev.setdefault(name, []).append((self_.a, b))
                return False
        return _Ctx()

    def means(self):
        self.torch.cuda.synchronize()
        return {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in self.ev.items()}


def make_workload(name):
    import scenegen
    t0 = time.time()
    sc = scenegen.make_config(name)
    if name in ("C4", "C5"):
        nv = sc["viewmat"].shape[0]
        batches = scenegen.batch_views(int(name[1]), nv, 4, 4)
        targets = [scenegen.view_targets(int(name[1]), sc["wh"], b) for b in batches]
    else:
        batches = [np.arange(sc["viewmat"].shape[0])]
        targets = [sc["target"]]
        n = sc["means"].shape[1]
        sc["X"] = np.zeros((0, 3), np.float32)
        sc["obs_cam"] = np.zeros(0, np.int32)
        sc["obs_pt"] = np.zeros(0, np.int32)
        sc["obs_xy"] = np.zeros((0, 2), np.float32)
        del n
    log(f"[bench] generated {name} in {time.time() - t0:.1f}s")
    return sc, batches, targets


def run_joint(torch, name, steps, warmup, tune=True, tile=None, order=0, graph=True,
              lambda_ssim=0.2, lazy_lists=True, overlap_track=True):
    from paper_2603_04847_amd import _lib as L
    from paper_2603_04847_amd.autotune import autotune
    from paper_2603_04847_amd.step import JointStep
    sc, batches, targets = make_workload(name)
    P = max(int(sum(int(sc["wh"][v, 0]) * int(sc["wh"][v, 1]) for v in b)) for b in batches)
    st = JointStep(sc, batches, targets, max_isect=min(2**30 - 65536, 48 * P),
                   lambda_ssim=lambda_ssim, lazy_lists=lazy_lists, overlap_track=overlap_track)
    tuning = None
    if tile is not None:
        st.settings = L.default_settings(tile_w=tile[0], tile_h=tile[1], tile_order=order)
    if tune and tile is None:
        results, best = autotune(st)
        tuning = dict(best=f"{best['tile'][0]}x{best['tile'][1]} order={best['order']}",
                      candidates={f"{r['tile'][0]}x{r['tile'][1]}/{'-' if r['order'] is None else r['order']}":
                                  (round(r["ms"], 3) if r["ms"] is not None else r["skipped"])
                                  for r in results})
    else:
        need = 0
        for b in range(len(batches)):
            st.forward_backward(b)
            need = max(need, st.ctx.status()["n_isect_needed"])
        st.set_capacity(int(need * 1.15) + 4096)
    log(f"[bench] {name}: settings {st.settings.tile_w}x{st.settings.tile_h} "
        f"order={st.settings.tile_order}, capacity {st.ctx.cap.max_isect}")
    timer = EventTimer(torch)
    for i in range(warmup):
        st.run(i % len(batches))
    torch.cuda.synchronize()
    st.ctx.reset_status()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b_ = torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(steps):
        st.run(i % len(batches), timer=timer)
    b_.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b_) / steps
    per_call = timer.means()
    status = st.ctx.status()
    # the same steps replayed from captured HIP graphs (one per batch)
    graph_ms = None
    step_ms = None
    try:
        if not graph:
            raise RuntimeError("graph replay skipped (--no-graph)")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for bb in range(len(batches)):
                st.run(bb)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graphs = []
        for bb in range(len(batches)):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                st.run(bb)  # the device step counter advances on every replay
            graphs.append(g)
        torch.cuda.synchronize()
        for g in graphs:  # untimed first replays (graph upload)
            g.replay()
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        a.record()
        evs[0].record()
        for i in range(steps):
            graphs[i % len(batches)].replay()
            evs[i + 1].record()
        b_.record()
        torch.cuda.synchronize()
        graph_ms = a.elapsed_time(b_) / steps
        step_ms = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
        del graphs
        status = st.ctx.status()  # flags of the eager and the replayed steps
    except Exception as e:  # report, do not hide
        log(f"[bench] graph replay failed: {e!r}")
    # workload sizes for the roofline (outside the timed region; the forward's
    # evaluation counts come from its counting variant)
    timed_settings = st.settings
    st.settings = L.default_settings(tile_w=timed_settings.tile_w, tile_h=timed_settings.tile_h,
                                     tile_order=timed_settings.tile_order, eval_stats=1)
    st.forward_backward(0)
    torch.cuda.synchronize()
    st.settings = timed_settings
    stat0 = st.ctx.status()
    wh_b = st.wh_all[batches[0]]
    P = int((wh_b[:, 0].astype(np.int64) * wh_b[:, 1]).sum())
    ts = L.gs_ctx_tile_stats(st.ctx)
    nt = ts["n_tiles"]
    tile_sum = lambda key: int(L.copy_to_host(ts[key], nt, np.int32).astype(np.int64).sum())
    # list entries the tiles read, (pixel, entry) evaluations the definition
    # makes up to each pixel's last contributor, contributing pairs
    C_f = tile_sum("tile_entries")
    n_eval = tile_sum("tile_evals")
    n_contrib = tile_sum("tile_contrib")
    sizes = dict(P=P, N=st.N, V=len(batches[0]), K=(st.sh_degree + 1) ** 2,
                 n_visible=stat0["n_visible"], n_isect=stat0["n_isect"], C_f=C_f,
                 n_eval=n_eval, n_contrib=n_contrib,
                 M=int(st.obs_cam.shape[0]), Pt=int(st.X.shape[0]),
                 n_params=int(sum(v.numel() for v in st._opt_params().values())),
                 n_adam=int(st.twist.numel() + st.X.numel()))
    return dict(ms=ms, graph_ms=graph_ms, step_ms=step_ms, per_call=per_call, status=status, sizes=sizes, st=st,
                sc=sc, batches=batches, tuning=tuning)


def algorithmic_bytes(sz):
    """Bytes each call must move at least (per launch), by the model of the
    hot-path table: parameter streams, records up to tile termination, pixel
    I/O, per-pair 2D gradients, intersections through one sort pass."""
    pg = 44 + 12 * sz["K"]
    return {
        "project": sz["N"] * pg + sz["n_visible"] * 48,
        "bin_sort": sz["n_isect"] * 36,
        "render_fwd": sz["C_f"] * 40 + sz["P"] * 20,
        "l1": sz["P"] * 36,
        # images in, gradient out (the SSIM window sums stay in LDS)
        "photo": sz["P"] * 36,
        "raster_bwd": sz["C_f"] * 40 + sz["P"] * 20 + sz["n_visible"] * 36,
        "project_bwd": sz["n_visible"] * 36 + 2 * sz["N"] * pg,
        # 2D gradients in; parameters, first and second moments in and out
        "project_bwd_adam": sz["n_visible"] * 36 + 6 * sz["N"] * pg,
        "track": sz["M"] * 28 + 2 * sz["Pt"] * 12,
        # twists and track points (the Gaussians step inside project_bwd_adam)
        "adam": sz["n_adam"] * 28,
    }


# Arithmetic of the definition, one per add, multiply, compare, select, min,
# exp2 or reciprocal and two per fused multiply-add: per (pixel, list entry)
# evaluation (offset 2, exponent 8, exp2, opacity, clamp, gate = 14) and per
# contributing (pixel, splat) pair (forward: 1 - alpha, T update, stop test,
# weight, colour 3 fma = 10; backward: 1 - alpha, rcp, T, weight, colour
# gradient 3 fma, dL/dC.c, dL/dalpha, dL/dC.S update, q with clamp, opacity
# gradient, five moments = 34)
FLOPS_EVAL = 14
FLOPS_CONTRIB = {"render_fwd": 10, "raster_bwd": 34}
FP32_PEAK_TFLOPS = 157.3
ALU_KERNELS = ("render_fwd", "raster_bwd")
# calls that launch one kernel (the others are sequences: bin_sort is ~25)
SINGLE_KERNEL = ("project", "render_fwd", "l1", "photo", "raster_bwd", "track", "adam")
KERNEL_SOURCE = {"render_fwd": "raster.hip", "raster_bwd": "raster.hip", "project": "project.hip",
                 "project_bwd": "project.hip", "project_bwd_adam": "project.hip",
                 "bin_sort": "bin.hip", "track": "track.hip",
                 "adam": "optim.hip", "l1": "raster.hip", "photo": "photo.hip"}


# calls whose kernels HBM traffic bounds (the raster pair is VALU-bound, the
# binning sequence latency- and VALU-bound)
HBM_BOUND_CALLS = ("project", "project_bwd_adam", "l1", "adam")
# the steps of one forward + backward with pose gradients (a2-a8), and the
# whole step (a1-a10: adds the track term and Adam on twists and points)
A2_A8 = ("project", "bin_sort", "render_fwd", "l1", "photo", "raster_bwd", "project_bwd",
         "project_bwd_adam")
STEP_CALLS = A2_A8 + ("track", "adam")


def algorithmic_flops(sz, call):
    return sz["n_eval"] * FLOPS_EVAL + sz["n_contrib"] * FLOPS_CONTRIB[call]


def hbm_step(alg, per_call, step_ms):
    a = [k for k in A2_A8 if k in per_call and k in alg]
    w = [k for k in STEP_CALLS if k in per_call and k in alg]
    b_a, t_a = sum(alg[k] for k in a), sum(per_call[k] for k in a)
    b_w = sum(alg[k] for k in w)
    return {"a2_a8": {"bytes": int(b_a), "ms": round(t_a, 4),
                      "gbs": round(b_a / (t_a * 1e-3) / 1e9, 1),
                      "frac": round(b_a / (t_a * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)},
            "step": {"bytes": int(b_w), "ms": round(step_ms, 4),
                     "gbs": round(b_w / (step_ms * 1e-3) / 1e9, 1),
                     "frac": round(b_w / (step_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)},
            "bytes_by_call": {k: int(alg[k]) for k in w},
            "model": ("project N(44+12K) + 48 N_v; bin_sort 36 I; render_fwd 40 C_f + 20 P; "
                      "photo / l1 36 P; raster_bwd 40 C_f + 20 P + 36 N_v; project_bwd_adam "
                      "36 N_v + 6 N(44+12K); track 28 M + 24 Pt; adam 28 per parameter")}


def source_sha(call):
    """Hash of the source of a call's kernels (its file and the shared header)."""
    import hashlib
    h = hashlib.sha256()
    for f in (KERNEL_SOURCE[call], "gs_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2603_04847_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(call, workload):
    """HBM bytes per launch from the committed counter runs, if they were taken
    on the current source of that call's kernels (else None)."""
    f = os.path.join(ROOT, "profiles", f"kernels_{workload}_hbm_traffic.json")
    if not os.path.exists(f):
        return None
    d = json.load(open(f))
    e = d.get(call)
    if not e or e.get("src_sha") != source_sha(call):
        return None
    return int(e["fetch_bytes"] + e["write_bytes"])


def batched_vs_per_view(torch, steps, warmup):
    """fwd+bwd (pose grads included) over the 8 uneven views of C3: one batched
    call per stage vs the same library called once per view.  The tile shape
    and launch order are the fastest of the candidates for the batched call
    (timed here); the per-view path runs at the same settings."""
    import scenegen
    import paper_2603_04847_amd as P
    from paper_2603_04847_amd import _lib as L
    sc = scenegen.make_config("C3")
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda().float()
    params = {k: f(sc[k]) for k in ("means", "log_scales", "quats", "opacity_logit", "sh")}
    N = params["means"].shape[1]
    V = sc["viewmat"].shape[0]
    wh = sc["wh"]
    Ptot = int((wh[:, 0].astype(np.int64) * wh[:, 1]).sum())
    vm, intr = f(sc["viewmat"]), f(sc["intr"])
    target = f(sc["target"])
    g = L.make_gaussians(*(params[k] for k in ("means", "log_scales", "quats", "opacity_logit", "sh")), 3)
    grads = {k: torch.empty_like(v) for k, v in params.items()}
    gg = L.make_grads(*(grads[k] for k in ("means", "log_scales", "quats", "opacity_logit", "sh")))
    rgb = torch.empty((Ptot, 3), device="cuda")
    T = torch.empty((Ptot,), device="cuda")
    last = torch.empty((Ptot,), device="cuda", dtype=torch.int32)
    v_rgb = torch.empty((Ptot, 3), device="cuda")
    loss = torch.zeros(1, device="cuda")
    v_tw = torch.zeros((V, 6), device="cuda")
    pix_off = np.concatenate([[0], np.cumsum(wh[:, 0].astype(np.int64) * wh[:, 1])])
    cams_b = L.Cameras(vm, intr, wh)
    cams_v = [L.Cameras(vm[v:v + 1], intr[v:v + 1], wh[v:v + 1]) for v in range(V)]
    cap_max = 2**30 - 65536

    def make_ctx(tile):
        tiles = int(sum(((w + tile[0] - 1) // tile[0]) * ((h + tile[1] - 1) // tile[1]) for w, h in wh))
        ctx = P.Context(max_pairs=V * N, max_isect=cap_max, max_tiles=tiles, max_views=V)
        s = L.default_settings(tile_w=tile[0], tile_h=tile[1])
        L.gs_project(ctx, g, cams_b, s)
        L.gs_bin_sort(ctx, cams_b, N, s)
        st = ctx.status()
        need = st["n_isect_needed"]
        ctx.close()
        if st["flags"] & L.GS_FLAG_ISECT_OVERFLOW or need * 1.1 + 4096 > cap_max:
            return None, need
        return P.Context(max_pairs=V * N, max_isect=int(need * 1.1) + 4096, max_tiles=tiles,
                         max_views=V), need

    def timed(fn, n):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    def batched(ctx, s):
        L.gs_project(ctx, g, cams_b, s)
        L.gs_bin_sort(ctx, cams_b, N, s)
        L.gs_render_fwd(ctx, cams_b, s, None, rgb, T, last)
        L.gs_l1_loss_grad(ctx, cams_b, rgb, target, v_rgb, loss)
        L.gs_render_bwd(ctx, g, cams_b, s, None, T, last, v_rgb, gg, v_tw)

    def per_view(ctx, s):
        s_acc = L.default_settings(tile_w=s.tile_w, tile_h=s.tile_h, tile_order=s.tile_order,
                                   grad_accumulate=1, lazy_lists=1)
        for v in range(V):
            a, b = int(pix_off[v]), int(pix_off[v + 1])
            c = cams_v[v]
            L.gs_project(ctx, g, c, s)
            L.gs_bin_sort(ctx, c, N, s)
            L.gs_render_fwd(ctx, c, s, None, rgb[a:b], T[a:b], last[a:b])
            L.gs_l1_loss_grad(ctx, c, rgb[a:b], target[a:b], v_rgb[a:b], loss)
            L.gs_render_bwd(ctx, g, c, s if v == 0 else s_acc, None, T[a:b], last[a:b],
                            v_rgb[a:b], gg, v_tw[v:v + 1])

    cand = {}
    best = None
    for tile in ((16, 16), (32, 16), (16, 8)):
        ctx, need = make_ctx(tile)
        if ctx is None:
            cand[f"{tile[0]}x{tile[1]}"] = "lists exceed the capacity limit"
            continue
        for order in (0, 1, 2):
            s = L.default_settings(tile_w=tile[0], tile_h=tile[1], tile_order=order, lazy_lists=1)
            ms = timed(lambda: batched(ctx, s), max(2, steps // 2))
            cand[f"{tile[0]}x{tile[1]}/{order}"] = round(ms, 3)
            if best is None or ms < best[0]:
                best = (ms, tile, order, need)
        ctx.close()
    _, tile, order, need = best
    ctx, need = make_ctx(tile)
    s = L.default_settings(tile_w=tile[0], tile_h=tile[1], tile_order=order, lazy_lists=1)
    out = {}
    for name, fn in (("batched", lambda: batched(ctx, s)), ("per_view", lambda: per_view(ctx, s))):
        ms = timed(fn, steps)
        out[name] = dict(ms=round(ms, 3), mp_s=round(Ptot / ms / 1e3, 1))
    out["speedup"] = round(out["per_view"]["ms"] / out["batched"]["ms"], 2)
    out["config"] = WORKLOADS["C3"]
    out["tile"] = f"{tile[0]}x{tile[1]}"
    out["tile_order"] = order
    out["autotune_ms"] = cand
    out["n_isect"] = int(need)
    # the stated load imbalance on the exact tile lists
    L.gs_project(ctx, g, cams_b, s)
    L.gs_bin_sort(ctx, cams_b, N, s)
    b = ctx.buffers()
    nt = b["n_tiles"]
    rng = L.copy_to_host(b["tile_ranges"], 2 * nt, np.int32).reshape(nt, 2)
    lens = (rng[:, 1] - rng[:, 0]).astype(np.int64)
    nz = lens[lens > 0]
    out["tile_list_len_max_over_median"] = round(float(nz.max() / np.median(nz)), 1)
    ctx.close()
    return out


def next_rows(torch, res, reps=5):
    """The calls around the joint step on the same scene: Gaussians from the
    track points (k = 4 nearest neighbours), one Levenberg-Marquardt step of
    bundle adjustment over all observations, MCMC relocation (a fifth of the
    Gaussians dead) and the MCMC noise on the means.  Inputs resident; HIP
    events on the launch stream; mean of `reps` calls after one warm-up."""
    from paper_2603_04847_amd import _lib as L
    st, sc = res["st"], res["sc"]
    sz = res["sizes"]
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    Pt = int(st.X.shape[0])
    K = (st.sh_degree + 1) ** 2
    rgb = torch.rand((Pt, 3), device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    ms = timed(lambda: L.gs_init_gaussians(st.ctx, st.X, rgb, sh_degree=st.sh_degree))
    byt = Pt * 24 + Pt * (44 + 12 * K)
    out["init_gaussians"] = dict(points=Pt, ms=round(ms, 4), algorithmic_gbs=round(byt / (ms * 1e-3) / 1e9, 1))
    if st.pt_index is not None and Pt > 0:
        ba = L.BundleAdjuster(Pt, st.n_cams)
        dtw = torch.empty((st.n_cams, 6), device="cuda")
        dX = torch.empty((Pt, 3), device="cuda")
        stats = torch.zeros(5, device="cuda")
        call = lambda: L.gs_ba_lm_step(ba, st.X, st.viewmat, st.intr, st.obs_cam, st.obs_pt,
                                       st.obs_xy, st.pt_index, 1.0, 1e-2, 0.01, 100, 1e-8, dtw, dX,
                                       stats)
        ms = timed(call)
        s5 = stats.cpu().numpy()
        it = int(s5[0])
        # per conjugate-gradient iteration two passes over the observations
        # (~30 B each: camera, point, pixel and the point's coordinates)
        out["ba_lm_step"] = dict(cameras=st.n_cams, points=Pt, observations=sz["M"], ms=round(ms, 4),
                                 pcg_iterations=it, relative_residual=float(s5[1]),
                                 ms_per_pcg_iteration=round(ms / max(it + 3, 1), 4))
        ba.close()
    N = st.N
    g = {k: st.params[k].clone() for k in ("means", "log_scales", "quats", "opacity_logit", "sh")}
    gen = torch.Generator("cuda").manual_seed(2)
    dead = torch.rand(N, device="cuda", generator=gen) < 0.2
    base_logit = g["opacity_logit"].clone()
    base_logit[dead] = -9.0
    m1 = [torch.zeros_like(g[k]) for k in g]
    m2 = [torch.zeros_like(g[k]) for k in g]
    u = torch.rand(N, device="cuda", generator=gen)
    P = [g[k] for k in g]

    def reloc():
        g["opacity_logit"].copy_(base_logit)
        L.gs_mcmc_relocate(st.ctx, P, m1, m2, st.sh_degree, u)
    ms_copy = timed(lambda: g["opacity_logit"].copy_(base_logit))
    ms = timed(reloc) - ms_copy
    out["mcmc_relocate"] = dict(gaussians=N, dead_fraction=0.2, ms=round(ms, 4))
    eta = torch.randn((3, N), device="cuda", generator=gen)
    ms = timed(lambda: L.gs_mcmc_noise(g["means"], g["log_scales"], g["quats"], g["opacity_logit"],
                                       eta, 1e-3))
    byt = N * (12 + 12 + 16 + 4 + 12) + N * 12
    out["mcmc_noise"] = dict(gaussians=N, ms=round(ms, 4),
                             algorithmic_gbs=round(byt / (ms * 1e-3) / 1e9, 1))
    return out


def copy_bandwidth(torch, mib=1024, reps=5):
    """Device copy rate (GB/s, bytes read + written) of a plain elementwise
    copy of `mib` MiB, beside the 8 TB/s HBM peak."""
    n = mib * (1 << 20) // 4
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del x, y
    return round(2 * n * 4 / (ms * 1e-3) / 1e9, 1)


def cpu_baseline(res, seconds_target=12.0, lambda_ssim=0.2, max_gaussians=1_000_000,
                 max_obs=2_000_000):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload: the projection and its backward for the batch's views, the track
    term, and compositing (with backward) of a random sample of pixels; the
    compositing time is fitted over sample sizes and taken at all pixels.  On
    scenes of more than `max_gaussians` Gaussians (or `max_obs` observations)
    the oracle runs on the first ones and its per-Gaussian (per-observation)
    times are scaled to the whole scene: every part of it is linear in them."""
    import oracle
    sc, b = res["sc"], res["batches"][0]
    st = res["st"]
    sz = res["sizes"]
    vm = st.viewmat.cpu().numpy()[b]
    intr = sc["intr"][b]
    wh = sc["wh"][b]
    t_start = time.time()
    Ns = min(sz["N"], max_gaussians)
    fN = sz["N"] / Ns
    sub = dict(sc, viewmat=vm, intr=intr, wh=wh)
    for k in ("means", "log_scales", "quats"):
        sub[k] = np.ascontiguousarray(sc[k][:, :Ns])
    sub["opacity_logit"] = np.ascontiguousarray(sc["opacity_logit"][:Ns])
    sub["sh"] = np.ascontiguousarray(sc["sh"][:, :, :Ns])
    t0 = time.time()
    proj = oracle.project(sub)
    t_proj = (time.time() - t0) * fN
    rng = np.random.default_rng(0)
    # the oracle's compositing time is a fixed part (per-view set-up) plus a
    # part per pixel: two calibration sizes give the per-pixel cost, a third,
    # larger sample (most of the time budget) the fit used for all pixels
    def timed(n):
        pix = rng.choice(sz["P"], size=n, replace=False)
        t0 = time.time()
        r = oracle.render(proj, wh, pix=pix, v_rgb=np.ones((n, 3)))
        return time.time() - t0, r
    timed(64)  # untimed: first-call set-up
    n1, n2 = 256, 1024
    t1, _ = timed(n1)
    t2, _ = timed(n2)
    # per-pixel cost for sizing: the marginal one, but never below half the
    # mean (timing noise must not size a sample that runs for minutes)
    b0 = max((t2 - t1) / (n2 - n1), 0.5 * t2 / n2, 1e-9)
    n_pix = int(max(2 * n2, min(400000, 0.6 * seconds_target / b0)))
    log(f"[bench] oracle: {n1} px {t1:.1f}s, {n2} px {t2:.1f}s; sampling {n_pix} px")
    t_pix, r = timed(n_pix)
    log(f"[bench] oracle: {n_pix} px {t_pix:.1f}s")
    per_px = max((t_pix - t1) / (n_pix - n1), 1e-12)
    fixed = max(t1 - per_px * n1, 0.0)
    t_pix_all = (fixed + per_px * sz["P"]) * fN
    t0 = time.time()
    oracle.project_bwd(sub, r["v2d"])
    t_pbwd = (time.time() - t0) * fN
    t_track, Ms = 0.0, 0
    if sz["M"] > 0:
        Ms = min(sz["M"], max_obs)
        t0 = time.time()
        oracle.track(sc["X"], st.viewmat.cpu().numpy(), sc["intr"], sc["obs_cam"][:Ms],
                     sc["obs_pt"][:Ms], sc["obs_xy"][:Ms], jacobians=False)
        t_track = (time.time() - t0) * sz["M"] / Ms
    # the photometric loss on a crop of view 0 (its cost is linear in pixels)
    t_photo, n_crop = 0.0, 0
    if lambda_ssim > 0:
        W0, H0 = int(wh[0, 0]), int(wh[0, 1])
        cw, ch = min(W0, 400), min(H0, 300)
        img = st.rgb[:W0 * H0].cpu().numpy().reshape(H0, W0, 3)[:ch, :cw].reshape(-1, 3)
        tgt = st.targets[0][:W0 * H0].cpu().numpy().reshape(H0, W0, 3)[:ch, :cw].reshape(-1, 3)
        n_crop = cw * ch
        t0 = time.time()
        oracle.photo_loss(img, tgt, np.array([[cw, ch]], np.int32), lam=lambda_ssim)
        t_photo = (time.time() - t0) * sz["P"] / n_crop
    t_step = t_proj + t_pix_all + t_pbwd + t_track + t_photo
    # one thread: the same three pieces (compositing of 256 pixels, the
    # projection of the first 50k Gaussians, the track term on the first 100k
    # observations) timed on all threads and on one; the all-core estimate
    # divided by that ratio
    cores = oracle.num_threads()

    def pieces():
        t0 = time.time()
        pix = np.random.default_rng(1).choice(sz["P"], size=256, replace=False)
        oracle.render(proj, wh, pix=pix, v_rgb=np.ones((256, 3)))
        s1 = dict(sub)
        for k in ("means", "log_scales", "quats"):
            s1[k] = np.ascontiguousarray(sub[k][:, :50000])
        s1["opacity_logit"] = np.ascontiguousarray(sub["opacity_logit"][:50000])
        s1["sh"] = np.ascontiguousarray(sub["sh"][:, :, :50000])
        oracle.project(s1)
        if sz["M"] > 0:
            m1 = min(sz["M"], 100000)
            oracle.track(sc["X"], st.viewmat.cpu().numpy(), sc["intr"], sc["obs_cam"][:m1],
                         sc["obs_pt"][:m1], sc["obs_xy"][:m1], jacobians=False)
        return time.time() - t0
    t_all = pieces()
    oracle.set_num_threads(1)
    try:
        t_one = pieces()
    finally:
        oracle.set_num_threads(cores)
    ratio = t_one / max(t_all, 1e-9)
    single = dict(value=round(sz["P"] / (t_step * ratio) / 1e6, 7), unit="MP/s", cores=1,
                  all_cores_speedup=round(ratio, 2),
                  sample=(f"the all-core estimate divided by the one-thread / all-thread time "
                          f"ratio of compositing 256 pixels, projecting 50k Gaussians and the "
                          f"track term on 100k observations ({t_one:.1f}s vs {t_all:.2f}s)"))
    return dict(value=round(sz["P"] / t_step / 1e6, 6), unit="MP/s", cores=cores,
                kind="oracle", single_thread=single,
                sample=(f"batch 0 of the workload on its first {Ns} of {sz['N']} Gaussians and "
                        f"first {Ms} of {sz['M']} observations (times scaled by {fN:.2f} and "
                        f"{(sz['M'] / Ms) if Ms else 0:.2f}): projection + its backward of "
                        f"{sz['V']} views, track term, and compositing + backward of {n_pix} "
                        f"random pixels of {sz['P']} (its time fitted as {fixed:.2f}s + "
                        f"{per_px * 1e3:.3f} ms per pixel from samples of {n1}, {n2} and {n_pix} "
                        f"pixels, then taken at all pixels)"
                        + (f", and the photometric loss (L1 + SSIM) on a {n_crop}-pixel crop of "
                           f"view 0 scaled to all pixels" if n_crop else "")
                        + f"; measured {time.time() - t_start:.1f}s"))


# -------------------------------------------------------------- counter summaries

# the counter passes: one rocprofv3 run each (a pass holds at most 4 TCC, 4 TCP
# and 8 SQ counters); FETCH_SIZE and WRITE_SIZE also on the copy probe
COUNTER_PASSES = {
    "fetch": ["FETCH_SIZE"],
    "write": ["WRITE_SIZE"],
    "l2": ["TCC_HIT_sum", "TCC_MISS_sum", "TCC_ATOMIC_sum", "TCP_TCC_ATOMIC_WITH_RET_REQ_sum",
           "TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum"],
    "lds": ["SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "SQ_INSTS_LDS", "SQ_WAIT_INST_LDS",
            "SQ_LDS_ADDR_CONFLICT", "SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES"],
    "valu": ["SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_THREAD_CYCLES_VALU", "SQ_WAIT_ANY",
             "SQ_ACTIVE_INST_ANY", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_INSTS_SALU",
             "GRBM_GUI_ACTIVE"],
}
N_CU, N_XCD, WAVE = 256, 8, 64


def _short_kernel(name):
    n = name[5:] if name.startswith("void ") else name
    n = n.replace("gs::(anonymous namespace)::", "")
    depth, out = 0, ""
    for ch in n:
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out += ch
    return out


def _read_pass(raw, name):
    """Dispatches of one counter pass in launch order: [(kernel, {counter: value}, ns)]."""
    import csv
    import glob
    files = glob.glob(os.path.join(raw, name, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter file under {os.path.join(raw, name)}")
    disp = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            d = disp.setdefault(int(r["Dispatch_Id"]), [r["Kernel_Name"], {},
                                                          int(r["End_Timestamp"]) - int(r["Start_Timestamp"])])
            d[1][r["Counter_Name"]] = d[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [tuple(disp[k]) for k in sorted(disp)]


def _bench_line(raw, name):
    for ln in open(os.path.join(raw, name + ".log")):
        if ln.startswith("{"):
            return json.loads(ln)
    return None


# the kernels of each timed call (bin_sort: every dispatch from k_count to k_chunk_expand)
CALL_KERNELS = {
    "project": lambda k: k.startswith("k_project_fwd<"),
    "render_fwd": lambda k: k.startswith("k_render_fwd<") and k.endswith("false>"),
    "raster_bwd": lambda k: k.startswith("k_render_bwd<"),
    "photo": lambda k: k == "k_photo",
    "project_bwd_adam": lambda k: k in ("k_project_bwd_color<3, true>", "k_project_bwd_geom<true>"),
    "track": lambda k: k in ("k_track", "k_track_points", "k_track_pm", "k_track_pm_reduce"),
    "adam": lambda k: k == "k_adam",
}


def _per_call(disp, counter):
    """Per-launch totals of one counter for each timed call."""
    out = {}
    for call, sel in CALL_KERNELS.items():
        tot = [v.get(counter, 0.0) for k, v, _ in disp if sel(_short_kernel(k))]
        first = [k for k, _, _ in disp if sel(_short_kernel(k))]
        n_first = sum(1 for k in first if _short_kernel(k) == _short_kernel(first[0])) if first else 0
        if n_first:
            out[call] = sum(tot) / n_first
    segs, cur = [], None
    for k, v, _ in disp:
        sk = _short_kernel(k)
        if sk == "k_count":
            cur = 0.0
        if cur is not None:
            cur += v.get(counter, 0.0)
        if sk == "k_chunk_expand" and cur is not None:
            segs.append(cur)
            cur = None
    if segs:
        out["bin_sort"] = sum(segs) / len(segs)
    return out


def summarize_counters(raw, workload):
    """profiles/kernels_<workload>_hbm_traffic.json (HBM bytes per launch of each
    timed call, FETCH_SIZE and WRITE_SIZE scaled by what they read for a 1 GiB
    streaming copy) and profiles/kernels_<workload>_counters.md (per kernel:
    HBM bytes, L2 hit rate, atomics, LDS bank conflicts, VALU busy and lanes
    active) from the rocprofv3 passes under `raw`."""
    cf = [v["FETCH_SIZE"] for k, v, _ in _read_pass(raw, "copy_fetch")
          if "AUnaryFunctor" in k or "MulFunctor" in k or "BinaryFunctor" in k]
    cw = [v["WRITE_SIZE"] for k, v, _ in _read_pass(raw, "copy_write")
          if "AUnaryFunctor" in k or "MulFunctor" in k or "BinaryFunctor" in k]
    gib_kib = float(1 << 20)
    f_scale = gib_kib / float(np.median(cf))
    w_scale = gib_kib / float(np.median(cw))
    P = {n: _read_pass(raw, f"{workload}_{n}") for n in COUNTER_PASSES}
    line = _bench_line(raw, f"{workload}_fetch") or {}
    alg = (line.get("hbm_step") or {}).get("bytes_by_call", {})
    fetch = _per_call(P["fetch"], "FETCH_SIZE")
    write = _per_call(P["write"], "WRITE_SIZE")
    traffic = {"workload": workload, "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
               "note": ("HBM bytes per launch of each timed call: FETCH_SIZE and WRITE_SIZE (KiB) "
                        "times 1024 times the copy-probe factor; src_sha is the hash of the call's "
                        "kernel sources when the counters were taken")}
    for call in fetch:
        if call in write:
            traffic[call] = {"src_sha": source_sha(call),
                             "fetch_bytes": int(fetch[call] * 1024 * f_scale),
                             "write_bytes": int(write[call] * 1024 * w_scale),
                             "algorithmic_bytes": alg.get(call)}
    with open(os.path.join(ROOT, "profiles", f"kernels_{workload}_hbm_traffic.json"), "w") as fh:
        json.dump(traffic, fh, indent=1)
        fh.write("\n")
    # per kernel, averaged over its dispatches in each pass
    agg = {}
    for n, disp in P.items():
        for k, v, ns in disp:
            a = agg.setdefault(_short_kernel(k), {"_n": {}, "_ns": []})
            a["_n"][n] = a["_n"].get(n, 0) + 1
            if n == "valu":
                a["_ns"].append(ns)
            for c, x in v.items():
                a[c] = a.get(c, 0.0) + x
    rows = []
    for k, a in agg.items():
        if not a["_ns"] or np.mean(a["_ns"]) < 20e3:
            continue

        def per(c, n):
            return a.get(c, 0.0) / max(a["_n"].get(n, 0), 1)
        hit, miss = per("TCC_HIT_sum", "l2"), per("TCC_MISS_sum", "l2")
        lds_act = per("SQ_LDS_IDX_ACTIVE", "lds")
        act_valu = per("SQ_ACTIVE_INST_VALU", "valu")
        grbm = per("GRBM_GUI_ACTIVE", "valu") / N_XCD
        rows.append((np.mean(a["_ns"]), k, a["_n"].get("valu", 0),
                     per("FETCH_SIZE", "fetch") * 1024 * f_scale / 1e6,
                     per("WRITE_SIZE", "write") * 1024 * w_scale / 1e6,
                     hit / max(hit + miss, 1.0),
                     per("TCC_ATOMIC_sum", "l2"),
                     per("TCP_TCC_ATOMIC_WITH_RET_REQ_sum", "l2") + per("TCP_TCC_ATOMIC_WITHOUT_RET_REQ_sum", "l2"),
                     per("SQ_LDS_BANK_CONFLICT", "lds") / lds_act if lds_act else 0.0,
                     per("SQ_INSTS_LDS", "lds"),
                     act_valu / N_CU / grbm if grbm else 0.0,
                     per("SQ_THREAD_CYCLES_VALU", "valu") / (act_valu * WAVE) if act_valu else 0.0,
                     per("SQ_WAIT_ANY", "valu") / max(per("SQ_WAVE_CYCLES", "lds"), 1.0)))
    rows.sort(reverse=True)
    cmd_pass = ("cd /tmp && rocprofv3 --pmc <counters of the pass> --output-format csv -d "
                "/root/repo/gpurun_out/pmc/{W}_<pass> -o run -- python3 /root/repo/bench.py --workload {W} "
                "--steps 2 --warmup 1 --tile {T} --order 0 --no-compare --no-cpu-baseline --no-extra "
                "--no-graph").format(W=workload, T=(line.get("config") or {}).get("tile", "?"))
    md = [f"# Counters of the joint step, {workload}, per kernel (rocprofv3 --pmc)", "",
          "Passes (one rocprofv3 run each; the counters of a pass in brackets):", ""]
    md += [f"- `{n}`: " + " ".join(c) for n, c in COUNTER_PASSES.items()]
    md += ["", "Command of a pass, and of the copy probe that calibrates FETCH_SIZE / WRITE_SIZE "
           "(passes `copy_fetch`, `copy_write`):", "", "```", cmd_pass,
           "cd /tmp && rocprofv3 --pmc FETCH_SIZE --output-format csv -d /root/repo/gpurun_out/pmc/copy_fetch "
           "-o run -- python3 /root/repo/bench.py --copy-probe 1024", "```", "",
           "Summary written by `python bench.py --summarize-counters gpurun_out/pmc --workload "
           f"{workload}` (also writes `kernels_{workload}_hbm_traffic.json`).", "",
           f"Copy probe (1 GiB read and 1 GiB written per launch): FETCH_SIZE reads "
           f"{1 / f_scale:.3f} of the bytes read, WRITE_SIZE {1 / w_scale:.3f} of the bytes written; "
           "the HBM columns below are scaled by the inverse.", "",
           "| kernel | launches | us (under counters) | HBM read MB | HBM write MB | L2 hit | "
           "TCC atomics | TCP->TCC atomic req | LDS bank-conflict cycles / LDS active | LDS insts | "
           "VALU busy | VALU lanes active | wait share |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        md.append(f"| `{r[1]}` | {r[2]} | {r[0] / 1e3:.1f} | {r[3]:.1f} | {r[4]:.1f} | {r[5]:.3f} | "
                  f"{r[6]:.3g} | {r[7]:.3g} | {r[8]:.4f} | {r[9]:.3g} | {r[10]:.3f} | {r[11]:.3f} | "
                  f"{r[12]:.3f} |")
    md += ["", "Per timed call, HBM bytes per launch against the algorithmic bytes of the bench's "
           "model (the same run's bench line):", "",
           "| call | HBM read MB | HBM write MB | algorithmic MB | measured / algorithmic |",
           "|---|---:|---:|---:|---:|"]
    for call in ("project", "bin_sort", "render_fwd", "photo", "raster_bwd", "project_bwd_adam",
                 "track", "adam"):
        t = traffic.get(call)
        if not t:
            continue
        a = t["algorithmic_bytes"]
        tot = t["fetch_bytes"] + t["write_bytes"]
        md.append(f"| {call} | {t['fetch_bytes'] / 1e6:.1f} | {t['write_bytes'] / 1e6:.1f} | "
                  f"{(a or 0) / 1e6:.1f} | {(tot / a if a else float('nan')):.2f} |")
    md += ["", "Columns: L2 hit = TCC_HIT / (TCC_HIT + TCC_MISS); VALU busy = SQ_ACTIVE_INST_VALU / "
           f"{N_CU} CUs / (GRBM_GUI_ACTIVE / {N_XCD} XCDs); VALU lanes active = SQ_THREAD_CYCLES_VALU / "
           "(SQ_ACTIVE_INST_VALU x 64); wait share = SQ_WAIT_ANY / SQ_WAVE_CYCLES (two passes of "
           "the same work). Kernels under 20 us left out."]
    with open(os.path.join(ROOT, "profiles", f"kernels_{workload}_counters.md"), "w") as fh:
        fh.write("\n".join(md) + "\n")
    print(json.dumps(traffic, indent=1))


def summarize_trace(raw, workload, cmd, stem=None):
    """profiles/<stem or joint_step_<workload>>_kernel_trace.md from a rocprofv3
    --kernel-trace --stats run of this bench (`cmd`): per kernel, launches and
    durations, and the live HIP-event time of the dominant kernel from the same
    run's bench line beside the trace's average for it."""
    import csv
    import glob
    f = glob.glob(os.path.join(raw, "**", "*kernel_stats.csv"), recursive=True)
    if not f:
        raise SystemExit(f"no kernel_stats.csv under {raw}")
    rows = list(csv.DictReader(open(f[0])))
    line = None
    for ln in open(os.path.join(raw + ".json")) if os.path.exists(raw + ".json") else []:
        if ln.startswith("{"):
            line = json.loads(ln)
    title = f"Joint step, {workload}" if not stem else stem.replace("_", " ")
    md = [f"# {title}: per-kernel durations (rocprofv3 kernel trace)", "",
          "Command (the repository at /root/repo; the bench line goes to the .json beside the "
          "trace directory):", "", "```", cmd, "```", "",
          f"Summary written by `python bench.py --summarize-trace {raw} --workload {workload}"
          + (f" --trace-name {stem}" if stem else "") + "`.", "",
          "| kernel | calls | total ms | avg us | min us | max us | % |",
          "|---|---:|---:|---:|---:|---:|---:|"]
    trace_avg = {}
    for r in rows:
        name = _short_kernel(r["Name"])
        trace_avg[name] = float(r["AverageNs"]) / 1e3
        if float(r["Percentage"]) < 0.05:
            continue
        md.append(f"| `{name[:70]}` | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.3f} | "
                  f"{float(r['AverageNs']) / 1e3:.1f} | {int(r['MinNs']) / 1e3:.1f} | "
                  f"{int(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    if line:
        roof = line.get("roofline") or {}
        dom = roof.get("kernel")
        kname = {"raster_bwd": "k_render_bwd", "render_fwd": "k_render_fwd"}.get(dom)
        tr = [v for k, v in trace_avg.items() if kname and k.startswith(kname) and not k.endswith("true>")]
        md += ["", f"Workload: {line['config']['workload']}; tile {line['config']['tile']}, order "
               f"{line['config']['tile_order']}.", "",
               f"Agreement with the live timing: the same run's bench line measured `{dom}` at "
               f"{roof.get('avg_ms', 0) * 1e3:.1f} us per call (HIP events on its stream, under the "
               f"profiler: {line['value']} MP/s); the trace average of its kernel is "
               + (f"{max(tr):.1f} us." if tr else "not found.")]
    out = os.path.join(ROOT, "profiles", f"{stem or 'joint_step_' + workload}_kernel_trace.md")
    with open(out, "w") as fh:
        fh.write("\n".join(md) + "\n")
    print(out)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C5", choices=sorted(WORKLOADS))
    ap.add_argument("--lambda-ssim", type=float, default=0.2,
                    help="weight of the SSIM term in the photometric loss (0: L1 alone)")
    ap.add_argument("--no-extra", action="store_true", help="skip the extra C4 timing")
    ap.add_argument("--no-tune", action="store_true", help="keep 16x16 tiles, natural order")
    ap.add_argument("--tile", default=None, help="fixed tile shape WxH (skips the autotuner)")
    ap.add_argument("--order", type=int, default=0, help="tile launch order with --tile")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized buffer 5 times with an elementwise kernel (counter calibration) and exit")
    ap.add_argument("--print-sha", action="store_true",
                    help="print the kernel source hashes used to validate stored counters")
    ap.add_argument("--no-compare", action="store_true", help="skip batched vs per-view (C3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replay timing")
    ap.add_argument("--full-lists", action="store_true",
                    help="bin into complete tile lists (gs_settings.lazy_lists = 0)")
    ap.add_argument("--serial-track", action="store_true",
                    help="run the track term in line instead of on a second stream")
    ap.add_argument("--summarize-counters", default=None, metavar="DIR",
                    help="write the counter summaries under profiles/ from the rocprofv3 passes in DIR "
                         "(no GPU needed) and exit")
    ap.add_argument("--summarize-trace", default=None, metavar="DIR",
                    help="write profiles/joint_step_<workload>_kernel_trace.md from the rocprofv3 "
                         "kernel trace in DIR (and the bench line in DIR.json) and exit")
    ap.add_argument("--trace-cmd", default="", help="the command that made the trace (for the summary)")
    ap.add_argument("--trace-name", default=None,
                    help="file name stem of the trace summary (default joint_step_<workload>)")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.workload)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.workload, args.trace_cmd, args.trace_name)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the hot path "
              "here has no multi-GPU code", file=sys.stderr)
        sys.exit(2)
    if args.print_sha:
        print(json.dumps({k: source_sha(k) for k in KERNEL_SOURCE}))
        return
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)  # a plain streaming copy: reads and writes MIB each
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_probe} MiB x 5")
        return
    import paper_2603_04847_amd as P
    P.load()

    tile = tuple(int(x) for x in args.tile.split("x")) if args.tile else None
    res = run_joint(torch, args.workload, args.steps, args.warmup, tune=not args.no_tune,
                    tile=tile, order=args.order, graph=not args.no_graph,
                    lambda_ssim=args.lambda_ssim, lazy_lists=not args.full_lists,
                    overlap_track=not args.serial_track)
    sz = res["sizes"]
    # the timed steps: replayed from captured HIP graphs (the production mode:
    # the same kernels, no per-call host work between them), else eager
    ms_eager = res["ms"]
    ms = res["graph_ms"] if res["graph_ms"] is not None else ms_eager
    value = sz["P"] / ms / 1e3  # megapixels / s
    per_call = {k: round(v, 4) for k, v in res["per_call"].items()}
    alg = algorithmic_bytes(sz)
    roof = None
    if per_call:
        # the dominant kernel: the slowest call that is a single kernel launch
        dom = max((k for k in per_call if k in SINGLE_KERNEL), key=lambda k: per_call[k])
        t = per_call[dom] * 1e-3
        if dom in ALU_KERNELS:
            ach = algorithmic_flops(sz, dom) / t / 1e12
            roof = {"bound": "alu", "kernel": dom, "achieved": round(ach, 2),
                    "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(ach / FP32_PEAK_TFLOPS, 4),
                    "algorithmic_flops": int(algorithmic_flops(sz, dom)),
                    "hbm_gbs_algorithmic": round(alg[dom] / t / 1e9, 1)}
        else:
            ach = alg[dom] / t / 1e9
            roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "algorithmic_bytes": int(alg[dom])}
        roof["traffic"] = measured_traffic(dom, args.workload)
        roof["avg_ms"] = per_call[dom]
    line = {
        "metric": "fwd+bwd megapixels/sec with pose grads (batched vs per-view), %HBM roofline",
        "value": round(value, 2), "unit": "MP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                   "views_per_step": sz["V"], "pixels_per_step": sz["P"], "gaussians": sz["N"],
                   "observations": sz["M"],
                   "tile": f"{res['st'].settings.tile_w}x{res['st'].settings.tile_h}",
                   "tile_order": int(res["st"].settings.tile_order),
                   "tile_lists": "lazy" if res["st"].lazy_lists else "full",
                   "track_stream": "second" if res["st"].overlap_track else "in line"},
        "roofline": roof,
        "per_call_ms": per_call,
        "per_call_algorithmic_gbs": {k: round(alg[k] / (per_call[k] * 1e-3) / 1e9, 1)
                                     for k in per_call if k in alg},
        # the calls bound by HBM: their algorithmic rate against the 8 TB/s peak
        "hbm_frac_by_call": {k: round(alg[k] / (per_call[k] * 1e-3) / 8e12, 3)
                             for k in HBM_BOUND_CALLS if k in alg and k in per_call},
        # the step's algorithmic HBM bytes against its time and the 8 TB/s peak:
        # a2-a8 (forward + backward with pose gradients) over the sum of those
        # calls' eager times, and the whole step (plus track and Adam) over the
        # replayed step time
        "hbm_step": hbm_step(alg, per_call, ms),
        "timed_as": "hip_graph_replay" if res["graph_ms"] is not None else "eager",
        "eager_ms_per_step": round(ms_eager, 4),
        "step_ms_p10_p50_p90": (None if res["step_ms"] is None else
                                [round(float(np.percentile(res["step_ms"], q)), 4) for q in (10, 50, 90)]),
        # the raster kernels are VALU-bound: their algorithmic rate against the FP32 peak
        "raster_alu_tflops": {k: round(algorithmic_flops(sz, k) / (per_call[k] * 1e-3) / 1e12, 2)
                              for k in ALU_KERNELS if k in per_call},
        # track reprojection (a9) as a share of the step (the paper quotes about 3 %)
        "track_share": (round(per_call["track"] / res["ms"], 4) if "track" in per_call else None),
        "copy_gbs": copy_bandwidth(torch),
        "autotune": res["tuning"],
        "sizes": {k: int(v) for k, v in sz.items()},
    }
    if res["status"]["flags"]:
        line["status_flags"] = res["status"]["flags"]
    if not args.no_compare:
        log("[bench] batched vs per-view on C3")
        line["batched_vs_per_view"] = batched_vs_per_view(torch, max(2, args.steps // 4), 1)
    if not args.no_extra:
        log("[bench] init, bundle adjustment and MCMC calls on the same scene")
        line["next_rows"] = next_rows(torch, res)
    if not args.no_cpu_baseline:
        log("[bench] oracle CPU baseline")
        line["cpu_baseline"] = cpu_baseline(res, lambda_ssim=args.lambda_ssim)
    if not args.no_extra and args.workload != "C4":
        # the joint step of 150 cameras at 1237x822 and 1M Gaussians, at the tile
        # shape and order its autotuning picks (16x16, heaviest tile first)
        del res
        torch.cuda.empty_cache()
        log("[bench] extra workload C4")
        r4 = run_joint(torch, "C4", args.steps, args.warmup, tune=False, tile=(16, 16), order=1,
                       graph=not args.no_graph, lambda_ssim=args.lambda_ssim,
                       lazy_lists=not args.full_lists, overlap_track=not args.serial_track)
        ms4 = r4["graph_ms"] if r4["graph_ms"] is not None else r4["ms"]
        pc4 = {k: round(v, 4) for k, v in r4["per_call"].items()}
        line["extra_workloads"] = {"C4": {
            "workload": f"C4: {WORKLOADS['C4']}", "value": round(r4["sizes"]["P"] / ms4 / 1e3, 2),
            "unit": "MP/s", "ms_per_step": round(ms4, 4),
            "timed_as": "hip_graph_replay" if r4["graph_ms"] is not None else "eager",
            "eager_ms_per_step": round(r4["ms"], 4), "tile": "16x16", "tile_order": 1,
            "per_call_ms": pc4, "hbm_step": hbm_step(algorithmic_bytes(r4["sizes"]), pc4, ms4),
            "status_flags": r4["status"]["flags"]}}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
