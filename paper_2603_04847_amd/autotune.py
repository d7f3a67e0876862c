"""Pick the tile shape and the tile launch order for a workload by timing them.

Every candidate runs the forward + backward of the joint step (a1-a9) at a
context sized for its own intersection count; the fastest wins.  The image
does not depend on the choice (the tile lists are truncation-free), so this
only trades binning work (more, smaller tiles) against raster work (fewer,
larger tiles).
"""

from __future__ import annotations

import torch

from . import _lib as L

TILE_SHAPES = ((16, 16), (16, 8), (32, 16), (8, 8))


def _need(step, b):
    step.forward_backward(b)
    st = step.ctx.status()
    return st["n_isect_needed"]


def autotune(step, shapes=TILE_SHAPES, orders=(0, 1, 2), iters=3, big=None):
    """Time each (tile shape, order) on `step` (a JointStep) over every batch
    of views (`iters` rounds; their loads differ) and leave the fastest in
    step.settings with a tight capacity.  A shape whose lists do not fit the
    library's capacity limit is skipped.  Returns the timings."""
    P = max(c.n_pixels for c in step.cams)
    cap_max = 2**30 - 65536  # the largest list capacity a context takes
    big = big or min(cap_max, 64 * P)
    results = []
    for tw, th in shapes:
        step.settings = L.default_settings(tile_w=tw, tile_h=th)
        step.set_capacity(big)
        need = max(_need(step, b) for b in range(len(step.batches)))
        if need >= big and big < cap_max:
            # at or past `big` the count may be a lower bound (an overflowed
            # stage): count again at the largest capacity
            step.set_capacity(cap_max)
            need = max(_need(step, b) for b in range(len(step.batches)))
        cap = int(need * 1.15) + 4096
        if need >= cap_max or cap > cap_max:
            results.append(dict(tile=(tw, th), order=None, need=int(need), ms=None,
                                skipped="lists exceed the capacity limit"))
            continue
        step.set_capacity(cap)
        for order in orders:
            step.settings = L.default_settings(tile_w=tw, tile_h=th, tile_order=order)
            nb = len(step.batches)
            for bb in range(nb):
                step.forward_backward(bb)
            torch.cuda.synchronize()
            if step.ctx.status()["flags"] & L.GS_FLAG_ISECT_OVERFLOW:
                results.append(dict(tile=(tw, th), order=order, need=int(need), ms=None,
                                    skipped="capacity overflow"))
                step.ctx.reset_status()
                continue
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(iters):
                for bb in range(nb):
                    step.forward_backward(bb)
            b.record()
            torch.cuda.synchronize()
            results.append(dict(tile=(tw, th), order=order, need=int(need),
                                ms=a.elapsed_time(b) / (iters * nb)))
    timed = [r for r in results if r["ms"] is not None]
    if not timed:
        raise RuntimeError("autotune: no tile shape fits the capacity limit")
    best = min(timed, key=lambda r: r["ms"])
    tw, th = best["tile"]
    step.settings = L.default_settings(tile_w=tw, tile_h=th, tile_order=best["order"])
    step.set_capacity(int(best["need"] * 1.15) + 4096)
    return results, best
