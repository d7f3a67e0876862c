// Tile binning and key sort.
//
//  1. count:   per pair, the tiles its alpha >= alpha_min ellipse meets (an exact
//              ellipse/rectangle test inside the splat's bounding box), and its
//              depth key (float32 depth bits; positive floats order like their
//              bits).  Culled pairs get key 0xFFFFFFFF and no tiles.
//  2. sort the pairs by depth key (stable LSD radix from pair order, so equal
//     depths stay in pair order): this is the (depth, pair) order.
//  3. scan the tile counts in that order and emit one (tile, pair) entry per
//     intersection; entries of one pair are contiguous, pairs in depth order.
//  4. stable radix sort of the entries on the tile id only: inside every tile
//     the depth order of step 2 survives, so each tile list ends up in
//     ascending (depth, pair) order without sorting on depth again.
//  5. tile ranges from the boundaries of the sorted tile ids.
#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_count(const float4* __restrict__ rec, int N,
                                                  ViewTable vt, RasterParams rp,
                                                  uint32_t* __restrict__ cnt,
                                                  uint32_t* __restrict__ key,
                                                  uint32_t* __restrict__ val,
                                                  uint32_t* __restrict__ diag) {
    const int64_t pair = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t npairs = (int64_t)vt.V * N;
    bool vis = false;
    if (pair < npairs) {
        const int v = (int)(pair / N);
        const float4 a = rec[3 * pair];
        uint32_t c = 0;
        const float4 b = rec[3 * pair + 1];
        const bool fin = isfinite(a.x) && isfinite(a.y) && isfinite(a.z) && isfinite(a.w) &&
                         isfinite(b.x) && isfinite(b.y) && isfinite(b.z) && b.x > 0.f && b.z > 0.f &&
                         b.x * b.z > b.y * b.y;
        if (fin && a.w > rp.alpha_min && a.w <= 1.f) {
            c = for_each_tile(a, b, vt.W[v], vt.H[v], vt.gx[v], rp.tile_w, rp.tile_h,
                              rp.alpha_min, [](int) {});
        }
        vis = c > 0;
        cnt[pair] = c;
        key[pair] = vis ? __float_as_uint(a.z) : 0xFFFFFFFFu;
        val[pair] = (uint32_t)pair;
    }
    const uint64_t m = __ballot(vis);
    if (__lane_id() == 0 && m) atomicAdd(&diag[kDiagVisible], (uint32_t)__popcll(m));
}

__global__ __launch_bounds__(kBlock) void k_gather_cnt(const uint32_t* __restrict__ order,
                                                       const uint32_t* __restrict__ cnt,
                                                       uint32_t* __restrict__ out, int64_t n) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r < n) out[r] = cnt[order[r]];
}

__global__ void k_isect_total(const uint32_t* __restrict__ total, int64_t cap,
                              uint32_t* __restrict__ used, uint32_t* __restrict__ diag) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint32_t t = *total;
        const bool over = (int64_t)t > cap;
        *used = over ? 0u : t;
        diag[kDiagIsectTotal] = t;
        diag[kDiagIsectUsed] = over ? 0u : t;
        if (over) atomicOr(&diag[kDiagFlags], (uint32_t)GS_FLAG_ISECT_OVERFLOW);
    }
}

__global__ __launch_bounds__(kBlock) void k_emit(const float4* __restrict__ rec, int N, ViewTable vt,
                                                 RasterParams rp, const uint32_t* __restrict__ order,
                                                 const uint32_t* __restrict__ off,
                                                 const uint32_t* __restrict__ cnt, int64_t n,
                                                 const uint32_t* __restrict__ used,
                                                 uint32_t* __restrict__ okey,
                                                 uint32_t* __restrict__ oval) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= n) return;
    if (*used == 0) return;  // nothing fits (overflow) or nothing visible
    const uint32_t pair = order[r];
    const float4 a = rec[3 * (int64_t)pair];
    if (!(a.w > rp.alpha_min)) return;
    const float4 b = rec[3 * (int64_t)pair + 1];
    const int v = (int)(pair / (uint32_t)N);
    const uint32_t toff = (uint32_t)vt.tile_off[v];
    uint32_t o = off[r];
    const uint32_t o_end = o + cnt[pair];  // never write outside this pair's slots
    for_each_tile(a, b, vt.W[v], vt.H[v], vt.gx[v], rp.tile_w, rp.tile_h, rp.alpha_min,
                  [&](int t) {
                      if (o < o_end) {
                          okey[o] = toff + (uint32_t)t;
                          oval[o] = pair;
                      }
                      o++;
                  });
}

__global__ __launch_bounds__(kBlock) void k_ranges(const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ used,
                                                   int32_t* __restrict__ ranges) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t n = *used;
    if (i >= n) return;
    const uint32_t k = keys[i];
    if (i == 0 || keys[i - 1] != k) ranges[2 * (int64_t)k] = (int32_t)i;
    if (i == n - 1 || keys[i + 1] != k) ranges[2 * (int64_t)k + 1] = (int32_t)i + 1;
}

}  // namespace

hipError_t launch_bin(Ctx* c, const ViewTable& vt, int N, const RasterParams& rp,
                      const float* records, hipStream_t st) {
    const int64_t npairs = (int64_t)vt.V * N;
    const float4* rec = reinterpret_cast<const float4*>(records ? records : c->rec);
    const int64_t T = vt.tile_off[vt.V];
    hipError_t e = hipSuccess;
    // tile ranges start empty
    if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(c->ranges), 0u, 2 * T, st)) != hipSuccess)
        return e;
    if ((e = launch_fill_u32(c->diag + kDiagVisible, 0u, 1, st)) != hipSuccess) return e;
    if (npairs > 0) {
        const unsigned gp = (unsigned)((npairs + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_count, dim3(gp), dim3(kBlock), 0, st, rec, N, vt, rp, c->cnt, c->pk[0],
                           c->pv[0], c->diag);
        const int side = radix_sort_pairs(c->pk[0], c->pv[0], c->pk[1], c->pv[1], npairs, nullptr,
                                          0, 32, c->hist, c->scan_scratch, st, &e);
        if (e != hipSuccess) return e;
        const uint32_t* order = c->pv[side];
        hipLaunchKernelGGL(k_gather_cnt, dim3(gp), dim3(kBlock), 0, st, order, c->cnt, c->off,
                           npairs);
        uint32_t* total = c->scalars + 0;
        uint32_t* used = c->scalars + 1;
        if ((e = exclusive_scan_u32(c->off, npairs, total, c->scan_scratch, st)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_isect_total, dim3(1), dim3(64), 0, st, total, c->cap.max_isect, used,
                           c->diag);
        hipLaunchKernelGGL(k_emit, dim3(gp), dim3(kBlock), 0, st, rec, N, vt, rp, order, c->off,
                           c->cnt, npairs, used, c->ik[0], c->iv[0]);
        int tbits = 1;
        while (((int64_t)1 << tbits) < T) tbits++;
        const int side2 = radix_sort_pairs(c->ik[0], c->iv[0], c->ik[1], c->iv[1],
                                           c->cap.max_isect, used, 0, tbits, c->hist,
                                           c->scan_scratch, st, &e);
        if (e != hipSuccess) return e;
        const unsigned gi = (unsigned)((c->cap.max_isect + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_ranges, dim3(gi), dim3(kBlock), 0, st, c->ik[side2], used, c->ranges);
        c->ids = reinterpret_cast<const int32_t*>(c->iv[side2]);
    } else {
        c->ids = reinterpret_cast<const int32_t*>(c->iv[0]);
    }
    c->n_tiles = T;
    c->bin_V = vt.V;
    c->bin_N = N;
    c->bin_tw = rp.tile_w;
    c->bin_th = rp.tile_h;
    return hipGetLastError();
}

}  // namespace gs
