// Front-to-back compositing over the depth-sorted tile lists, its backward,
// and the photometric L1 term.
//
// One wave (64 lanes) owns one tile of TW x TH pixels, PPL = TW*TH/64 pixels per
// lane, laid out so that each of a lane's pixel slots stays in fixed tile
// quadrants; every list entry carries the quadrants its splat reaches, and a
// slot whose quadrants the splat misses is skipped by the whole wave.  The
// tile's list is consumed in batches of 64: each lane loads one splat record
// (a gather of 40 B) and stages it in the wave's own LDS region; the wave then
// walks the batch reading each splat's parameters with broadcast LDS loads
// (one address for all lanes), synchronising only with itself.  Loads run two
// batches ahead: while a batch composites, the next batch's records and the
// list entries of the one after it are in flight.  The backward walks the same
// lists back to front from each pixel's last contributor, recovering the
// transmittance by division, and sums each splat's nine 2D gradients over the
// whole wave (DPP and lane-swap steps) before one lane per component issues
// the global atomic.
#include <algorithm>

#include "gs_internal.h"

namespace gs {

namespace {

__device__ __forceinline__ int tile_view(const ViewTable& vt, int t) {
    int v = 0;
    while (v + 1 < vt.V && t >= vt.tile_off[v + 1]) v++;
    return v;
}

// Pixel of slot k of a lane inside a TW x TH tile, and the quadrants (TW/2 x
// TH/2 blocks, bit qx + 2 qy) that slot's 64 pixels lie in.  Slots are laid out
// so each one stays inside fixed quadrants: a splat whose entry mask misses
// them is skipped by the whole wave at once.
template <int TW, int TH>
struct TileMap {
    static constexpr int PPL = TW * TH / kWave;
    static_assert(PPL == 1 || PPL == 2 || PPL == 4 || PPL == 8, "tile shape");
    __device__ static __forceinline__ void pixel(int l, int k, int& x, int& y) {
        if constexpr (PPL == 1) {          // 8x8
            x = l % 8;
            y = l / 8;
        } else if constexpr (PPL == 2) {   // 16x8: two 8x8 halves
            x = 8 * k + l % 8;
            y = l / 8;
        } else if constexpr (PPL == 4) {   // 16x16: one 8x8 quadrant per slot
            x = (k % 2) * 8 + l % 8;
            y = (k / 2) * 8 + l / 8;
        } else {                            // 32x16: two 16x4 bands per 16x8 quadrant
            const int q = k / 2;
            x = (q % 2) * 16 + l % 16;
            y = (q / 2) * 8 + (k % 2) * 4 + l / 16;
        }
    }
    static constexpr uint32_t quads(int k) {
        return PPL == 1 ? 0xFu : PPL == 2 ? ((1u << k) | (1u << (k + 2)))
                        : PPL == 4 ? (1u << k) : (1u << (k / 2));
    }
};

// The tile of this workgroup.  Orders 0 and 1 number the workgroups like the
// tiles (1 through the heaviest-first permutation).  Order 2 is for the L2
// caches: workgroups are dealt round-robin over the chip's 8 XCDs, each with
// its own L2, so workgroups b, b + 8, b + 16, ... share one.  Tiles are walked
// block by block (4 x 4 tiles, row-major inside the block) and each block's
// 16 tiles go to 16 consecutive workgroups of one XCD: neighbouring tiles,
// which share most of their splats, read them through the same L2.  Returns
// false for a workgroup whose slot falls outside the view (edge blocks).
constexpr int kXcds = 8;
constexpr int kBlockTileCount = kBlockTiles * kBlockTiles;

__device__ __forceinline__ bool block_tile(const uint32_t* order, int mode, const ViewTable& vt, int& t) {
    const int b = blockIdx.x;
    if (mode != 2) {
        t = order ? (int)order[b] : b;
        return true;
    }
    const int x = b % kXcds, j = b / kXcds;
    const int s = ((j / kBlockTileCount) * kXcds + x) * kBlockTileCount + j % kBlockTileCount;
    const int gb = s / kBlockTileCount, w = s % kBlockTileCount;
    if (gb >= vt.block_off[vt.V]) return false;
    int v = 0;
    while (v + 1 < vt.V && gb >= vt.block_off[v + 1]) v++;
    const int lb = gb - vt.block_off[v];
    const int tx = (lb % vt.bx[v]) * kBlockTiles + w % kBlockTiles;
    const int ty = (lb / vt.bx[v]) * kBlockTiles + w / kBlockTiles;
    const int gy = (vt.tile_off[v + 1] - vt.tile_off[v]) / vt.gx[v];
    if (tx >= vt.gx[v] || ty >= gy) return false;
    t = vt.tile_off[v] + ty * vt.gx[v] + tx;
    return true;
}

// One splat record as a lane loads it: position, opacity, the base-2 conic,
// colour.
struct LaneSplat {
    float mx, my, o, a, b, c, cr, cg, cb;
};

__device__ __forceinline__ LaneSplat load_splat(const float4* __restrict__ rec, uint32_t pair) {
    const int64_t p = pair;
    const float4 ra = rec[3 * p], rb = rec[3 * p + 1];
    const float2 rc = *reinterpret_cast<const float2*>(rec + 3 * p + 2);
    const ConicE2 q = conic_e2(rb.x, rb.y, rb.z);
    return {ra.x, ra.y, ra.w, q.a, q.b, q.c, rb.w, rc.x, rc.y};
}

// A batch's splats staged in LDS, one entry per lane as three float4:
// (mx, my, o, -), (a, b, c, r), (g, b, -, -).  Entry i is then read by the
// whole wave from one address (a broadcast), not gathered by readlane.
struct BatchLds {
    float4 f[3][kWave];
};

__device__ __forceinline__ void stage_splat(BatchLds& sb, const LaneSplat& ls) {
    const int lane = threadIdx.x;
    sb.f[0][lane] = make_float4(ls.mx, ls.my, ls.o, 0.f);
    sb.f[1][lane] = make_float4(ls.a, ls.b, ls.c, ls.cr);
    sb.f[2][lane] = make_float4(ls.cg, ls.cb, 0.f, 0.f);
}

// One batch's list entries, loaded by every lane (index clamped into the
// list, which is not empty) and zeroed outside [s, e): the load stays
// unconditional, so the compiler's wait bookkeeping sees it on every path.
__device__ __forceinline__ uint32_t batch_ids(const int32_t* __restrict__ ids, int b, int s, int e) {
    const int j = b + (int)threadIdx.x;
    const uint32_t id = (uint32_t)ids[min(max(j, s), e - 1)];
    return (j >= s && j < e) ? id : 0u;
}

// Where a forward over lazy lists draws its tiles' entries from: the sorted
// block lists (pair; low and high 32 bits of the 64-bit quadrant mask), the
// block ranges, and the tile lists it writes what it reads into.
struct BlockSrc {
    const uint32_t* pair;
    const uint32_t* mlo;
    const uint32_t* mhi;
    const int32_t* branges;
    uint32_t* tids;
};

// Block-list entries a lazy forward keeps in flight (loads of 64 each), and
// the LDS ring its filtered entries queue in: at most 63 waiting plus one
// refill of kPull * 64.
constexpr int kPull = 8;
constexpr uint32_t kRing = 1024;
static_assert(kRing >= kWave - 1 + kPull * kWave, "ring");

template <int TW, int TH, bool EVALS, bool LAZY>
__global__ __launch_bounds__(64) void k_render_fwd(const float4* __restrict__ rec,
                                                   const int32_t* __restrict__ ids,
                                                   const int32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ order, ViewTable vt,
                                                   RasterParams rp, const float* __restrict__ bg,
                                                   float* __restrict__ out_rgb,
                                                   float* __restrict__ out_T,
                                                   int32_t* __restrict__ out_last,
                                                   int32_t* __restrict__ tile_contrib,
                                                   int32_t* __restrict__ tile_entries,
                                                   int32_t* __restrict__ tile_evals, int mode,
                                                   BlockSrc src) {
    using TM = TileMap<TW, TH>;
    constexpr int PPL = TM::PPL;
    int t;
    if (!block_tile(order, mode, vt, t)) return;
    const int v = tile_view(vt, t);
    const int lt = t - vt.tile_off[v];
    const int gx = vt.gx[v], W = vt.W[v], H = vt.H[v];
    const int tx = lt % gx, ty = lt / gx;
    const int lane = threadIdx.x;
    const float amin = rp.alpha_min, amax = rp.alpha_max, tmin = rp.t_min;
    float fx[PPL], fy[PPL], T[PPL], C0[PPL], C1[PPL], C2[PPL];
    int last[PPL];
    // per slot: entries met so far whose mask covers the slot's quadrants (the
    // same for the whole wave), and its value at each pixel's last contributor
    int qn[PPL], lastq[PPL];
    // the pixel's alpha gate: alpha_min while it composites, 2 (above every
    // alpha) once it has stopped or when it lies outside the view, so one
    // compare both gates and skips
    float gmin[PPL];
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        int x, y;
        TM::pixel(lane, k, x, y);
        const int px = tx * TW + x, py = ty * TH + y;
        fx[k] = px + 0.5f;
        fy[k] = py + 0.5f;
        gmin[k] = (px < W && py < H) ? amin : 2.f;
        T[k] = 1.f;
        C0[k] = C1[k] = C2[k] = 0.f;
        last[k] = 0;
        qn[k] = lastq[k] = 0;
    }
    const int s = ranges[2 * t];
    int e = ranges[2 * t + 1];
    int ncontrib = 0, nent = 0;
    __shared__ BatchLds sb;
    // Lazy lists: the tile's list is its block's list filtered by the tile's
    // four mask bits (the definition of the tile lists).  Block entries are
    // loaded kPull * 64 at a time, one load ahead; the entries that meet the
    // tile queue in an LDS ring in list order (qt queued, qh handed out, both
    // wave-uniform) and are handed out 64 at a time, each batch written to the
    // tile list as it is drawn, so the backward finds every entry up to the
    // last contributor.
    __shared__ uint32_t s_ring[LAZY ? kRing : 1];
    uint32_t lp[kPull], lm[kPull];
    int bpf = 0, bend = 0, msh = 0;
    uint32_t qh = 0, qt = 0;
    const uint32_t* mw = nullptr;
    auto pull = [&](int p0) {
        bpf = p0;
#pragma unroll
        for (int u = 0; u < kPull; u++) {
            const int j = min(p0 + u * kWave + lane, bend - 1);
            lp[u] = src.pair[j];
            lm[u] = mw[j];
        }
    };
    auto take = [&]() {
#pragma unroll
        for (int u = 0; u < kPull; u++) {
            const uint32_t w = lm[u];
            uint32_t m4 = ((w >> msh) & 3u) | (((w >> (msh + 8)) & 3u) << 2);
            m4 = bpf + u * kWave + lane < bend ? m4 : 0u;
            const uint64_t bal = __ballot(m4 != 0u);
            // set bits of bal below this lane
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            if (m4) s_ring[(qt + below) % kRing] = lp[u] | (m4 << kPairBits);
            qt += (uint32_t)__popcll(bal);
        }
        bpf += kPull * kWave;
    };
    // the next `want` entries (got < want only if the block list ran out
    // first, which the exact list lengths rule out)
    auto draw = [&](int want, int& got) -> uint32_t {
        while ((int)(qt - qh) < want && bpf < bend) {
            take();
            if (bpf < bend) pull(bpf);
        }
        got = min(want, (int)(qt - qh));
        wave_lds_sync();
        const uint32_t id = lane < got ? s_ring[(qh + (uint32_t)lane) % kRing] : 0u;
        qh += (uint32_t)got;
        return id;
    };
    // Two-deep pipeline: while a batch composites, the next batch's records
    // are in flight (their entries arrived during the batch before) and the
    // entries of the batch after that are requested.
    uint32_t id_cur = 0u, id_nxt = 0u;
    if constexpr (LAZY) {
        const int sx = tx % kBlockTiles, sy = ty % kBlockTiles;
        const int B = vt.block_off[v] + (ty / kBlockTiles) * vt.bx[v] + tx / kBlockTiles;
        // the block's entries are requested without waiting for the tile range
        bend = src.branges[2 * B + 1];
        bpf = src.branges[2 * B];
        mw = sy < 2 ? src.mlo : src.mhi;
        msh = 16 * (sy % 2) + 2 * sx;
        if (bpf < bend) pull(bpf);
        if (s < e) {
            const int want = min(kWave, e - s);
            int got;
            id_cur = draw(want, got);
            if (got < want) e = s + got;
            if (lane < got) src.tids[s + lane] = id_cur;
        }
    } else {
        id_cur = s < e ? batch_ids(ids, s, s, e) : 0u;
        id_nxt = s < e ? batch_ids(ids, s + kWave, s, e) : 0u;
    }
    LaneSplat ls_cur = {};
    if (lane < e - s) ls_cur = load_splat(rec, id_cur & kPairMask);
    for (int b = s; b < e; b += kWave) {
        bool alive = false;
#pragma unroll
        for (int k = 0; k < PPL; k++) alive |= gmin[k] <= 1.f;
        if (__ballot(alive) == 0) break;
        const uint32_t id = id_cur;
        const int nb = min(kWave, e - b);
        wave_lds_sync();  // the previous batch is read
        stage_splat(sb, ls_cur);
        ls_cur = {};
        if constexpr (LAZY) {
            const int want = min(kWave, e - (b + kWave));
            if (want > 0) {
                int got;
                id_cur = draw(want, got);
                if (got < want) e = b + kWave + got;
                if (lane < got) {
                    src.tids[b + kWave + lane] = id_cur;
                    ls_cur = load_splat(rec, id_cur & kPairMask);
                }
            }
        } else {
            if (lane < e - (b + kWave)) ls_cur = load_splat(rec, id_nxt & kPairMask);
            id_cur = id_nxt;
            id_nxt = batch_ids(ids, b + 2 * kWave, s, e);
        }
        wave_lds_sync();
        nent += nb;
        for (int i = 0; i < nb; i++) {
            const uint32_t m = (uint32_t)bcast((int)id, i) >> kPairBits;
            const float4 f0 = sb.f[0][i], f1 = sb.f[1][i], f2 = sb.f[2][i];
            const float mx = f0.x, my = f0.y, o = f0.z;
            const float qa = f1.x, qb = f1.y, qc = f1.z, cr = f1.w, cg = f2.x, cb = f2.y;
            const int pos = b + i - s + 1;
#pragma unroll
            for (int k = 0; k < PPL; k++) {
                if (!(m & TM::quads(k))) continue;  // wave-uniform
                if (EVALS) qn[k]++;
                if (__ballot(gmin[k] <= 1.f) == 0) continue;  // wave-uniform: the slot has stopped
                const float dx = mx - fx[k];
                const float dy = my - fy[k];
                // listed splats have positive-definite conics (binning drops the
                // rest), so sigma >= 0 needs no test of its own
                const float e2 = splat_e2(qa, qb, qc, dx, dy);
                // min(amax, o 2^e2) as one median (the product is >= 0)
                const float alpha = __builtin_amdgcn_fmed3f(o * __builtin_amdgcn_exp2f(e2), 0.f, amax);
                const float Tn = T[k] * (1.f - alpha);
                // the gate (never passed by a stopped pixel); then the splat
                // that would take T below t_min stops the pixel instead of
                // contributing.  Decided without branches, one branch for the
                // update.
                const bool gate = alpha >= gmin[k];
                const bool stop = gate && Tn < tmin;
                gmin[k] = stop ? 2.f : gmin[k];
                if (gate && !stop) {
                    const float w = alpha * T[k];
                    C0[k] = __builtin_fmaf(cr, w, C0[k]);
                    C1[k] = __builtin_fmaf(cg, w, C1[k]);
                    C2[k] = __builtin_fmaf(cb, w, C2[k]);
                    T[k] = Tn;
                    last[k] = pos;
                    if (EVALS) {
                        lastq[k] = qn[k];
                        ncontrib++;
                    }
                }
            }
        }
    }
    // workload statistics of the tile (the counting variant only): contributing
    // (pixel, splat) pairs, list entries read, and (pixel, entry) evaluations
    // up to each pixel's last contributor over the entries covering its quadrant
    if (EVALS) {
        int nev = 0;
#pragma unroll
        for (int k = 0; k < PPL; k++) nev += lastq[k];
        for (int sh = 32; sh > 0; sh >>= 1) {
            ncontrib += __shfl_xor(ncontrib, sh, kWave);
            nev += __shfl_xor(nev, sh, kWave);
        }
        if (lane == 0) {
            tile_contrib[t] = ncontrib;
            tile_entries[t] = nent;
            tile_evals[t] = nev;
        }
    }
    const float b0 = bg ? bg[0] : 0.f, b1 = bg ? bg[1] : 0.f, b2 = bg ? bg[2] : 0.f;
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        int x, y;
        TM::pixel(lane, k, x, y);
        const int px = tx * TW + x, py = ty * TH + y;
        if (px < W && py < H) {
            const int64_t pix = (int64_t)vt.pix_off[v] + (int64_t)py * W + px;
            out_rgb[3 * pix] = C0[k] + T[k] * b0;
            out_rgb[3 * pix + 1] = C1[k] + T[k] * b1;
            out_rgb[3 * pix + 2] = C2[k] + T[k] * b2;
            out_T[pix] = T[k];
            out_last[pix] = last[k];
        }
    }
}

template <int TW, int TH>
__global__ __launch_bounds__(64) void k_render_bwd(const float4* __restrict__ rec,
                                                   const int32_t* __restrict__ ids,
                                                   const int32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ order, ViewTable vt,
                                                   RasterParams rp, const float* __restrict__ bg,
                                                   const float* __restrict__ T_final,
                                                   const int32_t* __restrict__ last_in,
                                                   const float* __restrict__ v_rgb,
                                                   float* __restrict__ grad_geo,
                                                   float* __restrict__ grad_col, int mode) {
    using TM = TileMap<TW, TH>;
    constexpr int PPL = TM::PPL;
    int t;
    if (!block_tile(order, mode, vt, t)) return;
    const int v = tile_view(vt, t);
    const int lt = t - vt.tile_off[v];
    const int gx = vt.gx[v], W = vt.W[v], H = vt.H[v];
    const int tx = lt % gx, ty = lt / gx;
    const int lane = threadIdx.x;
    const float b0 = bg ? bg[0] : 0.f, b1 = bg ? bg[1] : 0.f, b2 = bg ? bg[2] : 0.f;
    float fx[PPL], fy[PPL], Tc[PPL], V0[PPL], V1[PPL], V2[PPL], VS[PPL];
    int L[PPL];
    int lmax = 0;
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        int x, y;
        TM::pixel(lane, k, x, y);
        const int px = tx * TW + x, py = ty * TH + y;
        fx[k] = px + 0.5f;
        fy[k] = py + 0.5f;
        L[k] = 0;
        Tc[k] = 1.f;
        V0[k] = V1[k] = V2[k] = 0.f;
        if (px < W && py < H) {
            const int64_t pix = (int64_t)vt.pix_off[v] + (int64_t)py * W + px;
            L[k] = last_in[pix];
            Tc[k] = T_final[pix];
            V0[k] = v_rgb[3 * pix];
            V1[k] = v_rgb[3 * pix + 1];
            V2[k] = v_rgb[3 * pix + 2];
        }
        // VS = dL/dC . S, S = sum over later splats of colour alpha T, plus
        // T_final bg (the background term seeds it)
        VS[k] = Tc[k] * (V0[k] * b0 + V1[k] * b1 + V2[k] * b2);
        lmax = max(lmax, L[k]);
    }
    // per slot, the largest `last` of its pixels: past it the whole wave skips
    // the slot (all its pixels are behind their last contributor)
    // (wave-uniform: read from the first lane, so the loops below stay scalar)
    int Lk[PPL];
#pragma unroll
    for (int k = 0; k < PPL; k++) Lk[k] = __builtin_amdgcn_readfirstlane(wave_max_i(L[k]));
    lmax = __builtin_amdgcn_readfirstlane(wave_max_i(lmax));
    const int s = ranges[2 * t], e = ranges[2 * t + 1];
    lmax = min(lmax, e - s);  // a pixel's last contributor lies inside its tile's list
    if (lmax <= 0) return;
    const float amin = rp.alpha_min, amax = rp.alpha_max;
    const int top = s + lmax;  // entries [s, top) can matter
    // The gradient component this lane adds after each splat's wave sum E
    // (lanes 0-7 hold value sum8_index(lane), lane 16 the blue sum; the rest
    // add none): 0 mean.x, 1 mean.y, 2 A, 3 B, 4 C, 5 opacity, 6 r, 7 g, 8 b.
    // It is E (kS o + kE) + o ln2 ((ua a + ub b) QX + (vb b + vc c) QY) with
    // QX, QY the first two moments, so every lane runs the same instructions.
    const int comp = lane < 8 ? sum8_index(lane) : lane == 16 ? 8 : -1;
    const float kS = (comp == 2 || comp == 4) ? -0.5f : comp == 3 ? -1.f : 0.f;
    const float kE = comp >= 5 ? 1.f : 0.f;
    const float ua = comp == 0 ? 2.f : 0.f, ub = comp == 1 ? 1.f : 0.f;
    const float vb = comp == 0 ? 1.f : 0.f, vc = comp == 1 ? 2.f : 0.f;
    __shared__ BatchLds sb;
    int b = s + ((lmax - 1) / kWave) * kWave;
    // the same two-deep pipeline as the forward, walking down: the batches
    // after the first (partial) one are full
    uint32_t id_cur = batch_ids(ids, b, s, top);
    uint32_t id_nxt = batch_ids(ids, b - kWave, s, top);
    LaneSplat ls_cur = {};
    if (lane < top - b) ls_cur = load_splat(rec, id_cur & kPairMask);
    // per-lane sums over the lane's pixels for the current splat: colour
    // weights, q = dL/dalpha e^-sigma (zero where alpha is clamped), and the
    // moments q dx, q dy, q dx^2, q dx dy, q dy^2; the exponent's gradient is
    // -o q, so the mean and conic gradients follow from these after the wave
    // sum.  They are zero at every splat's start: a splat nobody contributes
    // to leaves them untouched, one that is summed clears them afterwards.
    float g_r = 0.f, g_g = 0.f, g_b = 0.f, g_o = 0.f;
    float m_x = 0.f, m_y = 0.f, m_xx = 0.f, m_xy = 0.f, m_yy = 0.f;
    bool any = false;
    for (; b >= s; b -= kWave) {
        const uint32_t id = id_cur;
        const int nb = min(kWave, top - b);
        wave_lds_sync();  // the previous batch is read
        stage_splat(sb, ls_cur);
        ls_cur = {};
        if (b - kWave >= s) ls_cur = load_splat(rec, id_nxt & kPairMask);
        id_cur = id_nxt;
        id_nxt = batch_ids(ids, b - 2 * kWave, s, top);
        wave_lds_sync();
        for (int i = nb - 1; i >= 0; i--) {
            const uint32_t idb = (uint32_t)bcast((int)id, i);
            const uint32_t m = idb >> kPairBits;
            const float4 f0 = sb.f[0][i], f1 = sb.f[1][i], f2 = sb.f[2][i];
            const float mx = f0.x, my = f0.y, o = f0.z;
            const float qa = f1.x, qb = f1.y, qc = f1.z, cr = f1.w, cg = f2.x, cb = f2.y;
            const int pos = b + i - s;
#pragma unroll
            for (int k = 0; k < PPL; k++) {
                if (!(m & TM::quads(k)) || pos >= Lk[k]) continue;  // wave-uniform
                const float dx = mx - fx[k];
                const float dy = my - fy[k];
                const float e2 = splat_e2(qa, qb, qc, dx, dy);
                const float ex = __builtin_amdgcn_exp2f(e2);
                const float araw = o * ex;
                const float alpha = __builtin_amdgcn_fmed3f(araw, 0.f, amax);
                // same decisions as the forward: before the pixel's last
                // contributor and above the alpha gate
                const bool live = pos < L[k] && alpha >= amin;
                if (live) {
                    any = true;
                    const float iom = __builtin_amdgcn_rcpf(1.f - alpha);
                    const float Tb = Tc[k] * iom;  // transmittance in front of this splat
                    const float w = alpha * Tb;
                    g_r = __builtin_fmaf(w, V0[k], g_r);
                    g_g = __builtin_fmaf(w, V1[k], g_g);
                    g_b = __builtin_fmaf(w, V2[k], g_b);
                    const float Vc = __builtin_fmaf(V2[k], cb, __builtin_fmaf(V1[k], cg, V0[k] * cr));
                    // dL/dalpha = T (dL/dC . c) - (dL/dC . S) / (1 - alpha)
                    const float va = __builtin_fmaf(Tb, Vc, -(iom * VS[k]));
                    VS[k] = __builtin_fmaf(w, Vc, VS[k]);
                    Tc[k] = Tb;
                    const float q = araw < amax ? va * ex : 0.f;  // clamped alpha passes no gradient
                    g_o += q;
                    const float qx = q * dx, qy = q * dy;
                    m_x += qx;
                    m_y += qy;
                    m_xx = __builtin_fmaf(qx, dx, m_xx);
                    m_xy = __builtin_fmaf(qx, dy, m_xy);
                    m_yy = __builtin_fmaf(qy, dy, m_yy);
                }
            }
            if (__ballot(any) == 0) continue;
            // wave totals of the nine sums in one transposed butterfly
            const float E = wave_sum9_t(m_x, m_y, m_xx, m_xy, m_yy, g_o, g_r, g_g, g_b);
            const float QX = bcast(E, 0), QY = bcast(E, 4);  // lanes holding m_x, m_y
            if (comp >= 0) {
                // With vs = -o q the sums of vs dx, vs dy, ... are -o times the
                // moments; A = -2 a / log2(e), B = -b / log2(e), C = -2 c / log2(e).
                const float mean = __builtin_fmaf(__builtin_fmaf(ua, qa, ub * qb), QX,
                                                  __builtin_fmaf(vb, qb, vc * qc) * QY);
                const float val = __builtin_fmaf(o * kLn2, mean, E * __builtin_fmaf(kS, o, kE));
                const int64_t p = idb & kPairMask;
                atomicAdd(comp < kGradGeo ? grad_geo + kGradGeo * p + comp
                                          : grad_col + kGradCol * p + (comp - kGradGeo), val);
            }
            g_r = g_g = g_b = g_o = 0.f;
            m_x = m_y = m_xx = m_xy = m_yy = 0.f;
            any = false;
        }
    }
}

constexpr int kL1Blocks = 1024;

__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ rgb,
                                            const float* __restrict__ target,
                                            float* __restrict__ v_rgb, ViewTable vt,
                                            double* __restrict__ loss_acc) {
    __shared__ float s_w[4];
    const int64_t P = vt.pix_off[vt.V];
    float part = 0.f;
    for (int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x; pix < P;
         pix += (int64_t)gridDim.x * 256) {
        int v = 0;
        while (v + 1 < vt.V && pix >= vt.pix_off[v + 1]) v++;
        const float wgt = 1.f / (3.f * (float)(vt.pix_off[v + 1] - vt.pix_off[v]) * (float)vt.V);
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            const float d = rgb[3 * pix + ch] - target[3 * pix + ch];
            v_rgb[3 * pix + ch] = d > 0.f ? wgt : (d < 0.f ? -wgt : 0.f);
            part += fabsf(d) * wgt;
        }
    }
    // one double atomic per block
    const float s = wave_sum(part);
    if (__lane_id() == 0) s_w[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double tot = (double)s_w[0] + s_w[1] + s_w[2] + s_w[3];
        if (tot != 0.0) atomicAdd(loss_acc, tot);
    }
}

// workgroups of a raster launch: one per tile, or for the XCD order one per
// slot of every 4 x 4 block, rounded to whole rounds over the XCDs
unsigned raster_grid(const Ctx* c, const ViewTable& vt, int mode) {
    if (mode != 2) return (unsigned)c->n_tiles;
    const int64_t slots = (int64_t)vt.block_off[vt.V] * kBlockTileCount;
    const int64_t round = (int64_t)kXcds * kBlockTileCount;
    return (unsigned)((slots + round - 1) / round * round);
}

template <int TW, int TH, bool EVALS, bool LAZY>
void fwd_launch(Ctx* c, const ViewTable& vt, const RasterParams& rp, const float* bg, float* rgb,
                float* T_final, int32_t* last, const uint32_t* order, int mode, const BlockSrc& src,
                hipStream_t st) {
    hipLaunchKernelGGL((k_render_fwd<TW, TH, EVALS, LAZY>), dim3(raster_grid(c, vt, mode)), dim3(64), 0,
                       st, reinterpret_cast<const float4*>(c->rec), reinterpret_cast<const int32_t*>(c->tids),
                       c->tranges, order, vt, rp, bg, rgb, T_final, last, c->tile_contrib,
                       c->tile_entries, c->tile_evals, mode, src);
}

template <int TW, int TH>
hipError_t fwd_impl(Ctx* c, const ViewTable& vt, const RasterParams& rp, const float* bg,
                    float* rgb, float* T_final, int32_t* last, const uint32_t* order, int mode,
                    hipStream_t st) {
    BlockSrc src = {};
    if (c->lists_lazy) {
        const int sd = c->block_side;
        src = {c->iv[sd], c->im[sd], c->im[sd] + c->cap.max_isect, c->ranges, c->tids};
        if (rp.eval_stats) fwd_launch<TW, TH, true, true>(c, vt, rp, bg, rgb, T_final, last, order, mode, src, st);
        else fwd_launch<TW, TH, false, true>(c, vt, rp, bg, rgb, T_final, last, order, mode, src, st);
    } else {
        if (rp.eval_stats) fwd_launch<TW, TH, true, false>(c, vt, rp, bg, rgb, T_final, last, order, mode, src, st);
        else fwd_launch<TW, TH, false, false>(c, vt, rp, bg, rgb, T_final, last, order, mode, src, st);
    }
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess && c->lists_lazy) c->lists_filled = true;
    return e;
}

template <int TW, int TH>
hipError_t bwd_impl(Ctx* c, const ViewTable& vt, const RasterParams& rp, const float* bg,
                    const float* T_final, const int32_t* last, const float* v_rgb,
                    const uint32_t* order, int mode, hipStream_t st) {
    hipLaunchKernelGGL((k_render_bwd<TW, TH>), dim3(raster_grid(c, vt, mode)), dim3(64), 0, st,
                       reinterpret_cast<const float4*>(c->rec), reinterpret_cast<const int32_t*>(c->tids), c->tranges, order,
                       vt, rp, bg, T_final, last, v_rgb, c->grad2d,
                       c->grad2d + kGradGeo * c->cap.max_pairs, mode);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_render_fwd(Ctx* c, const ViewTable& vt, const RasterParams& rp, const float* bg,
                             float* rgb, float* T_final, int32_t* last, hipStream_t st) {
    if (c->n_tiles <= 0) return hipSuccess;
    const uint32_t* order = c->ordered ? c->tile_order : nullptr;
    const int mode = rp.tile_order == 2 ? 2 : (order ? 1 : 0);
    const int TW = rp.tile_w, TH = rp.tile_h;
    if (TW == 16 && TH == 16) return fwd_impl<16, 16>(c, vt, rp, bg, rgb, T_final, last, order, mode, st);
    if (TW == 16 && TH == 8) return fwd_impl<16, 8>(c, vt, rp, bg, rgb, T_final, last, order, mode, st);
    if (TW == 8 && TH == 8) return fwd_impl<8, 8>(c, vt, rp, bg, rgb, T_final, last, order, mode, st);
    if (TW == 32 && TH == 16) return fwd_impl<32, 16>(c, vt, rp, bg, rgb, T_final, last, order, mode, st);
    return hipErrorInvalidValue;
}

hipError_t launch_render_bwd(Ctx* c, const ViewTable& vt, const RasterParams& rp, const float* bg,
                             const float* T_final, const int32_t* last, const float* v_rgb,
                             hipStream_t st) {
    if (c->n_tiles <= 0) return hipSuccess;
    // lazy lists with no forward since the bin step: write them in full first
    if (c->lists_lazy && !c->lists_filled) {
        const hipError_t e = launch_expand_lists(c, st);
        if (e != hipSuccess) return e;
    }
    const uint32_t* order = c->ordered ? c->tile_order : nullptr;
    const int mode = rp.tile_order == 2 ? 2 : (order ? 1 : 0);
    const int TW = rp.tile_w, TH = rp.tile_h;
    if (TW == 16 && TH == 16) return bwd_impl<16, 16>(c, vt, rp, bg, T_final, last, v_rgb, order, mode, st);
    if (TW == 16 && TH == 8) return bwd_impl<16, 8>(c, vt, rp, bg, T_final, last, v_rgb, order, mode, st);
    if (TW == 8 && TH == 8) return bwd_impl<8, 8>(c, vt, rp, bg, T_final, last, v_rgb, order, mode, st);
    if (TW == 32 && TH == 16) return bwd_impl<32, 16>(c, vt, rp, bg, T_final, last, v_rgb, order, mode, st);
    return hipErrorInvalidValue;
}

hipError_t launch_l1(Ctx* c, const ViewTable& vt, const float* rgb, const float* target,
                     float* v_rgb, float* loss, hipStream_t st) {
    const int64_t P = vt.pix_off[vt.V];
    if (P > 0) {
        const unsigned nb = (unsigned)std::min<int64_t>((P + 255) / 256, kL1Blocks);
        hipLaunchKernelGGL(k_l1, dim3(nb), dim3(256), 0, st, rgb, target, v_rgb, vt, c->loss_acc);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_flush_acc(c->loss_acc, loss, 1, st);
}

}  // namespace gs
