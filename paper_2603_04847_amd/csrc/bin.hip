// Tile binning and key sort, kept per block of 4 x 4 tiles.
//
//  1. count:   per pair, an upper bound of the blocks its alpha >= alpha_min
//              ellipse meets (one block row at a time, from the ellipse's
//              x-span over the row's whole band), and its depth key (float32
//              depth bits; positive floats order like their bits).  Culled
//              pairs get key 0xFFFFFFFF and no blocks.
//  2. sort the pairs by depth key (stable LSD radix from pair order, so equal
//     depths stay in pair order): this is the (depth, pair) order.  The pair
//     index and its block count travel with the key, packed in one word.
//  3. scan the block counts in that order and emit one (block, pair, 64-bit
//     quadrant mask) entry per block met, from the exact per-quadrant-row
//     spans; entries of one pair are contiguous, pairs in depth order, and the
//     slots the bound over-counts (at the end of each wave's range) get a
//     sentinel block id that sorts after every block.
//  4. stable radix sort of the entries on the block id only: inside every block
//     the depth order of step 2 survives, so each block list ends up in
//     ascending (depth, pair) order without sorting on depth again.
//  5. block ranges from the boundaries of the sorted block ids.
//  6. expand to tile lists, the definition: a tile's list is its block's list
//     restricted to the entries whose mask meets one of the tile's four
//     quadrants.  Per 256-entry chunk of the sorted block array, the entries
//     touching each of a block's 16 tiles are counted; scans of those counts
//     and of the tile totals place every entry, written as (pair | 4-bit mask
//     << 28) in block-list order.  Sorting (block, pair) entries instead of (tile, pair)
//     ones moves about a quarter of the data through the radix passes.
//     Lazy lists stop before the entries of step 6 (the ranges are kept): the
//     forward filters each tile's entries out of its block's list itself and
//     writes the part it reads.
#include <algorithm>

#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;

// Valid, finite record with a positive-definite conic and a splat that can
// pass the alpha gate.
__device__ __forceinline__ bool record_ok(const float4& a, const float4& b, float alpha_min) {
    return isfinite(a.x) && isfinite(a.y) && isfinite(a.z) && isfinite(a.w) && isfinite(b.x) &&
           isfinite(b.y) && isfinite(b.z) && b.x > 0.f && b.z > 0.f && b.x * b.z > b.y * b.y &&
           a.w > alpha_min && a.w <= 1.f;
}

// Work of one wave, flattened: its 64 splats' block rows ("units") are laid end
// to end and handed to the lanes in turn, so a wave costs its total number of
// block rows rather than 64 times its tallest splat.
struct WaveUnits {
    SplatSpan sp[kWave];
    int v[kWave];
    uint32_t upre[kWave + 1];  // exclusive prefix of units per splat
};

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x, uint32_t& total) {
    const int lane = __lane_id();
    uint32_t inc = x;
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t t = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += t;
    }
    total = __shfl(inc, kWave - 1, kWave);
    return inc - x;
}

// largest q in [0, n) with pre[q] <= j (the entry of the segment holding j)
__device__ __forceinline__ int seg_search(const uint32_t* pre, int n, uint32_t j) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= j) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void wave_units_load(WaveUnits& wu, int lane, bool ok, const float4& a,
                                                const float4& b, int v, const ViewTable& vt,
                                                const RasterParams& rp, uint32_t& total) {
    uint32_t units = 0;
    if (ok) {
        const SplatSpan sp = splat_span(a, b, vt.H[v], quad_grid(rp.tile_w, rp.tile_h), rp.alpha_min);
        wu.sp[lane] = sp;
        if (sp.r0 <= sp.r1) units = (uint32_t)(sp.r1 / kBlockQuads - sp.r0 / kBlockQuads + 1);
    }
    wu.v[lane] = v;
    const uint32_t ex = wave_excl_scan(units, total);
    wu.upre[lane] = ex;
    if (lane == 0) wu.upre[kWave] = total;
}

__global__ __launch_bounds__(kBlock) void k_count(const float4* __restrict__ rec, int N,
                                                  ViewTable vt, RasterParams rp,
                                                  uint32_t* __restrict__ cnt,
                                                  uint32_t* __restrict__ key,
                                                  uint32_t* __restrict__ val,
                                                  int32_t* __restrict__ branges, int64_t nbr,
                                                  int pbits) {
    // the block ranges start empty (the sorted keys fill the blocks that have entries)
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nbr; k += (int64_t)gridDim.x * kBlock)
        branges[k] = 0;
    const int64_t pair = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (pair >= (int64_t)vt.V * N) return;
    const int v = (int)(pair / N);
    const float4 a = rec[3 * pair], b = rec[3 * pair + 1];
    // an upper bound per block row (the emit pass fills what it over-counts),
    // each lane over its own splat's rows
    uint32_t c = 0;
    if (record_ok(a, b, rp.alpha_min)) {
        const SplatSpan sp = splat_span(a, b, vt.H[v], quad_grid(rp.tile_w, rp.tile_h), rp.alpha_min);
        if (sp.r0 <= sp.r1)
            for (int br = sp.r0 / kBlockQuads; br <= sp.r1 / kBlockQuads; br++)
                c += (uint32_t)unit_band_count(sp, br, vt.W[v], vt.H[v], quad_grid(rp.tile_w, rp.tile_h));
    }
    cnt[pair] = c;
    key[pair] = c > 0 ? __float_as_uint(a.z) : 0xFFFFFFFFu;
    // the pair index in the low pbits, the count above it (all ones when it
    // does not fit: the full count is then read back from cnt)
    val[pair] = (uint32_t)pair | (min(c, ~0u >> pbits) << pbits);
}

// Masks of four block columns of a unit from q0 = 8 c on: row i's quadrant
// columns inside [q0, q0 + 32) as one run of bits counted from q0, so that
// byte k of run i is row i of the mask of block column c + k.
__device__ __forceinline__ void unit_runs4(const BlockUnit& u, int c, uint32_t (&S)[kBlockQuads]) {
    const int base = kBlockQuads * c;
#pragma unroll
    for (int i = 0; i < kBlockQuads; i++) {
        const int a = max(u.c0[i] - base, 0), b = min(u.c1[i] - base, 31);
        S[i] = (u.c0[i] <= u.c1[i] && a <= b) ? ((2u << (b - a)) - 1u) << a : 0u;
    }
}

// The mask of block column c + k from the runs: byte k of runs 0-7 gathered with
// byte permutes (v_perm_b32 selector values 0-3 take bytes of its second
// operand, 4-7 of its first, 12 gives zero); equal to block_unit_mask.
__device__ __forceinline__ uint64_t runs_mask4(const uint32_t (&S)[kBlockQuads], int k) {
    const uint32_t sa = 0x0C0C0400u + 0x0101u * (uint32_t)k;      // bytes 0, 1
    const uint32_t sb = 0x04000C0Cu + 0x01010000u * (uint32_t)k;  // bytes 2, 3
    const uint32_t lo = __builtin_amdgcn_perm(S[1], S[0], sa) | __builtin_amdgcn_perm(S[3], S[2], sb);
    const uint32_t hi = __builtin_amdgcn_perm(S[5], S[4], sa) | __builtin_amdgcn_perm(S[7], S[6], sb);
    return ((uint64_t)hi << 32) | lo;
}

// One (block key; pair, mask) entry per block met, pairs in depth order: rank
// r's entries fill [off[r], off[r + 1]) (the last rank ends at the total).  The
// 64 ranks of a wave own one contiguous output range; in each round every lane
// takes one unit (block row) and writes its entries at the unit's place in the
// wave's range.  Counts come from adjacent offsets, so the only access by pair
// index is the record.  Also reports the number of visible pairs (their depth
// keys sort before the culled ones' 0xFFFFFFFF).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7))) void k_emit(const float4* __restrict__ rec, int N, ViewTable vt,
                                                 RasterParams rp, const uint32_t* __restrict__ order,
                                                 uint32_t pmask, const uint32_t* __restrict__ off,
                                                 const uint32_t* __restrict__ keys, int64_t n,
                                                 const uint32_t* __restrict__ used,
                                                 uint32_t* __restrict__ okey,
                                                 uint32_t* __restrict__ opair,
                                                 uint32_t* __restrict__ omlo,
                                                 uint32_t* __restrict__ omhi,
                                                 uint32_t* __restrict__ diag) {
    __shared__ WaveUnits s_wu[kWaves];
    __shared__ uint32_t s_pair[kWaves][kWave];
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    WaveUnits& wu = s_wu[w];
    const QuadGrid qg = quad_grid(rp.tile_w, rp.tile_h);
    const uint32_t lim = *used;    // nothing is written after an overflow
    const bool any = lim != 0u;
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
    int v = 0;
    bool ok = false;
    uint32_t pair = 0, c = 0, o0 = 0xFFFFFFFFu;
    if (r < n) {
        const bool vis = keys[r] != 0xFFFFFFFFu;
        const bool next_vis = r + 1 < n && keys[r + 1] != 0xFFFFFFFFu;
        if (r == 0 && !vis) diag[kDiagVisible] = 0;
        if (vis && !next_vis) diag[kDiagVisible] = (uint32_t)(r + 1);
    }
    if (r < n && any) {
        pair = order[r] & pmask;
        o0 = off[r];
        const uint32_t o1 = r + 1 < n ? off[r + 1] : lim;
        c = o1 > o0 ? o1 - o0 : 0u;
        if (c > 0) {
            a = rec[3 * (int64_t)pair];
            b = rec[3 * (int64_t)pair + 1];
            v = (int)(pair / (uint32_t)N);
            ok = record_ok(a, b, rp.alpha_min);
        }
    }
    // the wave's output range: [first offset, first offset + sum of counts)
    uint32_t base = o0;
    for (int sh = 32; sh > 0; sh >>= 1) base = min(base, (uint32_t)__shfl_xor((int)base, sh, kWave));
    uint32_t wave_total = c;
    for (int sh = 32; sh > 0; sh >>= 1) wave_total += (uint32_t)__shfl_xor((int)wave_total, sh, kWave);
    uint32_t U;
    wave_units_load(wu, lane, ok, a, b, v, vt, rp, U);
    s_pair[w][lane] = pair;
    __syncthreads();
    uint32_t done = 0;  // entries of the wave written so far
    bool bound_broken = false;
    for (uint32_t ub = 0; ub < U; ub += kWave) {
        const uint32_t j = ub + lane;
        BlockUnit u;
        u.bc0 = 1;
        u.bc1 = 0;
        int q = 0, br = 0;
        uint32_t ne = 0;
        if (j < U) {
            q = seg_search(wu.upre, kWave, j);
            const int vq = wu.v[q];
            br = wu.sp[q].r0 / kBlockQuads + (int)(j - wu.upre[q]);
            u = block_unit(wu.sp[q], br, vt.W[vq], vt.H[vq], qg);
            ne = (uint32_t)block_unit_count(u);
        }
        uint32_t rt;
        uint32_t o = done + wave_excl_scan(ne, rt);
        if (ne) {
            const int vq = wu.v[q];
            const uint32_t brow = (uint32_t)vt.block_off[vq] + (uint32_t)(br * vt.bx[vq]);
            const uint32_t pq = s_pair[w][q];
            auto put = [&](int bc, uint64_t m) {
                if (m == 0) return;
                if (o < wave_total && base + o < lim) {  // never outside the wave's slots
                    okey[base + o] = brow + (uint32_t)bc;
                    opair[base + o] = pq;
                    omlo[base + o] = (uint32_t)m;
                    omhi[base + o] = (uint32_t)(m >> 32);
                } else {
                    bound_broken = true;
                }
                o++;
            };
            // four block columns at a time: per-row bit runs, then four byte
            // permutes per block instead of eight clamped rows
            for (int c = u.bc0; c <= u.bc1; c += 4) {
                uint32_t S[kBlockQuads];
                unit_runs4(u, c, S);
                const int kn = min(3, u.bc1 - c);
                for (int k = 0; k <= kn; k++) put(c + k, runs_mask4(S, k));
            }
        }
        done += rt;
    }
    // slots the count's bound left over get a sentinel block id past every
    // block and no mask, so no list ever reads them
    for (uint32_t o = done + lane; o < wave_total && base + o < lim; o += kWave) {
        okey[base + o] = (uint32_t)vt.block_off[vt.V];
        opair[base + o] = s_pair[w][0];
        omlo[base + o] = 0;
        omhi[base + o] = 0;
    }
    // the bound must hold; if it ever did not, entries were dropped: say so
    if (bound_broken) atomicOr(&diag[kDiagFlags], (uint32_t)GS_FLAG_COUNT_BOUND);
}

// block ranges from the boundaries of the sorted keys, four keys per thread
__global__ __launch_bounds__(kBlock) void k_ranges(const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ used,
                                                   int32_t* __restrict__ ranges, uint32_t T) {
    const int64_t n = *used;
    const int64_t nq = (n + 3) / 4;
    for (int64_t qd = (int64_t)blockIdx.x * kBlock + threadIdx.x; qd < nq;
         qd += (int64_t)gridDim.x * kBlock) {
        const int64_t i0 = 4 * qd;
        uint32_t k[6];
        k[0] = i0 > 0 ? keys[i0 - 1] : 0xFFFFFFFFu;
        if (i0 + 4 <= n) {
            const uint4 q4 = *reinterpret_cast<const uint4*>(keys + i0);
            k[1] = q4.x;
            k[2] = q4.y;
            k[3] = q4.z;
            k[4] = q4.w;
        } else {
            for (int t = 0; t < 4; t++) k[1 + t] = i0 + t < n ? keys[i0 + t] : 0xFFFFFFFFu;
        }
        k[5] = i0 + 4 < n ? keys[i0 + 4] : 0xFFFFFFFFu;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int64_t i = i0 + t;
            const uint32_t kk = k[1 + t];
            if (i >= n || kk >= T) continue;
            if (i == 0 || k[t] != kk) ranges[2 * (int64_t)kk] = (int32_t)i;
            if (i == n - 1 || k[2 + t] != kk) ranges[2 * (int64_t)kk + 1] = (int32_t)i + 1;
        }
    }
}

// Block B's place: view, and block column / row in it.
__device__ __forceinline__ void block_place(const ViewTable& vt, int B, int& v, int& bxi, int& byi) {
    v = 0;
    while (v + 1 < vt.V && B >= vt.block_off[v + 1]) v++;
    const int lb = B - vt.block_off[v];
    bxi = lb % vt.bx[v];
    byi = lb / vt.bx[v];
}

constexpr int kBlockSub = kBlockTiles * kBlockTiles;  // tiles per block (sub-tile q = 4 sy + sx)
constexpr int kChunk = 256;                           // block-list entries per expansion workgroup

// The tile lists come out of the sorted block lists through 16 prefix counts:
// P_q(j) = entries before position j whose mask touches sub-tile q of their own
// block.  Entry j of block B lands in the list of B's sub-tile q (if it touches
// it) at P_q(j) - P_q(start of B); that list has P_q(end of B) - P_q(start of
// B) entries.  P_q is kept per 256-entry chunk (a scan of the chunk counts) and
// finished inside a chunk with ballots.

// touch bits of sub-tile q of a block mask
__device__ __forceinline__ bool touches(uint64_t m, int q) {
    return tile_bits(m, q % kBlockTiles, q / kBlockTiles) != 0;
}

// All sixteen at once: bit q (= 4 sy + sx) set iff the mask meets sub-tile q.
// Per 32-bit half (quadrant rows 4 h .. 4 h + 3): OR each tile's quadrant pair
// in a row, then the row below into it, keep bit 2 sx of bytes 0 and 2 and
// pack those eight bits into two nibbles.
__device__ __forceinline__ uint32_t touch_half(uint32_t x) {
    x |= x >> 1;
    x |= x >> 8;
    x &= 0x00550055u;
    x = (x | (x >> 1)) & 0x00330033u;
    x = (x | (x >> 2)) & 0x000F000Fu;
    return (x & 0xFu) | ((x >> 12) & 0xF0u);
}
__device__ __forceinline__ uint32_t tile_touch16(uint64_t m) {
    return touch_half((uint32_t)m) | (touch_half((uint32_t)(m >> 32)) << 8);
}

// Column stride of the chunk counts: one slot per chunk of the live entries
// and a last one that stays 0, so the prefix at the very end of the list is
// still read inside its column.
__device__ __forceinline__ int64_t chunk_stride(const uint32_t* used) {
    return ((int64_t)*used + kChunk - 1) / kChunk + 1;
}

// Per chunk and sub-tile: entries touching it.  ccnt is [16][stride] (column q
// contiguous), scanned as one array: every prefix that is used is a
// difference inside one column.
// One wave per chunk: its 256 entries are read four per lane, all loads in
// flight together, and counted by ballots; nothing is exchanged between waves.
constexpr int kChunkSteps = kChunk / kWave;

__global__ __launch_bounds__(kBlock) void k_chunk_count(const uint32_t* __restrict__ mlo,
                                                        const uint32_t* __restrict__ mhi,
                                                        const uint32_t* __restrict__ used,
                                                        uint32_t* __restrict__ ccnt) {
    const int64_t n = *used;
    const int64_t stride = chunk_stride(used);
    const int lane = threadIdx.x % kWave;
    if (blockIdx.x == 0 && threadIdx.x < kBlockSub) ccnt[(int64_t)threadIdx.x * stride + stride - 1] = 0u;
    const int64_t nw = (int64_t)gridDim.x * kWaves;
    for (int64_t c = (int64_t)blockIdx.x * kWaves + threadIdx.x / kWave; c * kChunk < n; c += nw) {
        uint64_t m[kChunkSteps];
#pragma unroll
        for (int u = 0; u < kChunkSteps; u++) {
            const int64_t j = c * kChunk + u * kWave + lane;
            const int64_t jc = min(j, n - 1);  // unconditional loads, zeroed past the end
            const uint64_t mm = ((uint64_t)mhi[jc] << 32) | mlo[jc];
            m[u] = j < n ? mm : 0ull;
        }
        uint32_t t[kChunkSteps];
#pragma unroll
        for (int u = 0; u < kChunkSteps; u++) t[u] = tile_touch16(m[u]);
        uint32_t cn = 0;
#pragma unroll
        for (int q = 0; q < kBlockSub; q++) {
            uint32_t k = 0;
#pragma unroll
            for (int u = 0; u < kChunkSteps; u++) k += (uint32_t)__popcll(__ballot((t[u] >> q) & 1u));
            cn = lane == q ? k : cn;  // lane q holds count q
        }
        if (lane < kBlockSub) ccnt[(int64_t)lane * stride + c] = cn;
    }
}

// P_q at list position x (x <= used): the chunk prefix plus the entries of x's
// chunk before x, counted by one wave.  Returns the value for q = lane (lanes < 16).
__device__ __forceinline__ uint32_t prefix_at(const uint32_t* __restrict__ mlo,
                                              const uint32_t* __restrict__ mhi,
                                              const uint32_t* __restrict__ cpre, int64_t stride,
                                              int64_t x) {
    const int lane = __lane_id();
    const int64_t c = x / kChunk, c0 = c * kChunk;
    uint32_t part = 0;
    for (int64_t j0 = c0; j0 < x; j0 += kWave) {
        const int64_t j = j0 + lane;
        uint64_t m = 0;
        if (j < x) m = ((uint64_t)mhi[j] << 32) | mlo[j];
#pragma unroll
        for (int q = 0; q < kBlockSub; q++) {
            const uint32_t n = (uint32_t)__popcll(__ballot(touches(m, q)));
            if (lane == q) part += n;
        }
    }
    return lane < kBlockSub ? cpre[(int64_t)lane * stride + c] + part : 0u;
}

// Per block (one wave): the prefixes at its list's start, its sub-tiles' list
// lengths, and where its tiles are (first tile, row stride, tiles per side).
__global__ __launch_bounds__(kWave) void k_block_tiles(const int32_t* __restrict__ branges,
                                                       const uint32_t* __restrict__ mlo,
                                                       const uint32_t* __restrict__ mhi,
                                                       const uint32_t* __restrict__ cpre,
                                                       const uint32_t* __restrict__ used,
                                                       ViewTable vt, int TH,
                                                       uint32_t* __restrict__ bpre,
                                                       int4* __restrict__ bplace,
                                                       uint32_t* __restrict__ tcnt) {
    const int B = blockIdx.x, lane = threadIdx.x;
    int v, bxi, byi;
    block_place(vt, B, v, bxi, byi);
    const int gy = (vt.H[v] + TH - 1) / TH;
    const int nx = min(kBlockTiles, vt.gx[v] - kBlockTiles * bxi);
    const int ny = min(kBlockTiles, gy - kBlockTiles * byi);
    const int tile0 = vt.tile_off[v] + kBlockTiles * byi * vt.gx[v] + kBlockTiles * bxi;
    if (lane == 0) bplace[B] = make_int4(tile0, vt.gx[v], nx, ny);
    const int rs = branges[2 * B], re = branges[2 * B + 1];
    uint32_t ps = 0, pe = 0;
    if (rs < re) {
        const int64_t stride = chunk_stride(used);
        ps = prefix_at(mlo, mhi, cpre, stride, rs);
        pe = prefix_at(mlo, mhi, cpre, stride, re);
    }
    if (lane < kBlockSub) {
        bpre[(int64_t)B * kBlockSub + lane] = ps;
        const int sx = lane % kBlockTiles, sy = lane / kBlockTiles;
        if (sx < nx && sy < ny) tcnt[tile0 + sy * vt.gx[v] + sx] = pe - ps;
    }
}

// Launch order of the tiles, heaviest first.  The weight is a log-scale bucket
// of the list length, exact in integers: 16 buckets per octave from the leading
// bit and the four bits after it (0 for an empty list).  Inside a bucket the
// order is free: tiles are independent, so it never changes a result.
__device__ __forceinline__ uint32_t length_bucket(uint32_t len) {
    if (len == 0) return 0;
    const int msb = 31 - __clz(len);
    const uint32_t frac = msb >= 4 ? (len >> (msb - 4)) & 15u : (len << (4 - msb)) & 15u;
    return 1u + 16u * (uint32_t)msb + frac;  // <= 1 + 16*31 + 15 = 512
}
// Tile ranges from the scanned counts (empty everywhere after an overflow),
// for each (block, sub-tile) the base that turns a prefix P_q(j) into the
// entry's slot: tile start - P_q(start of the block), and, if `bucket` is set,
// each tile's launch-order weight.
__global__ __launch_bounds__(kBlock) void k_tile_ranges(const uint32_t* __restrict__ toff,
                                                        const uint32_t* __restrict__ total,
                                                        const uint32_t* __restrict__ used,
                                                        ViewTable vt, int TH, int64_t T,
                                                        const uint32_t* __restrict__ bpre,
                                                        int32_t* __restrict__ tranges,
                                                        uint32_t* __restrict__ tbase,
                                                        uint32_t* __restrict__ bucket) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= T) return;
    const bool ok = *used != 0u || *total == 0u;
    const int32_t ts = ok ? (int32_t)toff[t] : 0;
    const int32_t te = ok ? (int32_t)(t + 1 < T ? toff[t + 1] : *total) : 0;
    tranges[2 * t] = ts;
    tranges[2 * t + 1] = te;
    // the launch-order weight of the tile (when an order is asked for)
    if (bucket) bucket[t] = length_bucket((uint32_t)max(te - ts, 0));
    int v = 0;
    while (v + 1 < vt.V && t >= vt.tile_off[v + 1]) v++;
    const int lt = (int)t - vt.tile_off[v];
    const int tx = lt % vt.gx[v], ty = lt / vt.gx[v];
    const int64_t B = vt.block_off[v] + (ty / kBlockTiles) * vt.bx[v] + tx / kBlockTiles;
    const int q = (ty % kBlockTiles) * kBlockTiles + tx % kBlockTiles;
    tbase[B * kBlockSub + q] = toff[t] - bpre[B * kBlockSub + q];
    (void)TH;
}

// Per chunk and sub-tile q, the place in q's list of the chunk's first entry
// of q, for the block of the chunk's first entry: tbase of that block plus the
// chunk prefix (cb[16 c + q]).  Chunks whose entries all lie in that block
// (nearly all) need nothing else.
__global__ __launch_bounds__(kBlock) void k_chunk_bases(const uint32_t* __restrict__ bkey,
                                                        const uint32_t* __restrict__ used,
                                                        const uint32_t* __restrict__ cpre,
                                                        const uint32_t* __restrict__ tbase,
                                                        uint32_t NB, int64_t max_chunks,
                                                        uint32_t* __restrict__ cb) {
    const int64_t n = *used;
    const int64_t stride = chunk_stride(used);
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t c = g / kBlockSub;
    const int q = (int)(g % kBlockSub);
    if (c >= max_chunks || c * kChunk >= n) return;
    const uint32_t B0 = bkey[c * kChunk];
    if (B0 < NB) cb[g] = tbase[(int64_t)B0 * kBlockSub + q] + cpre[(int64_t)q * stride + c];
}

// The tile lists: each block-list entry copied, as (pair | 4-bit mask << 28),
// to every sub-tile of its block it touches, at the place the prefixes give.
// One wave per chunk, four entries per lane, every load of the chunk (entries
// and its sub-tiles' bases) issued at once; the running counts per sub-tile
// are wave-uniform.  A chunk inside one block (nearly all) is staged in LDS
// grouped by sub-tile (the group sizes are differences of the chunk prefixes)
// and written out with dense stores, 64 consecutive staged entries per store,
// which land in at most a few contiguous runs; chunks that span blocks, or
// whose entries would overflow the stage, store each entry directly.
constexpr int kStage = 2048;  // staged tile entries per wave

__global__ __launch_bounds__(kBlock) void k_chunk_expand(
    const uint32_t* __restrict__ bkey, const uint32_t* __restrict__ pairs,
    const uint32_t* __restrict__ mlo, const uint32_t* __restrict__ mhi,
    const uint32_t* __restrict__ used, const uint32_t* __restrict__ tused,
    const uint32_t* __restrict__ cpre, const uint32_t* __restrict__ tbase,
    const uint32_t* __restrict__ cb, uint32_t NB, uint32_t* __restrict__ tids) {
    __shared__ uint32_t s_stage[kWaves][kStage];
    __shared__ uint32_t s_gpre[kWaves][kBlockSub + 1];  // group starts in the stage
    __shared__ uint32_t s_gbase[kWaves][kBlockSub];     // group starts in the lists
    const uint32_t tcap = *tused;  // list entries; every write stays below
    if (tcap == 0u) return;        // nothing is written after an overflow
    const int64_t n = *used;
    const int64_t stride = chunk_stride(used);
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const uint64_t lt = lanemask_lt();
    const int64_t nw = (int64_t)gridDim.x * kWaves;
    for (int64_t c = (int64_t)blockIdx.x * kWaves + w; c * kChunk < n; c += nw) {
        uint64_t m[kChunkSteps];
        uint32_t B[kChunkSteps], pr[kChunkSteps];
#pragma unroll
        for (int u = 0; u < kChunkSteps; u++) {
            const int64_t j = c * kChunk + u * kWave + lane;
            const int64_t jc = min(j, n - 1);  // unconditional loads, dropped past the end
            const uint64_t mm = ((uint64_t)mhi[jc] << 32) | mlo[jc];
            B[u] = bkey[jc];
            pr[u] = pairs[jc];
            // sentinel entries (unfilled slots) have B = NB and no mask
            m[u] = (j < n && B[u] < NB) ? mm : 0ull;
        }
        const int ql = lane % kBlockSub;
        const uint32_t cbq = cb[c * kBlockSub + ql];
        // this chunk's entries touching sub-tile ql: a difference of its prefixes
        const uint32_t cq = cpre[(int64_t)ql * stride + c + 1] - cpre[(int64_t)ql * stride + c];
        const uint32_t B0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)B[0]);
        bool other = false;
#pragma unroll
        for (int u = 0; u < kChunkSteps; u++) other |= m[u] != 0 && B[u] != B0;
        uint32_t run[kBlockSub];  // entries of the chunk so far touching sub-tile q
#pragma unroll
        for (int q = 0; q < kBlockSub; q++) run[q] = 0;
        // group starts: exclusive prefix of the counts over sub-tiles (lanes 0-15)
        uint32_t inc = lane < kBlockSub ? cq : 0u;
#pragma unroll
        for (int off = 1; off < kBlockSub; off <<= 1) {
            const uint32_t t = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += t;
        }
        const uint32_t staged = (uint32_t)__builtin_amdgcn_readlane((int)inc, kBlockSub - 1);
        if (__ballot(other) == 0 && staged <= (uint32_t)kStage) {
            if (lane < kBlockSub) {
                s_gpre[w][lane + 1] = inc;
                s_gbase[w][lane] = cbq;
            }
            if (lane == 0) s_gpre[w][0] = 0u;
#pragma unroll
            for (int u = 0; u < kChunkSteps; u++) {
#pragma unroll
                for (int q = 0; q < kBlockSub; q++) {
                    const uint64_t bal = __ballot(touches(m[u], q));
                    if (bal == 0) continue;  // wave-uniform
                    const uint32_t m4 = tile_bits(m[u], q % kBlockTiles, q / kBlockTiles);
                    // group q starts after the counts of sub-tiles 0 .. q-1
                    const uint32_t g0 = q == 0 ? 0u : (uint32_t)__builtin_amdgcn_readlane((int)inc, q - 1);
                    const uint32_t si = g0 + run[q] + (uint32_t)__popcll(bal & lt);
                    if (m4 && si < (uint32_t)kStage) s_stage[w][si] = pr[u] | (m4 << kPairBits);
                    run[q] += (uint32_t)__popcll(bal);
                }
            }
            wave_lds_sync();
            // staged entry f belongs to the group whose start is the last <= f
            for (uint32_t f = lane; f < staged; f += kWave) {
                int q = 0;
#pragma unroll
                for (int h = kBlockSub / 2; h > 0; h >>= 1)
                    if (s_gpre[w][q + h] <= f) q += h;
                const uint32_t ti = s_gbase[w][q] + (f - s_gpre[w][q]);
                if (ti < tcap) tids[ti] = s_stage[w][f];
            }
            wave_lds_sync();  // the stage is read before the next chunk's writes
        } else if (__ballot(other) == 0) {
#pragma unroll
            for (int u = 0; u < kChunkSteps; u++) {
#pragma unroll
                for (int q = 0; q < kBlockSub; q++) {
                    const uint64_t bal = __ballot(touches(m[u], q));
                    if (bal == 0) continue;  // wave-uniform
                    const uint32_t m4 = tile_bits(m[u], q % kBlockTiles, q / kBlockTiles);
                    const uint32_t base = (uint32_t)__builtin_amdgcn_readlane((int)cbq, q) + run[q];
                    const uint32_t ti = base + (uint32_t)__popcll(bal & lt);
                    if (m4 && ti < tcap) tids[ti] = pr[u] | (m4 << kPairBits);
                    run[q] += (uint32_t)__popcll(bal);
                }
            }
        } else {
            // entries of several blocks: every base gathered per lane
#pragma unroll
            for (int u = 0; u < kChunkSteps; u++) {
                const uint32_t Bq = m[u] != 0 ? B[u] : B0;
#pragma unroll
                for (int q = 0; q < kBlockSub; q++) {
                    const uint64_t bal = __ballot(touches(m[u], q));
                    if (bal == 0) continue;  // wave-uniform
                    const uint32_t m4 = tile_bits(m[u], q % kBlockTiles, q / kBlockTiles);
                    if (m4) {
                        const uint32_t base = tbase[(int64_t)Bq * kBlockSub + q] +
                                              cpre[(int64_t)q * stride + c] + run[q];
                        const uint32_t ti = base + (uint32_t)__popcll(bal & lt);
                        if (ti < tcap) tids[ti] = pr[u] | (m4 << kPairBits);
                    }
                    run[q] += (uint32_t)__popcll(bal);
                }
            }
        }
    }
}

constexpr int kOrderBuckets = 513;
constexpr int kOrderThreads = 1024;

// One block: histogram of the buckets, their scan from the heaviest down, and
// a scatter through LDS cursors.  For up to 2^20 tiles.  The bucket scan
// runs over all threads at once.
__global__ __launch_bounds__(kOrderThreads) void k_tile_order(const uint32_t* __restrict__ bucket,
                                                               int64_t T,
                                                               uint32_t* __restrict__ order) {
    __shared__ uint32_t s_n[kOrderBuckets];
    __shared__ uint32_t s_w[kOrderThreads / kWave];
    for (int q = threadIdx.x; q < kOrderBuckets; q += kOrderThreads) s_n[q] = 0;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < T; t += kOrderThreads) atomicAdd(&s_n[bucket[t]], 1u);
    __syncthreads();
    {
        // exclusive scan from the heaviest bucket down, over all threads:
        // thread i takes bucket kOrderBuckets - 1 - i
        const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
        const int qb = kOrderBuckets - 1 - tid;
        const uint32_t c = qb >= 0 ? s_n[qb] : 0u;
        uint32_t inc = c;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t x = __shfl_up(inc, off, kWave);
            if (lane >= off) inc += x;
        }
        if (lane == kWave - 1) s_w[w] = inc;
        __syncthreads();
        uint32_t before = 0;
        for (int i = 0; i < w; i++) before += s_w[i];
        if (qb >= 0) s_n[qb] = before + inc - c;
    }
    __syncthreads();
    for (int64_t t = threadIdx.x; t < T; t += kOrderThreads) {
        const uint32_t pos = atomicAdd(&s_n[bucket[t]], 1u);
        order[pos] = (uint32_t)t;
    }
}

// Larger tile counts: key = 2^24 - 1 - min(list length, 2^24 - 1) through the
// stable radix sort (exact lengths, which also orders the buckets)
__global__ __launch_bounds__(kBlock) void k_tile_keys(const int32_t* __restrict__ tranges, int64_t T,
                                                      uint32_t* __restrict__ key,
                                                      uint32_t* __restrict__ val) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= T) return;
    const uint32_t len = (uint32_t)max(tranges[2 * t + 1] - tranges[2 * t], 0);
    key[t] = 0xFFFFFFu - min(len, 0xFFFFFFu);
    val[t] = (uint32_t)t;
}

}  // namespace

hipError_t launch_bin(Ctx* c, const ViewTable& vt, int N, const RasterParams& rp,
                      const float* records, int tile_order, hipStream_t st) {
    const int64_t npairs = (int64_t)vt.V * N;
    const float4* rec = reinterpret_cast<const float4*>(records ? records : c->rec);
    const int64_t T = vt.tile_off[vt.V];
    const int64_t NB = vt.block_off[vt.V];
    hipError_t e = hipSuccess;
    c->ordered = false;
    c->lists_lazy = false;
    c->lists_filled = false;
    if (npairs > 0) {
        const unsigned gp = (unsigned)((npairs + kBlock - 1) / kBlock);
        int pbits = 1;  // bits of a pair index (the capacity keeps it at most 26)
        while (((int64_t)1 << pbits) < npairs) pbits++;
        hipLaunchKernelGGL(k_count, dim3(gp), dim3(kBlock), 0, st, rec, N, vt, rp, c->cnt, c->pk[0],
                           c->pv[0], c->ranges, 2 * NB, pbits);
        // the pair and its entry count travel with the depth key as one word;
        // the sorted counts are then unpacked and scanned into the entry offsets
        const int side = radix_sort_pairs(c->pk[0], c->pv[0], c->pk[1], c->pv[1], npairs, nullptr, 0, 32,
                                          c->hist, c->scan_scratch, c->diag + kDiagFlags, st, &e);
        if (e != hipSuccess) return e;
        const uint32_t* order = c->pv[side];
        uint32_t* off = c->off;
        uint32_t* total = c->scalars + 0;
        uint32_t* used = c->scalars + 1;
        // the counts, unpacked as the scan loads them; its last tile checks
        // the block-entry total against the capacity
        const CapCheck chk_blocks = {c->cap.max_isect, used, c->diag, nullptr, nullptr};
        const ScanUnpack un = {order, c->cnt, pbits};
        if ((e = exclusive_scan_u32_unpack(off, un, npairs, total, c->scan_scratch, c->diag + kDiagFlags, st,
                                           &chk_blocks)) != hipSuccess)
            return e;
        const int64_t I = c->cap.max_isect;
        hipLaunchKernelGGL(k_emit, dim3(gp), dim3(kBlock), 0, st, rec, N, vt, rp, order,
                           (uint32_t)((1u << pbits) - 1u), off,
                           c->pk[side], npairs, used, c->ik[0], c->iv[0], c->im[0], c->im[0] + I, c->diag);
        int bbits = 1;  // block ids and the sentinel NB
        while (((int64_t)1 << bbits) <= NB) bbits++;
        // the pair and both mask words travel with the block key
        uint32_t* K[2] = {c->ik[0], c->ik[1]};
        uint32_t* Vv[3][2] = {{c->iv[0], c->iv[1]}, {c->im[0], c->im[1]}, {c->im[0] + I, c->im[1] + I}};
        const int side2 = radix_sort_kv3(K, Vv, I, used, 0, bbits, c->hist, c->scan_scratch, c->diag + kDiagFlags, st, &e);
        if (e != hipSuccess) return e;
        c->block_side = side2;
        const uint32_t* bmlo = c->im[side2];
        const uint32_t* bmhi = c->im[side2] + I;
        const unsigned gi = (unsigned)std::min<int64_t>((I + kBlock - 1) / kBlock, 4096);
        hipLaunchKernelGGL(k_ranges, dim3(gi), dim3(kBlock), 0, st, c->ik[side2], used, c->ranges,
                           (uint32_t)NB);
        // tile lists: chunk counts and their scan, per-block prefixes and tile
        // list lengths, the tile scan and ranges (the entries follow at the end)
        if (T > 0) {
            uint32_t* ttotal = c->scalars + 2;
            uint32_t* tused = c->scalars + 3;
            const int64_t nch = c->nchunks;
            // one wave per chunk, grid-stride beyond 32768 waves
            const unsigned gch = (unsigned)std::min<int64_t>((nch + kWaves - 1) / kWaves, 8192);
            hipLaunchKernelGGL(k_chunk_count, dim3(gch), dim3(kBlock), 0, st, bmlo, bmhi, used, c->ccnt);
            if ((e = exclusive_scan_u32_dev(c->ccnt, kBlockSub * (nch + 1), used, kChunk, kBlockSub, 1,
                                            nullptr, c->scan_scratch, c->diag + kDiagFlags, st)) != hipSuccess)
                return e;
            // every tile's count is written by its block's k_block_tiles
            if (NB > 0)
                hipLaunchKernelGGL(k_block_tiles, dim3((unsigned)NB), dim3(kWave), 0, st, c->ranges, bmlo,
                                   bmhi, c->ccnt, used, vt, rp.tile_h, c->bpre, c->bplace, c->tcnt);
            // the tile lists must fit too (their total replaces the block count)
            const CapCheck chk_tiles = {c->cap.max_isect, tused, c->diag, total, used};
            if ((e = exclusive_scan_u32(c->tcnt, T, ttotal, c->scan_scratch, c->diag + kDiagFlags, st,
                                        &chk_tiles)) != hipSuccess)
                return e;
            const unsigned gt = (unsigned)((T + kBlock - 1) / kBlock);
            const bool bucketed = tile_order && T <= ((int64_t)1 << 20);
            hipLaunchKernelGGL(k_tile_ranges, dim3(gt), dim3(kBlock), 0, st, c->tcnt, ttotal, tused, vt,
                               rp.tile_h, T, c->bpre, c->tranges, c->tbase, bucketed ? c->tk[0] : nullptr);
        }
        if (tile_order && T > 0 && T <= ((int64_t)1 << 20)) {
            // the weights were written with the tile ranges
            hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, st, c->tk[0], T,
                               c->tile_order);
            c->ordered = true;
        } else if (tile_order && T > 0) {
            hipLaunchKernelGGL(k_tile_keys, dim3((unsigned)((T + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                               st, c->tranges, T, c->tk[0], c->tile_order);
            // sort (key, tile) pairs: tile_order holds the values of the first buffer pair
            uint32_t* kk[2] = {c->tk[0], c->tk[1]};
            uint32_t* vv[2] = {c->tile_order, reinterpret_cast<uint32_t*>(c->tile_contrib)};
            const int side3 = radix_sort_pairs(kk[0], vv[0], kk[1], vv[1], T, nullptr, 0, 24, c->hist,
                                               c->scan_scratch, c->diag + kDiagFlags, st, &e);
            if (e != hipSuccess) return e;
            if (side3 == 1) {
                e = hipMemcpyAsync(c->tile_order, vv[1], sizeof(uint32_t) * T, hipMemcpyDeviceToDevice, st);
                if (e != hipSuccess) return e;
            }
            c->ordered = true;
        }
    } else if (T > 0) {
        // no pairs: every tile list is empty
        if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(c->tranges), 0u, 2 * T, st)) != hipSuccess)
            return e;
    }
    c->n_tiles = T;
    c->n_blocks = NB;
    c->bin_V = vt.V;
    c->bin_N = N;
    c->bin_tw = rp.tile_w;
    c->bin_th = rp.tile_h;
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the entries themselves: now, or drawn by the forward from the block lists
    if (npairs > 0 && T > 0) {
        if (rp.lazy_lists) c->lists_lazy = true;
        else return launch_expand_lists(c, st);
    }
    return hipSuccess;
}

hipError_t launch_expand_lists(Ctx* c, hipStream_t st) {
    const int64_t NB = c->n_blocks, nch = c->nchunks, I = c->cap.max_isect;
    const int side = c->block_side;
    const uint32_t* used = c->scalars + 1;
    const uint32_t* tused = c->scalars + 3;
    const unsigned gch = (unsigned)std::min<int64_t>((nch + kWaves - 1) / kWaves, 8192);
    hipLaunchKernelGGL(k_chunk_bases, dim3((unsigned)((nch * kBlockSub + kBlock - 1) / kBlock)),
                       dim3(kBlock), 0, st, c->ik[side], used, c->ccnt, c->tbase, (uint32_t)NB, nch,
                       c->cbase);
    hipLaunchKernelGGL(k_chunk_expand, dim3(gch), dim3(kBlock), 0, st, c->ik[side], c->iv[side],
                       c->im[side], c->im[side] + I, used, tused, c->ccnt, c->tbase, c->cbase,
                       (uint32_t)NB, c->tids);
    c->lists_lazy = false;
    return hipGetLastError();
}

}  // namespace gs
