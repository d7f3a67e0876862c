// Internal declarations of the gfx950 splatting library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gs.h"

namespace gs {

constexpr int kWave = 64;

// Per-view geometry of one call, passed by value as a kernel argument so a
// call needs no host->device copy (and stays capturable in a HIP graph).
struct ViewTable {
    int V;
    int W[GS_MAX_VIEWS];
    int H[GS_MAX_VIEWS];
    int gx[GS_MAX_VIEWS];
    int tile_off[GS_MAX_VIEWS + 1];  // first global tile of each view
    int pix_off[GS_MAX_VIEWS + 1];   // first packed pixel of each view
    int bx[GS_MAX_VIEWS];            // block columns of each view
    int block_off[GS_MAX_VIEWS + 1]; // first global block of each view
    int cam[GS_MAX_VIEWS];           // row of viewmat / intr / v_twist used by the view
};

struct RasterParams {
    float alpha_min, alpha_max, t_min;
    float near_plane, eps2d, fov_pad;
    int tile_w, tile_h;
    int eval_stats;
    int tile_order;
    int lazy_lists;
};

// Device status words (one array in the context).
enum DiagSlot {
    kDiagFlags = 0,        // GS_FLAG_* bits
    kDiagIsectTotal = 1,   // intersections the last bin step needed
    kDiagIsectUsed = 2,    // intersections it produced (0 on overflow)
    kDiagMasked = 3,       // masked track observations
    kDiagVisible = 4,      // pairs with >= 1 tile
    kDiagCount = 8,
};

struct Ctx;  // defined in gs_api.hip

constexpr int kAuxFloats = 8192;

// The per-pair 2D gradients live in two planes of one buffer: six floats per
// pair for the geometry (mean x, y, conic A, B, C, opacity) and, after the
// pair capacity's worth of those, three per pair for the colour, so the two
// halves of the projection backward each read only their own part.
constexpr int kGradGeo = 6;
constexpr int kGradCol = 3;

// ------------------------------------------------------------------ device helpers

__device__ __forceinline__ float bcast(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
__device__ __forceinline__ int bcast(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xF, false));
}

// Sum over the 64 lanes of a wave (all lanes must be active); the total is
// valid in lane 63 and returned uniformly.  DPP steps: quad xor 1, quad xor 2,
// half-row mirror, row mirror, then row broadcasts 15 and 31.
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    v += dpp_f<0x142, 0xA>(v);
    v += dpp_f<0x143, 0xC>(v);
    return bcast(v, 63);
}

// Wave totals of nine per-lane values in about a third of the instructions of
// nine separate sums.  The first eight are halved three times by exchanging
// with the quad partner lane^1 and lane^2 (keeping the half picked by that lane
// bit) and with the lane four places round the 16-lane row; the ninth is summed
// over its quads alone; both are then summed over the row (rotate by 8).  The
// last two steps need no LDS: v_permlane16_swap swaps the odd rows of one
// register with the even rows of another (rows 0 and 2 then hold the eight,
// rows 1 and 3 the ninth), and v_permlane32_swap the upper half of one with
// the lower half of another.  On return lanes 0-15 and 32-47 hold the total of
// value sum8_index(lane & 7), lanes 16-31 and 48-63 the total of a8.
__device__ __forceinline__ float wave_sum9_t(float a0, float a1, float a2, float a3, float a4, float a5,
                                             float a6, float a7, float a8) {
    const int lane = __lane_id();
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4;
    const float c0 = (b0 ? a4 : a0) + dpp_f<0xB1>(b0 ? a0 : a4);
    const float c1 = (b0 ? a5 : a1) + dpp_f<0xB1>(b0 ? a1 : a5);
    const float c2 = (b0 ? a6 : a2) + dpp_f<0xB1>(b0 ? a2 : a6);
    const float c3 = (b0 ? a7 : a3) + dpp_f<0xB1>(b0 ? a3 : a7);
    const float d0 = (b1 ? c2 : c0) + dpp_f<0x4E>(b1 ? c0 : c2);
    const float d1 = (b1 ? c3 : c1) + dpp_f<0x4E>(b1 ? c1 : c3);
    float e = (b2 ? d1 : d0) + dpp_f<0x124>(b2 ? d0 : d1);  // row_ror:4
    e += dpp_f<0x128>(e);                                     // row_ror:8
    float z = a8 + dpp_f<0xB1>(a8);
    z += dpp_f<0x4E>(z);
    z += dpp_f<0x124>(z);
    z += dpp_f<0x128>(z);
    // (the pair's elements are copied out before any bit cast)
    const auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(e), __float_as_uint(z), false, false);
    const unsigned s0 = r16[0], s1 = r16[1];
    const float f = __uint_as_float(s0) + __uint_as_float(s1);
    const auto r32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(f), __float_as_uint(f), false, false);
    const unsigned t0 = r32[0], t1 = r32[1];
    return __uint_as_float(t0) + __uint_as_float(t1);
}

__device__ __forceinline__ int sum8_index(int lane) {
    return ((lane & 1) << 2) | (lane & 2) | ((lane >> 2) & 1);
}

__device__ __forceinline__ int wave_max_i(int v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    return v;
}

// Orders one wave's own LDS accesses (its stores before its later loads) with
// no workgroup barrier, which would also wait for the loads in flight.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Gaussian falloff exponent sigma = 0.5 (A dx^2 + C dy^2) + B dx dy with a
// fixed operation order, shared by the forward and the backward raster so both
// take identical alpha-gate decisions.
// The exponent of a splat in base 2: e2 = -log2(e) sigma(dx, dy), sigma = A dx^2 / 2
// + B dx dy + C dy^2 / 2, with the conic scaled once per splat (a = -log2(e) A / 2,
// b = -log2(e) B, c = -log2(e) C / 2) so a pixel pays three operations and the
// hardware exp2.  The forward and the backward evaluate it with this one fixed
// operation order, so both take the same decisions.
constexpr float kLog2E = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

struct ConicE2 {
    float a, b, c;
};

__device__ __forceinline__ ConicE2 conic_e2(float A, float B, float C) {
    return {-0.5f * kLog2E * A, -kLog2E * B, -0.5f * kLog2E * C};
}

__device__ __forceinline__ float splat_e2(float a, float b, float c, float dx, float dy) {
    const float q = __builtin_fmaf(a * dx, dx, c * dy * dy);
    return __builtin_fmaf(b * dx, dy, q);
}

// Tile-space footprint of a splat, by spans.  The tile is split into four
// quadrants (TW/2 x TH/2); a quadrant row is a band of pixel-centre rows.  In a
// band the splat's alpha >= alpha_min ellipse covers one x-interval, found in
// closed form (the ellipse boundary is convex on the left, concave on the
// right, with its extremes at the leftmost / rightmost points), so a splat's
// quadrants follow from O(bands) work with no per-tile test.  The threshold is
// made conservative (relative 1e-4 plus 1e-4, and 1e-3 px on every interval)
// so float rounding can only add quadrants that contribute nothing.
struct SplatSpan {
    float mx, my, B, iA, t2A, det, ey, dyL;
    int r0, r1;  // quadrant rows that may be met (r0 > r1: none)
};

constexpr float kSpanEps = 1e-3f;

// Quadrant geometry of a call: half-tile sizes and their reciprocals (exact,
// powers of two), so no division is left in the per-row work.
struct QuadGrid {
    int hw, hh;
    float ihw, ihh;
};

__host__ __device__ __forceinline__ QuadGrid quad_grid(int TW, int TH) {
    QuadGrid g;
    g.hw = TW / 2;
    g.hh = TH / 2;
    g.ihw = 1.f / (float)g.hw;
    g.ihh = 1.f / (float)g.hh;
    return g;
}

// Contraction stays off in the span arithmetic: the count and the emit pass
// evaluate it separately and must agree to the bit.
__device__ __forceinline__ SplatSpan splat_span(const float4& a, const float4& b, int H,
                                                const QuadGrid& g, float alpha_min) {
#pragma clang fp contract(off)
    SplatSpan s;
    s.mx = a.x;
    s.my = a.y;
    const float A = b.x, B = b.y, C = b.z;
    const float t = __logf(a.w / alpha_min) * 1.0001f + 1e-4f;
    s.B = B;
    s.iA = 1.f / A;
    s.t2A = 2.f * A * t;
    s.det = A * C - B * B;
    const float idet = 1.f / s.det;
    // Sigma2D = [[C, -B], [-B, A]] / det; vertical half-extent sqrt(2 t Syy) and
    // the height of the leftmost point -Sxy sqrt(2 t / Sxx)
    s.ey = __builtin_amdgcn_sqrtf(2.f * t * A * idet);
    s.dyL = B * idet * __builtin_amdgcn_sqrtf(2.f * t * s.det / C);
    const int nrows = (H + g.hh - 1) / g.hh;
    s.r0 = max((int)floorf((s.my - s.ey - kSpanEps) * g.ihh), 0);
    s.r1 = min((int)floorf((s.my + s.ey + kSpanEps) * g.ihh), nrows - 1);
    return s;
}

// Quadrant columns [c0, c1] of quadrant row r met by the splat (c0 > c1:
// none); ncols = quadrant columns of the view.
__device__ __forceinline__ void span_cols(const SplatSpan& s, int r, int W, int H, const QuadGrid& g,
                                          int ncols, int& c0, int& c1) {
#pragma clang fp contract(off)
    c0 = 1;
    c1 = 0;
    const float ya = r * g.hh + 0.5f, yb = (float)min(r * g.hh + g.hh, H) - 0.5f;
    float la = fmaxf(ya - s.my, -s.ey), lb = fminf(yb - s.my, s.ey);
    if (la > lb + kSpanEps) return;
    if (la > lb) la = lb = 0.5f * (la + lb);
    // x offsets of the ellipse boundary at height dy: (-B dy -/+ sqrt(2 A t - det dy^2)) / A
    const float dl = fminf(fmaxf(s.dyL, la), lb), dr = fminf(fmaxf(-s.dyL, la), lb);
    const float ql = __builtin_amdgcn_sqrtf(fmaxf(s.t2A - s.det * dl * dl, 0.f));
    const float qr = __builtin_amdgcn_sqrtf(fmaxf(s.t2A - s.det * dr * dr, 0.f));
    const float xl = s.mx + (-s.B * dl - ql) * s.iA - kSpanEps;
    const float xr = s.mx + (-s.B * dr + qr) * s.iA + kSpanEps;
    if (!(xl <= (float)W - 0.5f) || !(xr >= 0.5f)) return;
    c0 = max((int)ceilf((xl + 0.5f) * g.ihw - 1.f), 0);
    c1 = min((int)floorf((xr - 0.5f) * g.ihw), ncols - 1);
}

// One Adam step of one element (Algorithm 1 update step): bias-corrected
// moments through ibc1 = 1 / (1 - b1^t), ibc2 = 1 / (1 - b2^t).  Every Adam
// in the library goes through this one function.
__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float lr, float b1,
                                         float b2, float eps, float ibc1, float ibc2) {
    m = b1 * m + (1.f - b1) * g;
    v = b2 * v + (1.f - b2) * g * g;
    p -= lr * (m * ibc1) / (sqrtf(v * ibc2) + eps);
}

// The bias corrections 1 / (1 - b^t) of Adam step t, read from the device
// counter when there is one (a captured step then takes the step number the
// counter holds at replay), else from the value passed; t < 1 counts as 1.
// b^t by repeated squaring in double, then rounded once.
__device__ __forceinline__ void adam_bias(const int32_t* step_dev, int step, float b1, float b2,
                                          float& ibc1, float& ibc2) {
    int t = step_dev ? *step_dev : step;
    t = t < 1 ? 1 : t;
    double p1 = 1.0, p2 = 1.0, q1 = b1, q2 = b2;
    for (int e = t; e > 0; e >>= 1) {
        if (e & 1) {
            p1 *= q1;
            p2 *= q2;
        }
        q1 *= q1;
        q2 *= q2;
    }
    ibc1 = (float)(1.0 / (1.0 - p1));
    ibc2 = (float)(1.0 / (1.0 - p2));
}

// Adam state of the five Gaussian arrays (means, log_scales, quats,
// opacity_logit, sh) for the projection backward that also steps them.
struct AdamGauss {
    float* p[5];
    float* m[5];
    float* v[5];
    float lr[5];
    float b1, b2, eps;
    float ibc1, ibc2;          // set in the kernel from the step
    const int32_t* step_dev;   // device step counter, or NULL: `step`
    int step;
};

// A tile-list entry carries the pair index in its low 28 bits and the
// quadrant mask in the top 4.
constexpr uint32_t kPairBits = 28;
constexpr uint32_t kPairMask = (1u << kPairBits) - 1u;

// Blocks: 4 x 4 tiles, i.e. 8 x 8 quadrants.  The lists are kept per block; an
// entry is a splat (its pair index) with the 64-bit mask of the block's
// quadrants it meets, bit 8 qr + qc for quadrant row qr and column qc inside
// the block.  A tile's list is the block list filtered to the entries with a
// non-zero mask on the tile's four quadrants.
constexpr int kBlockTiles = 4;                  // tiles per block side
constexpr int kBlockQuads = 2 * kBlockTiles;    // quadrants per block side

// The four quadrant bits (qx + 2 qy) of tile (sx, sy) of a block in a block mask.
__device__ __forceinline__ uint32_t tile_bits(uint64_t m, int sx, int sy) {
    const int sh = 16 * sy + 2 * sx;
    return (uint32_t)((m >> sh) & 3u) | ((uint32_t)((m >> (sh + 8)) & 3u) << 2);
}

// One block row of a splat's footprint ("unit"): the quadrant-column interval
// of each of its (up to 8) quadrant rows, and the block columns they span.
struct BlockUnit {
    int c0[kBlockQuads], c1[kBlockQuads];  // quadrant columns per row (c0 > c1: none)
    int bc0, bc1;                          // block columns to scan (bc0 > bc1: none)
};

__device__ __forceinline__ BlockUnit block_unit(const SplatSpan& s, int br, int W, int H,
                                                const QuadGrid& g) {
    BlockUnit u;
    const int ncols = (W + g.hw - 1) / g.hw;
    u.bc0 = 1 << 30;
    u.bc1 = -1;
#pragma unroll
    for (int i = 0; i < kBlockQuads; i++) {
        const int r = kBlockQuads * br + i;
        u.c0[i] = 1;
        u.c1[i] = 0;
        // r <= s.r1 keeps r inside the view's quadrant rows
        if (r >= s.r0 && r <= s.r1) span_cols(s, r, W, H, g, ncols, u.c0[i], u.c1[i]);
        if (u.c0[i] <= u.c1[i]) {
            u.bc0 = min(u.bc0, u.c0[i] / kBlockQuads);
            u.bc1 = max(u.bc1, u.c1[i] / kBlockQuads);
        }
    }
    return u;
}

// The block mask of unit u in block column bc (0: the splat misses the block).
// Row i's byte is the run of quadrant columns [c0 - q0, c1 - q0] clipped to
// [0, 7], built without branches: (0xFF << lo) & (0xFF >> (7 - hi)) with lo
// clamped to [0, 8] and hi to [-1, 7] is empty whenever lo > hi.
__device__ __forceinline__ uint64_t block_unit_mask(const BlockUnit& u, int bc) {
    const int q0 = kBlockQuads * bc;
    uint32_t lo32 = 0, hi32 = 0;
#pragma unroll
    for (int i = 0; i < kBlockQuads; i++) {
        const int lo = min(max(u.c0[i] - q0, 0), 8);
        const int hi = min(max(u.c1[i] - q0, -1), 7);
        const uint32_t byte = (0xFFu << lo) & (0xFFu >> (7 - hi));
        if (i < 4) lo32 |= byte << (8 * i);
        else hi32 |= byte << (8 * (i - 4));
    }
    return ((uint64_t)hi32 << 32) | lo32;
}

// Entries of a unit: block columns met by some row (a row meets the block
// columns c0/8 .. c1/8), counted on a bitmask of the columns from bc0 while
// they fit in 64 bits, one column at a time beyond.
__device__ __forceinline__ int block_unit_count(const BlockUnit& u) {
    if (u.bc0 > u.bc1) return 0;
    if (u.bc1 - u.bc0 < 64) {
        uint64_t cols = 0;
#pragma unroll
        for (int i = 0; i < kBlockQuads; i++) {
            if (u.c0[i] > u.c1[i]) continue;
            const int a = u.c0[i] / kBlockQuads - u.bc0, b = u.c1[i] / kBlockQuads - u.bc0;
            const uint64_t hi = b >= 63 ? ~0ull : (2ull << b) - 1ull;
            cols |= hi & ~((1ull << a) - 1ull);
        }
        return __popcll(cols);
    }
    int n = 0;
    for (int bc = u.bc0; bc <= u.bc1; bc++) n += block_unit_mask(u, bc) != 0;
    return n;
}

// Upper bound of a unit's entries, for sizing only: the block columns met by
// the ellipse over the unit's whole band of quadrant rows (one x-span instead
// of eight).  The band covers every row's pixel-centre range, and the minimum
// (maximum) of a convex (concave) boundary over a larger interval is no larger
// (smaller), so the band's columns contain each row's; kBandEps absorbs the
// rounding of the two evaluations.  The emit pass fills slots the bound
// over-counts with entries that no list reads.
constexpr float kBandEps = 0.125f;

__device__ __forceinline__ int unit_band_count(const SplatSpan& s, int br, int W, int H,
                                               const QuadGrid& g) {
#pragma clang fp contract(off)
    const int ra = max(s.r0, kBlockQuads * br), rb = min(s.r1, kBlockQuads * br + kBlockQuads - 1);
    if (ra > rb) return 0;
    const float ya = ra * g.hh + 0.5f, yb = (float)min(rb * g.hh + g.hh, H) - 0.5f;
    float la = fmaxf(ya - s.my, -s.ey), lb = fminf(yb - s.my, s.ey);
    if (la > lb + kSpanEps) return 0;
    if (la > lb) la = lb = 0.5f * (la + lb);
    const float dl = fminf(fmaxf(s.dyL, la), lb), dr = fminf(fmaxf(-s.dyL, la), lb);
    const float ql = __builtin_amdgcn_sqrtf(fmaxf(s.t2A - s.det * dl * dl, 0.f));
    const float qr = __builtin_amdgcn_sqrtf(fmaxf(s.t2A - s.det * dr * dr, 0.f));
    const float xl = s.mx + (-s.B * dl - ql) * s.iA - (kSpanEps + kBandEps);
    const float xr = s.mx + (-s.B * dr + qr) * s.iA + (kSpanEps + kBandEps);
    if (!(xl <= (float)W - 0.5f) || !(xr >= 0.5f)) return 0;
    const int ncols = (W + g.hw - 1) / g.hw;
    const int c0 = max((int)ceilf((xl + 0.5f) * g.ihw - 1.f), 0);
    const int c1 = min((int)floorf((xr - 0.5f) * g.ihw), ncols - 1);
    return c0 <= c1 ? c1 / kBlockQuads - c0 / kBlockQuads + 1 : 0;
}

// ------------------------------------------------------------------ host launchers

ViewTable make_view_table(const int32_t* wh, int V, int TW, int TH, const int32_t* index = nullptr);
RasterParams make_raster_params(const gs_settings* s);

// scan.hip / sort.hip
size_t scan_scratch_words(int64_t max_n);
// Exclusive scan in place (mod 2^32); total_out (device, nullable) gets the
// total.  scratch: scan_scratch_words(n) words, zero before the first scan and
// left zero by every scan; flags (device, nullable) gets GS_FLAG_SCAN_STALLED
// if a look-back gave up.
// Capacity check of a list total, run by the scan's last tile: used = total
// if it fits cap, else 0 with GS_FLAG_ISECT_OVERFLOW; the totals go to
// diag[kDiagIsectTotal / kDiagIsectUsed].  Once an earlier stage (prev_total,
// prev_used; both may be NULL) overflowed, its counts stay (a lower bound of
// the need) and this stage only sets used = 0.
struct CapCheck {
    int64_t cap;
    uint32_t* used;  // NULL: no check
    uint32_t* diag;
    const uint32_t* prev_total;
    const uint32_t* prev_used;
};
hipError_t exclusive_scan_u32(uint32_t* data, int64_t n, uint32_t* total_out, uint32_t* scratch,
                              uint32_t* flags, hipStream_t st, const CapCheck* chk = nullptr);
// The same, with the input unpacked on load from words that hold an index in
// their low pbits and a count above it: the count, or cnt[index] where the
// count field is all ones.  The scan is written to data (not to src).
struct ScanUnpack {
    const uint32_t* src;
    const uint32_t* cnt;
    int pbits;
};
hipError_t exclusive_scan_u32_unpack(uint32_t* data, const ScanUnpack& un, int64_t n, uint32_t* total_out,
                                     uint32_t* scratch, uint32_t* flags, hipStream_t st, const CapCheck* chk);
// The same over a length the device holds: mul * (ceil(*d_cnt / per) + add),
// at most max_n (the launch covers max_n).
hipError_t exclusive_scan_u32_dev(uint32_t* data, int64_t max_n, const uint32_t* d_cnt, int64_t per,
                                  int64_t mul, int64_t add, uint32_t* total_out, uint32_t* scratch,
                                  uint32_t* flags, hipStream_t st);
size_t radix_hist_words(int64_t max_n);
// Stable LSD radix sort of (key, value) u32 pairs on bits [lo, hi). n items
// (device count d_n if non-null, clamped to max_n). Returns the buffer pair
// holding the result: 0 = (ka, va), 1 = (kb, vb).
int radix_sort_pairs(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t max_n,
                     const uint32_t* d_n, int lo, int hi, uint32_t* hist, uint32_t* scan_scratch,
                     uint32_t* flags, hipStream_t st, hipError_t* err);
// The same with three value words per item (separate arrays): K[side],
// V[word][side]; returns the side holding the result.
int radix_sort_kv3(uint32_t* K[2], uint32_t* V[3][2], int64_t max_n, const uint32_t* d_n, int lo,
                   int hi, uint32_t* hist, uint32_t* scan_scratch, uint32_t* flags, hipStream_t st,
                   hipError_t* err);

// bin.hip
hipError_t launch_bin(Ctx* c, const ViewTable& vt, int N, const RasterParams& rp,
                      const float* records, int tile_order, hipStream_t st);

// project.hip
hipError_t launch_project_fwd(Ctx* c, const gs_gaussians* g, const gs_cameras* cams,
                              const ViewTable& vt, const RasterParams& rp, hipStream_t st);
// with adam non-null the Gaussian gradients are not written: each one takes
// its Adam step in place instead
hipError_t launch_project_bwd(Ctx* c, const gs_gaussians* g, const gs_cameras* cams,
                              const ViewTable& vt, const RasterParams& rp, const AdamGauss* adam,
                              gs_gaussians_grad* grads, int accumulate, float* v_twist,
                              hipStream_t st);

// raster.hip
// The tile lists in full from the block lists of the last bin step (for a
// backward after a lazy bin step with no forward in between).
hipError_t launch_expand_lists(Ctx* c, hipStream_t st);
hipError_t launch_render_fwd(Ctx* c, const ViewTable& vt, const RasterParams& rp, const float* bg,
                             float* rgb, float* T_final, int32_t* last, hipStream_t st);
hipError_t launch_render_bwd(Ctx* c, const ViewTable& vt, const RasterParams& rp, const float* bg,
                             const float* T_final, const int32_t* last, const float* v_rgb,
                             hipStream_t st);
hipError_t launch_l1(Ctx* c, const ViewTable& vt, const float* rgb, const float* target,
                     float* v_rgb, float* loss, hipStream_t st);

// init.hip: Gaussians from points (k-nearest-neighbour scales); uses the
// pair-sized sort buffers, records, counts and aux of the context
hipError_t launch_init_gaussians(Ctx* c, const float* pts, const float* rgb, int n, int k,
                                 float opacity, int sh_degree, float* means, float* log_scales,
                                 float* quats, float* logit, float* sh, hipStream_t st);

// mcmc.hip: relocation of dead Gaussians and noise on the means
hipError_t launch_mcmc_relocate(Ctx* c, const gs_gaussian_adam* state, int N, int sh_degree,
                                const float* u, float t_dead, int32_t* src, int32_t* n_moved,
                                hipStream_t st);
hipError_t launch_mcmc_noise(float* means, const float* log_scales, const float* quats,
                             const float* logit, int N, const float* eta, float scale, float k, float t,
                             hipStream_t st);

// ba.hip: one Levenberg-Marquardt step of bundle adjustment
struct BaInputs {
    const float* X;
    const float* viewmat;
    const float* intr;
    const int32_t* obs_cam;
    const int32_t* obs_pt;
    const float* obs_xy;
    const int32_t* pt_off;
    const int32_t* pt_obs;
    const int32_t* pm_cam;  // point-major copies (or NULL: read through pt_obs)
    const float* pm_xy;
    int Pt, n_cams, M, max_iter;
    float delta, lambda, near_plane, tol;
};
hipError_t launch_ba_step(gs_ba* ba, const BaInputs& in, float* d_twist, float* d_X, float* stats,
                          hipStream_t st);

// photo.hip: (1 - lambda) L1 + lambda (1 - SSIM) and its image gradient
hipError_t launch_photo(Ctx* c, const ViewTable& vt, const float* rgb, const float* target,
                        float lambda, float* v_rgb, float* loss, hipStream_t st);

// track.hip
// Workgroups of the point-major track pass (each keeps its twist sums in LDS).
constexpr int kTrackPmBlocks = 512;
hipError_t launch_track(Ctx* c, const float* X, int Pt, const float* viewmat, const float* intr,
                        int n_cams, const int32_t* obs_cam, const int32_t* obs_pt,
                        const float* obs_xy, int M, float delta, float lambda, float near_plane,
                        float* residual, float* loss, float* v_X, float* v_twist, float* J_pose,
                        float* J_X, const int32_t* pt_off, const int32_t* pt_obs,
                        const int32_t* pm_cam, const float* pm_xy, hipStream_t st);
// The same with the accumulators given explicitly: twist_acc [n_cams][6] and
// loss_acc [1] (double, zero on entry, left zero), diag [kDiagCount] (the
// masked count is added to diag[kDiagMasked]).
struct TrackScratch {
    double* twist_acc;
    double* loss_acc;
    uint32_t* diag;
};
hipError_t launch_track_scratch(const TrackScratch& sc, const float* X, int Pt, const float* viewmat,
                                const float* intr, int n_cams, const int32_t* obs_cam,
                                const int32_t* obs_pt, const float* obs_xy, int M, float delta,
                                float lambda, float near_plane, float* residual, float* loss,
                                float* v_X, float* v_twist, float* J_pose, float* J_X,
                                const int32_t* pt_off, const int32_t* pt_obs, hipStream_t st);
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t st);
// Point-major index of the observations for launch_track: pt_off[Pt + 1],
// pt_obs[M] (each point's observations ascending; out-of-range points left
// out), and optionally the cameras and pixels in that order (pm_cam, pm_xy
// from obs_cam, obs_xy).  Uses c->cnt (>= Pt words) and the scan scratch
// (>= Pt + 1 items).
hipError_t launch_track_index(Ctx* c, const int32_t* obs_pt, int M, int Pt, int32_t* pt_off,
                              int32_t* pt_obs, const int32_t* obs_cam, const float* obs_xy,
                              int32_t* pm_cam, float* pm_xy, hipStream_t st);

// optim.hip
hipError_t launch_pose_compose(int V, const float* twist, const float* base, float* out,
                               hipStream_t st);
hipError_t launch_pose_compose_bwd(int V, const float* twist, const float* g, float* out,
                                   hipStream_t st);
hipError_t launch_adam(const gs_adam_group* groups, int n, int step, const int32_t* step_dev,
                       float b1, float b2, float eps, hipStream_t st);
hipError_t launch_step_advance(int32_t* step_dev, hipStream_t st);
hipError_t launch_flush_acc(double* acc, float* out, int n, hipStream_t st);
// out[6 * rows[v] + e] += acc[6 * v + e]; acc cleared (twists of a sampled batch)
hipError_t launch_flush_twist_rows(double* acc, float* out, const ViewTable& vt, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);

// The context (workspace), shared by the launchers.
struct Ctx {
    gs_capacity cap;
    int device;
    float* rec;            // [max_pairs][12]
    float* grad2d;         // [max_pairs][6] geometry, then [max_pairs][3] colour; kept zero
                           // between backward calls
    float* vmu_dir;        // [3][max_pairs] the colour's share of the mean gradient (backward)
    uint32_t* cnt;         // [max_pairs] list entries per pair
    uint32_t* off;         // [max_pairs] entry counts in depth order, then their scan
    uint32_t* pk[2];       // [max_pairs] depth keys (ping-pong)
    uint32_t* pv[2];       // [max_pairs] pair indices (ping-pong)
    uint32_t* ik[2];       // [max_isect] block keys (ping-pong)
    uint32_t* iv[2];       // [max_isect] pair indices (ping-pong)
    uint32_t* im[2];       // [2][max_isect] block masks, low then high words (ping-pong)
    int32_t* ranges;       // [max_tiles][2] block list ranges (blocks <= tiles)
    uint32_t* tcnt;        // [max_tiles] tile list lengths, then their scan
    uint32_t* ccnt;        // [16][ceil(used / 256) + 1] sub-tile counts per 256-entry chunk, then their scan
    int64_t nchunks;       // max_isect / 256 + 1
    int64_t scan_max;      // longest array the scan scratch covers
    uint32_t* cbase;       // [nchunks][16] list place of each chunk's first entry per sub-tile
    uint32_t* bpre;        // [max_tiles][16] sub-tile prefixes at each block's list start
    int4* bplace;          // [max_tiles] first tile, row stride, tiles across / down per block
    uint32_t* tbase;       // [max_tiles][16] tile start - prefix at the block start
    int32_t* tranges;      // [max_tiles][2] tile list ranges
    uint32_t* tids;        // [max_isect] tile lists: pair | quadrant mask << 28
    uint32_t* tile_order;  // [max_tiles] launch order of the tiles (heaviest first)
    uint32_t* tk[2];       // [max_tiles] sort scratch for the tile order
    int32_t* tile_contrib; // [max_tiles] contributing (pixel, splat) pairs per tile
    int32_t* tile_entries; // [max_tiles] list entries each tile's forward consumed
    int32_t* tile_evals;   // [max_tiles] (pixel, entry) evaluations up to the last contributors
    uint32_t* hist;        // radix histograms
    uint32_t* scan_scratch;
    uint32_t* scalars;     // small device counters
    double* twist_render;  // [max_views][6]
    double* twist_track;   // [max_cams][6]
    float* track_part;     // [kTrackPmBlocks][6 pm_cams] per-workgroup twist sums (point-major pass)
    double* track_loss_part;  // [kTrackPmBlocks] per-workgroup loss sums
    int pm_cams;           // cameras the point-major pass can hold (0: none)
    double* loss_acc;      // [4]
    float* aux;            // [kAuxFloats] small per-call device scratch (bounding boxes, grid)
    uint32_t* diag;        // [kDiagCount]
    // state of the last bin step
    int64_t n_tiles, n_blocks;
    int bin_V, bin_N, bin_tw, bin_th;
    bool ordered;          // tile_order holds the order of the last bin step
    // lazy lists: the last bin step stopped at the block lists (block_side is
    // the ping-pong side they ended on); filled: a forward has written the
    // part of each tile list a backward reads
    bool lists_lazy, lists_filled;
    int block_side;
    int64_t generation;    // gs_bin_sort calls enqueued so far
};

}  // namespace gs
