// Device-wide exclusive scan and stable LSD radix sort of (u32 key, u32 value)
// pairs, written for wave64: digit ranks inside a wave come from ballots
// (match-any over the digit bits), across waves from LDS counters, and each
// block stages its items in LDS so the global scatter writes contiguous runs.
#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // 4096 items per block
constexpr int kWaves = kThreads / kWave;

// ------------------------------------------------------------------ scan

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = __lane_id();
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t t = __shfl_up(v, off, kWave);
        if (lane >= off) v += t;
    }
    return v;
}

// exclusive scan of one value per thread over the block; returns the block total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_w, uint32_t& total) {
    const int lane = __lane_id(), w = threadIdx.x / kWave;
    uint32_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) s_w[w] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); i++) {
        if (i < w) before += s_w[i];
        tot += s_w[i];
    }
    __syncthreads();
    total = tot;
    return before + inc - v;
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                          uint32_t* __restrict__ part) {
    __shared__ uint32_t s_w[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        int64_t j = base + i;
        if (j < n) s += in[j];
    }
    uint32_t tot;
    block_excl_scan(s, s_w, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// one block of 1024 threads scans up to 16384 block partials
__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t* __restrict__ part, int nparts,
                                                        uint32_t* __restrict__ total_out) {
    __shared__ uint32_t s_w[16];
    const int per = (nparts + 1023) / 1024;
    const int b = threadIdx.x * per;
    uint32_t loc[16];
    uint32_t s = 0;
    for (int i = 0; i < per; i++) {
        loc[i] = (b + i < nparts) ? part[b + i] : 0u;
        s += loc[i];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(s, s_w, tot);
    for (int i = 0; i < per; i++) {
        if (b + i < nparts) part[b + i] = ex;
        ex += loc[i];
    }
    if (threadIdx.x == 0 && total_out) *total_out = tot;
}

__global__ __launch_bounds__(kThreads) void k_scan_apply(uint32_t* __restrict__ data, int64_t n,
                                                         const uint32_t* __restrict__ part) {
    __shared__ uint32_t s_w[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        int64_t j = base + i;
        v[i] = (j < n) ? data[j] : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(s, s_w, tot) + part[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kItems; i++) {
        int64_t j = base + i;
        if (j < n) data[j] = ex;
        ex += v[i];
    }
}

// ------------------------------------------------------------------ radix sort

__device__ __forceinline__ uint32_t dev_count(const uint32_t* d_n, int64_t max_n) {
    if (!d_n) return (uint32_t)max_n;
    uint32_t n = *d_n;
    return n < (uint64_t)max_n ? n : (uint32_t)max_n;
}

// lanes of the wave holding the same digit of `bits` bits (among lanes with `valid`)
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid, int bits) {
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// Items of a block: wave w owns the contiguous chunk [base + 64 ITEMS w,
// base + 64 ITEMS (w+1)), read 64 at a time; so (wave, step, lane) order is
// index order and ranks can be kept per wave without block barriers.
template <int ITEMS>
__device__ __forceinline__ int64_t item_index(int64_t base, int w, int i, int lane) {
    return base + (int64_t)w * (kWave * ITEMS) + i * kWave + lane;
}

// Per-block digit counts, digit-major: hist[d * nblocks + block].  All loads
// of a thread are issued before the first ballot.
template <int ITEMS>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                         const uint32_t* __restrict__ d_n,
                                                         int64_t max_n, int shift, int bits,
                                                         uint32_t* __restrict__ hist,
                                                         uint32_t nblocks) {
    constexpr int TILE = kThreads * ITEMS;
    __shared__ uint32_t s_h[kWaves][256];
    const uint32_t n = dev_count(d_n, max_n);
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const uint32_t mask = (1u << bits) - 1u;
    for (int q = 0; q < kWaves; q++) s_h[q][tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * TILE;
    if (base < n) {
        uint32_t k[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const int64_t j = item_index<ITEMS>(base, w, i, lane);
            k[i] = j < n ? keys[j] : 0u;
        }
#pragma unroll
        for (int i = 0; i < ITEMS; i++) {
            const bool valid = item_index<ITEMS>(base, w, i, lane) < n;
            const uint32_t d = (k[i] >> shift) & mask;
            const uint64_t peers = match_digit(d, valid, bits);
            // one lane per digit adds the digit's count in this wave's histogram
            if (valid && (peers & lanemask_lt()) == 0) s_h[w][d] += (uint32_t)__popcll(peers);
        }
    }
    __syncthreads();
    if (tid <= (int)mask)
        hist[(int64_t)tid * nblocks + blockIdx.x] = s_h[0][tid] + s_h[1][tid] + s_h[2][tid] + s_h[3][tid];
}

// Value arrays moved with the keys: NV words per item, one array each.
template <int NV>
struct ValArrays {
    const uint32_t* in[NV];
    uint32_t* out[NV];
};

template <int ITEMS, int NV>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(
    const uint32_t* __restrict__ kin, uint32_t* __restrict__ kout, ValArrays<NV> va,
    const uint32_t* __restrict__ d_n, int64_t max_n, int shift, int bits,
    const uint32_t* __restrict__ hist, uint32_t nblocks) {
    constexpr int TILE = kThreads * ITEMS;
    __shared__ uint32_t s_h[kWaves][256];  // per-wave digit counts, then offsets
    __shared__ uint32_t s_start[256];
    __shared__ uint32_t s_glob[256];
    __shared__ uint32_t s_w[kWaves];
    __shared__ uint32_t s_key[TILE];
    __shared__ uint32_t s_val[NV][TILE];
    const uint32_t n = dev_count(d_n, max_n);
    const int64_t base = (int64_t)blockIdx.x * TILE;
    if (base >= n) return;  // uniform over the block
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t k[ITEMS], v[NV][ITEMS];
    uint16_t rank[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const int64_t j = item_index<ITEMS>(base, w, i, lane);
        k[i] = j < n ? kin[j] : 0u;
#pragma unroll
        for (int c = 0; c < NV; c++) v[c][i] = j < n ? va.in[c][j] : 0u;
    }
    for (int q = 0; q < kWaves; q++) s_h[q][tid] = 0;
    s_glob[tid] = tid <= (int)mask ? hist[(int64_t)tid * nblocks + blockIdx.x] : 0u;
    __syncthreads();
    // stable rank inside the wave's chunk: earlier steps (LDS count) + earlier lanes
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const bool valid = item_index<ITEMS>(base, w, i, lane) < n;
        const uint32_t d = (k[i] >> shift) & mask;
        const uint64_t peers = match_digit(d, valid, bits);
        const uint32_t before = s_h[w][d];
        rank[i] = (uint16_t)(before + (uint32_t)__popcll(peers & lanemask_lt()));
        if (valid && (peers & lanemask_lt()) == 0) s_h[w][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: offsets of the waves, then the block-wide exclusive scan
    uint32_t run = 0;
    for (int q = 0; q < kWaves; q++) {
        const uint32_t c = s_h[q][tid];
        s_h[q][tid] = run;
        run += c;
    }
    uint32_t tot;
    s_start[tid] = block_excl_scan(run, s_w, tot);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        if (item_index<ITEMS>(base, w, i, lane) < n) {
            const uint32_t d = (k[i] >> shift) & mask;
            const uint32_t pos = s_start[d] + s_h[w][d] + rank[i];
            s_key[pos] = k[i];
#pragma unroll
            for (int c = 0; c < NV; c++) s_val[c][pos] = v[c][i];
        }
    }
    __syncthreads();
    const uint32_t cnt = (uint32_t)min((int64_t)TILE, (int64_t)n - base);
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const uint32_t j = i * kThreads + tid;
        if (j < cnt) {
            const uint32_t key = s_key[j];
            const uint32_t d = (key >> shift) & mask;
            const uint32_t g = s_glob[d] + (j - s_start[d]);
            kout[g] = key;
#pragma unroll
            for (int c = 0; c < NV; c++) va.out[c][g] = s_val[c][j];
        }
    }
}

}  // namespace

size_t scan_scratch_words(int64_t max_n) { return (size_t)((max_n + kTile - 1) / kTile) + 16; }

hipError_t exclusive_scan_u32(uint32_t* data, int64_t n, uint32_t* total_out, uint32_t* scratch,
                              hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kTile - 1) / kTile;
    if (nb > 16384) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kThreads), 0, st, data, n, scratch);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, st, scratch, (int)nb, total_out);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kThreads), 0, st, data, n, scratch);
    return hipGetLastError();
}

size_t radix_hist_words(int64_t max_n) { return (size_t)256 * ((max_n + kTile - 1) / kTile) + 16; }

namespace {

// one pass over `bits` bits at `shift`; blocks of 256 x ITEMS items
template <int ITEMS, int NV>
hipError_t radix_pass(const uint32_t* ki, uint32_t* ko, const ValArrays<NV>& va, int64_t max_n,
                      const uint32_t* d_n, int shift, int bits, uint32_t* hist,
                      uint32_t* scan_scratch, hipStream_t st) {
    const uint32_t nb = (uint32_t)((max_n + kThreads * ITEMS - 1) / (kThreads * ITEMS));
    hipLaunchKernelGGL(k_radix_hist<ITEMS>, dim3(nb), dim3(kThreads), 0, st, ki, d_n, max_n, shift,
                       bits, hist, nb);
    hipError_t e = exclusive_scan_u32(hist, ((int64_t)1 << bits) * nb, nullptr, scan_scratch, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_radix_scatter<ITEMS, NV>), dim3(nb), dim3(kThreads), 0, st, ki, ko, va,
                       d_n, max_n, shift, bits, hist, nb);
    return hipGetLastError();
}

// LSD passes of equal digit widths (at most 8 bits) over [lo, hi); K[2] and
// V[c][2] are the ping-pong buffers; returns the side holding the result
template <int NV>
int radix_sort_impl(uint32_t* K[2], uint32_t* V[NV][2], int64_t max_n, const uint32_t* d_n, int lo,
                    int hi, uint32_t* hist, uint32_t* scan_scratch, hipStream_t st, hipError_t* err) {
    *err = hipSuccess;
    if (max_n <= 0 || hi <= lo) return 0;
    const int total = hi - lo;
    const int passes = (total + 7) / 8;
    int cur = 0;
    int shift = lo;
    for (int p = 0; p < passes; p++) {
        const int bits = (total - (shift - lo) + (passes - p) - 1) / (passes - p);
        ValArrays<NV> va;
        for (int c = 0; c < NV; c++) {
            va.in[c] = V[c][cur];
            va.out[c] = V[c][cur ^ 1];
        }
        // large single-value inputs: 8192 items per block (longer runs per
        // digit in the scatter); wider payloads keep 4096 for the LDS staging
        if (NV == 1 && max_n > ((int64_t)1 << 22))
            *err = radix_pass<32, NV>(K[cur], K[cur ^ 1], va, max_n, d_n, shift, bits, hist,
                                      scan_scratch, st);
        else
            *err = radix_pass<16, NV>(K[cur], K[cur ^ 1], va, max_n, d_n, shift, bits, hist,
                                      scan_scratch, st);
        if (*err != hipSuccess) return cur;
        shift += bits;
        cur ^= 1;
    }
    return cur;
}

}  // namespace

int radix_sort_pairs(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t max_n,
                     const uint32_t* d_n, int lo, int hi, uint32_t* hist, uint32_t* scan_scratch,
                     hipStream_t st, hipError_t* err) {
    uint32_t* K[2] = {ka, kb};
    uint32_t* V[1][2] = {{va, vb}};
    return radix_sort_impl<1>(K, V, max_n, d_n, lo, hi, hist, scan_scratch, st, err);
}

int radix_sort_kv3(uint32_t* K[2], uint32_t* V[3][2], int64_t max_n, const uint32_t* d_n, int lo,
                   int hi, uint32_t* hist, uint32_t* scan_scratch, hipStream_t st, hipError_t* err) {
    return radix_sort_impl<3>(K, V, max_n, d_n, lo, hi, hist, scan_scratch, st, err);
}

}  // namespace gs
