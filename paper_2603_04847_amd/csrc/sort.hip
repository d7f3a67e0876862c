// Device-wide exclusive scan (single pass) and stable LSD radix sort of (u32 key, u32 value)
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

// Single-pass scan with decoupled look-back.  Tiles of kScanTile items are taken
// in launch order from a counter, so every tile a workgroup waits on belongs
// to a workgroup that is already running.  A tile publishes its own total
// (flag kAgg), then its first wave reads the words of the 64 preceding tiles
// at once and adds back to the nearest one that carries an inclusive prefix
// (flag kIncl), which it then publishes for itself.  The last workgroup to
// finish clears the words and counters, so the workspace is clean for the
// next scan without a separate fill.
//
// Workspace (u32 words): [0] tile counter, [1] finished counter, then one
// 64-bit word per tile from word kScanHeader: flag << 32 | value.
constexpr int kScanHeader = 64;
constexpr uint32_t kAgg = 1u, kIncl = 2u;
// bound on the polls of one look-back (each ~1 us): a wait that never ends is
// reported (GS_FLAG_SCAN_STALLED) instead of hanging the device
constexpr int kSpinLimit = 1 << 21;

__device__ __forceinline__ uint64_t ld_word(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_word(uint64_t* p, uint32_t flag, uint32_t v) {
    __hip_atomic_store(p, ((uint64_t)flag << 32) | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Called by one whole wave: the sum of the values of tiles [0, t) (mod 2^32).
__device__ uint32_t wave_lookback(const uint64_t* words, int64_t t, uint32_t* flags) {
    const int lane = __lane_id();
    uint32_t excl = 0;
    int64_t top = t - 1;
    int polls = 0;
    while (top >= 0) {
        const int64_t idx = top - lane;
        const uint64_t w = idx >= 0 ? ld_word(words + idx) : ((uint64_t)kIncl << 32);
        const uint32_t flag = (uint32_t)(w >> 32);
        const uint64_t incl = __ballot(flag == kIncl);
        const uint64_t none = __ballot(flag == 0u);
        const int first = incl ? __builtin_ctzll(incl) : kWave;  // nearest inclusive tile
        const uint64_t need = first >= kWave - 1 ? ~0ull : ((2ull << first) - 1ull);
        if (none & need) {
            if (++polls > kSpinLimit) {
                if (lane == 0 && flags) {
                    atomicOr(flags, (uint32_t)GS_FLAG_SCAN_STALLED);
                    __atomic_thread_fence(__ATOMIC_RELEASE);
                }
                return excl;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        excl += wave_sum_u32(lane <= first ? (uint32_t)w : 0u);
        if (first < kWave) break;
        top -= kWave;
    }
    return excl;
}

// A scan whose look-back gave up (GS_FLAG_SCAN_STALLED) has offsets that are
// not to be trusted: the check then treats the list as overflowed, so every
// later stage writes nothing.
__device__ __forceinline__ void cap_check(uint32_t t, const CapCheck& c, const uint32_t* flags) {
    if (!c.used) return;
    const bool stalled =
        flags && (__hip_atomic_load(flags, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) &
                  (uint32_t)GS_FLAG_SCAN_STALLED) != 0u;
    const bool prev_over = c.prev_total && *c.prev_total != 0u && *c.prev_used == 0u;
    const bool over = prev_over || stalled || (int64_t)t > c.cap;
    *c.used = over ? 0u : t;
    if (prev_over) return;
    c.diag[kDiagIsectTotal] = t;
    c.diag[kDiagIsectUsed] = over ? 0u : t;
    if (over) atomicOr(&c.diag[kDiagFlags], (uint32_t)GS_FLAG_ISECT_OVERFLOW);
}

// 32 items per thread, read and written as 16-byte vectors: 8192 per tile of
// 256 threads.  Scans past kWideScan items use tiles of 1024 threads (32768
// items): the tickets and the look-back chain are per tile, and on the 20M
// offsets of the large scene the wide tiles take 0.05 ms off the binning
// (smaller scans lose parallelism with them).
constexpr int kScanItems = 32;
constexpr int kScanTile = kThreads * kScanItems;
constexpr int kWideThreads = 1024;
constexpr int64_t kWideScan = (int64_t)1 << 23;

// The length is max_n, or, with d_cnt, mul * (ceil(*d_cnt / per) + add)
// clamped to max_n (a count only the device knows: the grid covers max_n and
// tiles past the length only take their tickets).
template <int THREADS, bool UNPACK = false>
__global__ __launch_bounds__(THREADS) void k_scan(uint32_t* __restrict__ data, int64_t max_n,
                                                   const uint32_t* __restrict__ d_cnt, int64_t per,
                                                   int64_t mul, int64_t add,
                                                   uint32_t* __restrict__ total_out,
                                                   uint32_t* __restrict__ ws,
                                                   uint32_t* __restrict__ flags, CapCheck chk,
                                                   ScanUnpack un) {
    constexpr int TILE = THREADS * kScanItems;
    __shared__ uint32_t s_w[THREADS / kWave];
    __shared__ uint32_t s_t, s_excl, s_last;
    uint64_t* words = reinterpret_cast<uint64_t*>(ws + kScanHeader);
    int64_t n = max_n;
    if (d_cnt) n = min(max_n, mul * (((int64_t)*d_cnt + per - 1) / per + add));
    const int64_t ntiles = (n + TILE - 1) / TILE;
    if (threadIdx.x == 0) s_t = atomicAdd(&ws[0], 1u);
    __syncthreads();
    const int64_t t = s_t;
    if (t >= ntiles) {
        if (t == 0 && threadIdx.x == 0) {
            if (total_out) *total_out = 0u;
            cap_check(0u, chk, flags);
        }
    } else {
        const int64_t base = t * TILE + (int64_t)threadIdx.x * kScanItems;
        const bool full = base + kScanItems <= n;
        uint32_t v[kScanItems];
        const uint32_t* in = UNPACK ? un.src : data;
        if (full) {
            const uint4* p = reinterpret_cast<const uint4*>(in + base);
#pragma unroll
            for (int i = 0; i < kScanItems / 4; i++) {
                const uint4 q = p[i];
                v[4 * i] = q.x;
                v[4 * i + 1] = q.y;
                v[4 * i + 2] = q.z;
                v[4 * i + 3] = q.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < kScanItems; i++) v[i] = base + i < n ? in[base + i] : 0u;
        }
        if (UNPACK) {
            const uint32_t esc = ~0u >> un.pbits, pmask = (1u << un.pbits) - 1u;
#pragma unroll
            for (int i = 0; i < kScanItems; i++) {
                const uint32_t c = v[i] >> un.pbits;
                v[i] = c == esc ? un.cnt[v[i] & pmask] : c;
            }
        }
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) s += v[i];
        uint32_t tot;
        uint32_t ex = block_excl_scan(s, s_w, tot);
        if (threadIdx.x < kWave) {
            if (threadIdx.x == 0) st_word(words + t, t == 0 ? kIncl : kAgg, tot);
            const uint32_t excl = t > 0 ? wave_lookback(words, t, flags) : 0u;
            if (threadIdx.x == 0) {
                if (t > 0) st_word(words + t, kIncl, excl + tot);
                s_excl = excl;
                if (t == ntiles - 1) {
                    if (total_out) *total_out = excl + tot;
                    cap_check(excl + tot, chk, flags);
                }
            }
        }
        __syncthreads();
        ex += s_excl;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            const uint32_t x = v[i];
            v[i] = ex;
            ex += x;
        }
        if (full) {
            uint4* p = reinterpret_cast<uint4*>(data + base);
#pragma unroll
            for (int i = 0; i < kScanItems / 4; i++)
                p[i] = make_uint4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
        } else {
#pragma unroll
            for (int i = 0; i < kScanItems; i++)
                if (base + i < n) data[base + i] = v[i];
        }
    }
    // every tile has finished its look-back once all have taken a ticket here
    if (threadIdx.x == 0) s_last = atomicAdd(&ws[1], 1u) == gridDim.x - 1;
    __syncthreads();
    if (s_last) {
        for (int64_t k = threadIdx.x; k < ntiles; k += THREADS) st_word(words + k, 0u, 0u);
        if (threadIdx.x == 0) {
            __hip_atomic_store(&ws[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ws[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
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

// Per-block digit counts, digit-major: hist[d * nb + block] with nb the number
// of blocks that hold items (the live count), so the scan covers only those.
// All loads of a thread are issued before the first count.  Counts need no
// ranks: for 7- and 8-bit digits each item is one LDS add, and a wave whose
// valid items share one digit (common in the top digit of clustered keys)
// adds them at once; narrower digits of clustered keys (the block ids) would
// pile many adds onto a few addresses, so there one lane per distinct digit
// adds the count its ballot match found.
template <int ITEMS>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                         const uint32_t* __restrict__ d_n,
                                                         int64_t max_n, int shift, int bits,
                                                         uint32_t* __restrict__ hist) {
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
            if (bits > 6) {
                const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
                if (__ballot(valid && d != d0) == 0) {
                    const uint64_t live = __ballot(valid);
                    if (lane == 0 && live) atomicAdd(&s_h[w][d0], (uint32_t)__popcll(live));
                } else if (valid) {
                    atomicAdd(&s_h[w][d], 1u);
                }
            } else {
                const uint64_t peers = match_digit(d, valid, bits);
                if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&s_h[w][d], (uint32_t)__popcll(peers));
            }
        }
    }
    __syncthreads();
    const int64_t nb = ((int64_t)n + TILE - 1) / TILE;
    if (tid <= (int)mask && (int64_t)blockIdx.x < nb)
        hist[(int64_t)tid * nb + blockIdx.x] = s_h[0][tid] + s_h[1][tid] + s_h[2][tid] + s_h[3][tid];
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
    const uint32_t* __restrict__ hist) {
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
    const int64_t nb = ((int64_t)n + TILE - 1) / TILE;
    s_glob[tid] = tid <= (int)mask ? hist[(int64_t)tid * nb + blockIdx.x] : 0u;
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
            if (g < n) {  // always, unless a digit scan gave up (flagged)
                kout[g] = key;
#pragma unroll
                for (int c = 0; c < NV; c++) va.out[c][g] = s_val[c][j];
            }
        }
    }
}

}  // namespace

size_t scan_scratch_words(int64_t max_n) {
    return (size_t)kScanHeader + 2 * (size_t)((max_n + kScanTile - 1) / kScanTile) + 16;
}

namespace {

hipError_t scan_launch(uint32_t* data, int64_t max_n, const uint32_t* d_cnt, int64_t per, int64_t mul,
                       int64_t add, uint32_t* total_out, uint32_t* scratch, uint32_t* flags,
                       hipStream_t st, const CapCheck* chk, const ScanUnpack* un = nullptr) {
    CapCheck ck = {};
    if (chk) ck = *chk;
    // nothing to scan: done, unless a capacity check must still see the 0 total
    if (max_n <= 0 && !ck.used) return hipSuccess;
    if (max_n < 0) max_n = 0;
    // whole-tile vector accesses need 16-byte alignment
    if (reinterpret_cast<uintptr_t>(data) % 16 != 0 || (d_cnt && (per <= 0 || mul <= 0 || add < 0)) ||
        (un && (reinterpret_cast<uintptr_t>(un->src) % 16 != 0 || un->pbits < 1 || un->pbits > 31)))
        return hipErrorInvalidValue;
    const ScanUnpack u = un ? *un : ScanUnpack{nullptr, nullptr, 1};
    if (max_n > kWideScan) {
        const int64_t ntw = (max_n + kWideThreads * kScanItems - 1) / (kWideThreads * kScanItems);
        if (un)
            hipLaunchKernelGGL((k_scan<kWideThreads, true>), dim3((unsigned)ntw), dim3(kWideThreads), 0, st, data,
                               max_n, d_cnt, per, mul, add, total_out, scratch, flags, ck, u);
        else
            hipLaunchKernelGGL((k_scan<kWideThreads, false>), dim3((unsigned)ntw), dim3(kWideThreads), 0, st, data,
                               max_n, d_cnt, per, mul, add, total_out, scratch, flags, ck, u);
        return hipGetLastError();
    }
    const int64_t nt = std::max<int64_t>((max_n + kScanTile - 1) / kScanTile, 1);
    if (nt > ((int64_t)1 << 31)) return hipErrorInvalidValue;
    if (un)
        hipLaunchKernelGGL((k_scan<kThreads, true>), dim3((unsigned)nt), dim3(kThreads), 0, st, data, max_n, d_cnt,
                           per, mul, add, total_out, scratch, flags, ck, u);
    else
        hipLaunchKernelGGL((k_scan<kThreads, false>), dim3((unsigned)nt), dim3(kThreads), 0, st, data, max_n, d_cnt,
                           per, mul, add, total_out, scratch, flags, ck, u);
    return hipGetLastError();
}

}  // namespace

hipError_t exclusive_scan_u32_dev(uint32_t* data, int64_t max_n, const uint32_t* d_cnt, int64_t per,
                                  int64_t mul, int64_t add, uint32_t* total_out, uint32_t* scratch,
                                  uint32_t* flags, hipStream_t st) {
    return scan_launch(data, max_n, d_cnt, per, mul, add, total_out, scratch, flags, st, nullptr);
}

hipError_t exclusive_scan_u32(uint32_t* data, int64_t n, uint32_t* total_out, uint32_t* scratch,
                              uint32_t* flags, hipStream_t st, const CapCheck* chk) {
    return scan_launch(data, n, nullptr, 1, 1, 0, total_out, scratch, flags, st, chk);
}

hipError_t exclusive_scan_u32_unpack(uint32_t* data, const ScanUnpack& un, int64_t n, uint32_t* total_out,
                                     uint32_t* scratch, uint32_t* flags, hipStream_t st, const CapCheck* chk) {
    return scan_launch(data, n, nullptr, 1, 1, 0, total_out, scratch, flags, st, chk, &un);
}

// sized for the smallest block (2048 items)
size_t radix_hist_words(int64_t max_n) { return (size_t)256 * ((max_n + kTile / 2 - 1) / (kTile / 2)) + 16; }

namespace {

// one pass over `bits` bits at `shift`; blocks of 256 x ITEMS items
template <int ITEMS, int NV>
hipError_t radix_pass(const uint32_t* ki, uint32_t* ko, const ValArrays<NV>& va, int64_t max_n,
                      const uint32_t* d_n, int shift, int bits, uint32_t* hist,
                      uint32_t* scan_scratch, uint32_t* flags, hipStream_t st) {
    const uint32_t nb = (uint32_t)((max_n + kThreads * ITEMS - 1) / (kThreads * ITEMS));
    hipLaunchKernelGGL(k_radix_hist<ITEMS>, dim3(nb), dim3(kThreads), 0, st, ki, d_n, max_n, shift,
                       bits, hist);
    hipError_t e = exclusive_scan_u32_dev(hist, ((int64_t)1 << bits) * nb, d_n, kThreads * ITEMS,
                                          (int64_t)1 << bits, 0, nullptr, scan_scratch, flags, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_radix_scatter<ITEMS, NV>), dim3(nb), dim3(kThreads), 0, st, ki, ko, va,
                       d_n, max_n, shift, bits, hist);
    return hipGetLastError();
}

// LSD passes of equal digit widths (at most 8 bits) over [lo, hi); K[2] and
// V[c][2] are the ping-pong buffers; returns the side holding the result
template <int NV>
int radix_sort_impl(uint32_t* K[2], uint32_t* V[NV][2], int64_t max_n, const uint32_t* d_n, int lo,
                    int hi, uint32_t* hist, uint32_t* scan_scratch, uint32_t* flags, hipStream_t st,
                    hipError_t* err) {
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
        // large single-value inputs (the depth sort, whose one value word
        // packs the pair and its entry count): 4096 items per block (on the
        // 20M pairs of the large scene 0.06 ms faster over the four passes
        // than 8192, and 0.08 ms faster than 2048); the block sort of a list
        // capacity past 2^27 4096 (fewer digit counts to scan); the others
        // 2048: a sort of a few million items still gives every CU several
        // blocks, and a block sort of tens of millions of entries gains from
        // the shorter blocks (measured: at 70M capacity 2048 beats 4096 by
        // 15 us, at 333M it loses by 120 us)
        if (NV == 1 && max_n > ((int64_t)1 << 22))
            *err = radix_pass<16, NV>(K[cur], K[cur ^ 1], va, max_n, d_n, shift, bits, hist,
                                      scan_scratch, flags, st);
        else if (NV == 3 && max_n > ((int64_t)1 << 27))
            *err = radix_pass<16, NV>(K[cur], K[cur ^ 1], va, max_n, d_n, shift, bits, hist,
                                      scan_scratch, flags, st);
        else
            *err = radix_pass<8, NV>(K[cur], K[cur ^ 1], va, max_n, d_n, shift, bits, hist,
                                     scan_scratch, flags, st);
        if (*err != hipSuccess) return cur;
        shift += bits;
        cur ^= 1;
    }
    return cur;
}

}  // namespace

int radix_sort_pairs(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t max_n,
                     const uint32_t* d_n, int lo, int hi, uint32_t* hist, uint32_t* scan_scratch,
                     uint32_t* flags, hipStream_t st, hipError_t* err) {
    uint32_t* K[2] = {ka, kb};
    uint32_t* V[1][2] = {{va, vb}};
    return radix_sort_impl<1>(K, V, max_n, d_n, lo, hi, hist, scan_scratch, flags, st, err);
}

int radix_sort_kv3(uint32_t* K[2], uint32_t* V[3][2], int64_t max_n, const uint32_t* d_n, int lo,
                   int hi, uint32_t* hist, uint32_t* scan_scratch, uint32_t* flags, hipStream_t st,
                   hipError_t* err) {
    return radix_sort_impl<3>(K, V, max_n, d_n, lo, hi, hist, scan_scratch, flags, st, err);
}

}  // namespace gs
