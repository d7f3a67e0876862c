// The stochastic density control of the joint step (MCMC densification):
// relocation of dead Gaussians onto live ones drawn in proportion to their
// opacity, with the opacity and scale rule that keeps a source's combined
// contribution, and the noise added to the means after an update.  The
// random numbers come in as arguments.
//
// Draws are exact integer arithmetic: each live Gaussian weighs
// floor(o 2^24) (o from the logit in double), the weights' inclusive prefix
// sums are 64-bit (a block pass, one workgroup for the block totals, a block
// pass again), and dead Gaussian j takes the first index whose prefix exceeds
// floor(u_j W), found by binary search.
#include <math.h>

#include <algorithm>

#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kBlock = 1024;      // items (and threads) per block of the prefix sums
constexpr int kMaxCopies = 51;    // copies counted in the opacity and scale rule
constexpr double kWeightScale = 16777216.0;  // 2^24

struct McState {
    float* p[5];
    float* m[5];
    float* v[5];
    int rows[5];
    int N;
};

__device__ __forceinline__ double opacity_of(float logit) { return 1.0 / (1.0 + exp(-(double)logit)); }

__device__ __forceinline__ uint64_t block_incl_scan_u64(uint64_t v, uint64_t* s, uint64_t& total) {
    // inclusive scan over kBlock threads: waves by shuffles, then the waves' totals
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t t = __shfl_up(v, off, kWave);
        if (lane >= off) v += t;
    }
    if (lane == kWave - 1) s[w] = v;
    __syncthreads();
    uint64_t before = 0, tot = 0;
    for (int q = 0; q < kBlock / kWave; q++) {
        if (q < w) before += s[q];
        tot += s[q];
    }
    __syncthreads();
    total = tot;
    return v + before;
}

// per item: its weight; per block: the sum
__global__ __launch_bounds__(kBlock) void k_mc_weights(const float* __restrict__ logit, int N, float t_dead,
                                                       uint64_t* __restrict__ cdf,
                                                       uint64_t* __restrict__ bsum) {
    __shared__ uint64_t s[kBlock / kWave];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    uint64_t w = 0;
    if (i < N) {
        const double o = opacity_of(logit[i]);
        if (o > (double)t_dead) w = (uint64_t)floor(o * kWeightScale);
    }
    uint64_t tot;
    const uint64_t inc = block_incl_scan_u64(w, s, tot);
    if (i < N) cdf[i] = inc;  // the block-local prefix; the block offset is added below
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// one workgroup: exclusive prefix of the block sums, the total last
__global__ __launch_bounds__(kBlock) void k_mc_block_offsets(uint64_t* __restrict__ bsum, int nb) {
    __shared__ uint64_t s[kBlock / kWave];
    uint64_t carry = 0;
    for (int base = 0; base < nb; base += kBlock) {
        const int b = base + threadIdx.x;
        const uint64_t v = b < nb ? bsum[b] : 0;
        uint64_t tot;
        const uint64_t inc = block_incl_scan_u64(v, s, tot);
        if (b < nb) bsum[b] = carry + inc - v;
        carry += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(kBlock) void k_mc_cdf(uint64_t* __restrict__ cdf, int N,
                                                   const uint64_t* __restrict__ bsum,
                                                   uint32_t* __restrict__ count) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < N) {
        cdf[i] += bsum[blockIdx.x];
        count[i] = 0u;
    }
}

// each dead Gaussian draws its source
__global__ __launch_bounds__(kBlock) void k_mc_draw(const float* __restrict__ logit, int N, float t_dead,
                                                    const float* __restrict__ u,
                                                    const uint64_t* __restrict__ cdf,
                                                    const uint64_t* __restrict__ total_p,
                                                    int32_t* __restrict__ src, uint32_t* __restrict__ count,
                                                    int32_t* __restrict__ n_moved) {
    __shared__ int s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < N) {
        const uint64_t W = *total_p;
        int s = -1;
        if (W > 0 && !(opacity_of(logit[i]) > (double)t_dead)) {
            const uint64_t tv = (uint64_t)floor((double)u[i] * (double)W);
            int lo = 0, hi = N;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (cdf[mid] > tv) hi = mid;
                else lo = mid + 1;
            }
            s = min(lo, N - 1);
            atomicAdd(&count[s], 1u);
            atomicAdd(&s_cnt, 1);
        }
        src[i] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt && n_moved) atomicAdd(n_moved, s_cnt);
}

__device__ __forceinline__ void reset_moments(const McState& st, int i) {
#pragma unroll
    for (int q = 0; q < 5; q++)
        for (int r = 0; r < st.rows[q]; r++) {
            st.m[q][(int64_t)r * st.N + i] = 0.f;
            st.v[q][(int64_t)r * st.N + i] = 0.f;
        }
}

// sources: the opacity and scale of their n copies
__global__ __launch_bounds__(256) void k_mc_sources(McState st, const uint32_t* __restrict__ count) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= st.N || count[i] == 0u) return;
    const int n = (int)min(count[i] + 1u, (uint32_t)kMaxCopies);
    const double o = opacity_of(st.p[3][i]);
    const double op = 1.0 - pow(1.0 - o, 1.0 / n);
    double denom = 0.0;
    for (int a = 1; a <= n; a++) {
        double c = 1.0, pw = op;  // C(a-1, k), op^(k+1)
        for (int k = 0; k <= a - 1; k++) {
            denom += ((k & 1) ? -c : c) * pw * rsqrt((double)(k + 1));
            c = c * (double)(a - 1 - k) / (double)(k + 1);
            pw *= op;
        }
    }
    const double lf = log(o / denom);
    st.p[3][i] = (float)log(op / (1.0 - op));
#pragma unroll
    for (int a = 0; a < 3; a++) {
        float& ls = st.p[1][(int64_t)a * st.N + i];
        ls = (float)((double)ls + lf);
    }
    reset_moments(st, i);
}

// dead Gaussians: copies of their (updated) source
__global__ __launch_bounds__(256) void k_mc_copy(McState st, const int32_t* __restrict__ src) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= st.N) return;
    const int s = src[i];
    if (s < 0) return;
#pragma unroll
    for (int q = 0; q < 5; q++)
        for (int r = 0; r < st.rows[q]; r++)
            st.p[q][(int64_t)r * st.N + i] = st.p[q][(int64_t)r * st.N + s];
    reset_moments(st, i);
}

// mu += scale sigmoid(-k (o - t)) Sigma eta
__global__ __launch_bounds__(256) void k_mc_noise(float* __restrict__ means, const float* __restrict__ ls,
                                                  const float* __restrict__ quats,
                                                  const float* __restrict__ logit, int N,
                                                  const float* __restrict__ eta, float scale, float k,
                                                  float t) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    float q[4];
    float qn = 0.f;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        q[a] = quats[(int64_t)a * N + i];
        qn += q[a] * q[a];
    }
    const float iq = rsqrtf(qn);
    const float w = q[0] * iq, x = q[1] * iq, y = q[2] * iq, z = q[3] * iq;
    const float R[9] = {1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
                        2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
                        2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)};
    float s2[3];
#pragma unroll
    for (int a = 0; a < 3; a++) s2[a] = expf(2.f * ls[(int64_t)a * N + i]);
    const float o = 1.f / (1.f + expf(-logit[i]));
    const float gate = 1.f / (1.f + expf(k * (o - t)));
    const float e[3] = {eta[i], eta[(int64_t)N + i], eta[2 * (int64_t)N + i]};
    // Sigma eta = R diag(s^2) R^T eta
    float rt[3];
#pragma unroll
    for (int c = 0; c < 3; c++) rt[c] = s2[c] * (R[c] * e[0] + R[3 + c] * e[1] + R[6 + c] * e[2]);
#pragma unroll
    for (int a = 0; a < 3; a++)
        means[(int64_t)a * N + i] += scale * gate * (R[3 * a] * rt[0] + R[3 * a + 1] * rt[1] + R[3 * a + 2] * rt[2]);
}

}  // namespace

hipError_t launch_mcmc_relocate(Ctx* c, const gs_gaussian_adam* state, int N, int sh_degree,
                                const float* u, float t_dead, int32_t* src, int32_t* n_moved,
                                hipStream_t st) {
    if (N <= 0) return hipSuccess;
    McState s;
    const int K = (sh_degree + 1) * (sh_degree + 1);
    const int rows[5] = {3, 3, 4, 1, 3 * K};
    for (int q = 0; q < 5; q++) {
        s.p[q] = state->params[q];
        s.m[q] = state->exp_avg[q];
        s.v[q] = state->exp_avg_sq[q];
        s.rows[q] = rows[q];
    }
    s.N = N;
    // workspace in the record buffer: cdf (8 B per item), counts (4 B), block
    // sums; the caller's src array, or one in the workspace
    char* base = reinterpret_cast<char*>(c->rec);
    uint64_t* cdf = reinterpret_cast<uint64_t*>(base);
    uint32_t* count = reinterpret_cast<uint32_t*>(base + 8 * (size_t)N);
    int32_t* srcw = reinterpret_cast<int32_t*>(base + 12 * (size_t)N);
    uint64_t* bsum = reinterpret_cast<uint64_t*>(base + 16 * (size_t)((N + 1) / 2 * 2));
    if (!src) src = srcw;
    const int nb = (N + kBlock - 1) / kBlock;
    if (n_moved) {
        hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(n_moved), 0u, 1, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_mc_weights, dim3(nb), dim3(kBlock), 0, st, s.p[3], N, t_dead, cdf, bsum);
    hipLaunchKernelGGL(k_mc_block_offsets, dim3(1), dim3(kBlock), 0, st, bsum, nb);
    hipLaunchKernelGGL(k_mc_cdf, dim3(nb), dim3(kBlock), 0, st, cdf, N, bsum, count);
    hipLaunchKernelGGL(k_mc_draw, dim3(nb), dim3(kBlock), 0, st, s.p[3], N, t_dead, u, cdf, bsum + nb, src,
                       count, n_moved);
    const unsigned g = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(k_mc_sources, dim3(g), dim3(256), 0, st, s, count);
    hipLaunchKernelGGL(k_mc_copy, dim3(g), dim3(256), 0, st, s, src);
    return hipGetLastError();
}

hipError_t launch_mcmc_noise(float* means, const float* log_scales, const float* quats,
                             const float* logit, int N, const float* eta, float scale, float k, float t,
                             hipStream_t st) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mc_noise, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, means, log_scales,
                       quats, logit, N, eta, scale, k, t);
    return hipGetLastError();
}

}  // namespace gs
