// Gaussians from SfM points: mean = the point, an isotropic scale equal to
// the mean distance to its k nearest other points, identity rotation, one
// opacity, and the point's colour in the degree-0 SH band.
//
// The k nearest neighbours come from a uniform grid: the points' bounding box
// is cut into cubic cells of side h (about four points per cell on average),
// the points are sorted by cell id (x fastest), and each point visits the
// cells around its own in shells of growing Chebyshev radius r.  Once it holds
// k candidates and the k-th distance is at most r h, no point outside the
// shells seen can be nearer (every such point lies at least r h away), so the
// search stops: the result is exact.  In the sorted order the cells of one
// grid row are contiguous, so a shell is a set of row ranges, each found by
// one binary search.  A point still short of that after kMaxRing shells (an
// outlier far from the rest) falls back to a scan of all points.  Points are
// processed in sorted order and gathered into it first, so neighbouring
// threads read the same cells.
#include <math.h>

#include <algorithm>

#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxK = GS_INIT_MAX_K;
constexpr int kMaxRing = 6;
constexpr int kMaxDim = 1024;       // cells per axis (ids fit in 30 bits)
constexpr int kBoxBlocks = 1024;    // blocks of the bounding-box reduction
constexpr float kSMin = 1e-7f;      // smallest scale (coincident points)

struct Grid {
    float ox, oy, oz, h, ih;
    int nx, ny, nz;
};

// per block: min and max of x, y, z
__global__ __launch_bounds__(kBlock) void k_box_partial(const float* __restrict__ pts, int n,
                                                        float* __restrict__ part) {
    __shared__ float s[6][kBlock / kWave];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const float v = pts[3 * (int64_t)i + a];
            lo[a] = fminf(lo[a], v);
            hi[a] = fmaxf(hi[a], v);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; a++)
        for (int off = 32; off > 0; off >>= 1) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], off, kWave));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off, kWave));
        }
    const int w = threadIdx.x / kWave;
    if (__lane_id() == 0)
        for (int a = 0; a < 3; a++) {
            s[a][w] = lo[a];
            s[3 + a][w] = hi[a];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        const bool mx = threadIdx.x >= 3;
        float v = s[threadIdx.x][0];
        for (int q = 1; q < kBlock / kWave; q++) v = mx ? fmaxf(v, s[threadIdx.x][q]) : fminf(v, s[threadIdx.x][q]);
        part[6 * blockIdx.x + threadIdx.x] = v;
    }
}

// The grid: cell side from the box volume per point (about four points per
// cell), at most kMaxDim cells per axis.
__global__ void k_grid(const float* __restrict__ part, int nb, int n, Grid* __restrict__ g) {
    if (threadIdx.x != 0) return;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < nb; b++)
        for (int a = 0; a < 3; a++) {
            lo[a] = fminf(lo[a], part[6 * b + a]);
            hi[a] = fmaxf(hi[a], part[6 * b + 3 + a]);
        }
    const float ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    const float emax = fmaxf(ex, fmaxf(ey, ez));
    // a degenerate box (a plane, a line, a point) still gets a positive volume
    const float fl = fmaxf(emax * 1e-3f, 1e-20f);
    const double vol = (double)fmaxf(ex, fl) * fmaxf(ey, fl) * fmaxf(ez, fl);
    float h = (float)cbrt(4.0 * vol / (double)(n > 0 ? n : 1));
    h = fmaxf(h, emax / (float)(kMaxDim - 1));
    if (!(h > 0.f)) h = 1.f;  // all points coincide
    Grid G;
    G.ox = lo[0];
    G.oy = lo[1];
    G.oz = lo[2];
    G.h = h;
    G.ih = 1.f / h;
    G.nx = min((int)(ex * G.ih) + 1, kMaxDim);
    G.ny = min((int)(ey * G.ih) + 1, kMaxDim);
    G.nz = min((int)(ez * G.ih) + 1, kMaxDim);
    *g = G;
}

__device__ __forceinline__ int cell_of(float v, float o, float ih, int nd) {
    return min(max((int)((v - o) * ih), 0), nd - 1);
}

__global__ __launch_bounds__(kBlock) void k_cell_keys(const float* __restrict__ pts, int n,
                                                      const Grid* __restrict__ gp,
                                                      uint32_t* __restrict__ keys,
                                                      uint32_t* __restrict__ vals) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const Grid g = *gp;
    const int cx = cell_of(pts[3 * (int64_t)i], g.ox, g.ih, g.nx);
    const int cy = cell_of(pts[3 * (int64_t)i + 1], g.oy, g.ih, g.ny);
    const int cz = cell_of(pts[3 * (int64_t)i + 2], g.oz, g.ih, g.nz);
    keys[i] = (uint32_t)cx + (uint32_t)g.nx * ((uint32_t)cy + (uint32_t)g.ny * (uint32_t)cz);
    vals[i] = (uint32_t)i;
}

// points in sorted order (x, y, z, -)
__global__ __launch_bounds__(kBlock) void k_gather(const float* __restrict__ pts, int n,
                                                   const uint32_t* __restrict__ vals,
                                                   float4* __restrict__ sp) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int64_t q = vals[j];
    sp[j] = make_float4(pts[3 * q], pts[3 * q + 1], pts[3 * q + 2], 0.f);
}

__device__ __forceinline__ int lower_bound(const uint32_t* __restrict__ a, int n, uint32_t key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// the K smallest squared distances seen, ascending (K >= k: the first k of
// them are the k nearest)
template <int K>
struct TopK {
    float d[K];
    int cnt;
    __device__ void init() {
#pragma unroll
        for (int i = 0; i < K; i++) d[i] = INFINITY;
        cnt = 0;
    }
    __device__ void push(float v) {
        if (!(v < d[K - 1])) return;
        float x = v;
#pragma unroll
        for (int i = 0; i < K; i++) {
            if (x < d[i]) {
                const float t = d[i];
                d[i] = x;
                x = t;
            }
        }
        cnt = min(cnt + 1, K);
    }
    // the i-th smallest (i < K), by selects (no dynamic register index)
    __device__ float at(int i) const {
        float r = d[0];
#pragma unroll
        for (int q = 1; q < K; q++) r = q == i ? d[q] : r;
        return r;
    }
};

template <int K>
__device__ __forceinline__ void scan_range(const uint32_t* __restrict__ keys,
                                           const float4* __restrict__ sp, int n, uint32_t k0,
                                           uint32_t k1, int self, float4 p, TopK<K>& best) {
    for (int j = lower_bound(keys, n, k0); j < n && keys[j] <= k1; j++) {
        if (j == self) continue;
        const float4 o = sp[j];
        const float dx = o.x - p.x, dy = o.y - p.y, dz = o.z - p.z;
        best.push(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)));
    }
}

// one thread per point, in sorted order; the mean of the k nearest distances
// goes to s[original index]
template <int K>
__global__ __launch_bounds__(kBlock) void k_knn(const uint32_t* __restrict__ keys,
                                                const uint32_t* __restrict__ vals,
                                                const float4* __restrict__ sp, int n, int k,
                                                const Grid* __restrict__ gp, float* __restrict__ s) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const Grid g = *gp;
    const float4 p = sp[j];
    const uint32_t key = keys[j];
    const int cx = (int)(key % (uint32_t)g.nx);
    const int cy = (int)((key / (uint32_t)g.nx) % (uint32_t)g.ny);
    const int cz = (int)(key / ((uint32_t)g.nx * (uint32_t)g.ny));
    const int kk = min(k, n - 1);
    TopK<K> best;
    best.init();
    bool done = kk <= 0;
    // a point outside the shells seen so far is at least r h away; the margin
    // covers the rounding of the cell assignment
    for (int r = 0; r <= kMaxRing && !done; r++) {
        for (int dz = -r; dz <= r; dz++) {
            const int z = cz + dz;
            if (z < 0 || z >= g.nz) continue;
            for (int dy = -r; dy <= r; dy++) {
                const int y = cy + dy;
                if (y < 0 || y >= g.ny) continue;
                const uint32_t row = (uint32_t)g.nx * ((uint32_t)y + (uint32_t)g.ny * (uint32_t)z);
                if (dz == -r || dz == r || dy == -r || dy == r) {
                    const int x0 = max(cx - r, 0), x1 = min(cx + r, g.nx - 1);
                    scan_range<K>(keys, sp, n, row + x0, row + x1, j, p, best);
                } else {
                    if (cx - r >= 0) scan_range<K>(keys, sp, n, row + cx - r, row + cx - r, j, p, best);
                    if (cx + r < g.nx) scan_range<K>(keys, sp, n, row + cx + r, row + cx + r, j, p, best);
                }
            }
        }
        const float reach = (float)r * g.h * (1.f - 1e-4f);
        done = best.cnt >= kk && best.at(kk - 1) <= reach * reach;
        // every cell of the grid seen: nothing is left
        if (cx - r <= 0 && cy - r <= 0 && cz - r <= 0 && cx + r >= g.nx - 1 && cy + r >= g.ny - 1 &&
            cz + r >= g.nz - 1)
            done = true;
    }
    if (!done) {
        best.init();
        for (int i = 0; i < n; i++) {
            if (i == j) continue;
            const float4 o = sp[i];
            const float dx = o.x - p.x, dy = o.y - p.y, dz = o.z - p.z;
            best.push(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz)));
        }
    }
    float m = 0.f;
#pragma unroll
    for (int i = 0; i < K; i++) m += i < kk ? sqrtf(best.d[i]) : 0.f;
    m = kk > 0 ? m / (float)kk : 0.f;
    s[vals[j]] = fmaxf(m, kSMin);
}

// the Gaussians, coalesced in the original order
__global__ __launch_bounds__(kBlock) void k_init_write(const float* __restrict__ pts,
                                                       const float* __restrict__ rgb, int n, int K,
                                                       float opacity_logit,
                                                       const float* __restrict__ s,
                                                       float* __restrict__ means,
                                                       float* __restrict__ log_scales,
                                                       float* __restrict__ quats,
                                                       float* __restrict__ logit,
                                                       float* __restrict__ sh) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    // rgb = 0.5 + C0 sh_0 with C0 = 1 / (2 sqrt(pi)), the renderer's colour rule
    constexpr float kInvC0 = 3.5449077018110318f;  // 2 sqrt(pi)
    const float ls = logf(s[i]);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        means[(int64_t)a * n + i] = pts[3 * (int64_t)i + a];
        log_scales[(int64_t)a * n + i] = ls;
    }
    quats[i] = 1.f;
    quats[(int64_t)n + i] = 0.f;
    quats[2 * (int64_t)n + i] = 0.f;
    quats[3 * (int64_t)n + i] = 0.f;
    logit[i] = opacity_logit;
    for (int c = 0; c < K; c++)
#pragma unroll
        for (int ch = 0; ch < 3; ch++)
            sh[((int64_t)c * 3 + ch) * n + i] = c == 0 ? (rgb[3 * (int64_t)i + ch] - 0.5f) * kInvC0 : 0.f;
}

}  // namespace

hipError_t launch_init_gaussians(Ctx* c, const float* pts, const float* rgb, int n, int k,
                                 float opacity, int sh_degree, float* means, float* log_scales,
                                 float* quats, float* logit, float* sh, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int nb = std::min((n + kBlock - 1) / kBlock, kBoxBlocks);
    float* part = c->aux;
    Grid* grid = reinterpret_cast<Grid*>(c->aux + 6 * kBoxBlocks);
    hipLaunchKernelGGL(k_box_partial, dim3(nb), dim3(kBlock), 0, st, pts, n, part);
    hipLaunchKernelGGL(k_grid, dim3(1), dim3(64), 0, st, part, nb, n, grid);
    const unsigned g = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_cell_keys, dim3(g), dim3(kBlock), 0, st, pts, n, grid, c->pk[0], c->pv[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int side = radix_sort_pairs(c->pk[0], c->pv[0], c->pk[1], c->pv[1], n, nullptr, 0, 30,
                                      c->hist, c->scan_scratch, c->diag + kDiagFlags, st, &e);
    if (e != hipSuccess) return e;
    const uint32_t* keys = c->pk[side];
    const uint32_t* vals = c->pv[side];
    float4* sp = reinterpret_cast<float4*>(c->rec);
    float* s = reinterpret_cast<float*>(c->cnt);
    hipLaunchKernelGGL(k_gather, dim3(g), dim3(kBlock), 0, st, pts, n, vals, sp);
    if (k <= 4)
        hipLaunchKernelGGL(k_knn<4>, dim3(g), dim3(kBlock), 0, st, keys, vals, sp, n, k, grid, s);
    else
        hipLaunchKernelGGL(k_knn<kMaxK>, dim3(g), dim3(kBlock), 0, st, keys, vals, sp, n, k, grid, s);
    const float lg = logf(opacity / (1.f - opacity));
    const int K = (sh_degree + 1) * (sh_degree + 1);
    hipLaunchKernelGGL(k_init_write, dim3(g), dim3(kBlock), 0, st, pts, rgb, n, K, lg, s, means,
                       log_scales, quats, logit, sh);
    return hipGetLastError();
}

}  // namespace gs
