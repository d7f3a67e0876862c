// Gaussians from SfM points: mean = the point, an isotropic scale equal to
// the mean distance to its k nearest other points, identity rotation, one
// opacity, and the point's colour in the degree-0 SH band.
//
// The k nearest neighbours are exact and come from a bounding-volume
// hierarchy over the points in Morton order (10 bits per axis over the
// bounding cube).  Leaves hold kLeaf consecutive points of that order; the
// tree over the leaves is complete and implicit (heap numbering: node v has
// children 2v and 2v+1, the leaves are NL..2NL-1, padded with empty boxes) and
// stores each node's axis-aligned box of its points.  Because the boxes are
// the points' own boxes and the leaves split by count, not by space, the
// search adapts to the density: clustered scenes (dense blobs next to sparse
// outliers) cost about the same per point as uniform ones.  Each point first
// takes the kWin points on either side of it in the sorted order (almost
// always near it) as candidates, which bounds its k-th distance, then walks
// the tree depth first without a stack (left child first; after a subtree,
// climb while on a right child, then step to the sibling) and skips every
// box farther than the current k-th distance.  The box distance is computed
// with the same float operations as the point distances and is monotone in
// them, so no point nearer than the bound is ever skipped.
#include <math.h>

#include <algorithm>

#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxK = GS_INIT_MAX_K;
constexpr int kLeaf = 8;           // points per leaf
constexpr int kWin = 8;            // sorted neighbours taken on each side first
constexpr int kBoxBlocks = 1024;   // blocks of the bounding-box reduction
constexpr int kUpBlock = 256;      // nodes per block in the bottom-up box pass
constexpr float kSMin = 1e-7f;     // smallest scale (coincident points)

static_assert(2 * kWin >= kMaxK, "the window must hold k candidates");

// Morton cells: origin and 1024 / (side of the bounding cube)
struct Grid {
    float ox, oy, oz, ih;
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

// The Morton grid: 1024 cells per axis over the bounding cube (the order only
// serves locality; the search does not depend on the cells).
__global__ void k_grid(const float* __restrict__ part, int nb, Grid* __restrict__ g) {
    if (threadIdx.x != 0) return;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < nb; b++)
        for (int a = 0; a < 3; a++) {
            lo[a] = fminf(lo[a], part[6 * b + a]);
            hi[a] = fmaxf(hi[a], part[6 * b + 3 + a]);
        }
    const float e = fmaxf(hi[0] - lo[0], fmaxf(hi[1] - lo[1], hi[2] - lo[2]));
    Grid G;
    G.ox = lo[0];
    G.oy = lo[1];
    G.oz = lo[2];
    G.ih = (e > 0.f && e < INFINITY) ? 1024.f / e : 0.f;  // all points coincide: one cell
    *g = G;
}

__device__ __forceinline__ uint32_t cell_of(float v, float o, float ih) {
    const float c = (v - o) * ih;
    return c >= 1023.f ? 1023u : (c > 0.f ? (uint32_t)c : 0u);  // NaN goes to 0
}

// 10 bits spread to every third bit
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 1023u;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ __launch_bounds__(kBlock) void k_cell_keys(const float* __restrict__ pts, int n,
                                                      const Grid* __restrict__ gp,
                                                      uint32_t* __restrict__ keys,
                                                      uint32_t* __restrict__ vals) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const Grid g = *gp;
    const uint32_t cx = cell_of(pts[3 * (int64_t)i], g.ox, g.ih);
    const uint32_t cy = cell_of(pts[3 * (int64_t)i + 1], g.oy, g.ih);
    const uint32_t cz = cell_of(pts[3 * (int64_t)i + 2], g.oz, g.ih);
    keys[i] = spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2);
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

// leaf boxes: tree[2v] = (min x, y, z, -), tree[2v + 1] = (max x, y, z, -);
// padded leaves get an empty box (+inf, -inf), which every bound skips
__global__ __launch_bounds__(kBlock) void k_leaf_box(const float4* __restrict__ sp, int n, int NL,
                                                     float4* __restrict__ tree) {
    const int l = blockIdx.x * kBlock + threadIdx.x;
    if (l >= NL) return;
    float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
    float4 hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
    const int a = l * kLeaf, b = min(n, a + kLeaf);
    for (int i = a; i < b; i++) {
        const float4 p = sp[i];
        lo.x = fminf(lo.x, p.x);
        lo.y = fminf(lo.y, p.y);
        lo.z = fminf(lo.z, p.z);
        hi.x = fmaxf(hi.x, p.x);
        hi.y = fmaxf(hi.y, p.y);
        hi.z = fmaxf(hi.z, p.z);
    }
    tree[2 * (int64_t)(NL + l)] = lo;
    tree[2 * (int64_t)(NL + l) + 1] = hi;
}

// Boxes of the inner nodes from their children, up to nine levels per launch:
// block b makes the nodes m + 256 b .. m + 256 b + 255 of level [m, 2m) (the
// level below is done), then their parents from its own results in LDS, and
// so on while it holds more than one node.  m is a power of two.
__global__ __launch_bounds__(kUpBlock) void k_tree_up(float4* __restrict__ tree, int m) {
    __shared__ float4 slo[kUpBlock], shi[kUpBlock];
    const int t = threadIdx.x;
    int cnt = min(kUpBlock, m);
    int base = m + blockIdx.x * kUpBlock;
    float4 lo, hi;
    if (t < cnt) {
        const int64_t c = 2 * (int64_t)(base + t);
        const float4 l0 = tree[2 * c], h0 = tree[2 * c + 1], l1 = tree[2 * c + 2], h1 = tree[2 * c + 3];
        lo = make_float4(fminf(l0.x, l1.x), fminf(l0.y, l1.y), fminf(l0.z, l1.z), 0.f);
        hi = make_float4(fmaxf(h0.x, h1.x), fmaxf(h0.y, h1.y), fmaxf(h0.z, h1.z), 0.f);
        tree[2 * (int64_t)(base + t)] = lo;
        tree[2 * (int64_t)(base + t) + 1] = hi;
        slo[t] = lo;
        shi[t] = hi;
    }
    while (cnt > 1) {
        __syncthreads();
        cnt >>= 1;
        base >>= 1;
        if (t < cnt) {
            const float4 l0 = slo[2 * t], h0 = shi[2 * t], l1 = slo[2 * t + 1], h1 = shi[2 * t + 1];
            lo = make_float4(fminf(l0.x, l1.x), fminf(l0.y, l1.y), fminf(l0.z, l1.z), 0.f);
            hi = make_float4(fmaxf(h0.x, h1.x), fmaxf(h0.y, h1.y), fmaxf(h0.z, h1.z), 0.f);
        }
        __syncthreads();
        if (t < cnt) {
            slo[t] = lo;
            shi[t] = hi;
            tree[2 * (int64_t)(base + t)] = lo;
            tree[2 * (int64_t)(base + t) + 1] = hi;
        }
    }
}

__device__ __forceinline__ float dist2(float4 o, float4 p) {
    const float dx = o.x - p.x, dy = o.y - p.y, dz = o.z - p.z;
    return __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
}

// squared distance from p to a box; for any point q in the box each axis
// difference is at least the box's, in float too (rounding is monotone), so
// this never exceeds dist2(q, p)
__device__ __forceinline__ float box_dist2(float4 lo, float4 hi, float4 p) {
    const float ex = fmaxf(fmaxf(lo.x - p.x, p.x - hi.x), 0.f);
    const float ey = fmaxf(fmaxf(lo.y - p.y, p.y - hi.y), 0.f);
    const float ez = fmaxf(fmaxf(lo.z - p.z, p.z - hi.z), 0.f);
    return __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez));
}

// one thread per point, in sorted order; the mean of the k nearest distances
// goes to s[original index].  With n <= 2 kWin + 1 the window holds every
// point and there is no tree.
template <int K>
__global__ __launch_bounds__(kBlock) void k_knn(const uint32_t* __restrict__ vals,
                                                const float4* __restrict__ sp, int n, int k,
                                                const float4* __restrict__ tree, int NL,
                                                float* __restrict__ s) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const float4 p = sp[j];
    const int kk = min(k, n - 1);
    TopK<K> best;
    best.init();
    const int j1 = min(n - 1, max(j - kWin, 0) + 2 * kWin);
    const int j0 = max(0, j1 - 2 * kWin);
    for (int i = j0; i <= j1; i++)
        if (i != j) best.push(dist2(sp[i], p));
    float bound = kk > 0 ? best.at(kk - 1) : 0.f;
    if (n > 2 * kWin + 1 && bound > 0.f) {
        int v = 1;
        while (true) {
            bool go = box_dist2(tree[2 * (int64_t)v], tree[2 * (int64_t)v + 1], p) <= bound;
            if (go && v >= NL) {
                const int a = (v - NL) * kLeaf, b = min(n, a + kLeaf);
                for (int i = a; i < b; i++)
                    if (i < j0 || i > j1) best.push(dist2(sp[i], p));
                bound = best.at(kk - 1);
                go = false;
            }
            if (go) {
                v = 2 * v;
                continue;
            }
            while (v & 1) v >>= 1;  // finished a right child: climb
            if (v == 0) break;      // climbed past the root
            v += 1;                 // the right sibling
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
    hipLaunchKernelGGL(k_grid, dim3(1), dim3(64), 0, st, part, nb, grid);
    const unsigned g = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_cell_keys, dim3(g), dim3(kBlock), 0, st, pts, n, grid, c->pk[0], c->pv[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int side = radix_sort_pairs(c->pk[0], c->pv[0], c->pk[1], c->pv[1], n, nullptr, 0, 30,
                                      c->hist, c->scan_scratch, c->diag + kDiagFlags, st, &e);
    if (e != hipSuccess) return e;
    const uint32_t* vals = c->pv[side];
    // sorted points, then the tree, in the record buffer (12 floats per pair):
    // 16 n bytes and 32 * 2 NL <= 16 n + 48 bytes (NL < 2 ceil(n / 8))
    float4* sp = reinterpret_cast<float4*>(c->rec);
    float4* tree = sp + n;
    float* s = reinterpret_cast<float*>(c->cnt);
    hipLaunchKernelGGL(k_gather, dim3(g), dim3(kBlock), 0, st, pts, n, vals, sp);
    int NL = 0;
    if (n > 2 * kWin + 1) {
        const int nl = (n + kLeaf - 1) / kLeaf;
        NL = 1;
        while (NL < nl) NL *= 2;
        hipLaunchKernelGGL(k_leaf_box, dim3((NL + kBlock - 1) / kBlock), dim3(kBlock), 0, st, sp, n, NL,
                           tree);
        for (int m = NL / 2; m >= 1; m /= 2 * kUpBlock)
            hipLaunchKernelGGL(k_tree_up, dim3(std::max(1, m / kUpBlock)), dim3(kUpBlock), 0, st, tree, m);
    }
    if (k <= 4)
        hipLaunchKernelGGL(k_knn<4>, dim3(g), dim3(kBlock), 0, st, vals, sp, n, k, tree, NL, s);
    else
        hipLaunchKernelGGL(k_knn<kMaxK>, dim3(g), dim3(kBlock), 0, st, vals, sp, n, k, tree, NL, s);
    const float lg = logf(opacity / (1.f - opacity));
    const int K = (sh_degree + 1) * (sh_degree + 1);
    hipLaunchKernelGGL(k_init_write, dim3(g), dim3(kBlock), 0, st, pts, rgb, n, K, lg, s, means,
                       log_scales, quats, logit, sh);
    return hipGetLastError();
}

}  // namespace gs
