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
};

struct RasterParams {
    float alpha_min, alpha_max, t_min;
    float near_plane, eps2d, fov_pad;
    int tile_w, tile_h;
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

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ int wave_max_i(int v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    return v;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Gaussian falloff exponent sigma = 0.5 (A dx^2 + C dy^2) + B dx dy with a
// fixed operation order, shared by the forward and the backward raster so both
// take identical alpha-gate decisions.
__device__ __forceinline__ float splat_sigma(float A, float B, float C, float dx, float dy) {
    const float q = __builtin_fmaf(A * dx, dx, C * dy * dy);
    return __builtin_fmaf(B * dx, dy, 0.5f * q);
}

__device__ __forceinline__ float fast_exp_neg(float s) {
    // e^-s = 2^(-s log2 e) on the hardware exp2
    return __builtin_amdgcn_exp2f(-s * 1.4426950408889634f);
}

// Minimum of sigma(d) over the rectangle [x0,x1]x[y0,y1] of pixel centres for a
// splat at (mx,my): 0 if the centre is inside, else the smallest value on the
// four edges (sigma is convex).
__device__ __forceinline__ float edge_min_x(float A, float B, float C, float fx, float lo, float hi) {
    // x fixed at fx, y in [lo,hi]: 0.5 A fx^2 + B fx y + 0.5 C y^2
    float y = fminf(fmaxf(-B * fx / C, lo), hi);
    return 0.5f * (A * fx * fx + C * y * y) + B * fx * y;
}
__device__ __forceinline__ float edge_min_y(float A, float B, float C, float fy, float lo, float hi) {
    float x = fminf(fmaxf(-B * fy / A, lo), hi);
    return 0.5f * (A * x * x + C * fy * fy) + B * x * fy;
}
__device__ __forceinline__ float rect_sigma_min(float A, float B, float C, float mx, float my,
                                                float x0, float x1, float y0, float y1) {
    if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return 0.f;
    const float lx = x0 - mx, hx = x1 - mx, ly = y0 - my, hy = y1 - my;
    float q = edge_min_x(A, B, C, lx, ly, hy);
    q = fminf(q, edge_min_x(A, B, C, hx, ly, hy));
    q = fminf(q, edge_min_y(A, B, C, ly, lx, hx));
    q = fminf(q, edge_min_y(A, B, C, hy, lx, hx));
    return q;
}

// Iterate the tiles of view `v` met by the splat's alpha >= alpha_min ellipse.
// `fn(tile_local)` is called in row-major order.  Shared by the counting and the
// emitting pass so both see exactly the same tiles.
template <typename F>
__device__ __forceinline__ int for_each_tile(const float4& a, const float4& b, int W, int H,
                                             int gx, int TW, int TH, float alpha_min, F&& fn) {
    const float mx = a.x, my = a.y, o = a.w;
    const float A = b.x, B = b.y, C = b.z;
    const float thr = __logf(o / alpha_min);
    // conservative threshold: a splat is kept in a tile if its minimum exponent
    // there is within a relative 1e-4 (plus 1e-4) of the gate
    const float thr_c = thr * 1.0001f + 1e-4f;
    const float detc = A * C - B * B;
    const float sxx = C / detc, syy = A / detc;  // Sigma2D diagonal
    const float ex = sqrtf(2.f * thr_c * sxx) + 0.01f;
    const float ey = sqrtf(2.f * thr_c * syy) + 0.01f;
    const int gy = (H + TH - 1) / TH;
    int tx0 = (int)floorf((mx - ex) / TW), tx1 = (int)floorf((mx + ex) / TW);
    int ty0 = (int)floorf((my - ey) / TH), ty1 = (int)floorf((my + ey) / TH);
    tx0 = max(tx0, 0);
    ty0 = max(ty0, 0);
    tx1 = min(tx1, gx - 1);
    ty1 = min(ty1, gy - 1);
    int n = 0;
    for (int ty = ty0; ty <= ty1; ty++) {
        const float y0 = ty * TH + 0.5f;
        const float y1 = (float)min(ty * TH + TH, H) - 0.5f;
        for (int tx = tx0; tx <= tx1; tx++) {
            const float x0 = tx * TW + 0.5f;
            const float x1 = (float)min(tx * TW + TW, W) - 0.5f;
            if (rect_sigma_min(A, B, C, mx, my, x0, x1, y0, y1) <= thr_c) {
                fn(ty * gx + tx);
                n++;
            }
        }
    }
    return n;
}

// ------------------------------------------------------------------ host launchers

ViewTable make_view_table(const int32_t* wh, int V, int TW, int TH);
RasterParams make_raster_params(const gs_settings* s);

// scan.hip / sort.hip
size_t scan_scratch_words(int64_t max_n);
hipError_t exclusive_scan_u32(uint32_t* data, int64_t n, uint32_t* total_out, uint32_t* scratch,
                              hipStream_t st);
size_t radix_hist_words(int64_t max_n);
// Stable LSD radix sort of (key, value) u32 pairs on bits [lo, hi). n items
// (device count d_n if non-null, clamped to max_n). Returns the buffer pair
// holding the result: 0 = (ka, va), 1 = (kb, vb).
int radix_sort_pairs(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, int64_t max_n,
                     const uint32_t* d_n, int lo, int hi, uint32_t* hist, uint32_t* scan_scratch,
                     hipStream_t st, hipError_t* err);

// bin.hip
hipError_t launch_bin(Ctx* c, const ViewTable& vt, int N, const RasterParams& rp,
                      const float* records, hipStream_t st);

// project.hip
hipError_t launch_project_fwd(Ctx* c, const gs_gaussians* g, const gs_cameras* cams,
                              const ViewTable& vt, const RasterParams& rp, hipStream_t st);
hipError_t launch_project_bwd(Ctx* c, const gs_gaussians* g, const gs_cameras* cams,
                              const ViewTable& vt, const RasterParams& rp,
                              gs_gaussians_grad* grads, int accumulate, float* v_twist,
                              hipStream_t st);

// raster.hip
hipError_t launch_render_fwd(Ctx* c, const ViewTable& vt, const RasterParams& rp, const float* bg,
                             float* rgb, float* T_final, int32_t* last, hipStream_t st);
hipError_t launch_render_bwd(Ctx* c, const ViewTable& vt, const RasterParams& rp, const float* bg,
                             const float* T_final, const int32_t* last, const float* v_rgb,
                             hipStream_t st);
hipError_t launch_l1(Ctx* c, const ViewTable& vt, const float* rgb, const float* target,
                     float* v_rgb, float* loss, hipStream_t st);

// track.hip
hipError_t launch_track(Ctx* c, const float* X, int Pt, const float* viewmat, const float* intr,
                        int n_cams, const int32_t* obs_cam, const int32_t* obs_pt,
                        const float* obs_xy, int M, float delta, float lambda, float near_plane,
                        float* residual, float* loss, float* v_X, float* v_twist, float* J_pose,
                        float* J_X, hipStream_t st);

// optim.hip
hipError_t launch_pose_compose(int V, const float* twist, const float* base, float* out,
                               hipStream_t st);
hipError_t launch_pose_compose_bwd(int V, const float* twist, const float* g, float* out,
                                   hipStream_t st);
hipError_t launch_adam(const gs_adam_group* groups, int n, int step, float b1, float b2,
                       float eps, hipStream_t st);
hipError_t launch_flush_acc(double* acc, float* out, int n, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);

// The context (workspace), shared by the launchers.
struct Ctx {
    gs_capacity cap;
    int device;
    float* rec;            // [max_pairs][12]
    float* grad2d;         // [max_pairs][9], kept zero between backward calls
    uint32_t* cnt;         // [max_pairs] tiles per pair
    uint32_t* off;         // [max_pairs] tile counts in depth order, then their scan
    uint32_t* pk[2];       // [max_pairs] depth keys (ping-pong)
    uint32_t* pv[2];       // [max_pairs] pair indices (ping-pong)
    uint32_t* ik[2];       // [max_isect] tile keys (ping-pong)
    uint32_t* iv[2];       // [max_isect] pair indices (ping-pong)
    int32_t* ranges;       // [max_tiles][2]
    uint32_t* tile_order;  // [max_tiles]
    uint32_t* hist;        // radix histograms
    uint32_t* scan_scratch;
    uint32_t* scalars;     // small device counters
    double* twist_render;  // [max_views][6]
    double* twist_track;   // [max_cams][6]
    double* loss_acc;      // [4]
    uint32_t* diag;        // [kDiagCount]
    // state of the last bin step
    const int32_t* ids;    // sorted pair indices (points into iv[])
    int64_t n_tiles;
    int bin_V, bin_N, bin_tw, bin_th;
};

}  // namespace gs
