// EWA projection of 3D Gaussians for every view of a call, and its backward.
//
// One thread per Gaussian: its parameters (44 + 12K bytes, planar, coalesced)
// are read once and projected into all V views of the call, so a batched call
// streams the parameters once where a per-view loop streams them V times.  The
// backward mirrors this: per-pair 2D gradients are chained to the parameters
// and summed over the views in registers (no atomics for Gaussian gradients),
// and each view's twist gradient is reduced wave -> block -> one double atomic
// per block.
#include <algorithm>

#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kBlock = 256;

// Real SH basis, Condon-Shortley phase, l-major with m = -l..l, evaluated as
// polynomials in the unit direction (x, y, z).  Normalisations:
// Y00 = 1/(2 sqrt(pi)); degree 1: sqrt(3/(4 pi)); degree 2: sqrt(15/pi)/2,
// sqrt(5/pi)/4, sqrt(15/pi)/4; degree 3: sqrt(35/(2 pi))/4, sqrt(105/pi)/2,
// sqrt(21/(2 pi))/4, sqrt(7/pi)/4, sqrt(105/pi)/4.
constexpr float kY0 = 0.28209479177387814f;
constexpr float kY1 = 0.48860251190291992f;
constexpr float kY2a = 1.0925484305920792f;
constexpr float kY2b = 0.31539156525252005f;
constexpr float kY2c = 0.54627421529603959f;
constexpr float kY3a = 0.59004358992664352f;
constexpr float kY3b = 2.8906114426405538f;
constexpr float kY3c = 0.45704579946446572f;
constexpr float kY3d = 0.3731763325901154f;
constexpr float kY3e = 1.4453057213202769f;

__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float* Y) {
    Y[0] = kY0;
    if (deg < 1) return;
    Y[1] = -kY1 * y;
    Y[2] = kY1 * z;
    Y[3] = -kY1 * x;
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kY2a * x * y;
    Y[5] = -kY2a * y * z;
    Y[6] = kY2b * (2.f * zz - xx - yy);
    Y[7] = -kY2a * x * z;
    Y[8] = kY2c * (xx - yy);
    if (deg < 3) return;
    Y[9] = -kY3a * y * (3.f * xx - yy);
    Y[10] = kY3b * x * y * z;
    Y[11] = -kY3c * y * (4.f * zz - xx - yy);
    Y[12] = kY3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = -kY3c * x * (4.f * zz - xx - yy);
    Y[14] = kY3e * z * (xx - yy);
    Y[15] = -kY3a * x * (xx - 3.f * yy);
}

// v_dir += s_k * grad Y_k for the polynomial basis above.
__device__ __forceinline__ void sh_basis_grad(int deg, float x, float y, float z, const float* s,
                                              float& gx, float& gy, float& gz) {
    if (deg < 1) return;
    gx += -kY1 * s[3];
    gy += -kY1 * s[1];
    gz += kY1 * s[2];
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    gx += kY2a * y * s[4] - 2.f * kY2b * x * s[6] - kY2a * z * s[7] + 2.f * kY2c * x * s[8];
    gy += kY2a * x * s[4] - kY2a * z * s[5] - 2.f * kY2b * y * s[6] - 2.f * kY2c * y * s[8];
    gz += -kY2a * y * s[5] + 4.f * kY2b * z * s[6] - kY2a * x * s[7];
    if (deg < 3) return;
    gx += -6.f * kY3a * x * y * s[9] + kY3b * y * z * s[10] + 2.f * kY3c * x * y * s[11] -
          6.f * kY3d * x * z * s[12] - kY3c * (4.f * zz - 3.f * xx - yy) * s[13] +
          2.f * kY3e * x * z * s[14] - 3.f * kY3a * (xx - yy) * s[15];
    gy += -3.f * kY3a * (xx - yy) * s[9] + kY3b * x * z * s[10] -
          kY3c * (4.f * zz - xx - 3.f * yy) * s[11] - 6.f * kY3d * y * z * s[12] +
          2.f * kY3c * x * y * s[13] - 2.f * kY3e * y * z * s[14] + 6.f * kY3a * x * y * s[15];
    gz += kY3b * x * y * s[10] - 8.f * kY3c * y * z * s[11] +
          kY3d * (6.f * zz - 3.f * xx - 3.f * yy) * s[12] - 8.f * kY3c * x * z * s[13] +
          kY3e * (xx - yy) * s[14];
}

struct Cam {
    float R[9], t[3], fx, fy, cx, cy;
};

__device__ __forceinline__ Cam load_cam(const float* __restrict__ viewmat,
                                        const float* __restrict__ intr, int v) {
    Cam c;
#pragma unroll
    for (int i = 0; i < 3; i++) {
#pragma unroll
        for (int j = 0; j < 3; j++) c.R[3 * i + j] = viewmat[12 * v + 4 * i + j];
        c.t[i] = viewmat[12 * v + 4 * i + 3];
    }
    c.fx = intr[4 * v];
    c.fy = intr[4 * v + 1];
    c.cx = intr[4 * v + 2];
    c.cy = intr[4 * v + 3];
    return c;
}

// Per-Gaussian quantities that do not depend on the view.  The covariance
// and everything the EWA step derives from it are formed per view in double
// precision (see project_one), from the raw parameters kept here.
struct GaussLocal {
    float mu[3], q[4], s[3];
    float o;
};

__device__ __forceinline__ void load_gaussian(const gs_gaussians& g, int i, GaussLocal& G) {
    const int N = g.N;
#pragma unroll
    for (int k = 0; k < 3; k++) G.mu[k] = g.means[k * N + i];
#pragma unroll
    for (int k = 0; k < 4; k++) G.q[k] = g.quats[k * N + i];
#pragma unroll
    for (int k = 0; k < 3; k++) G.s[k] = __expf(g.log_scales[k * N + i]);
    G.o = 1.f / (1.f + __expf(-g.opacity_logit[i]));
}

__device__ __forceinline__ double symd(const double* S, int i, int j) {
    // symmetric 3x3 stored as 00 01 02 11 12 22
    const int a = min(i, j), b = max(i, j);
    return a == 0 ? S[b] : (a == 1 ? S[2 + b] : S[5]);
}

// View direction (unit) and distance from the camera centre -R^T t to the mean.
__device__ __forceinline__ void view_dir(const GaussLocal& G, const Cam& cam, float* dir, float& dist) {
    float cc[3];
#pragma unroll
    for (int j = 0; j < 3; j++)
        cc[j] = -(cam.R[j] * cam.t[0] + cam.R[3 + j] * cam.t[1] + cam.R[6 + j] * cam.t[2]);
    const float d[3] = {G.mu[0] - cc[0], G.mu[1] - cc[1], G.mu[2] - cc[2]};
    dist = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const float id = 1.f / dist;
#pragma unroll
    for (int j = 0; j < 3; j++) dir[j] = d[j] * id;
}

// Per-(view, Gaussian) projection state, recomputed identically in the
// backward.  The EWA chain runs in double: for needle-like splats the 2D
// covariance and its inverse are ill-conditioned (eigenvalue ratios of 1e5
// and more), and in float the conic's small eigenvalue, and the gradients that
// project onto the needle's axis, lose most of their digits.
struct Proj {
    bool valid;
    double p[3], iz;      // camera-frame mean and 1 / z
    double qn[4], qnorm;  // unit quaternion and the raw norm
    float Rq[9];          // its rotation (rounded from double)
    double Sc[6];         // camera covariance (sym)
    float J00, J02, J11, J12;
    bool clx, cly;
    float tx, ty;         // clamped x/z, y/z
    double A, B, C;       // conic
    double mx, my;
    float dir[3], dist;
};

__device__ __forceinline__ void project_one(const GaussLocal& G, const Cam& cam, int W, int H,
                                            const RasterParams& rp, Proj& P) {
    P.valid = false;
#pragma unroll
    for (int i = 0; i < 3; i++)
        P.p[i] = (double)cam.R[3 * i] * G.mu[0] + (double)cam.R[3 * i + 1] * G.mu[1] +
                 (double)cam.R[3 * i + 2] * G.mu[2] + cam.t[i];
    // view direction from the camera centre (the colour's input: float)
    view_dir(G, cam, P.dir, P.dist);
    const double z = P.p[2];
    if (!(z >= rp.near_plane)) return;
    // rotation of the unit quaternion (w, x, y, z)
    P.qnorm = sqrt((double)G.q[0] * G.q[0] + (double)G.q[1] * G.q[1] + (double)G.q[2] * G.q[2] +
                   (double)G.q[3] * G.q[3]);
    const double inv = 1.0 / P.qnorm;
#pragma unroll
    for (int k = 0; k < 4; k++) P.qn[k] = G.q[k] * inv;
    double Rq[9];
    {
        const double w = P.qn[0], x = P.qn[1], y = P.qn[2], zq = P.qn[3];
        Rq[0] = 1.0 - 2.0 * (y * y + zq * zq);
        Rq[1] = 2.0 * (x * y - w * zq);
        Rq[2] = 2.0 * (x * zq + w * y);
        Rq[3] = 2.0 * (x * y + w * zq);
        Rq[4] = 1.0 - 2.0 * (x * x + zq * zq);
        Rq[5] = 2.0 * (y * zq - w * x);
        Rq[6] = 2.0 * (x * zq - w * y);
        Rq[7] = 2.0 * (y * zq + w * x);
        Rq[8] = 1.0 - 2.0 * (x * x + y * y);
    }
#pragma unroll
    for (int k = 0; k < 9; k++) P.Rq[k] = (float)Rq[k];
    // Sc = (R Rq S)(R Rq S)^T
    double RM[9];  // R Rq S
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            RM[3 * i + j] = ((double)cam.R[3 * i] * Rq[j] + (double)cam.R[3 * i + 1] * Rq[3 + j] +
                             (double)cam.R[3 * i + 2] * Rq[6 + j]) * G.s[j];
    int k = 0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = i; j < 3; j++)
            P.Sc[k++] = RM[3 * i] * RM[3 * j] + RM[3 * i + 1] * RM[3 * j + 1] + RM[3 * i + 2] * RM[3 * j + 2];
    const double iz = 1.0 / z;
    P.iz = iz;
    // the x/z, y/z clamp limits of J (1.3x the field of view): per view, in float
    const float ifx = 1.f / cam.fx, ify = 1.f / cam.fy;
    const float padx = rp.fov_pad * 0.5f * W * ifx, pady = rp.fov_pad * 0.5f * H * ify;
    const double lxp = ((float)W - cam.cx) * ifx + padx, lxn = cam.cx * ifx + padx;
    const double lyp = ((float)H - cam.cy) * ify + pady, lyn = cam.cy * ify + pady;
    const double rx = P.p[0] * iz, ry = P.p[1] * iz;
    const double tx = fmin(fmax(rx, -lxn), lxp), ty = fmin(fmax(ry, -lyn), lyp);
    P.tx = (float)tx;
    P.ty = (float)ty;
    P.clx = (rx > lxp) || (rx < -lxn);
    P.cly = (ry > lyp) || (ry < -lyn);
    const double J00 = cam.fx * iz, J02 = -cam.fx * tx * iz, J11 = cam.fy * iz, J12 = -cam.fy * ty * iz;
    P.J00 = (float)J00;
    P.J02 = (float)J02;
    P.J11 = (float)J11;
    P.J12 = (float)J12;
    // U = J R Rq S (2 x 3): cov2d = U U^T + eps I.  det without the
    // cancellation of a c - b^2: a' c' - b^2 = |u0 x u1|^2 (Lagrange).
    double u0[3], u1[3];
#pragma unroll
    for (int j = 0; j < 3; j++) {
        u0[j] = J00 * RM[j] + J02 * RM[6 + j];
        u1[j] = J11 * RM[3 + j] + J12 * RM[6 + j];
    }
    const double ap = u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2];
    const double cp = u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2];
    const double b = u0[0] * u1[0] + u0[1] * u1[1] + u0[2] * u1[2];
    const double x0 = u0[1] * u1[2] - u0[2] * u1[1], x1 = u0[2] * u1[0] - u0[0] * u1[2],
                 x2 = u0[0] * u1[1] - u0[1] * u1[0];
    const double eps = rp.eps2d;
    const double det = (x0 * x0 + x1 * x1 + x2 * x2) + eps * (ap + cp) + eps * eps;
    if (!(det > 0.0)) return;
    const double idet = 1.0 / det;
    P.A = (cp + eps) * idet;
    P.B = -b * idet;
    P.C = (ap + eps) * idet;
    P.mx = cam.fx * rx + cam.cx;
    P.my = cam.fy * ry + cam.cy;
    P.valid = true;
}

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_project_fwd(gs_gaussians g, const float* __restrict__ viewmat,
                                                        const float* __restrict__ intr, ViewTable vt,
                                                        RasterParams rp, float4* __restrict__ rec,
                                                        uint32_t* __restrict__ diag) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= g.N) return;
    GaussLocal G;
    load_gaussian(g, i, G);
    float sh[K][3];
#pragma unroll
    for (int k = 0; k < K; k++)
#pragma unroll
        for (int ch = 0; ch < 3; ch++) sh[k][ch] = g.sh[((int64_t)k * 3 + ch) * g.N + i];
    // a Gaussian with any non-finite parameter is culled in every view (and
    // flagged): it contributes nothing, so it receives no gradient
    bool bad = !isfinite(g.opacity_logit[i]);
#pragma unroll
    for (int k = 0; k < 3; k++) bad |= !isfinite(G.mu[k]) || !isfinite(g.log_scales[k * g.N + i]);
#pragma unroll
    for (int k = 0; k < 4; k++) bad |= !isfinite(G.q[k]);
#pragma unroll
    for (int k = 0; k < K; k++)
#pragma unroll
        for (int ch = 0; ch < 3; ch++) bad |= !isfinite(sh[k][ch]);
    bool nonfinite = bad;
    for (int v = 0; v < vt.V; v++) {
        const Cam cam = load_cam(viewmat, intr, vt.cam[v]);
        Proj P;
        if (!bad) project_one(G, cam, vt.W[v], vt.H[v], rp, P);
        const int64_t pair = (int64_t)v * g.N + i;
        float4* r = rec + 3 * pair;
        if (bad || !P.valid || !(G.o > rp.alpha_min)) {
            r[0] = make_float4(0.f, 0.f, 0.f, 0.f);
            continue;
        }
        float Y[K];
        sh_basis(DEG, P.dir[0], P.dir[1], P.dir[2], Y);
        float col[3];
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < K; k++) s += Y[k] * sh[k][ch];
            col[ch] = fmaxf(s + 0.5f, 0.f);
        }
        // the record in float32, each value rounded once from double
        const float mx = (float)P.mx, my = (float)P.my, depth = (float)P.p[2];
        const float cA = (float)P.A, cB = (float)P.B, cC = (float)P.C;
        const bool fin = isfinite(mx) && isfinite(my) && isfinite(cA) && isfinite(cB) &&
                         isfinite(cC) && isfinite(col[0]) && isfinite(col[1]) &&
                         isfinite(col[2]) && isfinite(G.o) && isfinite(depth);
        if (!fin) {
            nonfinite = true;
            r[0] = make_float4(0.f, 0.f, 0.f, 0.f);
            continue;
        }
        r[0] = make_float4(mx, my, depth, G.o);
        r[1] = make_float4(cA, cB, cC, col[0]);
        r[2] = make_float4(col[1], col[2], 0.f, 0.f);
    }
    if (nonfinite) atomicOr(&diag[kDiagFlags], (uint32_t)GS_FLAG_NONFINITE);
}

// One Adam step (ADAM) or the gradient written / added (!ADAM) for n entries
// of one Gaussian: entry j is element i of row row(j) of array arr(j) (0
// means, 1 log_scales, 2 quats, 3 opacity_logit, 4 sh).  Adam batches issue
// every parameter and moment load of a batch before the batch's stores; each
// access is a uniform row base plus one 32-bit lane offset (N < 2^28).
template <bool ADAM, int NE, int BATCH = 20, bool HAS_P = false, typename Arr, typename Row>
__device__ __forceinline__ void step_entries(const float (&gr)[NE], Arr arr, Row row, int i, int N,
                                             const AdamGauss& adam, const gs_gaussians_grad& out,
                                             int accumulate, const float (&pval)[NE]) {
    const uint32_t off = (uint32_t)i * 4u;
    auto at = [&](float* base, int r) -> float& {
        return *reinterpret_cast<float*>(reinterpret_cast<char*>(base + (int64_t)r * N) + off);
    };
    if (ADAM) {
#pragma unroll
        for (int j0 = 0; j0 < NE; j0 += BATCH) {
            float pb[BATCH], mb[BATCH], vb[BATCH];
#pragma unroll
            for (int u = 0; u < BATCH; u++) {
                const int j = j0 + u;
                if (j < NE) {
                    // the parameter itself, when the caller still holds it
                    pb[u] = HAS_P ? pval[j] : at(adam.p[arr(j)], row(j));
                    mb[u] = at(adam.m[arr(j)], row(j));
                    vb[u] = at(adam.v[arr(j)], row(j));
                }
            }
#pragma unroll
            for (int u = 0; u < BATCH; u++) {
                const int j = j0 + u;
                if (j < NE) {
                    const int q = arr(j);
                    adam_one(pb[u], gr[j], mb[u], vb[u], adam.lr[q], adam.b1, adam.b2, adam.eps,
                             adam.ibc1, adam.ibc2);
                    at(adam.p[q], row(j)) = pb[u];
                    at(adam.m[q], row(j)) = mb[u];
                    at(adam.v[q], row(j)) = vb[u];
                }
            }
        }
    } else {
        float* dst[5] = {out.means, out.log_scales, out.quats, out.opacity_logit, out.sh};
#pragma unroll
        for (int j = 0; j < NE; j++) {
            float& d = at(dst[arr(j)], row(j));
            d = accumulate ? d + gr[j] : gr[j];
        }
    }
}

// The projection backward, one thread per Gaussian over the call's views, as
// two kernels so their register sets stay apart: the colour (SH coefficients,
// and the view direction's share of the mean and twist gradients: float),
// then the geometry (the EWA chain in double: mean, scales, rotation,
// opacity and the rest of the twist).  Each reads and clears its part of the
// per-pair 2D gradients; the colour's share of the mean gradient passes to
// the geometry through vmu_dir [3][N]; both add twist terms to one
// accumulator.
template <int DEG, bool ADAM>
__global__ __launch_bounds__(kBlock) void k_project_bwd_color(gs_gaussians g, const float* __restrict__ viewmat,
                                 const float* __restrict__ intr, ViewTable vt, RasterParams rp,
                                 float* __restrict__ grad_col, gs_gaussians_grad out, int accumulate,
                                 AdamGauss adam, float* __restrict__ vmu_dir,
                                 double* __restrict__ twist_acc) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    if (ADAM) adam_bias(adam.step_dev, adam.step, adam.b1, adam.b2, adam.ibc1, adam.ibc2);
    __shared__ double s_acc[6 * GS_MAX_VIEWS];  // this block's twist sums, all iterations
    for (int k = threadIdx.x; k < 6 * vt.V; k += kBlock) s_acc[k] = 0.0;
    __syncthreads();
    const int N = g.N;
    const int lane = threadIdx.x % kWave;
    // one view's twist terms: a wave sum, which the wave's first lane adds to
    // the block's double sums in LDS (no block barrier per view: the loads of
    // the waves that run ahead stay in flight)
    auto twist_reduce = [&](int v, const float* tw) {
#pragma unroll
        for (int e = 0; e < 6; e++) {
            const float sm = wave_sum(tw[e]);
            if (lane == 0 && sm != 0.f) atomicAdd(&s_acc[6 * v + e], (double)sm);
        }
    };
    // grid-stride over Gaussians: a bounded number of blocks keeps the twist
    // atomics (one per block, view and component) few
    for (int base = blockIdx.x * kBlock; base < N; base += gridDim.x * kBlock) {
        const int i = base + threadIdx.x;
        const bool active = i < N;
        GaussLocal G;
        if (active) load_gaussian(g, i, G);
        float v_mu[3] = {0.f, 0.f, 0.f};
        // ---- colour
        {
            float sh[3 * K];  // coefficient k, channel ch at 3 k + ch
            float v_sh[3 * K];
#pragma unroll
            for (int j = 0; j < 3 * K; j++) v_sh[j] = 0.f;
            if (active) {
#pragma unroll
                for (int k = 0; k < K; k++)
#pragma unroll
                    for (int ch = 0; ch < 3; ch++) sh[3 * k + ch] = g.sh[((int64_t)k * 3 + ch) * N + i];
            }
            // the next view's colour gradients are requested ahead, as above
            float gcn[3];
            {
                const float* gp0 = grad_col + kGradCol * (int64_t)(active ? i : 0);
#pragma unroll
                for (int k = 0; k < 3; k++) gcn[k] = (active && vt.V > 0) ? gp0[k] : 0.f;
            }
            for (int v = 0; v < vt.V; v++) {
                float tw[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                const float gc[3] = {gcn[0], gcn[1], gcn[2]};
                if (v + 1 < vt.V) {
                    const float* gq = grad_col + kGradCol * ((int64_t)(v + 1) * N + (active ? i : 0));
#pragma unroll
                    for (int k = 0; k < 3; k++) gcn[k] = active ? gq[k] : 0.f;
                }
                if (active) {
                    float* gp = grad_col + kGradCol * ((int64_t)v * N + i);
                    // a pair that was never rendered (culled, or outside every
                    // list) has no gradient at all
                    if (gc[0] != 0.f || gc[1] != 0.f || gc[2] != 0.f) {
                        gp[0] = gp[1] = gp[2] = 0.f;  // leave the accumulator clean
                        const Cam cam = load_cam(viewmat, intr, vt.cam[v]);
                        float dir[3], dist;
                        view_dir(G, cam, dir, dist);
                        // colour through SH (zero where the colour clamp is active)
                        float Y[K];
                        sh_basis(DEG, dir[0], dir[1], dir[2], Y);
                        float vr[3];
#pragma unroll
                        for (int ch = 0; ch < 3; ch++) {
                            float sm = 0.f;
#pragma unroll
                            for (int k = 0; k < K; k++) sm += Y[k] * sh[3 * k + ch];
                            vr[ch] = (sm + 0.5f > 0.f) ? gc[ch] : 0.f;
                        }
                        float sk[K];
#pragma unroll
                        for (int k = 0; k < K; k++) {
                            sk[k] = 0.f;
#pragma unroll
                            for (int ch = 0; ch < 3; ch++) {
                                v_sh[3 * k + ch] += Y[k] * vr[ch];
                                sk[k] += vr[ch] * sh[3 * k + ch];
                            }
                        }
                        float gd[3] = {0.f, 0.f, 0.f};
                        sh_basis_grad(DEG, dir[0], dir[1], dir[2], sk, gd[0], gd[1], gd[2]);
                        const float dd = dir[0] * gd[0] + dir[1] * gd[1] + dir[2] * gd[2];
                        const float idist = 1.f / dist;
                        float vmd[3];
#pragma unroll
                        for (int e = 0; e < 3; e++) {
                            vmd[e] = (gd[e] - dir[e] * dd) * idist;
                            v_mu[e] += vmd[e];
                        }
                        // the camera centre moves by -R^T rho under the left twist
#pragma unroll
                        for (int e = 0; e < 3; e++)
                            tw[e] += cam.R[3 * e] * vmd[0] + cam.R[3 * e + 1] * vmd[1] +
                                     cam.R[3 * e + 2] * vmd[2];
                    }
                }
                twist_reduce(v, tw);
            }
            if (active) {
#pragma unroll
                for (int e = 0; e < 3; e++) vmu_dir[(int64_t)e * N + i] = v_mu[e];
                step_entries<ADAM, 3 * K, 16, true>(v_sh, [](int) { return 4; }, [](int j) { return j; }, i, N,
                                                    adam, out, accumulate, sh);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 6 * vt.V; k += kBlock)
        if (s_acc[k] != 0.0) atomicAdd(&twist_acc[k], s_acc[k]);
}

template <bool ADAM>
__global__ __launch_bounds__(kBlock) void k_project_bwd_geom(gs_gaussians g, const float* __restrict__ viewmat,
                                 const float* __restrict__ intr, ViewTable vt, RasterParams rp,
                                 float* __restrict__ grad_geo, gs_gaussians_grad out, int accumulate,
                                 AdamGauss adam, float* __restrict__ vmu_dir,
                                 double* __restrict__ twist_acc) {
    if (ADAM) adam_bias(adam.step_dev, adam.step, adam.b1, adam.b2, adam.ibc1, adam.ibc2);
    __shared__ double s_acc[6 * GS_MAX_VIEWS];  // this block's twist sums, all iterations
    for (int k = threadIdx.x; k < 6 * vt.V; k += kBlock) s_acc[k] = 0.0;
    __syncthreads();
    const int N = g.N;
    const int lane = threadIdx.x % kWave;
    // one view's twist terms: a wave sum, which the wave's first lane adds to
    // the block's double sums in LDS (no block barrier per view: the loads of
    // the waves that run ahead stay in flight)
    auto twist_reduce = [&](int v, const float* tw) {
#pragma unroll
        for (int e = 0; e < 6; e++) {
            const float sm = wave_sum(tw[e]);
            if (lane == 0 && sm != 0.f) atomicAdd(&s_acc[6 * v + e], (double)sm);
        }
    };
    // grid-stride over Gaussians: a bounded number of blocks keeps the twist
    // atomics (one per block, view and component) few
    for (int base = blockIdx.x * kBlock; base < N; base += gridDim.x * kBlock) {
        const int i = base + threadIdx.x;
        const bool active = i < N;
        GaussLocal G;
        if (active) load_gaussian(g, i, G);
        float v_mu[3] = {0.f, 0.f, 0.f};
        // ---- geometry
        {
            if (active) {
#pragma unroll
                for (int e = 0; e < 3; e++) v_mu[e] = vmu_dir[(int64_t)e * N + i];
            }
            float v_ls[3] = {0.f, 0.f, 0.f}, v_q[4] = {0.f, 0.f, 0.f, 0.f};
            float v_logit = 0.f;
            // the next view's 2D gradients are requested before this view's
            // chain runs, so their latency hides behind it
            float G9n[6];
            {
                const float* gp0 = grad_geo + kGradGeo * (int64_t)(active ? i : 0);
#pragma unroll
                for (int k = 0; k < 6; k++) G9n[k] = (active && vt.V > 0) ? gp0[k] : 0.f;
            }
            for (int v = 0; v < vt.V; v++) {
                float tw[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                float G9[6];
#pragma unroll
                for (int k = 0; k < 6; k++) G9[k] = G9n[k];
                if (v + 1 < vt.V) {
                    const float* gq = grad_geo + kGradGeo * ((int64_t)(v + 1) * N + (active ? i : 0));
#pragma unroll
                    for (int k = 0; k < 6; k++) G9n[k] = active ? gq[k] : 0.f;
                }
                if (active) {
                    float* gp = grad_geo + kGradGeo * ((int64_t)v * N + i);
                    bool nz = false;
#pragma unroll
                    for (int k = 0; k < 6; k++) nz |= G9[k] != 0.f;
                    if (nz) {
#pragma unroll
                        for (int k = 0; k < 6; k++) gp[k] = 0.f;  // leave the accumulator clean
                        const Cam cam = load_cam(viewmat, intr, vt.cam[v]);
                        Proj P;
                        project_one(G, cam, vt.W[v], vt.H[v], rp, P);
                        if (P.valid) {
                            // opacity
                            v_logit += G9[5] * G.o * (1.f - G.o);
                // the EWA chain in double (the conic and covariances are
                            // ill-conditioned for needle-like splats)
                            // mean2d
                            const double x = P.p[0], y = P.p[1], z = P.p[2];
                            const double iz = P.iz, iz2 = iz * iz;
                            const double fx = cam.fx, fy = cam.fy;
                            double vp[3];
                            vp[0] = fx * iz * G9[0];
                            vp[1] = fy * iz * G9[1];
                            vp[2] = -(fx * x * G9[0] + fy * y * G9[1]) * iz2;
                            // conic -> cov2d: G2 = -Mc Gc Mc, Gc = [[vA, vB/2], [vB/2, vC]]
                            const double gA = G9[2], gB = 0.5 * G9[3], gC = G9[4];
                            const double t00 = P.A * gA + P.B * gB, t01 = P.A * gB + P.B * gC;
                            const double t10 = P.B * gA + P.C * gB, t11 = P.B * gB + P.C * gC;
                            const double G00 = -(t00 * P.A + t01 * P.B);
                            const double G01 = -(t00 * P.B + t01 * P.C);
                            const double G11 = -(t10 * P.B + t11 * P.C);
                            // J rows: (J00, 0, J02), (0, J11, J12)
                            const double* S = P.Sc;
                            double JS0[3], JS1[3];
#pragma unroll
                            for (int j = 0; j < 3; j++) {
                                JS0[j] = P.J00 * symd(S, 0, j) + P.J02 * symd(S, 2, j);
                                JS1[j] = P.J11 * symd(S, 1, j) + P.J12 * symd(S, 2, j);
                            }
                            // v_J = 2 G2 J Sc
                            const double vJ00 = 2.0 * (G00 * JS0[0] + G01 * JS1[0]);
                            const double vJ02 = 2.0 * (G00 * JS0[2] + G01 * JS1[2]);
                            const double vJ11 = 2.0 * (G01 * JS0[1] + G11 * JS1[1]);
                            const double vJ12 = 2.0 * (G01 * JS0[2] + G11 * JS1[2]);
                            vp[2] += -fx * iz2 * vJ00 - fy * iz2 * vJ11;
                            if (!P.clx) {
                                vp[0] += -fx * iz2 * vJ02;
                                vp[2] += 2.0 * fx * x * iz2 * iz * vJ02;
                            } else {
                                vp[2] += fx * P.tx * iz2 * vJ02;
                            }
                            if (!P.cly) {
                                vp[1] += -fy * iz2 * vJ12;
                                vp[2] += 2.0 * fy * y * iz2 * iz * vJ12;
                            } else {
                                vp[2] += fy * P.ty * iz2 * vJ12;
                            }
                            // v_Sc = J^T G2 J, symmetric: 00 01 02 11 12 22
                            double vSc[6];
                            vSc[0] = G00 * P.J00 * P.J00;
                            vSc[1] = G01 * P.J00 * P.J11;
                            vSc[2] = P.J00 * (G00 * P.J02 + G01 * P.J12);
                            vSc[3] = G11 * P.J11 * P.J11;
                            vSc[4] = P.J11 * (G01 * P.J02 + G11 * P.J12);
                            vSc[5] = G00 * P.J02 * P.J02 + 2.0 * G01 * P.J02 * P.J12 + G11 * P.J12 * P.J12;
                            // twist: rho gets v_p, phi gets p x v_p + 2 axial(Sc vSc), axial
                            // of W = Sc vSc: (W12 - W21, W20 - W02, W01 - W10)
                            auto Wrc = [&](int r, int c) {
                                return symd(S, r, 0) * symd(vSc, 0, c) + symd(S, r, 1) * symd(vSc, 1, c) +
                                       symd(S, r, 2) * symd(vSc, 2, c);
                            };
                            tw[0] += (float)vp[0];
                            tw[1] += (float)vp[1];
                            tw[2] += (float)vp[2];
                            tw[3] += (float)(y * vp[2] - z * vp[1] + 2.0 * (Wrc(1, 2) - Wrc(2, 1)));
                            tw[4] += (float)(z * vp[0] - x * vp[2] + 2.0 * (Wrc(2, 0) - Wrc(0, 2)));
                            tw[5] += (float)(x * vp[1] - y * vp[0] + 2.0 * (Wrc(0, 1) - Wrc(1, 0)));
                            // mean: p = R mu + t
#pragma unroll
                            for (int e = 0; e < 3; e++)
                                v_mu[e] += (float)(cam.R[e] * vp[0] + cam.R[3 + e] * vp[1] + cam.R[6 + e] * vp[2]);
                            // Sc = R Sig R^T, Sig = M M^T, M = Rq S.  Q = Rq^T vSig Rq
                            // = (R Rq)^T vSc (R Rq) (symmetric): the scale gradient is
                            // 2 s_c^2 Q_cc and vR = 2 vSig Rq S^2 = 2 Rq Q S^2
                            double Q[6];
                            {
                                double RR[9];  // R Rq
#pragma unroll
                                for (int r = 0; r < 3; r++)
#pragma unroll
                                    for (int c = 0; c < 3; c++)
                                        RR[3 * r + c] = cam.R[3 * r] * P.Rq[c] + cam.R[3 * r + 1] * P.Rq[3 + c] +
                                                        cam.R[3 * r + 2] * P.Rq[6 + c];
                                int k = 0;
#pragma unroll
                                for (int r = 0; r < 3; r++)
#pragma unroll
                                    for (int c = r; c < 3; c++) {
                                        double acc = 0.0;
#pragma unroll
                                        for (int m = 0; m < 3; m++)
#pragma unroll
                                            for (int n = 0; n < 3; n++)
                                                acc += RR[3 * m + r] * symd(vSc, m, n) * RR[3 * n + c];
                                        Q[k++] = acc;
                                    }
                            }
                            const double s2[3] = {(double)G.s[0] * G.s[0], (double)G.s[1] * G.s[1],
                                                  (double)G.s[2] * G.s[2]};
#pragma unroll
                            for (int c = 0; c < 3; c++) v_ls[c] += (float)(2.0 * symd(Q, c, c) * s2[c]);
                            double vR[9];  // 2 Rq Q S^2
#pragma unroll
                            for (int r = 0; r < 3; r++)
#pragma unroll
                                for (int c = 0; c < 3; c++)
                                    vR[3 * r + c] = 2.0 * (P.Rq[3 * r] * symd(Q, 0, c) + P.Rq[3 * r + 1] * symd(Q, 1, c) +
                                                           P.Rq[3 * r + 2] * symd(Q, 2, c)) * s2[c];
                            const double w = P.qn[0], qx = P.qn[1], qy = P.qn[2], qz = P.qn[3];
                            double vqn[4];
                            vqn[0] = 2.0 * (-qz * vR[1] + qy * vR[2] + qz * vR[3] - qx * vR[5] - qy * vR[6] +
                                            qx * vR[7]);
                            vqn[1] = 2.0 * (qy * vR[1] + qz * vR[2] + qy * vR[3] - w * vR[5] + qz * vR[6] +
                                            w * vR[7]) - 4.0 * qx * (vR[4] + vR[8]);
                            vqn[2] = 2.0 * (qx * vR[1] + w * vR[2] + qx * vR[3] + qz * vR[5] - w * vR[6] +
                                            qz * vR[7]) - 4.0 * qy * (vR[0] + vR[8]);
                            vqn[3] = 2.0 * (-w * vR[1] + qx * vR[2] + w * vR[3] + qy * vR[5] + qx * vR[6] +
                                            qy * vR[7]) - 4.0 * qz * (vR[0] + vR[4]);
                            const double qd = P.qn[0] * vqn[0] + P.qn[1] * vqn[1] + P.qn[2] * vqn[2] +
                                              P.qn[3] * vqn[3];
                            const double iq = 1.0 / P.qnorm;
#pragma unroll
                            for (int e = 0; e < 4; e++) v_q[e] += (float)((vqn[e] - P.qn[e] * qd) * iq);
                        }
                    }
                }
                twist_reduce(v, tw);
            }
            if (active) {
                const float gr[11] = {v_mu[0], v_mu[1], v_mu[2], v_ls[0], v_ls[1], v_ls[2],
                                      v_q[0],  v_q[1],  v_q[2],  v_q[3],  v_logit};
                step_entries<ADAM>(
                    gr, [](int j) { return j < 3 ? 0 : j < 6 ? 1 : j < 10 ? 2 : 3; },
                    [](int j) { return j < 3 ? j : j < 6 ? j - 3 : j < 10 ? j - 6 : 0; }, i, N, adam, out,
                    accumulate, gr);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 6 * vt.V; k += kBlock)
        if (s_acc[k] != 0.0) atomicAdd(&twist_acc[k], s_acc[k]);
}

}  // namespace

hipError_t launch_project_fwd(Ctx* c, const gs_gaussians* g, const gs_cameras* cams,
                              const ViewTable& vt, const RasterParams& rp, hipStream_t st) {
    if (g->N <= 0) return hipSuccess;
    const dim3 grid((g->N + kBlock - 1) / kBlock), block(kBlock);
    float4* rec = reinterpret_cast<float4*>(c->rec);
    switch (g->sh_degree) {
        case 0: hipLaunchKernelGGL(k_project_fwd<0>, grid, block, 0, st, *g, cams->viewmat, cams->intr, vt, rp, rec, c->diag); break;
        case 1: hipLaunchKernelGGL(k_project_fwd<1>, grid, block, 0, st, *g, cams->viewmat, cams->intr, vt, rp, rec, c->diag); break;
        case 2: hipLaunchKernelGGL(k_project_fwd<2>, grid, block, 0, st, *g, cams->viewmat, cams->intr, vt, rp, rec, c->diag); break;
        default: hipLaunchKernelGGL(k_project_fwd<3>, grid, block, 0, st, *g, cams->viewmat, cams->intr, vt, rp, rec, c->diag); break;
    }
    return hipGetLastError();
}

template <int DEG>
void project_bwd_impl(Ctx* c, const gs_gaussians* g, const gs_cameras* cams, const ViewTable& vt,
                      const RasterParams& rp, const AdamGauss* adam, const gs_gaussians_grad* grads,
                      int accumulate, hipStream_t st) {
    // at most 2048 blocks, grid-striding beyond: per block one double atomic
    // per view and twist component (measured on 1M Gaussians: 2048 blocks 2%
    // faster than 1024, one round of resident blocks 1% slower)
    const dim3 grid(std::min((g->N + kBlock - 1) / kBlock, 2048)), block(kBlock);
    const gs_gaussians_grad none{};
    const AdamGauss no_adam{};
    float* geo = c->grad2d;
    float* col = c->grad2d + kGradGeo * c->cap.max_pairs;
    if (adam) {
        hipLaunchKernelGGL((k_project_bwd_color<DEG, true>), grid, block, 0, st, *g, cams->viewmat,
                           cams->intr, vt, rp, col, none, 0, *adam, c->vmu_dir, c->twist_render);
        hipLaunchKernelGGL((k_project_bwd_geom<true>), grid, block, 0, st, *g, cams->viewmat, cams->intr,
                           vt, rp, geo, none, 0, *adam, c->vmu_dir, c->twist_render);
    } else {
        hipLaunchKernelGGL((k_project_bwd_color<DEG, false>), grid, block, 0, st, *g, cams->viewmat,
                           cams->intr, vt, rp, col, *grads, accumulate, no_adam, c->vmu_dir,
                           c->twist_render);
        hipLaunchKernelGGL((k_project_bwd_geom<false>), grid, block, 0, st, *g, cams->viewmat,
                           cams->intr, vt, rp, geo, *grads, accumulate, no_adam, c->vmu_dir,
                           c->twist_render);
    }
}

hipError_t launch_project_bwd(Ctx* c, const gs_gaussians* g, const gs_cameras* cams,
                              const ViewTable& vt, const RasterParams& rp, const AdamGauss* adam,
                              gs_gaussians_grad* grads, int accumulate, float* v_twist,
                              hipStream_t st) {
    if (g->N > 0) {
        switch (g->sh_degree) {
            case 0: project_bwd_impl<0>(c, g, cams, vt, rp, adam, grads, accumulate, st); break;
            case 1: project_bwd_impl<1>(c, g, cams, vt, rp, adam, grads, accumulate, st); break;
            case 2: project_bwd_impl<2>(c, g, cams, vt, rp, adam, grads, accumulate, st); break;
            default: project_bwd_impl<3>(c, g, cams, vt, rp, adam, grads, accumulate, st); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_flush_twist_rows(c->twist_render, v_twist, vt, st);
}

}  // namespace gs
