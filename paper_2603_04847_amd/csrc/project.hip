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

// Per-Gaussian quantities that do not depend on the view.
struct GaussLocal {
    float mu[3], qn[4], qnorm, s[3], Rq[9], Sig[6];  // Sig: 00 01 02 11 12 22
    float o;
};

__device__ __forceinline__ void load_gaussian(const gs_gaussians& g, int i, GaussLocal& G) {
    const int N = g.N;
#pragma unroll
    for (int k = 0; k < 3; k++) G.mu[k] = g.means[k * N + i];
    float q[4];
#pragma unroll
    for (int k = 0; k < 4; k++) q[k] = g.quats[k * N + i];
    G.qnorm = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float inv = 1.f / G.qnorm;
#pragma unroll
    for (int k = 0; k < 4; k++) G.qn[k] = q[k] * inv;
    const float w = G.qn[0], x = G.qn[1], y = G.qn[2], z = G.qn[3];
    G.Rq[0] = 1.f - 2.f * (y * y + z * z);
    G.Rq[1] = 2.f * (x * y - w * z);
    G.Rq[2] = 2.f * (x * z + w * y);
    G.Rq[3] = 2.f * (x * y + w * z);
    G.Rq[4] = 1.f - 2.f * (x * x + z * z);
    G.Rq[5] = 2.f * (y * z - w * x);
    G.Rq[6] = 2.f * (x * z - w * y);
    G.Rq[7] = 2.f * (y * z + w * x);
    G.Rq[8] = 1.f - 2.f * (x * x + y * y);
#pragma unroll
    for (int k = 0; k < 3; k++) G.s[k] = __expf(g.log_scales[k * N + i]);
    float M[9];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) M[3 * r + c] = G.Rq[3 * r + c] * G.s[c];
    G.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    G.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    G.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    G.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    G.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    G.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
    G.o = 1.f / (1.f + __expf(-g.opacity_logit[i]));
}

__device__ __forceinline__ float sym(const float* S, int i, int j) {
    // symmetric 3x3 stored as 00 01 02 11 12 22
    const int a = min(i, j), b = max(i, j);
    return a == 0 ? S[b] : (a == 1 ? S[2 + b] : S[5]);
}

// Per-(view, Gaussian) projection state, recomputed identically in the backward.
struct Proj {
    bool valid;
    float p[3];
    float Sc[6];          // camera covariance (sym)
    float J00, J02, J11, J12;
    bool clx, cly;
    float tx, ty;         // clamped x/z, y/z
    float a, b, c;        // cov2d
    float A, B, C;        // conic
    float mx, my;
    float dir[3], dist;
};

__device__ __forceinline__ void project_one(const GaussLocal& G, const Cam& cam, int W, int H,
                                            const RasterParams& rp, Proj& P) {
    P.valid = false;
#pragma unroll
    for (int i = 0; i < 3; i++)
        P.p[i] = cam.R[3 * i] * G.mu[0] + cam.R[3 * i + 1] * G.mu[1] + cam.R[3 * i + 2] * G.mu[2] +
                 cam.t[i];
    // view direction from the camera centre -R^T t
    float cc[3];
#pragma unroll
    for (int j = 0; j < 3; j++)
        cc[j] = -(cam.R[j] * cam.t[0] + cam.R[3 + j] * cam.t[1] + cam.R[6 + j] * cam.t[2]);
    float d[3] = {G.mu[0] - cc[0], G.mu[1] - cc[1], G.mu[2] - cc[2]};
    P.dist = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const float id = 1.f / P.dist;
#pragma unroll
    for (int j = 0; j < 3; j++) P.dir[j] = d[j] * id;
    const float z = P.p[2];
    if (!(z >= rp.near_plane)) return;
    // Sc = R Sig R^T
    float RS[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            RS[3 * i + j] = cam.R[3 * i] * sym(G.Sig, 0, j) + cam.R[3 * i + 1] * sym(G.Sig, 1, j) +
                            cam.R[3 * i + 2] * sym(G.Sig, 2, j);
    int k = 0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = i; j < 3; j++)
            P.Sc[k++] = RS[3 * i] * cam.R[3 * j] + RS[3 * i + 1] * cam.R[3 * j + 1] +
                        RS[3 * i + 2] * cam.R[3 * j + 2];
    const float iz = 1.f / z;
    const float lxp = (W - cam.cx) / cam.fx + rp.fov_pad * 0.5f * W / cam.fx;
    const float lxn = cam.cx / cam.fx + rp.fov_pad * 0.5f * W / cam.fx;
    const float lyp = (H - cam.cy) / cam.fy + rp.fov_pad * 0.5f * H / cam.fy;
    const float lyn = cam.cy / cam.fy + rp.fov_pad * 0.5f * H / cam.fy;
    const float rx = P.p[0] * iz, ry = P.p[1] * iz;
    P.tx = fminf(fmaxf(rx, -lxn), lxp);
    P.ty = fminf(fmaxf(ry, -lyn), lyp);
    P.clx = (rx > lxp) || (rx < -lxn);
    P.cly = (ry > lyp) || (ry < -lyn);
    P.J00 = cam.fx * iz;
    P.J02 = -cam.fx * P.tx * iz;
    P.J11 = cam.fy * iz;
    P.J12 = -cam.fy * P.ty * iz;
    const float* S = P.Sc;  // 00 01 02 11 12 22
    P.a = P.J00 * P.J00 * S[0] + 2.f * P.J00 * P.J02 * S[2] + P.J02 * P.J02 * S[5] + rp.eps2d;
    P.b = P.J00 * P.J11 * S[1] + P.J00 * P.J12 * S[2] + P.J02 * P.J11 * S[4] + P.J02 * P.J12 * S[5];
    P.c = P.J11 * P.J11 * S[3] + 2.f * P.J11 * P.J12 * S[4] + P.J12 * P.J12 * S[5] + rp.eps2d;
    const float det = P.a * P.c - P.b * P.b;
    if (!(det > 0.f)) return;
    const float idet = 1.f / det;
    P.A = P.c * idet;
    P.B = -P.b * idet;
    P.C = P.a * idet;
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
    bool nonfinite = false;
    for (int v = 0; v < vt.V; v++) {
        const Cam cam = load_cam(viewmat, intr, vt.cam[v]);
        Proj P;
        project_one(G, cam, vt.W[v], vt.H[v], rp, P);
        const int64_t pair = (int64_t)v * g.N + i;
        float4* r = rec + 3 * pair;
        if (!P.valid || !(G.o > rp.alpha_min)) {
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
        const bool fin = isfinite(P.mx) && isfinite(P.my) && isfinite(P.A) && isfinite(P.B) &&
                         isfinite(P.C) && isfinite(col[0]) && isfinite(col[1]) &&
                         isfinite(col[2]) && isfinite(G.o) && isfinite(P.p[2]);
        if (!fin) {
            nonfinite = true;
            r[0] = make_float4(0.f, 0.f, 0.f, 0.f);
            continue;
        }
        r[0] = make_float4(P.mx, P.my, P.p[2], G.o);
        r[1] = make_float4(P.A, P.B, P.C, col[0]);
        r[2] = make_float4(col[1], col[2], 0.f, 0.f);
    }
    if (nonfinite) atomicOr(&diag[kDiagFlags], (uint32_t)GS_FLAG_NONFINITE);
}

template <int DEG, bool ADAM>
__global__ __launch_bounds__(kBlock) void k_project_bwd(gs_gaussians g, const float* __restrict__ viewmat,
                                                        const float* __restrict__ intr, ViewTable vt,
                                                        RasterParams rp, float* __restrict__ grad2d,
                                                        gs_gaussians_grad out, int accumulate,
                                                        AdamGauss adam,
                                                        double* __restrict__ twist_acc) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    __shared__ float s_tw[kBlock / kWave][6];
    __shared__ double s_acc[6 * GS_MAX_VIEWS];  // this block's twist sums, all iterations
    for (int k = threadIdx.x; k < 6 * vt.V; k += kBlock) s_acc[k] = 0.0;
    __syncthreads();
    const int N = g.N;
    // grid-stride over Gaussians: a bounded number of blocks keeps the twist
    // atomics (one per block, view and component) few
    for (int base = blockIdx.x * kBlock; base < N; base += gridDim.x * kBlock) {
    const int i = base + threadIdx.x;
    const bool active = i < N;
    GaussLocal G;
    float sh[K][3];
    float v_sh[K][3];
    float v_mu[3] = {0.f, 0.f, 0.f}, v_ls[3] = {0.f, 0.f, 0.f}, v_q[4] = {0.f, 0.f, 0.f, 0.f};
    float v_logit = 0.f;
#pragma unroll
    for (int k = 0; k < K; k++)
#pragma unroll
        for (int ch = 0; ch < 3; ch++) v_sh[k][ch] = 0.f;
    if (active) {
        load_gaussian(g, i, G);
#pragma unroll
        for (int k = 0; k < K; k++)
#pragma unroll
            for (int ch = 0; ch < 3; ch++) sh[k][ch] = g.sh[((int64_t)k * 3 + ch) * N + i];
    }
    for (int v = 0; v < vt.V; v++) {
        float tw[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (active) {
            const int64_t pair = (int64_t)v * N + i;
            float* gp = grad2d + 9 * pair;
            float G9[9];
            bool nz = false;
#pragma unroll
            for (int k = 0; k < 9; k++) {
                G9[k] = gp[k];
                nz |= G9[k] != 0.f;
            }
            if (nz) {
#pragma unroll
                for (int k = 0; k < 9; k++) gp[k] = 0.f;  // leave the accumulator clean
                const Cam cam = load_cam(viewmat, intr, vt.cam[v]);
                Proj P;
                project_one(G, cam, vt.W[v], vt.H[v], rp, P);
                if (P.valid) {
                    // opacity
                    v_logit += G9[5] * G.o * (1.f - G.o);
                    // colour through SH (zero where the colour clamp is active)
                    float Y[K];
                    sh_basis(DEG, P.dir[0], P.dir[1], P.dir[2], Y);
                    float vr[3];
#pragma unroll
                    for (int ch = 0; ch < 3; ch++) {
                        float s = 0.f;
#pragma unroll
                        for (int k = 0; k < K; k++) s += Y[k] * sh[k][ch];
                        vr[ch] = (s + 0.5f > 0.f) ? G9[6 + ch] : 0.f;
                    }
                    float sk[K];
#pragma unroll
                    for (int k = 0; k < K; k++) {
                        sk[k] = 0.f;
#pragma unroll
                        for (int ch = 0; ch < 3; ch++) {
                            v_sh[k][ch] += Y[k] * vr[ch];
                            sk[k] += vr[ch] * sh[k][ch];
                        }
                    }
                    float gd[3] = {0.f, 0.f, 0.f};
                    sh_basis_grad(DEG, P.dir[0], P.dir[1], P.dir[2], sk, gd[0], gd[1], gd[2]);
                    const float dd = P.dir[0] * gd[0] + P.dir[1] * gd[1] + P.dir[2] * gd[2];
                    const float idist = 1.f / P.dist;
                    float vmd[3];
#pragma unroll
                    for (int e = 0; e < 3; e++) {
                        vmd[e] = (gd[e] - P.dir[e] * dd) * idist;
                        v_mu[e] += vmd[e];
                    }
                    // the camera centre moves by -R^T rho under the left twist
#pragma unroll
                    for (int e = 0; e < 3; e++)
                        tw[e] += cam.R[3 * e] * vmd[0] + cam.R[3 * e + 1] * vmd[1] +
                                 cam.R[3 * e + 2] * vmd[2];
                    // mean2d
                    const float x = P.p[0], y = P.p[1], z = P.p[2];
                    const float iz = 1.f / z, iz2 = iz * iz;
                    float vp[3];
                    vp[0] = cam.fx * iz * G9[0];
                    vp[1] = cam.fy * iz * G9[1];
                    vp[2] = -(cam.fx * x * G9[0] + cam.fy * y * G9[1]) * iz2;
                    // conic -> cov2d: G2 = -Mc Gc Mc, Gc = [[vA, vB/2], [vB/2, vC]]
                    const float gA = G9[2], gB = 0.5f * G9[3], gC = G9[4];
                    const float t00 = P.A * gA + P.B * gB, t01 = P.A * gB + P.B * gC;
                    const float t10 = P.B * gA + P.C * gB, t11 = P.B * gB + P.C * gC;
                    const float G00 = -(t00 * P.A + t01 * P.B);
                    const float G01 = -(t00 * P.B + t01 * P.C);
                    const float G11 = -(t10 * P.B + t11 * P.C);
                    // J rows: (J00, 0, J02), (0, J11, J12)
                    const float* S = P.Sc;
                    float JS0[3], JS1[3];
#pragma unroll
                    for (int j = 0; j < 3; j++) {
                        JS0[j] = P.J00 * sym(S, 0, j) + P.J02 * sym(S, 2, j);
                        JS1[j] = P.J11 * sym(S, 1, j) + P.J12 * sym(S, 2, j);
                    }
                    // v_J = 2 G2 J Sc
                    const float vJ00 = 2.f * (G00 * JS0[0] + G01 * JS1[0]);
                    const float vJ02 = 2.f * (G00 * JS0[2] + G01 * JS1[2]);
                    const float vJ11 = 2.f * (G01 * JS0[1] + G11 * JS1[1]);
                    const float vJ12 = 2.f * (G01 * JS0[2] + G11 * JS1[2]);
                    vp[2] += -cam.fx * iz2 * vJ00 - cam.fy * iz2 * vJ11;
                    if (!P.clx) {
                        vp[0] += -cam.fx * iz2 * vJ02;
                        vp[2] += 2.f * cam.fx * x * iz2 * iz * vJ02;
                    } else {
                        vp[2] += cam.fx * P.tx * iz2 * vJ02;
                    }
                    if (!P.cly) {
                        vp[1] += -cam.fy * iz2 * vJ12;
                        vp[2] += 2.f * cam.fy * y * iz2 * iz * vJ12;
                    } else {
                        vp[2] += cam.fy * P.ty * iz2 * vJ12;
                    }
                    // v_Sc = J^T G2 J (full 3x3, symmetric)
                    const float J0[3] = {P.J00, 0.f, P.J02}, J1[3] = {0.f, P.J11, P.J12};
                    float U0[3], U1[3];
#pragma unroll
                    for (int j = 0; j < 3; j++) {
                        U0[j] = G00 * J0[j] + G01 * J1[j];
                        U1[j] = G01 * J0[j] + G11 * J1[j];
                    }
                    float vSc[9];
#pragma unroll
                    for (int r = 0; r < 3; r++)
#pragma unroll
                        for (int c = 0; c < 3; c++) vSc[3 * r + c] = J0[r] * U0[c] + J1[r] * U1[c];
                    // twist: rho gets v_p, phi gets p x v_p + 2 axial(Sc vSc)
                    float Wm[9];
#pragma unroll
                    for (int r = 0; r < 3; r++)
#pragma unroll
                        for (int c = 0; c < 3; c++)
                            Wm[3 * r + c] = sym(S, r, 0) * vSc[c] + sym(S, r, 1) * vSc[3 + c] +
                                            sym(S, r, 2) * vSc[6 + c];
                    tw[0] += vp[0];
                    tw[1] += vp[1];
                    tw[2] += vp[2];
                    tw[3] += y * vp[2] - z * vp[1] + 2.f * (Wm[5] - Wm[7]);
                    tw[4] += z * vp[0] - x * vp[2] + 2.f * (Wm[6] - Wm[2]);
                    tw[5] += x * vp[1] - y * vp[0] + 2.f * (Wm[1] - Wm[3]);
                    // mean: p = R mu + t
#pragma unroll
                    for (int e = 0; e < 3; e++)
                        v_mu[e] += cam.R[e] * vp[0] + cam.R[3 + e] * vp[1] + cam.R[6 + e] * vp[2];
                    // Sc = R Sig R^T -> vSig = R^T vSc R
                    float T9[9], vS[9];
#pragma unroll
                    for (int r = 0; r < 3; r++)
#pragma unroll
                        for (int c = 0; c < 3; c++)
                            T9[3 * r + c] = cam.R[r] * vSc[c] + cam.R[3 + r] * vSc[3 + c] +
                                            cam.R[6 + r] * vSc[6 + c];
#pragma unroll
                    for (int r = 0; r < 3; r++)
#pragma unroll
                        for (int c = 0; c < 3; c++)
                            vS[3 * r + c] = T9[3 * r] * cam.R[c] + T9[3 * r + 1] * cam.R[3 + c] +
                                            T9[3 * r + 2] * cam.R[6 + c];
                    // Sig = M M^T, M = Rq S: vM = 2 vS M
                    float vM[9];
#pragma unroll
                    for (int r = 0; r < 3; r++)
#pragma unroll
                        for (int c = 0; c < 3; c++)
                            vM[3 * r + c] =
                                2.f * (vS[3 * r] * G.Rq[c] + vS[3 * r + 1] * G.Rq[3 + c] +
                                       vS[3 * r + 2] * G.Rq[6 + c]) * G.s[c];
#pragma unroll
                    for (int c = 0; c < 3; c++)
                        v_ls[c] += (G.Rq[c] * vM[c] + G.Rq[3 + c] * vM[3 + c] +
                                    G.Rq[6 + c] * vM[6 + c]) * G.s[c];
                    float vR[9];
#pragma unroll
                    for (int r = 0; r < 3; r++)
#pragma unroll
                        for (int c = 0; c < 3; c++) vR[3 * r + c] = vM[3 * r + c] * G.s[c];
                    const float w = G.qn[0], qx = G.qn[1], qy = G.qn[2], qz = G.qn[3];
                    float vqn[4];
                    vqn[0] = 2.f * (-qz * vR[1] + qy * vR[2] + qz * vR[3] - qx * vR[5] - qy * vR[6] +
                                    qx * vR[7]);
                    vqn[1] = 2.f * (qy * vR[1] + qz * vR[2] + qy * vR[3] - w * vR[5] + qz * vR[6] +
                                    w * vR[7]) - 4.f * qx * (vR[4] + vR[8]);
                    vqn[2] = 2.f * (qx * vR[1] + w * vR[2] + qx * vR[3] + qz * vR[5] - w * vR[6] +
                                    qz * vR[7]) - 4.f * qy * (vR[0] + vR[8]);
                    vqn[3] = 2.f * (-w * vR[1] + qx * vR[2] + w * vR[3] + qy * vR[5] + qx * vR[6] +
                                    qy * vR[7]) - 4.f * qz * (vR[0] + vR[4]);
                    const float qd = G.qn[0] * vqn[0] + G.qn[1] * vqn[1] + G.qn[2] * vqn[2] +
                                     G.qn[3] * vqn[3];
                    const float iq = 1.f / G.qnorm;
#pragma unroll
                    for (int e = 0; e < 4; e++) v_q[e] += (vqn[e] - G.qn[e] * qd) * iq;
                }
            }
        }
        // per-view twist: wave sum, then the block's waves, then one double atomic
        const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
#pragma unroll
        for (int e = 0; e < 6; e++) {
            const float s = wave_sum(tw[e]);
            if (lane == 0) s_tw[wv][e] = s;
        }
        __syncthreads();
        if (threadIdx.x < 6) {
            double s = 0.0;
            for (int q = 0; q < kBlock / kWave; q++) s += (double)s_tw[q][threadIdx.x];
            s_acc[6 * v + threadIdx.x] += s;
        }
        __syncthreads();
    }
    if (active && ADAM) {
        // the Gaussian's 11 + 3K gradients in one flat list (means, log_scales,
        // quats, opacity, sh); each Adam batch issues all its parameter and
        // moment loads before its first store, so the loads of a batch are in
        // flight together
        constexpr int NP = 11 + 3 * K;
        constexpr int BATCH = 20;
        float gr[NP];
#pragma unroll
        for (int e = 0; e < 3; e++) gr[e] = v_mu[e];
#pragma unroll
        for (int e = 0; e < 3; e++) gr[3 + e] = v_ls[e];
#pragma unroll
        for (int e = 0; e < 4; e++) gr[6 + e] = v_q[e];
        gr[10] = v_logit;
#pragma unroll
        for (int k = 0; k < K; k++)
#pragma unroll
            for (int ch = 0; ch < 3; ch++) gr[11 + 3 * k + ch] = v_sh[k][ch];
        // array and row of flat entry j
        auto arr = [](int j) { return j < 3 ? 0 : j < 6 ? 1 : j < 10 ? 2 : j < 11 ? 3 : 4; };
        auto row = [](int j) { return j < 3 ? j : j < 6 ? j - 3 : j < 10 ? j - 6 : j < 11 ? 0 : j - 11; };
        // element i of a row: the row start is uniform, the byte offset i * 4
        // one 32-bit lane value shared by every access (N < 2^28, as pairs are)
        const uint32_t off = (uint32_t)i * 4u;
        auto at = [&](float* base, int r) -> float& {
            return *reinterpret_cast<float*>(reinterpret_cast<char*>(base + (int64_t)r * N) + off);
        };
#pragma unroll
        for (int j0 = 0; j0 < NP; j0 += BATCH) {
            float pb[BATCH], mb[BATCH], vb[BATCH];
#pragma unroll
            for (int u = 0; u < BATCH; u++) {
                const int j = j0 + u;
                if (j < NP) {
                    pb[u] = at(adam.p[arr(j)], row(j));
                    mb[u] = at(adam.m[arr(j)], row(j));
                    vb[u] = at(adam.v[arr(j)], row(j));
                }
            }
#pragma unroll
            for (int u = 0; u < BATCH; u++) {
                const int j = j0 + u;
                if (j < NP) {
                    const int q = arr(j);
                    adam_one(pb[u], gr[j], mb[u], vb[u], adam.lr[q], adam.b1, adam.b2, adam.eps,
                             adam.ibc1, adam.ibc2);
                    at(adam.p[q], row(j)) = pb[u];
                    at(adam.m[q], row(j)) = mb[u];
                    at(adam.v[q], row(j)) = vb[u];
                }
            }
        }
    } else if (active) {
    auto put = [&](float* dst, int64_t idx, float val) {
        if (accumulate) dst[idx] += val;
        else dst[idx] = val;
    };
#pragma unroll
    for (int e = 0; e < 3; e++) put(out.means, (int64_t)e * N + i, v_mu[e]);
#pragma unroll
    for (int e = 0; e < 3; e++) put(out.log_scales, (int64_t)e * N + i, v_ls[e]);
#pragma unroll
    for (int e = 0; e < 4; e++) put(out.quats, (int64_t)e * N + i, v_q[e]);
    put(out.opacity_logit, i, v_logit);
#pragma unroll
    for (int k = 0; k < K; k++)
#pragma unroll
        for (int ch = 0; ch < 3; ch++) put(out.sh, ((int64_t)k * 3 + ch) * N + i, v_sh[k][ch]);
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
    const dim3 grid(std::min((g->N + kBlock - 1) / kBlock, 1024)), block(kBlock);
    const gs_gaussians_grad none{};
    const AdamGauss no_adam{};
    if (adam)
        hipLaunchKernelGGL((k_project_bwd<DEG, true>), grid, block, 0, st, *g, cams->viewmat, cams->intr,
                           vt, rp, c->grad2d, none, 0, *adam, c->twist_render);
    else
        hipLaunchKernelGGL((k_project_bwd<DEG, false>), grid, block, 0, st, *g, cams->viewmat,
                           cams->intr, vt, rp, c->grad2d, *grads, accumulate, no_adam, c->twist_render);
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
