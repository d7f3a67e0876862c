// One Levenberg-Marquardt step of bundle adjustment on the track
// reprojection term: poses (left twists at the current pose) and points,
// Huber cost on the squared reprojection error, iteratively reweighted.
//
// With r the residual of an observation, s = |r|^2, w = rho'(s) and
// J = [J_pose | J_X] its Jacobian, the normal equations are
//   [U  W] [dc]   [-g_c]      U = sum w J_pose^T J_pose (+ lambda diag),
//   [W' V] [dX] = [-g_X],     V = sum w J_X^T J_X (+ lambda diag),
//                             W = sum w J_pose^T J_X, g = sum w J^T r.
// Points are eliminated (V is block diagonal, 3x3 per point): the reduced
// camera system S dc = b with S = U - W V^-1 W', b = -g_c + W V^-1 g_X is
// solved by conjugate gradients preconditioned with the inverse 6x6 diagonal
// blocks of S, then dX = -V^-1 (g_X + W' dc).  S is never formed: a product
// S p is one pass over the observations by point (u_k = V_k^-1 sum W'_o p)
// and one by camera (U p - sum W_o u_k), recomputing each observation's
// Jacobian blocks from the parameters (about 30 B read per observation,
// instead of the 144 B its blocks would take).  All arithmetic is double.
// The iteration count is fixed at launch (a graph-capturable step); once the
// residual is below tol |b| a device flag turns the remaining launches into
// no-ops.
#include <math.h>

#include <algorithm>

#include "gs_internal.h"

struct gs_ba {
    int64_t max_points;
    int32_t max_cams;
    double* pt;       // [max_points][12]: V^-1 (6, sym), V^-1 g_X (3), u (3)
    double* cam;      // [max_cams][84]: U (21), L (21, Cholesky of S_ii), b, x, r, z, p, Ap (6 each)
    int32_t* cam_off; // [max_cams + 1]
    double* sc;       // [16] scalars
};

namespace gs {

namespace {

constexpr int kBlock = 256;
constexpr int kVec = 1024;  // threads of the single-workgroup vector kernels
constexpr int kPt = 12, kCam = 84;
constexpr int oU = 0, oL = 21, oB = 42, oX = 48, oR = 54, oZ = 60, oP = 66, oAp = 72;
// scalars
enum { sRZ = 0, sBB = 1, sDone = 2, sIt = 3, sCost = 4, sMasked = 5, sUnsorted = 6, sRR = 7 };

struct BaObs {
    const float* X;
    const float* viewmat;
    const float* intr;
    const int32_t* obs_cam;
    const int32_t* obs_pt;
    const float* obs_xy;
    int Pt, n_cams, M;
    double delta, near_plane, lambda;
};

struct Lin {
    bool ok;
    double r0, r1, w, rho;
    double Jp[12], Jx[6];
};

__device__ __forceinline__ void linearise(const BaObs& a, int o, int ci, int k, Lin& L) {
    double R[9], t[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
#pragma unroll
        for (int j = 0; j < 3; j++) R[3 * i + j] = a.viewmat[12 * ci + 4 * i + j];
        t[i] = a.viewmat[12 * ci + 4 * i + 3];
    }
    const double X0 = a.X[3 * (int64_t)k], X1 = a.X[3 * (int64_t)k + 1], X2 = a.X[3 * (int64_t)k + 2];
    double p[3];
#pragma unroll
    for (int i = 0; i < 3; i++) p[i] = R[3 * i] * X0 + R[3 * i + 1] * X1 + R[3 * i + 2] * X2 + t[i];
    L.ok = p[2] >= a.near_plane;
    if (!L.ok) return;
    const double fx = a.intr[4 * ci], fy = a.intr[4 * ci + 1], cx = a.intr[4 * ci + 2],
                 cy = a.intr[4 * ci + 3];
    const double iz = 1.0 / p[2], u = p[0] * iz, v = p[1] * iz;
    L.r0 = fx * u + cx - (double)a.obs_xy[2 * (int64_t)o];
    L.r1 = fy * v + cy - (double)a.obs_xy[2 * (int64_t)o + 1];
    const double s = L.r0 * L.r0 + L.r1 * L.r1;
    if (s <= a.delta * a.delta) {
        L.w = 1.0;
        L.rho = s;
    } else {
        const double rs = sqrt(s);
        L.w = a.delta / rs;
        L.rho = 2.0 * a.delta * rs - a.delta * a.delta;
    }
    // J_pi = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]]; J_pose = J_pi [I | -[p]x]
    const double a00 = fx * iz, a02 = -fx * u * iz, a11 = fy * iz, a12 = -fy * v * iz;
    L.Jp[0] = a00; L.Jp[1] = 0.0; L.Jp[2] = a02;
    L.Jp[3] = a02 * p[1];
    L.Jp[4] = a00 * p[2] - a02 * p[0];
    L.Jp[5] = -a00 * p[1];
    L.Jp[6] = 0.0; L.Jp[7] = a11; L.Jp[8] = a12;
    L.Jp[9] = -a11 * p[2] + a12 * p[1];
    L.Jp[10] = -a12 * p[0];
    L.Jp[11] = a11 * p[0];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        L.Jx[c] = a00 * R[c] + a02 * R[6 + c];
        L.Jx[3 + c] = a11 * R[3 + c] + a12 * R[6 + c];
    }
}

// symmetric 3x3 (00 01 02 11 12 22) and 6x6 (row-major lower triangle, 21)
__device__ __forceinline__ int tri6(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* s) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < NV; j++)
        for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_xor(v[j], off, kWave);
    if (lane == 0)
#pragma unroll
        for (int j = 0; j < NV; j++) s[w * NV + j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < NV; j++) {
            double t = 0.0;
            for (int q = 0; q < kBlock / kWave; q++) t += s[q * NV + j];
            v[j] = t;
        }
}

__device__ __forceinline__ int lower_bound_i(const int32_t* a, int n, int key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// camera ranges of the observations (sorted by camera) and the sort check
__global__ __launch_bounds__(kBlock) void k_ba_ranges(BaObs a, int32_t* __restrict__ cam_off,
                                                      double* __restrict__ sc) {
    const int tid = blockIdx.x * kBlock + threadIdx.x;
    if (tid <= a.n_cams) cam_off[tid] = lower_bound_i(a.obs_cam, a.M, tid);
    for (int o = tid; o + 1 < a.M; o += gridDim.x * kBlock)
        if (a.obs_cam[o] > a.obs_cam[o + 1]) sc[sUnsorted] = 1.0;
}

// per point: V (damped) inverted, V^-1 g_X; the cost and masked count
__global__ __launch_bounds__(kBlock) void k_ba_points(BaObs a, const int32_t* __restrict__ pt_off,
                                                      const int32_t* __restrict__ pt_obs,
                                                      double* __restrict__ pt, double* __restrict__ sc) {
    __shared__ double s_red[(kBlock / kWave) * 2];
    const int k = blockIdx.x * kBlock + threadIdx.x;
    double cost = 0.0, masked = 0.0;
    if (k < a.Pt) {
        double V[6] = {0, 0, 0, 0, 0, 0}, g[3] = {0, 0, 0};
        for (int j = pt_off[k]; j < pt_off[k + 1]; j++) {
            const int o = pt_obs ? pt_obs[j] : j;  // no index: the arrays are point-major
            const int ci = a.obs_cam[o];
            if (ci < 0 || ci >= a.n_cams) continue;
            Lin L;
            linearise(a, o, ci, k, L);
            if (!L.ok) {
                masked += 1.0;
                continue;
            }
            cost += L.rho;
            const double* J0 = L.Jx;
            const double* J1 = L.Jx + 3;
            V[0] += L.w * (J0[0] * J0[0] + J1[0] * J1[0]);
            V[1] += L.w * (J0[0] * J0[1] + J1[0] * J1[1]);
            V[2] += L.w * (J0[0] * J0[2] + J1[0] * J1[2]);
            V[3] += L.w * (J0[1] * J0[1] + J1[1] * J1[1]);
            V[4] += L.w * (J0[1] * J0[2] + J1[1] * J1[2]);
            V[5] += L.w * (J0[2] * J0[2] + J1[2] * J1[2]);
#pragma unroll
            for (int c = 0; c < 3; c++) g[c] += L.w * (J0[c] * L.r0 + J1[c] * L.r1);
        }
        V[0] *= 1.0 + a.lambda;
        V[3] *= 1.0 + a.lambda;
        V[5] *= 1.0 + a.lambda;
        // inverse by the adjugate; a point with no observation is held fixed
        const double c00 = V[3] * V[5] - V[4] * V[4], c01 = V[2] * V[4] - V[1] * V[5],
                     c02 = V[1] * V[4] - V[2] * V[3], c11 = V[0] * V[5] - V[2] * V[2],
                     c12 = V[1] * V[2] - V[0] * V[4], c22 = V[0] * V[3] - V[1] * V[1];
        const double det = V[0] * c00 + V[1] * c01 + V[2] * c02;
        double* q = pt + (int64_t)kPt * k;
        if (det > 0.0) {
            const double id = 1.0 / det;
            q[0] = c00 * id; q[1] = c01 * id; q[2] = c02 * id;
            q[3] = c11 * id; q[4] = c12 * id; q[5] = c22 * id;
        } else {
#pragma unroll
            for (int e = 0; e < 6; e++) q[e] = 0.0;
        }
        q[6] = q[0] * g[0] + q[1] * g[1] + q[2] * g[2];
        q[7] = q[1] * g[0] + q[3] * g[1] + q[4] * g[2];
        q[8] = q[2] * g[0] + q[4] * g[1] + q[5] * g[2];
    }
    double v[2] = {cost, masked};
    block_sum<2>(v, s_red);
    if (threadIdx.x == 0) {
        if (v[0] != 0.0) atomicAdd(&sc[sCost], v[0]);
        if (v[1] != 0.0) atomicAdd(&sc[sMasked], v[1]);
    }
}

// per camera (one workgroup): U (damped), S_ii = U - sum W V^-1 W' and its
// Cholesky factor, b = -g_c + sum W V^-1 g_X
__global__ __launch_bounds__(kBlock) void k_ba_cams(BaObs a, const int32_t* __restrict__ cam_off,
                                                    const double* __restrict__ pt,
                                                    double* __restrict__ cam) {
    __shared__ double s_red[(kBlock / kWave) * 54];
    const int c = blockIdx.x;
    double v[54];  // U (21), corr (21), g_c (6), W V^-1 g_X (6)
#pragma unroll
    for (int j = 0; j < 54; j++) v[j] = 0.0;
    for (int o = cam_off[c] + threadIdx.x; o < cam_off[c + 1]; o += kBlock) {
        const int k = a.obs_pt[o];
        if (k < 0 || k >= a.Pt) continue;
        Lin L;
        linearise(a, o, c, k, L);
        if (!L.ok) continue;
        const double* q = pt + (int64_t)kPt * k;
        // M2 = J_X V^-1 J_X' (2x2), e = J_X V^-1 g_X (2)
        double JV[2][3];
#pragma unroll
        for (int r = 0; r < 2; r++) {
            const double* J = L.Jx + 3 * r;
            JV[r][0] = J[0] * q[0] + J[1] * q[1] + J[2] * q[2];
            JV[r][1] = J[0] * q[1] + J[1] * q[3] + J[2] * q[4];
            JV[r][2] = J[0] * q[2] + J[1] * q[4] + J[2] * q[5];
        }
        const double m00 = JV[0][0] * L.Jx[0] + JV[0][1] * L.Jx[1] + JV[0][2] * L.Jx[2];
        const double m01 = JV[0][0] * L.Jx[3] + JV[0][1] * L.Jx[4] + JV[0][2] * L.Jx[5];
        const double m11 = JV[1][0] * L.Jx[3] + JV[1][1] * L.Jx[4] + JV[1][2] * L.Jx[5];
        const double e0 = L.Jx[0] * q[6] + L.Jx[1] * q[7] + L.Jx[2] * q[8];
        const double e1 = L.Jx[3] * q[6] + L.Jx[4] * q[7] + L.Jx[5] * q[8];
        const double w2 = L.w * L.w;
#pragma unroll
        for (int i = 0; i < 6; i++) {
            const double pi0 = L.Jp[i], pi1 = L.Jp[6 + i];
#pragma unroll
            for (int j = 0; j <= i; j++) {
                const double pj0 = L.Jp[j], pj1 = L.Jp[6 + j];
                v[tri6(i, j)] += L.w * (pi0 * pj0 + pi1 * pj1);
                v[21 + tri6(i, j)] += w2 * (pi0 * (m00 * pj0 + m01 * pj1) + pi1 * (m01 * pj0 + m11 * pj1));
            }
            v[42 + i] += L.w * (pi0 * L.r0 + pi1 * L.r1);
            v[48 + i] += L.w * (pi0 * e0 + pi1 * e1);
        }
    }
    block_sum<54>(v, s_red);
    if (threadIdx.x != 0) return;
    double* q = cam + (int64_t)kCam * c;
    bool live = false;
#pragma unroll
    for (int i = 0; i < 6; i++) live |= v[tri6(i, i)] > 0.0;
    double S[21];
#pragma unroll
    for (int e = 0; e < 21; e++) q[oU + e] = v[e];
#pragma unroll
    for (int i = 0; i < 6; i++) q[oU + tri6(i, i)] *= 1.0 + a.lambda;
#pragma unroll
    for (int e = 0; e < 21; e++) S[e] = q[oU + e] - v[21 + e];
    // Cholesky S = L L' (lower, packed like the matrix); a camera with no
    // observation (or a block that is not positive) is held fixed: L = 0
    bool ok = live;
    for (int i = 0; i < 6 && ok; i++) {
        for (int j = 0; j <= i; j++) {
            double sum = S[tri6(i, j)];
            for (int m = 0; m < j; m++) sum -= S[tri6(i, m)] * S[tri6(j, m)];
            if (i == j) {
                if (!(sum > 0.0)) {
                    ok = false;
                    break;
                }
                S[tri6(i, i)] = sqrt(sum);
            } else {
                S[tri6(i, j)] = sum / S[tri6(j, j)];
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 21; e++) q[oL + e] = ok ? S[e] : 0.0;
#pragma unroll
    for (int i = 0; i < 6; i++) q[oB + i] = ok ? -v[42 + i] + v[48 + i] : 0.0;
}

// z = (L L')^-1 r for camera c (0 for a fixed camera)
__device__ __forceinline__ void precond(const double* q, const double* r, double* z) {
    if (!(q[oL] > 0.0)) {
#pragma unroll
        for (int i = 0; i < 6; i++) z[i] = 0.0;
        return;
    }
    double y[6];
#pragma unroll
    for (int i = 0; i < 6; i++) {
        double s = r[i];
#pragma unroll
        for (int m = 0; m < i; m++) s -= q[oL + tri6(i, m)] * y[m];
        y[i] = s / q[oL + tri6(i, i)];
    }
#pragma unroll
    for (int i = 5; i >= 0; i--) {
        double s = y[i];
#pragma unroll
        for (int m = i + 1; m < 6; m++) s -= q[oL + tri6(m, i)] * z[m];
        z[i] = s / q[oL + tri6(i, i)];
    }
}

__device__ __forceinline__ double block_dot(double v, double* s) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) s[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int q = 0; q < kVec / kWave; q++) t += s[q];
    return t;
}

// x = 0, r = b, z = P r, p = z
__global__ __launch_bounds__(kVec) void k_ba_pcg_init(int n_cams, double* __restrict__ cam,
                                                      double* __restrict__ sc) {
    __shared__ double s[kVec / kWave];
    double rz = 0.0, bb = 0.0;
    for (int c = threadIdx.x; c < n_cams; c += kVec) {
        double* q = cam + (int64_t)kCam * c;
        double z[6];
        precond(q, q + oB, z);
#pragma unroll
        for (int i = 0; i < 6; i++) {
            q[oX + i] = 0.0;
            q[oR + i] = q[oB + i];
            q[oZ + i] = z[i];
            q[oP + i] = z[i];
            rz += q[oB + i] * z[i];
            bb += q[oB + i] * q[oB + i];
        }
    }
    rz = block_dot(rz, s);
    bb = block_dot(bb, s);
    if (threadIdx.x == 0) {
        sc[sRZ] = rz;
        sc[sBB] = bb;
        sc[sRR] = bb;
        sc[sIt] = 0.0;
        sc[sDone] = (bb > 0.0 && !(sc[sUnsorted] > 0.0)) ? 0.0 : 1.0;
    }
}

// u_k = V_k^-1 sum_o W_o' src_cam(o)   (src: offset of the camera vector)
__global__ __launch_bounds__(kBlock) void k_ba_pt_apply(BaObs a, const int32_t* __restrict__ pt_off,
                                                        const int32_t* __restrict__ pt_obs,
                                                        const double* __restrict__ cam, int src,
                                                        double* __restrict__ pt,
                                                        const double* __restrict__ sc, int force) {
    if (!force && sc[sDone] > 0.0) return;
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= a.Pt) return;
    double t[3] = {0, 0, 0};
    for (int j = pt_off[k]; j < pt_off[k + 1]; j++) {
        const int o = pt_obs ? pt_obs[j] : j;  // no index: the arrays are point-major
        const int ci = a.obs_cam[o];
        if (ci < 0 || ci >= a.n_cams) continue;
        Lin L;
        linearise(a, o, ci, k, L);
        if (!L.ok) continue;
        const double* x = cam + (int64_t)kCam * ci + src;
        double jp0 = 0.0, jp1 = 0.0;
#pragma unroll
        for (int i = 0; i < 6; i++) {
            jp0 += L.Jp[i] * x[i];
            jp1 += L.Jp[6 + i] * x[i];
        }
#pragma unroll
        for (int c = 0; c < 3; c++) t[c] += L.w * (L.Jx[c] * jp0 + L.Jx[3 + c] * jp1);
    }
    double* q = pt + (int64_t)kPt * k;
    q[9] = q[0] * t[0] + q[1] * t[1] + q[2] * t[2];
    q[10] = q[1] * t[0] + q[3] * t[1] + q[4] * t[2];
    q[11] = q[2] * t[0] + q[4] * t[1] + q[5] * t[2];
}

// Ap_c = U_c p_c - sum_o W_o u_k(o)   (one workgroup per camera)
__global__ __launch_bounds__(kBlock) void k_ba_cam_apply(BaObs a, const int32_t* __restrict__ cam_off,
                                                         const double* __restrict__ pt,
                                                         double* __restrict__ cam,
                                                         const double* __restrict__ sc) {
    __shared__ double s_red[(kBlock / kWave) * 6];
    if (sc[sDone] > 0.0) return;
    const int c = blockIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int o = cam_off[c] + threadIdx.x; o < cam_off[c + 1]; o += kBlock) {
        const int k = a.obs_pt[o];
        if (k < 0 || k >= a.Pt) continue;
        Lin L;
        linearise(a, o, c, k, L);
        if (!L.ok) continue;
        const double* u = pt + (int64_t)kPt * k + 9;
        const double e0 = L.Jx[0] * u[0] + L.Jx[1] * u[1] + L.Jx[2] * u[2];
        const double e1 = L.Jx[3] * u[0] + L.Jx[4] * u[1] + L.Jx[5] * u[2];
#pragma unroll
        for (int i = 0; i < 6; i++) v[i] -= L.w * (L.Jp[i] * e0 + L.Jp[6 + i] * e1);
    }
    block_sum<6>(v, s_red);
    if (threadIdx.x != 0) return;
    double* q = cam + (int64_t)kCam * c;
    const bool live = q[oL] > 0.0;
#pragma unroll
    for (int i = 0; i < 6; i++) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 6; j++) s += q[oU + tri6(i, j)] * q[oP + j];
        q[oAp + i] = live ? s + v[i] : 0.0;
    }
}

// one conjugate-gradient update; sets the done flag on convergence
__global__ __launch_bounds__(kVec) void k_ba_pcg_update(int n_cams, double* __restrict__ cam,
                                                        double* __restrict__ sc, double tol2) {
    __shared__ double s[kVec / kWave];
    if (sc[sDone] > 0.0) return;
    double pap = 0.0;
    for (int c = threadIdx.x; c < n_cams; c += kVec) {
        const double* q = cam + (int64_t)kCam * c;
#pragma unroll
        for (int i = 0; i < 6; i++) pap += q[oP + i] * q[oAp + i];
    }
    pap = block_dot(pap, s);
    const double rz = sc[sRZ];
    const double alpha = pap > 0.0 ? rz / pap : 0.0;
    double rr = 0.0;
    for (int c = threadIdx.x; c < n_cams; c += kVec) {
        double* q = cam + (int64_t)kCam * c;
#pragma unroll
        for (int i = 0; i < 6; i++) {
            q[oX + i] += alpha * q[oP + i];
            q[oR + i] -= alpha * q[oAp + i];
            rr += q[oR + i] * q[oR + i];
        }
    }
    rr = block_dot(rr, s);
    const bool done = !(pap > 0.0) || rr <= tol2 * sc[sBB];
    double rz1 = 0.0;
    if (!done) {
        for (int c = threadIdx.x; c < n_cams; c += kVec) {
            double* q = cam + (int64_t)kCam * c;
            double z[6];
            precond(q, q + oR, z);
#pragma unroll
            for (int i = 0; i < 6; i++) {
                q[oZ + i] = z[i];
                rz1 += q[oR + i] * z[i];
            }
        }
        rz1 = block_dot(rz1, s);
        const double beta = rz > 0.0 ? rz1 / rz : 0.0;
        for (int c = threadIdx.x; c < n_cams; c += kVec) {
            double* q = cam + (int64_t)kCam * c;
#pragma unroll
            for (int i = 0; i < 6; i++) q[oP + i] = q[oZ + i] + beta * q[oP + i];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        sc[sIt] += 1.0;
        sc[sRR] = rr;
        sc[sRZ] = rz1;
        if (done) sc[sDone] = 1.0;
    }
}

// the step: d_twist = x, d_X = -(V^-1 g_X + u(x)); statistics
__global__ __launch_bounds__(kBlock) void k_ba_finish(int n_cams, int Pt, const double* __restrict__ cam,
                                                      const double* __restrict__ pt,
                                                      const double* __restrict__ sc,
                                                      float* __restrict__ d_twist, float* __restrict__ d_X,
                                                      float* __restrict__ stats) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const bool bad = sc[sUnsorted] > 0.0;
    if (i < 6 * n_cams) d_twist[i] = bad ? 0.f : (float)cam[(int64_t)kCam * (i / 6) + oX + i % 6];
    if (i < 3 * Pt) {
        const double* q = pt + (int64_t)kPt * (i / 3);
        d_X[i] = bad ? 0.f : (float)(-(q[6 + i % 3] + q[9 + i % 3]));
    }
    if (i == 0 && stats) {
        stats[0] = (float)sc[sIt];
        stats[1] = sc[sBB] > 0.0 ? (float)sqrt(sc[sRR] / sc[sBB]) : 0.f;
        stats[2] = (float)sc[sCost];
        stats[3] = (float)sc[sMasked];
        stats[4] = bad ? 1.f : 0.f;
    }
}

__global__ void k_ba_clear(double* __restrict__ sc) {
    if (threadIdx.x < 16) sc[threadIdx.x] = 0.0;
}

}  // namespace

hipError_t launch_ba_step(gs_ba* ba, const BaInputs& in, float* d_twist, float* d_X, float* stats,
                          hipStream_t st) {
    BaObs a;
    a.X = in.X;
    a.viewmat = in.viewmat;
    a.intr = in.intr;
    a.obs_cam = in.obs_cam;
    a.obs_pt = in.obs_pt;
    a.obs_xy = in.obs_xy;
    a.Pt = in.Pt;
    a.n_cams = in.n_cams;
    a.M = in.M;
    a.delta = in.delta;
    a.near_plane = in.near_plane;
    a.lambda = in.lambda;
    // the point passes read the point-major copies in order when there are
    // some (no index then), else the caller's arrays through the index
    BaObs ap = a;
    const int32_t* pidx = in.pt_obs;
    if (in.pm_cam && in.pm_xy) {
        ap.obs_cam = in.pm_cam;
        ap.obs_xy = in.pm_xy;
        pidx = nullptr;
    }
    const unsigned gp = (unsigned)std::max((in.Pt + kBlock - 1) / kBlock, 1);
    const unsigned gr = (unsigned)std::min(std::max((std::max(in.M, in.n_cams + 1) + kBlock - 1) / kBlock, 1), 4096);
    hipLaunchKernelGGL(k_ba_clear, dim3(1), dim3(64), 0, st, ba->sc);
    hipLaunchKernelGGL(k_ba_ranges, dim3(gr), dim3(kBlock), 0, st, a, ba->cam_off, ba->sc);
    hipLaunchKernelGGL(k_ba_points, dim3(gp), dim3(kBlock), 0, st, ap, in.pt_off, pidx, ba->pt, ba->sc);
    if (in.n_cams > 0)
        hipLaunchKernelGGL(k_ba_cams, dim3(in.n_cams), dim3(kBlock), 0, st, a, ba->cam_off, ba->pt, ba->cam);
    hipLaunchKernelGGL(k_ba_pcg_init, dim3(1), dim3(kVec), 0, st, in.n_cams, ba->cam, ba->sc);
    for (int it = 0; it < in.max_iter; it++) {
        hipLaunchKernelGGL(k_ba_pt_apply, dim3(gp), dim3(kBlock), 0, st, ap, in.pt_off, pidx, ba->cam,
                           oP, ba->pt, ba->sc, 0);
        if (in.n_cams > 0)
            hipLaunchKernelGGL(k_ba_cam_apply, dim3(in.n_cams), dim3(kBlock), 0, st, a, ba->cam_off, ba->pt,
                               ba->cam, ba->sc);
        hipLaunchKernelGGL(k_ba_pcg_update, dim3(1), dim3(kVec), 0, st, in.n_cams, ba->cam, ba->sc,
                           (double)in.tol * (double)in.tol);
    }
    // back-substitution for the points with the final camera step
    hipLaunchKernelGGL(k_ba_pt_apply, dim3(gp), dim3(kBlock), 0, st, ap, in.pt_off, pidx, ba->cam, oX,
                       ba->pt, ba->sc, 1);
    const int nout = std::max(6 * in.n_cams, 3 * in.Pt);
    hipLaunchKernelGGL(k_ba_finish, dim3((unsigned)std::max((nout + kBlock - 1) / kBlock, 1)), dim3(kBlock), 0, st,
                       in.n_cams, in.Pt, ba->cam, ba->pt, ba->sc, d_twist, d_X, stats);
    return hipGetLastError();
}

}  // namespace gs

extern "C" {

gs_status gs_ba_create(gs_ba** out, int64_t max_points, int32_t max_cams) {
    if (!out) return GS_ERR_INVALID_ARG;
    *out = nullptr;
    if (max_points < 0 || max_cams < 0) return GS_ERR_INVALID_ARG;
    if (max_points > ((int64_t)1 << 28) || max_cams > GS_BA_MAX_CAMS) return GS_ERR_CAPACITY;
    gs_ba* b = new gs_ba();
    b->max_points = max_points;
    b->max_cams = max_cams;
    hipError_t e = hipMalloc((void**)&b->pt, sizeof(double) * 12 * (size_t)std::max<int64_t>(max_points, 1));
    if (e == hipSuccess)
        e = hipMalloc((void**)&b->cam, sizeof(double) * 84 * (size_t)std::max(max_cams, 1));
    if (e == hipSuccess) e = hipMalloc((void**)&b->cam_off, sizeof(int32_t) * ((size_t)max_cams + 1));
    if (e == hipSuccess) e = hipMalloc((void**)&b->sc, sizeof(double) * 16);
    if (e != hipSuccess) {
        gs_ba_destroy(b);
        return GS_ERR_HIP;
    }
    *out = b;
    return GS_OK;
}

gs_status gs_ba_destroy(gs_ba* b) {
    if (!b) return GS_ERR_INVALID_ARG;
    hipDeviceSynchronize();
    if (b->pt) hipFree(b->pt);
    if (b->cam) hipFree(b->cam);
    if (b->cam_off) hipFree(b->cam_off);
    if (b->sc) hipFree(b->sc);
    delete b;
    return GS_OK;
}

gs_status gs_ba_lm_step(gs_ba* b, const float* X, int32_t Pt, const float* viewmat, const float* intr,
                        int32_t n_cams, const int32_t* obs_cam, const int32_t* obs_pt,
                        const float* obs_xy, int32_t M, const int32_t* pt_off, const int32_t* pt_obs,
                        const int32_t* pm_cam, const float* pm_xy, float delta, float lm_lambda,
                        float near_plane, int32_t max_iter, float tol, float* d_twist, float* d_X,
                        float* stats, void* stream) {
    if (!b || Pt < 0 || n_cams < 0 || M < 0 || max_iter < 0) return GS_ERR_INVALID_ARG;
    if ((int64_t)Pt > b->max_points || n_cams > b->max_cams) return GS_ERR_CAPACITY;
    if (!(delta > 0.f) || !(lm_lambda > 0.f) || !(near_plane > 0.f) || !(tol >= 0.f)) return GS_ERR_INVALID_ARG;
    if ((n_cams > 0 && (!viewmat || !intr || !d_twist)) || (Pt > 0 && (!X || !pt_off || !d_X)) ||
        (M > 0 && (!obs_cam || !obs_pt || !obs_xy || !pt_obs)))
        return GS_ERR_INVALID_ARG;
    if ((pm_cam == nullptr) != (pm_xy == nullptr)) return GS_ERR_INVALID_ARG;  // both or neither
    gs::BaInputs in;
    in.X = X;
    in.viewmat = viewmat;
    in.intr = intr;
    in.obs_cam = obs_cam;
    in.obs_pt = obs_pt;
    in.obs_xy = obs_xy;
    in.pt_off = pt_off;
    in.pt_obs = pt_obs;
    in.pm_cam = pm_cam;
    in.pm_xy = pm_xy;
    in.Pt = Pt;
    in.n_cams = n_cams;
    in.M = M;
    in.delta = delta;
    in.lambda = lm_lambda;
    in.near_plane = near_plane;
    in.max_iter = max_iter;
    in.tol = tol;
    return gs::launch_ba_step(b, in, d_twist, d_X, stats, (hipStream_t)stream) == hipSuccess ? GS_OK
                                                                                           : GS_ERR_HIP;
}

}  // extern "C"
