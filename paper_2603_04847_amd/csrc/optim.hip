// Pose composition Exp(xi) T0 and its backward, the multi-tensor Adam step, and
// small utility kernels (accumulator flush, fill).
#include "gs_internal.h"

namespace gs {

namespace {

// Coefficients of the SO(3)/SE(3) exponential: A = sin t / t,
// B = (1 - cos t) / t^2, Cc = (t - sin t) / t^3, by their Taylor series for
// small angles (where the closed forms cancel catastrophically in float).
__device__ __forceinline__ void exp_coeffs(float th2, float& A, float& B, float& Cc) {
    if (th2 < 0.09f) {
        const float t2 = th2, t4 = t2 * t2, t6 = t4 * t2, t8 = t4 * t4;
        A = 1.f - t2 / 6.f + t4 / 120.f - t6 / 5040.f + t8 / 362880.f;
        B = 0.5f - t2 / 24.f + t4 / 720.f - t6 / 40320.f + t8 / 3628800.f;
        Cc = 1.f / 6.f - t2 / 120.f + t4 / 5040.f - t6 / 362880.f + t8 / 39916800.f;
    } else {
        const float th = sqrtf(th2), s = sinf(th), c = cosf(th);
        A = s / th;
        B = (1.f - c) / th2;
        Cc = (th - s) / (th2 * th);
    }
}

__device__ __forceinline__ void cross3(const float* a, const float* b, float* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__global__ void k_pose_compose(int V, const float* __restrict__ twist, const float* __restrict__ base,
                               float* __restrict__ out) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const float* x = twist + 6 * v;
    const float rho[3] = {x[0], x[1], x[2]}, phi[3] = {x[3], x[4], x[5]};
    float A, B, Cc;
    exp_coeffs(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2], A, B, Cc);
    // K = [phi]x, K2 = K K
    const float K[9] = {0.f, -phi[2], phi[1], phi[2], 0.f, -phi[0], -phi[1], phi[0], 0.f};
    float K2[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++)
            K2[3 * r + c] = K[3 * r] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
    float Re[9], Vm[9];
    for (int i = 0; i < 9; i++) {
        const float I = (i % 4 == 0) ? 1.f : 0.f;
        Re[i] = I + A * K[i] + B * K2[i];
        Vm[i] = I + B * K[i] + Cc * K2[i];
    }
    const float* b = base + 12 * v;
    float* o = out + 12 * v;
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++)
            o[4 * r + c] = Re[3 * r] * b[c] + Re[3 * r + 1] * b[4 + c] + Re[3 * r + 2] * b[8 + c];
        o[4 * r + 3] = Re[3 * r] * b[3] + Re[3 * r + 1] * b[7] + Re[3 * r + 2] * b[11] +
                       Vm[3 * r] * rho[0] + Vm[3 * r + 1] * rho[1] + Vm[3 * r + 2] * rho[2];
    }
}

// out = J_l(xi)^T g with J_l = sum_n ad_xi^n / (n+1)!, ad_xi = [[phi]x, [rho]x; 0, [phi]x]:
// (ad^T)(w1, w2) = (w1 x phi, w1 x rho + w2 x phi).
__global__ void k_pose_compose_bwd(int V, const float* __restrict__ twist, const float* __restrict__ g,
                                   float* __restrict__ out) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const float rho[3] = {twist[6 * v], twist[6 * v + 1], twist[6 * v + 2]};
    const float phi[3] = {twist[6 * v + 3], twist[6 * v + 4], twist[6 * v + 5]};
    float w1[3] = {g[6 * v], g[6 * v + 1], g[6 * v + 2]};
    float w2[3] = {g[6 * v + 3], g[6 * v + 4], g[6 * v + 5]};
    float acc[6] = {w1[0], w1[1], w1[2], w2[0], w2[1], w2[2]};
    float fact = 1.f;
    for (int n = 1; n < 30; n++) {
        float a[3], b1[3], b2[3];
        cross3(w1, phi, a);
        cross3(w1, rho, b1);
        cross3(w2, phi, b2);
        for (int e = 0; e < 3; e++) {
            w1[e] = a[e];
            w2[e] = b1[e] + b2[e];
        }
        fact /= (float)(n + 1);
        for (int e = 0; e < 3; e++) {
            acc[e] += w1[e] * fact;
            acc[3 + e] += w2[e] * fact;
        }
    }
    for (int e = 0; e < 6; e++) out[6 * v + e] = acc[e];
}

struct AdamArgs {
    float* p[GS_ADAM_MAX_GROUPS];
    const float* g[GS_ADAM_MAX_GROUPS];
    float* m[GS_ADAM_MAX_GROUPS];
    float* v[GS_ADAM_MAX_GROUPS];
    float lr[GS_ADAM_MAX_GROUPS];
    int64_t n[GS_ADAM_MAX_GROUPS];
    int64_t blk[GS_ADAM_MAX_GROUPS + 1];  // first block of each group
    int vec[GS_ADAM_MAX_GROUPS];          // all four arrays 16-byte aligned
    int ng;
};

constexpr int kAdamPerBlock = 256 * 4;

// Each block updates 1024 consecutive elements of one group (float4 loads
// when the group is 16-byte aligned).
__global__ __launch_bounds__(256) void k_adam(AdamArgs a, float b1, float b2, float eps,
                                              const int32_t* __restrict__ step_dev, int step) {
    float ibc1, ibc2;
    adam_bias(step_dev, step, b1, b2, ibc1, ibc2);
    int q = 0;
    while (q + 1 < a.ng && (int64_t)blockIdx.x >= a.blk[q + 1]) q++;
    const int64_t i0 = ((int64_t)blockIdx.x - a.blk[q]) * kAdamPerBlock;
    const int64_t n = a.n[q];
    const float lr = a.lr[q];
    if (a.vec[q] && i0 + kAdamPerBlock <= n) {
        const int64_t j = i0 / 4 + threadIdx.x;
        float4 p = reinterpret_cast<float4*>(a.p[q])[j];
        const float4 g = reinterpret_cast<const float4*>(a.g[q])[j];
        float4 m = reinterpret_cast<float4*>(a.m[q])[j];
        float4 v = reinterpret_cast<float4*>(a.v[q])[j];
        adam_one(p.x, g.x, m.x, v.x, lr, b1, b2, eps, ibc1, ibc2);
        adam_one(p.y, g.y, m.y, v.y, lr, b1, b2, eps, ibc1, ibc2);
        adam_one(p.z, g.z, m.z, v.z, lr, b1, b2, eps, ibc1, ibc2);
        adam_one(p.w, g.w, m.w, v.w, lr, b1, b2, eps, ibc1, ibc2);
        reinterpret_cast<float4*>(a.p[q])[j] = p;
        reinterpret_cast<float4*>(a.m[q])[j] = m;
        reinterpret_cast<float4*>(a.v[q])[j] = v;
    } else {
        for (int64_t j = i0 + threadIdx.x; j < min(n, i0 + kAdamPerBlock); j += 256)
            adam_one(a.p[q][j], a.g[q][j], a.m[q][j], a.v[q][j], lr, b1, b2, eps, ibc1, ibc2);
    }
}

__global__ void k_fill_f64(double* __restrict__ p, double v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_step_advance(int32_t* __restrict__ step_dev) {
    if (threadIdx.x == 0) *step_dev += 1;
}

__global__ void k_flush_acc(double* __restrict__ acc, float* __restrict__ out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        out[i] += (float)acc[i];
        acc[i] = 0.0;
    }
}

__global__ void k_flush_twist_rows(double* __restrict__ acc, float* __restrict__ out, ViewTable vt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 6 * vt.V) {
        const int v = i / 6, e = i % 6;
        out[6 * vt.cam[v] + e] += (float)acc[i];
        acc[i] = 0.0;
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

hipError_t launch_pose_compose(int V, const float* twist, const float* base, float* out,
                               hipStream_t st) {
    if (V <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pose_compose, dim3((V + 63) / 64), dim3(64), 0, st, V, twist, base, out);
    return hipGetLastError();
}

hipError_t launch_pose_compose_bwd(int V, const float* twist, const float* g, float* out,
                                   hipStream_t st) {
    if (V <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pose_compose_bwd, dim3((V + 63) / 64), dim3(64), 0, st, V, twist, g, out);
    return hipGetLastError();
}

hipError_t launch_adam(const gs_adam_group* groups, int n, int step, const int32_t* step_dev,
                       float b1, float b2, float eps, hipStream_t st) {
    AdamArgs a{};
    a.ng = n;
    a.blk[0] = 0;
    auto al = [](const void* p) { return ((uintptr_t)p & 15u) == 0; };
    for (int q = 0; q < n; q++) {
        a.p[q] = groups[q].param;
        a.g[q] = groups[q].grad;
        a.m[q] = groups[q].exp_avg;
        a.v[q] = groups[q].exp_avg_sq;
        a.lr[q] = groups[q].lr;
        a.n[q] = groups[q].n;
        a.vec[q] = al(a.p[q]) && al(a.g[q]) && al(a.m[q]) && al(a.v[q]);
        a.blk[q + 1] = a.blk[q] + (groups[q].n + kAdamPerBlock - 1) / kAdamPerBlock;
    }
    const int64_t blocks = a.blk[n];
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, st, a, b1, b2, eps, step_dev, step);
    return hipGetLastError();
}

hipError_t launch_step_advance(int32_t* step_dev, hipStream_t st) {
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, st, step_dev);
    return hipGetLastError();
}

hipError_t launch_flush_acc(double* acc, float* out, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flush_acc, dim3((n + 255) / 256), dim3(256), 0, st, acc, out, n);
    return hipGetLastError();
}

hipError_t launch_flush_twist_rows(double* acc, float* out, const ViewTable& vt, hipStream_t st) {
    if (vt.V <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flush_twist_rows, dim3((6 * vt.V + 255) / 256), dim3(256), 0, st, acc, out, vt);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

}  // namespace gs
