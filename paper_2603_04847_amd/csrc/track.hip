// Track reprojection residual, Huber loss and their gradients / Jacobian blocks.
//
// One thread per observation; each workgroup walks one contiguous range of
// observations.  Observations arrive sorted by camera, so a wave sees the same
// camera for many steps: it keeps per-lane twist sums while the camera stays
// and adds them (one wave sum, one double atomic per component) only when the
// camera changes and at the end, which keeps the atomics on each camera's six
// words few.  A step whose lanes straddle a camera boundary uses per-lane
// atomics.  Track-point gradients are
// scattered with three float atomics per observation (points are spread, so
// these rarely collide), or, given a point-major index of the observations,
// summed per point by a kernel of their own with no atomics.
//
// Given also the observations' cameras and pixels copied into point-major
// order (once per scene), the whole term is one pass over the points that
// reads every array in order: each workgroup keeps per-camera twist sums in
// LDS (float atomics there, no global atomics), writes them out once, and a
// second kernel sums the workgroups' rows in a fixed order in double.  Without the copies the
// camera-major pass gathers a random point per observation and the point
// pass a random observation per index entry.
#include <algorithm>

#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kBlock = 256;

constexpr int kTrackBlocks = 1024;

// One observation's terms, the same arithmetic for every kernel that needs
// them: camera point p = R X + t; masked if p_z < near; else the residual r,
// the Huber value rho and the 2D gradient g = d(lambda rho)/dr pushed through
// the projection: vp = J_pi^T g (the gradient at p).
struct ObsTerms {
    float R[9], p[3];
    float r0, r1, rho, j00, j02, j11, j12, vp[3];
    bool masked;
};

__device__ __forceinline__ void obs_terms(const float* __restrict__ X, int k,
                                          const float* __restrict__ viewmat,
                                          const float* __restrict__ intr, int ci,
                                          const float* __restrict__ obs_xy, int o, float delta,
                                          float lambda, float near_plane, ObsTerms& T) {
    float t[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
#pragma unroll
        for (int c = 0; c < 3; c++) T.R[3 * r + c] = viewmat[12 * ci + 4 * r + c];
        t[r] = viewmat[12 * ci + 4 * r + 3];
    }
    const float fx = intr[4 * ci], fy = intr[4 * ci + 1], cx = intr[4 * ci + 2], cy = intr[4 * ci + 3];
    const float Xk[3] = {X[3 * (int64_t)k], X[3 * (int64_t)k + 1], X[3 * (int64_t)k + 2]};
#pragma unroll
    for (int r = 0; r < 3; r++)
        T.p[r] = T.R[3 * r] * Xk[0] + T.R[3 * r + 1] * Xk[1] + T.R[3 * r + 2] * Xk[2] + t[r];
    T.masked = !(T.p[2] >= near_plane);
    if (T.masked) return;
    const float iz = 1.f / T.p[2];
    const float u = T.p[0] * iz, w = T.p[1] * iz;
    T.r0 = fx * u + cx - obs_xy[2 * (int64_t)o];
    T.r1 = fy * w + cy - obs_xy[2 * (int64_t)o + 1];
    const float s = T.r0 * T.r0 + T.r1 * T.r1;
    float drho;
    if (s <= delta * delta) {
        T.rho = s;
        drho = 1.f;
    } else {
        const float rs = sqrtf(s);
        T.rho = 2.f * delta * rs - delta * delta;
        drho = delta / rs;
    }
    // J_pi (2x3) = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]]
    T.j00 = fx * iz;
    T.j02 = -fx * u * iz;
    T.j11 = fy * iz;
    T.j12 = -fy * w * iz;
    const float g0 = 2.f * lambda * drho * T.r0, g1 = 2.f * lambda * drho * T.r1;
    T.vp[0] = T.j00 * g0;
    T.vp[1] = T.j11 * g1;
    T.vp[2] = T.j02 * g0 + T.j12 * g1;
}

__global__ __launch_bounds__(kBlock) void k_track(
    const float* __restrict__ X, int Pt, const float* __restrict__ viewmat,
    const float* __restrict__ intr, int n_cams, const int32_t* __restrict__ obs_cam,
    const int32_t* __restrict__ obs_pt, const float* __restrict__ obs_xy, int M, float delta,
    float lambda, float near_plane, float* __restrict__ residual, float* __restrict__ v_X,
    float* __restrict__ J_pose, float* __restrict__ J_X, double* __restrict__ twist_acc,
    double* __restrict__ loss_acc, uint32_t* __restrict__ diag) {
    __shared__ float s_loss[kBlock / kWave];
    __shared__ uint32_t s_mask[kBlock / kWave];
    const int lane = __lane_id();
    float lo_sum = 0.f;
    uint32_t n_masked = 0;
    // this workgroup's range, a multiple of the workgroup size long
    const int per = ((M + (int)gridDim.x - 1) / (int)gridDim.x + kBlock - 1) / kBlock * kBlock;
    const int lo = (int)min((int64_t)blockIdx.x * per, (int64_t)M);
    const int hi = min(lo + per, M);
    float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // lane sums for camera `cur`
    int cur = -1;                                   // wave-uniform
    auto flush = [&]() {
        if (cur >= 0) {
#pragma unroll
            for (int e = 0; e < 6; e++) {
                const float s = wave_sum(acc[e]);
                if (lane == e && s != 0.f) atomicAdd(twist_acc + 6 * (int64_t)cur + e, (double)s);
                acc[e] = 0.f;
            }
        }
    };
    // block-level sums of the loss and the masked count end in one atomic per block
    for (int base = lo; base < hi; base += kBlock) {
    const int o = base + threadIdx.x;
    const bool in = o < hi;
    int ci = 0, k = 0;
    if (in) {
        ci = obs_cam[o];
        k = obs_pt[o];
    }
    const bool ok_idx = in && ci >= 0 && ci < n_cams && k >= 0 && k < Pt;
    float tw[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    bool masked = false;
    if (ok_idx) {
        ObsTerms T;
        obs_terms(X, k, viewmat, intr, ci, obs_xy, o, delta, lambda, near_plane, T);
        masked = T.masked;
        if (masked) {
            n_masked++;
            if (residual) {
                residual[2 * (int64_t)o] = 0.f;
                residual[2 * (int64_t)o + 1] = 0.f;
            }
            if (J_pose)
                for (int e = 0; e < 12; e++) J_pose[12 * (int64_t)o + e] = 0.f;
            if (J_X)
                for (int e = 0; e < 6; e++) J_X[6 * (int64_t)o + e] = 0.f;
        } else {
            const float* R = T.R;
            const float* p = T.p;
            const float* vp = T.vp;
            lo_sum += lambda * T.rho;
            if (v_X) {
#pragma unroll
                for (int c = 0; c < 3; c++)
                    atomicAdd(v_X + 3 * (int64_t)k + c, R[c] * vp[0] + R[3 + c] * vp[1] + R[6 + c] * vp[2]);
            }
            tw[0] = vp[0];
            tw[1] = vp[1];
            tw[2] = vp[2];
            tw[3] = p[1] * vp[2] - p[2] * vp[1];
            tw[4] = p[2] * vp[0] - p[0] * vp[2];
            tw[5] = p[0] * vp[1] - p[1] * vp[0];
            if (residual) {
                residual[2 * (int64_t)o] = T.r0;
                residual[2 * (int64_t)o + 1] = T.r1;
            }
            const float j00 = T.j00, j02 = T.j02, j11 = T.j11, j12 = T.j12;
            if (J_pose) {
                // dr/dxi = J_pi [I | -[p]x]
                float* Jp = J_pose + 12 * (int64_t)o;
                Jp[0] = j00; Jp[1] = 0.f; Jp[2] = j02;
                Jp[3] = j02 * p[1];
                Jp[4] = j00 * p[2] - j02 * p[0];
                Jp[5] = -j00 * p[1];
                Jp[6] = 0.f; Jp[7] = j11; Jp[8] = j12;
                Jp[9] = -j11 * p[2] + j12 * p[1];
                Jp[10] = -j12 * p[0];
                Jp[11] = j11 * p[0];
            }
            if (J_X) {
                float* Jx = J_X + 6 * (int64_t)o;
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    Jx[c] = j00 * R[c] + j02 * R[6 + c];
                    Jx[3 + c] = j11 * R[3 + c] + j12 * R[6 + c];
                }
            }
        }
    }
    // twist: one camera for the whole wave is the common case
    const uint64_t live = __ballot(ok_idx && !masked);
    if (live != 0) {
        const int first = __builtin_ctzll(live);
        const int c0 = bcast(ci, first);
        const bool uniform = __ballot(ok_idx && !masked && ci != c0) == 0;
        if (uniform) {
            if (c0 != cur) {
                flush();
                cur = c0;
            }
#pragma unroll
            for (int e = 0; e < 6; e++) acc[e] += tw[e];
        } else if (ok_idx && !masked) {
#pragma unroll
            for (int e = 0; e < 6; e++) atomicAdd(twist_acc + 6 * (int64_t)ci + e, (double)tw[e]);
        }
    }
    }
    flush();
    const float ls = wave_sum(lo_sum);
    uint32_t nm = n_masked;
    for (int off = 32; off > 0; off >>= 1) nm += __shfl_xor(nm, off, kWave);
    if (lane == 0) {
        s_loss[threadIdx.x / kWave] = ls;
        s_mask[threadIdx.x / kWave] = nm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0.0;
        uint32_t tm = 0;
        for (int q = 0; q < kBlock / kWave; q++) {
            tot += s_loss[q];
            tm += s_mask[q];
        }
        if (tot != 0.0) atomicAdd(loss_acc, tot);
        if (tm) atomicAdd(&diag[kDiagMasked], tm);
    }
}

// The track points' gradients from a point-major index of the observations
// (pt_off[Pt + 1], pt_obs: a point's observations, ascending): one thread per
// point recomputes its observations' terms and adds their sum once, with no
// atomics, in a fixed order.
__global__ __launch_bounds__(kBlock) void k_track_points(
    const float* __restrict__ X, int Pt, const float* __restrict__ viewmat,
    const float* __restrict__ intr, int n_cams, const int32_t* __restrict__ obs_cam,
    const float* __restrict__ obs_xy, const int32_t* __restrict__ pt_off,
    const int32_t* __restrict__ pt_obs, float delta, float lambda, float near_plane,
    float* __restrict__ v_X, double* __restrict__ twist_acc, float* __restrict__ v_twist,
    double* __restrict__ loss_acc, float* __restrict__ loss) {
    // the first workgroup also drains k_track's twist and loss sums (that
    // kernel has finished: this one runs after it on the same stream)
    if (blockIdx.x == 0) {
        if (v_twist)
            for (int q = threadIdx.x; q < 6 * n_cams; q += kBlock) {
                v_twist[q] += (float)twist_acc[q];
                twist_acc[q] = 0.0;
            }
        if (loss && threadIdx.x == 0) {
            *loss += (float)*loss_acc;
            *loss_acc = 0.0;
        }
    }
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= Pt) return;
    float acc[3] = {0.f, 0.f, 0.f};
    const int j1 = pt_off[k + 1];
    for (int j = pt_off[k]; j < j1; j++) {
        const int o = pt_obs[j];
        const int ci = obs_cam[o];
        if (ci < 0 || ci >= n_cams) continue;
        ObsTerms T;
        obs_terms(X, k, viewmat, intr, ci, obs_xy, o, delta, lambda, near_plane, T);
        if (T.masked) continue;
#pragma unroll
        for (int c = 0; c < 3; c++) acc[c] += T.R[c] * T.vp[0] + T.R[3 + c] * T.vp[1] + T.R[6 + c] * T.vp[2];
    }
#pragma unroll
    for (int c = 0; c < 3; c++) v_X[3 * (int64_t)k + c] += acc[c];
}

// The point-major pass (see the file comment): one thread per point (grid
// stride), its observations' terms from the point-major copies; v_X written
// once per point; twist sums per workgroup in LDS, 6 n_cams floats.  (One
// thread per observation, the point found by a search of the chunk's offsets
// in LDS and its gradient gathered by LDS atomics, measured 30% slower: the
// search is a chain of dependent LDS loads and a point's observations collide
// on its three words.)
__global__ __launch_bounds__(kBlock) void k_track_pm(
    const float* __restrict__ X, int Pt, const float* __restrict__ viewmat,
    const float* __restrict__ intr, int n_cams, const int32_t* __restrict__ pt_off,
    const int32_t* __restrict__ pm_cam, const float* __restrict__ pm_xy, float delta, float lambda,
    float near_plane, float* __restrict__ v_X, float* __restrict__ part,
    double* __restrict__ loss_part, uint32_t* __restrict__ diag) {
    extern __shared__ float s_tw[];  // [n_cams][6]
    __shared__ float s_loss[kBlock / kWave];
    __shared__ uint32_t s_mask[kBlock / kWave];
    for (int q = threadIdx.x; q < 6 * n_cams; q += kBlock) s_tw[q] = 0.f;
    __syncthreads();
    float lo_sum = 0.f;
    uint32_t n_masked = 0;
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < Pt; k += gridDim.x * kBlock) {
        const int j0 = pt_off[k], j1 = pt_off[k + 1];
        if (j0 >= j1) continue;
        float acc[3] = {0.f, 0.f, 0.f};
        for (int j = j0; j < j1; j++) {
            const int ci = pm_cam[j];
            if (ci < 0 || ci >= n_cams) continue;
            ObsTerms T;
            obs_terms(X, k, viewmat, intr, ci, pm_xy, j, delta, lambda, near_plane, T);
            if (T.masked) {
                n_masked++;
                continue;
            }
            lo_sum += lambda * T.rho;
            const float* R = T.R;
            const float* p = T.p;
            const float* vp = T.vp;
#pragma unroll
            for (int c = 0; c < 3; c++) acc[c] += R[c] * vp[0] + R[3 + c] * vp[1] + R[6 + c] * vp[2];
            float* tw = s_tw + 6 * ci;
            atomicAdd(tw + 0, vp[0]);
            atomicAdd(tw + 1, vp[1]);
            atomicAdd(tw + 2, vp[2]);
            atomicAdd(tw + 3, p[1] * vp[2] - p[2] * vp[1]);
            atomicAdd(tw + 4, p[2] * vp[0] - p[0] * vp[2]);
            atomicAdd(tw + 5, p[0] * vp[1] - p[1] * vp[0]);
        }
#pragma unroll
        for (int c = 0; c < 3; c++) v_X[3 * (int64_t)k + c] += acc[c];
    }
    const float ls = wave_sum(lo_sum);
    uint32_t nm = n_masked;
    for (int off = 32; off > 0; off >>= 1) nm += __shfl_xor(nm, off, kWave);
    if (__lane_id() == 0) {
        s_loss[threadIdx.x / kWave] = ls;
        s_mask[threadIdx.x / kWave] = nm;
    }
    __syncthreads();
    float* row = part + (int64_t)blockIdx.x * 6 * n_cams;
    for (int q = threadIdx.x; q < 6 * n_cams; q += kBlock) row[q] = s_tw[q];
    if (threadIdx.x == 0) {
        double tot = 0.0;
        uint32_t tm = 0;
        for (int q = 0; q < kBlock / kWave; q++) {
            tot += s_loss[q];
            tm += s_mask[q];
        }
        loss_part[blockIdx.x] = tot;
        if (tm) atomicAdd(&diag[kDiagMasked], tm);
    }
}

// Sum of the point-major pass's workgroup rows, in double and a fixed order:
// 64 columns per workgroup, eight waves over interleaved rows; workgroup 0
// also sums the loss.
constexpr int kPmReduceWaves = 8;

__global__ __launch_bounds__(kWave * kPmReduceWaves) void k_track_pm_reduce(
    const float* __restrict__ part, const double* __restrict__ loss_part, int nblk, int n6,
    float* __restrict__ v_twist, float* __restrict__ loss) {
    __shared__ double s[kPmReduceWaves][kWave];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int q = blockIdx.x * kWave + lane;
    double a = 0.0;
    if (q < n6)
        for (int b = w; b < nblk; b += kPmReduceWaves) a += part[(int64_t)b * n6 + q];
    s[w][lane] = a;
    __syncthreads();
    if (w == 0 && q < n6) {
        double t = 0.0;
        for (int i = 0; i < kPmReduceWaves; i++) t += s[i][lane];
        v_twist[q] += (float)t;
    }
    if (blockIdx.x == 0) {
        __syncthreads();
        double l = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kWave * kPmReduceWaves) l += loss_part[b];
        s[w][lane] = l;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int i = 0; i < kPmReduceWaves; i++)
                for (int j = 0; j < kWave; j++) t += s[i][j];
            *loss += (float)t;
        }
    }
}

// The observations' cameras and pixels in the index's order.
__global__ __launch_bounds__(kBlock) void k_pm_gather(const int32_t* __restrict__ pt_off, int Pt,
                                                      const int32_t* __restrict__ pt_obs,
                                                      const int32_t* __restrict__ obs_cam,
                                                      const float2* __restrict__ obs_xy,
                                                      int32_t* __restrict__ pm_cam,
                                                      float2* __restrict__ pm_xy) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= pt_off[Pt]) return;
    const int o = pt_obs[j];
    pm_cam[j] = obs_cam[o];
    pm_xy[j] = obs_xy[o];
}

// The point-major index: counts per point, their scan, a fill through one
// cursor per point, then each point's observations sorted ascending.
__global__ __launch_bounds__(kBlock) void k_pt_count(const int32_t* __restrict__ obs_pt, int M, int Pt,
                                                     int32_t* __restrict__ cnt) {
    const int o = blockIdx.x * kBlock + threadIdx.x;
    if (o >= M) return;
    const int k = obs_pt[o];
    if (k >= 0 && k < Pt) atomicAdd(&cnt[k], 1);
}

__global__ __launch_bounds__(kBlock) void k_pt_fill(const int32_t* __restrict__ obs_pt, int M, int Pt,
                                                    const int32_t* __restrict__ pt_off,
                                                    uint32_t* __restrict__ cursor,
                                                    int32_t* __restrict__ pt_obs) {
    const int o = blockIdx.x * kBlock + threadIdx.x;
    if (o >= M) return;
    const int k = obs_pt[o];
    if (k >= 0 && k < Pt) pt_obs[pt_off[k] + (int)atomicAdd(&cursor[k], 1u)] = o;
}

__global__ __launch_bounds__(kBlock) void k_pt_sort(int Pt, const int32_t* __restrict__ pt_off,
                                                    int32_t* __restrict__ pt_obs) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= Pt) return;
    const int j0 = pt_off[k], j1 = pt_off[k + 1];
    for (int j = j0 + 1; j < j1; j++) {  // insertion sort: tracks are short
        const int v = pt_obs[j];
        int i = j - 1;
        while (i >= j0 && pt_obs[i] > v) {
            pt_obs[i + 1] = pt_obs[i];
            i--;
        }
        pt_obs[i + 1] = v;
    }
}

}  // namespace

hipError_t launch_track(Ctx* c, const float* X, int Pt, const float* viewmat, const float* intr,
                        int n_cams, const int32_t* obs_cam, const int32_t* obs_pt,
                        const float* obs_xy, int M, float delta, float lambda, float near_plane,
                        float* residual, float* loss, float* v_X, float* v_twist, float* J_pose,
                        float* J_X, const int32_t* pt_off, const int32_t* pt_obs,
                        const int32_t* pm_cam, const float* pm_xy, hipStream_t st) {
    const bool pm = pm_cam && pm_xy && pt_off && pt_obs && v_X && v_twist && loss && !residual &&
                    !J_pose && !J_X && n_cams <= c->pm_cams && c->track_part;
    if (pm && M > 0 && Pt > 0) {
        hipLaunchKernelGGL(k_track_pm, dim3(kTrackPmBlocks), dim3(kBlock), sizeof(float) * 6 * n_cams, st,
                           X, Pt, viewmat, intr, n_cams, pt_off, pm_cam, pm_xy, delta, lambda, near_plane,
                           v_X, c->track_part, c->track_loss_part, c->diag);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int n6 = 6 * n_cams;
        hipLaunchKernelGGL(k_track_pm_reduce, dim3((unsigned)std::max((n6 + kWave - 1) / kWave, 1)),
                           dim3(kWave * kPmReduceWaves), 0, st, c->track_part, c->track_loss_part,
                           kTrackPmBlocks, n6, v_twist, loss);
        return hipGetLastError();
    }
    const TrackScratch sc = {c->twist_track, c->loss_acc + 1, c->diag};
    return launch_track_scratch(sc, X, Pt, viewmat, intr, n_cams, obs_cam, obs_pt, obs_xy, M, delta,
                                lambda, near_plane, residual, loss, v_X, v_twist, J_pose, J_X, pt_off,
                                pt_obs, st);
}

hipError_t launch_track_scratch(const TrackScratch& sc, const float* X, int Pt, const float* viewmat,
                                const float* intr, int n_cams, const int32_t* obs_cam,
                                const int32_t* obs_pt, const float* obs_xy, int M, float delta,
                                float lambda, float near_plane, float* residual, float* loss,
                                float* v_X, float* v_twist, float* J_pose, float* J_X,
                                const int32_t* pt_off, const int32_t* pt_obs, hipStream_t st) {
    const bool indexed = pt_off && pt_obs && v_X;
    if (M > 0) {
        // with the point index the point gradients come from k_track_points
        hipLaunchKernelGGL(k_track, dim3(std::min((M + kBlock - 1) / kBlock, kTrackBlocks)),
                           dim3(kBlock), 0, st, X, Pt,
                           viewmat, intr, n_cams, obs_cam, obs_pt, obs_xy, M, delta, lambda,
                           near_plane, residual, indexed ? nullptr : v_X, J_pose, J_X, sc.twist_acc,
                           sc.loss_acc, sc.diag);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (indexed && Pt > 0) {
            // the point gradients, and the drain of the twist and loss sums
            hipLaunchKernelGGL(k_track_points, dim3((Pt + kBlock - 1) / kBlock), dim3(kBlock), 0, st, X,
                               Pt, viewmat, intr, n_cams, obs_cam, obs_xy, pt_off, pt_obs, delta, lambda,
                               near_plane, v_X, sc.twist_acc, v_twist, sc.loss_acc, loss);
            return hipGetLastError();
        }
    }
    hipError_t e = hipSuccess;
    if (v_twist && (e = launch_flush_acc(sc.twist_acc, v_twist, 6 * n_cams, st)) != hipSuccess)
        return e;
    if (loss) return launch_flush_acc(sc.loss_acc, loss, 1, st);
    return hipSuccess;
}

hipError_t launch_track_index(Ctx* c, const int32_t* obs_pt, int M, int Pt, int32_t* pt_off,
                              int32_t* pt_obs, const int32_t* obs_cam, const float* obs_xy,
                              int32_t* pm_cam, float* pm_xy, hipStream_t st) {
    // counts in pt_off[0, Pt) (pt_off[Pt] = 0), their exclusive scan (pt_off[Pt]
    // becomes the number indexed), then the fill through cursors in c->cnt
    hipError_t e;
    if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(pt_off), 0u, (int64_t)Pt + 1, st)) != hipSuccess)
        return e;
    if (Pt == 0) return hipSuccess;
    if ((e = launch_fill_u32(c->cnt, 0u, Pt, st)) != hipSuccess) return e;
    const unsigned gm = (unsigned)((M + kBlock - 1) / kBlock), gp = (unsigned)((Pt + kBlock - 1) / kBlock);
    if (M > 0) {
        hipLaunchKernelGGL(k_pt_count, dim3(gm), dim3(kBlock), 0, st, obs_pt, M, Pt, pt_off);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = exclusive_scan_u32(reinterpret_cast<uint32_t*>(pt_off), (int64_t)Pt + 1, nullptr,
                                c->scan_scratch, c->diag + kDiagFlags, st)) != hipSuccess)
        return e;
    if (M > 0) {
        hipLaunchKernelGGL(k_pt_fill, dim3(gm), dim3(kBlock), 0, st, obs_pt, M, Pt, pt_off, c->cnt, pt_obs);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_pt_sort, dim3(gp), dim3(kBlock), 0, st, Pt, pt_off, pt_obs);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (pm_cam && obs_cam && M > 0) {
        hipLaunchKernelGGL(k_pm_gather, dim3(gm), dim3(kBlock), 0, st, pt_off, Pt, pt_obs, obs_cam,
                           reinterpret_cast<const float2*>(obs_xy), pm_cam, reinterpret_cast<float2*>(pm_xy));
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace gs
