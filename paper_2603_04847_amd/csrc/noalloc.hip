// track_reproj_fwd_bwd_noalloc: the track reprojection term without a
// context, for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).  Its
// accumulators (the per-camera twist sums and the loss in double, and the
// status words) live in one fixed array of device memory below instead of a
// context's workspace.
#include <math.h>

#include <cmath>
#include <mutex>

#include "gs_internal.h"

namespace {

// cameras whose twist sums the fixed array holds
constexpr int kMaxCams = GS_NOALLOC_MAX_CAMS;
// twist sums [kMaxCams][6], the loss sum, then kDiagCount status words (as
// double slots: 8 u32 words take 4)
constexpr int kScratchDoubles = 6 * kMaxCams + 2 + (gs::kDiagCount + 1) / 2;

// One copy per GPU the library runs on, held until the process ends.  Host
// code never uses this name as an address: it uses the per-device pointer
// hipGetSymbolAddress returns.
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double* g_ptr[GS_NOALLOC_MAX_DEVICES] = {};

// The device address of this GPU's copy of `scratch`, looked up once per
// device with that device current (it is the current one here).
hipError_t scratch_ptr(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= GS_NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" gs_status track_reproj_fwd_bwd_noalloc(
    const float* X, int32_t Pt, const float* viewmat, const float* intr, int32_t n_cams,
    const int32_t* obs_cam, const int32_t* obs_pt, const float* obs_xy, int32_t M, float delta,
    float lambda, float near_plane, float* residual, float* loss, float* v_X, float* v_twist,
    float* J_pose, float* J_X, const int32_t* pt_off, const int32_t* pt_obs, void* stream) {
    if (Pt < 0 || n_cams < 0 || M < 0) return GS_ERR_INVALID_ARG;
    if (n_cams > kMaxCams) return GS_ERR_CAPACITY;
    if (M > 0 && (!X || !viewmat || !intr || !obs_cam || !obs_pt || !obs_xy)) return GS_ERR_INVALID_ARG;
    if (!(delta > 0.f) || !(near_plane > 0.f) || !std::isfinite(lambda)) return GS_ERR_INVALID_ARG;
    if (!v_twist && M > 0) return GS_ERR_INVALID_ARG;  // the twist sums must be drained
    if (!loss && M > 0) return GS_ERR_INVALID_ARG;
    if ((pt_off == nullptr) != (pt_obs == nullptr)) return GS_ERR_INVALID_ARG;
    double* base = nullptr;
    if (scratch_ptr(&base) != hipSuccess) return GS_ERR_HIP;
    const hipStream_t st = (hipStream_t)stream;
    // the sums this call uses start at zero whatever an earlier call left
    // (a fill kernel, not a memset node, so the call stays graph-capturable)
    const int64_t used = 6 * (int64_t)n_cams;
    double* twist_acc = base;
    double* loss_acc = base + 6 * kMaxCams;
    uint32_t* diag = reinterpret_cast<uint32_t*>(base + 6 * kMaxCams + 2);
    if (gs::launch_fill_f64(twist_acc, 0.0, used, st) != hipSuccess ||
        gs::launch_fill_f64(loss_acc, 0.0, 1, st) != hipSuccess ||
        gs::launch_fill_u32(diag, 0u, gs::kDiagCount, st) != hipSuccess)
        return GS_ERR_HIP;
    const gs::TrackScratch sc = {twist_acc, loss_acc, diag};
    return gs::launch_track_scratch(sc, X, Pt, viewmat, intr, n_cams, obs_cam, obs_pt, obs_xy, M,
                                    delta, lambda, near_plane, residual, loss, v_X, v_twist, J_pose,
                                    J_X, pt_off, pt_obs, st) == hipSuccess
               ? GS_OK
               : GS_ERR_HIP;
}
