// Front-to-back compositing over the depth-sorted tile lists, its backward, and
// the photometric L1 term.
//
// One wave (64 lanes) owns one tile of TW x TH pixels, PPL = TW*TH/64 pixels per
// lane.  The tile's list is consumed in batches of 64: each lane loads one
// splat record (a gather of 40 B) and the wave then walks the batch with the
// splat's parameters broadcast by readlane, i.e. held in scalar registers, so
// every pixel of the tile tests each splat with no LDS traffic at all.  The
// backward walks the same lists back to front from each pixel's last
// contributor, recovering the transmittance by division, and sums each
// splat's nine 2D gradients over the whole wave (DPP) before one lane per
// component issues the global atomic.
#include "gs_internal.h"

namespace gs {

namespace {

__device__ __forceinline__ int tile_view(const ViewTable& vt, int t) {
    int v = 0;
    while (v + 1 < vt.V && t >= vt.tile_off[v + 1]) v++;
    return v;
}

template <int TW, int TH>
__global__ __launch_bounds__(64) void k_render_fwd(const float4* __restrict__ rec,
                                                   const int32_t* __restrict__ ids,
                                                   const int32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ order, ViewTable vt,
                                                   RasterParams rp, const float* __restrict__ bg,
                                                   float* __restrict__ out_rgb,
                                                   float* __restrict__ out_T,
                                                   int32_t* __restrict__ out_last) {
    constexpr int PPL = TW * TH / kWave;
    constexpr int RSTEP = kWave / TW;
    const int t = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    const int v = tile_view(vt, t);
    const int lt = t - vt.tile_off[v];
    const int gx = vt.gx[v], W = vt.W[v], H = vt.H[v];
    const int tx = lt % gx, ty = lt / gx;
    const int lane = threadIdx.x;
    const int px = tx * TW + lane % TW;
    const int py0 = ty * TH + lane / TW;
    const float fx = px + 0.5f;
    float fy[PPL], T[PPL], C0[PPL], C1[PPL], C2[PPL];
    int last[PPL];
    bool done[PPL];
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        const int py = py0 + k * RSTEP;
        fy[k] = py + 0.5f;
        done[k] = !(px < W && py < H);
        T[k] = 1.f;
        C0[k] = C1[k] = C2[k] = 0.f;
        last[k] = 0;
    }
    const int s = ranges[2 * t], e = ranges[2 * t + 1];
    const float amin = rp.alpha_min, amax = rp.alpha_max, tmin = rp.t_min;
    for (int b = s; b < e; b += kWave) {
        bool alive = false;
#pragma unroll
        for (int k = 0; k < PPL; k++) alive |= !done[k];
        if (__ballot(alive) == 0) break;
        const int j = b + lane;
        float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb = ra;
        float2 rc = make_float2(0.f, 0.f);
        if (j < e) {
            const int64_t p = ids[j];
            ra = rec[3 * p];
            rb = rec[3 * p + 1];
            rc = *reinterpret_cast<const float2*>(rec + 3 * p + 2);
        }
        const int nb = min(kWave, e - b);
        for (int i = 0; i < nb; i++) {
            const float mx = bcast(ra.x, i), my = bcast(ra.y, i), o = bcast(ra.w, i);
            const float A = bcast(rb.x, i), B = bcast(rb.y, i), C = bcast(rb.z, i);
            const float cr = bcast(rb.w, i), cg = bcast(rc.x, i), cb = bcast(rc.y, i);
            const float dx = mx - fx;
#pragma unroll
            for (int k = 0; k < PPL; k++) {
                if (done[k]) continue;
                const float dy = my - fy[k];
                const float sig = splat_sigma(A, B, C, dx, dy);
                if (sig < 0.f) continue;
                const float alpha = fminf(amax, o * fast_exp_neg(sig));
                if (alpha < amin) continue;
                const float Tn = T[k] * (1.f - alpha);
                if (Tn < tmin) {
                    done[k] = true;
                    continue;
                }
                const float w = alpha * T[k];
                C0[k] = __builtin_fmaf(cr, w, C0[k]);
                C1[k] = __builtin_fmaf(cg, w, C1[k]);
                C2[k] = __builtin_fmaf(cb, w, C2[k]);
                T[k] = Tn;
                last[k] = b + i - s + 1;
            }
        }
    }
    const float b0 = bg ? bg[0] : 0.f, b1 = bg ? bg[1] : 0.f, b2 = bg ? bg[2] : 0.f;
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        const int py = py0 + k * RSTEP;
        if (px < W && py < H) {
            const int64_t pix = (int64_t)vt.pix_off[v] + (int64_t)py * W + px;
            out_rgb[3 * pix] = C0[k] + T[k] * b0;
            out_rgb[3 * pix + 1] = C1[k] + T[k] * b1;
            out_rgb[3 * pix + 2] = C2[k] + T[k] * b2;
            out_T[pix] = T[k];
            out_last[pix] = last[k];
        }
    }
}

template <int TW, int TH>
__global__ __launch_bounds__(64) void k_render_bwd(const float4* __restrict__ rec,
                                                   const int32_t* __restrict__ ids,
                                                   const int32_t* __restrict__ ranges,
                                                   const uint32_t* __restrict__ order, ViewTable vt,
                                                   RasterParams rp, const float* __restrict__ bg,
                                                   const float* __restrict__ T_final,
                                                   const int32_t* __restrict__ last_in,
                                                   const float* __restrict__ v_rgb,
                                                   float* __restrict__ grad2d) {
    constexpr int PPL = TW * TH / kWave;
    constexpr int RSTEP = kWave / TW;
    const int t = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    const int v = tile_view(vt, t);
    const int lt = t - vt.tile_off[v];
    const int gx = vt.gx[v], W = vt.W[v], H = vt.H[v];
    const int tx = lt % gx, ty = lt / gx;
    const int lane = threadIdx.x;
    const int px = tx * TW + lane % TW;
    const int py0 = ty * TH + lane / TW;
    const float fx = px + 0.5f;
    const float b0 = bg ? bg[0] : 0.f, b1 = bg ? bg[1] : 0.f, b2 = bg ? bg[2] : 0.f;
    float fy[PPL], Tc[PPL], Tf[PPL], V0[PPL], V1[PPL], V2[PPL], S0[PPL], S1[PPL], S2[PPL];
    int L[PPL];
    int lmax = 0;
#pragma unroll
    for (int k = 0; k < PPL; k++) {
        const int py = py0 + k * RSTEP;
        fy[k] = py + 0.5f;
        L[k] = 0;
        Tc[k] = Tf[k] = 1.f;
        V0[k] = V1[k] = V2[k] = 0.f;
        if (px < W && py < H) {
            const int64_t pix = (int64_t)vt.pix_off[v] + (int64_t)py * W + px;
            L[k] = last_in[pix];
            Tf[k] = Tc[k] = T_final[pix];
            V0[k] = v_rgb[3 * pix];
            V1[k] = v_rgb[3 * pix + 1];
            V2[k] = v_rgb[3 * pix + 2];
        }
        // S = sum_{later} colour alpha T + T_final bg (the background term seeds it)
        S0[k] = Tf[k] * b0;
        S1[k] = Tf[k] * b1;
        S2[k] = Tf[k] * b2;
        lmax = max(lmax, L[k]);
    }
    lmax = wave_max_i(lmax);
    const int s = ranges[2 * t], e = ranges[2 * t + 1];
    lmax = min(lmax, e - s);  // a pixel's last contributor lies inside its tile's list
    if (lmax <= 0) return;
    const float amin = rp.alpha_min, amax = rp.alpha_max;
    for (int b = s + ((lmax - 1) / kWave) * kWave; b >= s; b -= kWave) {
        const int j = b + lane;
        float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb = ra;
        float2 rc = make_float2(0.f, 0.f);
        int pid = 0;
        if (j < s + lmax) {
            pid = ids[j];
            const int64_t p = pid;
            ra = rec[3 * p];
            rb = rec[3 * p + 1];
            rc = *reinterpret_cast<const float2*>(rec + 3 * p + 2);
        }
        const int nb = min(kWave, s + lmax - b);
        for (int i = nb - 1; i >= 0; i--) {
            const float mx = bcast(ra.x, i), my = bcast(ra.y, i), o = bcast(ra.w, i);
            const float A = bcast(rb.x, i), B = bcast(rb.y, i), C = bcast(rb.z, i);
            const float cr = bcast(rb.w, i), cg = bcast(rc.x, i), cb = bcast(rc.y, i);
            const int pos = b + i - s;
            const float dx = mx - fx;
            float g_mx = 0.f, g_my = 0.f, g_A = 0.f, g_B = 0.f, g_C = 0.f, g_o = 0.f;
            float g_r = 0.f, g_g = 0.f, g_b = 0.f;
            bool any = false;
#pragma unroll
            for (int k = 0; k < PPL; k++) {
                if (pos >= L[k]) continue;
                const float dy = my - fy[k];
                const float sig = splat_sigma(A, B, C, dx, dy);
                if (sig < 0.f) continue;
                const float ex = fast_exp_neg(sig);
                const float araw = o * ex;
                const float alpha = fminf(amax, araw);
                if (alpha < amin) continue;
                any = true;
                const float om = 1.f - alpha;
                const float iom = 1.f / om;
                const float Tb = Tc[k] * iom;  // transmittance in front of this splat
                const float w = alpha * Tb;
                g_r = __builtin_fmaf(w, V0[k], g_r);
                g_g = __builtin_fmaf(w, V1[k], g_g);
                g_b = __builtin_fmaf(w, V2[k], g_b);
                const float va = V0[k] * (cr * Tb - S0[k] * iom) + V1[k] * (cg * Tb - S1[k] * iom) +
                                 V2[k] * (cb * Tb - S2[k] * iom);
                S0[k] = __builtin_fmaf(cr, w, S0[k]);
                S1[k] = __builtin_fmaf(cg, w, S1[k]);
                S2[k] = __builtin_fmaf(cb, w, S2[k]);
                Tc[k] = Tb;
                if (araw < amax) {
                    g_o = __builtin_fmaf(va, ex, g_o);
                    const float vs = -alpha * va;
                    g_mx += vs * (A * dx + B * dy);
                    g_my += vs * (B * dx + C * dy);
                    g_A += vs * 0.5f * dx * dx;
                    g_B += vs * dx * dy;
                    g_C += vs * 0.5f * dy * dy;
                }
            }
            if (__ballot(any) == 0) continue;
            const float s_mx = wave_sum(g_mx), s_my = wave_sum(g_my), s_A = wave_sum(g_A);
            const float s_B = wave_sum(g_B), s_C = wave_sum(g_C), s_o = wave_sum(g_o);
            const float s_r = wave_sum(g_r), s_g = wave_sum(g_g), s_b = wave_sum(g_b);
            if (lane < 9) {
                const float val = lane == 0 ? s_mx : lane == 1 ? s_my : lane == 2 ? s_A
                                : lane == 3 ? s_B : lane == 4 ? s_C : lane == 5 ? s_o
                                : lane == 6 ? s_r : lane == 7 ? s_g : s_b;
                const int64_t p = bcast(pid, i);
                atomicAdd(grad2d + 9 * p + lane, val);
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ rgb,
                                            const float* __restrict__ target,
                                            float* __restrict__ v_rgb, ViewTable vt,
                                            double* __restrict__ loss_acc) {
    const int64_t P = vt.pix_off[vt.V];
    const int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float part = 0.f;
    if (pix < P) {
        int v = 0;
        while (v + 1 < vt.V && pix >= vt.pix_off[v + 1]) v++;
        const float wgt = 1.f / (3.f * (float)(vt.pix_off[v + 1] - vt.pix_off[v]) * (float)vt.V);
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            const float d = rgb[3 * pix + ch] - target[3 * pix + ch];
            v_rgb[3 * pix + ch] = d > 0.f ? wgt : (d < 0.f ? -wgt : 0.f);
            part += fabsf(d) * wgt;
        }
    }
    const float s = wave_sum(part);
    if (__lane_id() == 0 && s != 0.f) atomicAdd(loss_acc, (double)s);
}

template <int TW, int TH>
hipError_t fwd_impl(Ctx* c, const ViewTable& vt, const RasterParams& rp, const float* bg,
                    float* rgb, float* T_final, int32_t* last, const uint32_t* order,
                    hipStream_t st) {
    hipLaunchKernelGGL((k_render_fwd<TW, TH>), dim3((unsigned)c->n_tiles), dim3(64), 0, st,
                       reinterpret_cast<const float4*>(c->rec), c->ids, c->ranges, order, vt, rp,
                       bg, rgb, T_final, last);
    return hipGetLastError();
}

template <int TW, int TH>
hipError_t bwd_impl(Ctx* c, const ViewTable& vt, const RasterParams& rp, const float* bg,
                    const float* T_final, const int32_t* last, const float* v_rgb,
                    const uint32_t* order, hipStream_t st) {
    hipLaunchKernelGGL((k_render_bwd<TW, TH>), dim3((unsigned)c->n_tiles), dim3(64), 0, st,
                       reinterpret_cast<const float4*>(c->rec), c->ids, c->ranges, order, vt, rp,
                       bg, T_final, last, v_rgb, c->grad2d);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_render_fwd(Ctx* c, const ViewTable& vt, const RasterParams& rp, const float* bg,
                             float* rgb, float* T_final, int32_t* last, hipStream_t st) {
    if (c->n_tiles <= 0) return hipSuccess;
    const uint32_t* order = nullptr;
    const int TW = rp.tile_w, TH = rp.tile_h;
    if (TW == 16 && TH == 16) return fwd_impl<16, 16>(c, vt, rp, bg, rgb, T_final, last, order, st);
    if (TW == 16 && TH == 8) return fwd_impl<16, 8>(c, vt, rp, bg, rgb, T_final, last, order, st);
    if (TW == 8 && TH == 8) return fwd_impl<8, 8>(c, vt, rp, bg, rgb, T_final, last, order, st);
    if (TW == 32 && TH == 16) return fwd_impl<32, 16>(c, vt, rp, bg, rgb, T_final, last, order, st);
    return hipErrorInvalidValue;
}

hipError_t launch_render_bwd(Ctx* c, const ViewTable& vt, const RasterParams& rp, const float* bg,
                             const float* T_final, const int32_t* last, const float* v_rgb,
                             hipStream_t st) {
    if (c->n_tiles <= 0) return hipSuccess;
    const uint32_t* order = nullptr;
    const int TW = rp.tile_w, TH = rp.tile_h;
    if (TW == 16 && TH == 16) return bwd_impl<16, 16>(c, vt, rp, bg, T_final, last, v_rgb, order, st);
    if (TW == 16 && TH == 8) return bwd_impl<16, 8>(c, vt, rp, bg, T_final, last, v_rgb, order, st);
    if (TW == 8 && TH == 8) return bwd_impl<8, 8>(c, vt, rp, bg, T_final, last, v_rgb, order, st);
    if (TW == 32 && TH == 16) return bwd_impl<32, 16>(c, vt, rp, bg, T_final, last, v_rgb, order, st);
    return hipErrorInvalidValue;
}

hipError_t launch_l1(Ctx* c, const ViewTable& vt, const float* rgb, const float* target,
                     float* v_rgb, float* loss, hipStream_t st) {
    const int64_t P = vt.pix_off[vt.V];
    if (P > 0) {
        hipLaunchKernelGGL(k_l1, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, rgb, target,
                           v_rgb, vt, c->loss_acc);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_flush_acc(c->loss_acc, loss, 1, st);
}

}  // namespace gs
