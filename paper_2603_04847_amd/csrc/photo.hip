// The photometric loss of the joint step, L_photo = (1 - lambda) L1 +
// lambda (1 - SSIM), and its image gradient, in one kernel.
//
// SSIM is taken per channel with an 11 x 11 Gaussian window (std 1.5, the
// outer product of the normalised 1D window), c1 = 0.01^2, c2 = 0.03^2, and
// zeros beyond the image border.  Its gradient at pixel q needs, for every
// pixel p whose window covers q, the partial derivatives of S(p) with respect
// to the three window sums that depend on x: mu_x, E_xx = w * x^2 and
// E_xy = w * (x y):
//   d SSIM / d x(q) = sum_p w(p - q) [dS/dmu_x(p) + 2 x(q) dS/dE_xx(p)
//                                      + y(q) dS/dE_xy(p)] / (3 P_v V).
// A workgroup owns a 32 x 32 tile of one view and keeps everything in LDS:
// the images with a 10-pixel halo, their five window sums over the tile plus
// a 5-pixel ring (separable: a horizontal pass, then a vertical one), the
// partial derivatives there (zero outside the image: the sum runs over image
// pixels only), and their window sums over the tile.  Nothing but the images
// and the gradient crosses HBM; the ring's window sums are computed again by
// the neighbouring tiles.  Each thread walks a run of consecutive outputs of
// one row or column with the window's inputs in registers, so every LDS value
// it loads serves up to 11 taps.
#include <math.h>

#include "gs_internal.h"

namespace gs {

namespace {

constexpr int kT = 32;                 // output tile side
constexpr int kR = 5;                  // window radius (11 taps)
constexpr int kTaps = 2 * kR + 1;
constexpr int kIn = kT + 4 * kR;       // input side with the 10-pixel halo: 52
constexpr int kMid = kT + 2 * kR;      // window sums over the tile and a 5-pixel ring: 42
constexpr int kThreads = 256;
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Window {
    float g[kTaps];
};

struct PhotoArgs {
    ViewTable vt;
    const float* rgb;
    const float* target;
    float* v_rgb;
    double* acc;     // [0] sum of the weighted |d|, [1] sum of the weighted S
    float lambda;    // weight of the SSIM term
    int tiles_x[GS_MAX_VIEWS];
    int tile_off[GS_MAX_VIEWS + 1];
};

// LDS: the two images of one channel (kIn x kIn each), then a region that
// holds the five horizontal window sums (kIn rows x kMid columns) and later,
// after a barrier, the three partial-derivative maps (kMid x kMid) and their
// horizontal window sums (kMid rows x kT columns).
struct PhotoLds {
    float X[kIn][kIn + 3];  // columns kIn.. are read only for outputs past kMid
    float Y[kIn][kIn + 3];
    union {
        float H[5][kIn][kMid + 1];
        struct {
            float D[3][kMid][kMid + 1];
            float E[3][kMid][kT + 1];
        } d;
    } u;
    float red[2][kThreads / kWave];
};

// Runs: horizontal passes write 11 (first) or 8 (partials) consecutive
// columns per work item, vertical passes 7 (first) or 4 (last) consecutive
// rows.
constexpr int kRunH = 11;  // 42 <= 4 x 11: 208 horizontal items, one per thread
constexpr int kGroupsH = (kMid + kRunH - 1) / kRunH;
constexpr int kRunA = 7;   // 42 = 6 x 7: 252 vertical items, one per thread
constexpr int kRunB = 8;  // 32 = 4 x 8
constexpr int kRunC = 4;  // the last vertical pass: 32 = 8 x 4, one item per thread

__global__ __launch_bounds__(kThreads) void k_photo(PhotoArgs a, Window win) {
    __shared__ PhotoLds s;
    const int tid = threadIdx.x;
    // tile -> view, tile position
    const int t = blockIdx.x;
    int v = 0;
    while (v + 1 < a.vt.V && t >= a.tile_off[v + 1]) v++;
    const int lt = t - a.tile_off[v];
    const int W = a.vt.W[v], H = a.vt.H[v];
    const int x0 = (lt % a.tiles_x[v]) * kT, y0 = (lt / a.tiles_x[v]) * kT;
    const int64_t poff = a.vt.pix_off[v];
    const float wv = 1.f / (3.f * (float)W * (float)H * (float)a.vt.V);
    const float lam = a.lambda;
    float l1_part = 0.f, s_part = 0.f;
    // the two images of a channel with the halo (zeros outside the view): all
    // of a thread's loads are issued at once, into registers, and stored to
    // LDS when the channel starts (one round trip to memory per channel, not
    // one per 256 pixels, and for the second and third channels hidden
    // behind the previous channel's work)
    constexpr int kLoads = (kIn * kIn + kThreads - 1) / kThreads;  // 11
    float ldx[kLoads], ldy[kLoads];
    auto issue = [&](int ch) {
        // the pixel indexes are formed anew per channel (kept opaque to the
        // compiler): held across the channel loop they would cost 44 registers
        int t0 = tid;
        asm volatile("" : "+v"(t0));
#pragma unroll
        for (int u = 0; u < kLoads; u++) {
            const int i = t0 + u * kThreads;
            const int r = i / kIn, c = i % kIn;
            const int px = x0 - 2 * kR + c, py = y0 - 2 * kR + r;
            ldx[u] = ldy[u] = 0.f;
            if (i < kIn * kIn && px >= 0 && px < W && py >= 0 && py < H) {
                const int64_t q = poff + (int64_t)py * W + px;
                ldx[u] = a.rgb[3 * q + ch];
                ldy[u] = a.target[3 * q + ch];
            }
        }
    };
    issue(0);
#pragma unroll 1
    for (int ch = 0; ch < 3; ch++) {
#pragma unroll
        for (int u = 0; u < kLoads; u++) {
            const int i = tid + u * kThreads;
            if (i < kIn * kIn) {
                s.X[i / kIn][i % kIn] = ldx[u];
                s.Y[i / kIn][i % kIn] = ldy[u];
            }
        }
        __syncthreads();
        // ---- horizontal window sums of x, y, x^2, y^2, x y: every row of the
        // halo, columns of the tile plus the ring
        // consecutive lanes take consecutive rows at one column run: the odd
        // row strides (53, 43 words) put their LDS words in distinct banks
        // (the last run's outputs past kMid are computed and dropped)
        for (int item = tid; item < kIn * kGroupsH; item += kThreads) {
            const int r = item % kIn, c0 = (item / kIn) * kRunH;
            // the run's inputs and their squares and products, formed once
            float xs[kRunH + kTaps - 1], ys[kRunH + kTaps - 1];
            float xx[kRunH + kTaps - 1], yy[kRunH + kTaps - 1], xy[kRunH + kTaps - 1];
#pragma unroll
            for (int k = 0; k < kRunH + kTaps - 1; k++) {
                xs[k] = s.X[r][c0 + k];
                ys[k] = s.Y[r][c0 + k];
                xx[k] = xs[k] * xs[k];
                yy[k] = ys[k] * ys[k];
                xy[k] = xs[k] * ys[k];
            }
#pragma unroll
            for (int j = 0; j < kRunH; j++) {
                if (c0 + j >= kMid) break;
                float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f;
#pragma unroll
                for (int k = 0; k < kTaps; k++) {
                    const float g = win.g[k];
                    m0 = __builtin_fmaf(g, xs[j + k], m0);
                    m1 = __builtin_fmaf(g, ys[j + k], m1);
                    m2 = __builtin_fmaf(g, xx[j + k], m2);
                    m3 = __builtin_fmaf(g, yy[j + k], m3);
                    m4 = __builtin_fmaf(g, xy[j + k], m4);
                }
                s.u.H[0][r][c0 + j] = m0;
                s.u.H[1][r][c0 + j] = m1;
                s.u.H[2][r][c0 + j] = m2;
                s.u.H[3][r][c0 + j] = m3;
                s.u.H[4][r][c0 + j] = m4;
            }
        }
        __syncthreads();
        // ---- vertical window sums over the tile and ring, then S and its
        // partial derivatives; held in registers until every thread has read
        // the horizontal sums (the partials take their place in LDS)
        constexpr int kItemsA = kMid * (kMid / kRunA);           // 252
        constexpr int kPerThreadA = (kItemsA + kThreads - 1) / kThreads;  // 2
        float dv[kPerThreadA][kRunA][3];
#pragma unroll
        for (int u = 0; u < kPerThreadA; u++) {
            const int item = tid + u * kThreads;
#pragma unroll
            for (int j = 0; j < kRunA; j++) dv[u][j][0] = dv[u][j][1] = dv[u][j][2] = 0.f;
            if (item < kItemsA) {
                const int c = item % kMid, r0 = (item / kMid) * kRunA;
                float mm[5][kRunA];
#pragma unroll
                for (int m = 0; m < 5; m++) {
                    float col[kRunA + kTaps - 1];
#pragma unroll
                    for (int k = 0; k < kRunA + kTaps - 1; k++) col[k] = s.u.H[m][r0 + k][c];
#pragma unroll
                    for (int j = 0; j < kRunA; j++) {
                        float acc = 0.f;
#pragma unroll
                        for (int k = 0; k < kTaps; k++) acc = __builtin_fmaf(win.g[k], col[j + k], acc);
                        mm[m][j] = acc;
                    }
                }
                const int px = x0 - kR + c;
#pragma unroll
                for (int j = 0; j < kRunA; j++) {
                    const int py = y0 - kR + r0 + j;
                    if (px < 0 || px >= W || py < 0 || py >= H) continue;  // not an image pixel
                    const float mx = mm[0][j], my = mm[1][j];
                    const float sxx = mm[2][j] - mx * mx, syy = mm[3][j] - my * my;
                    const float sxy = mm[4][j] - mx * my;
                    const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
                    const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
                    const float iD = 1.f / (B1 * B2);
                    const float S = A1 * A2 * iD;
                    // dS/dmu_x (through mu_x and the mu_x terms of s_xx, s_xy),
                    // dS/dE_xx, dS/dE_xy
                    dv[u][j][0] = 2.f * (my * (A2 - A1) - mx * S * (B2 - B1)) * iD;
                    dv[u][j][1] = -S / B2;
                    dv[u][j][2] = 2.f * A1 * iD;
                    // each pixel's S is counted by the tile that owns it
                    if (px >= x0 && px < x0 + kT && py >= y0 && py < y0 + kT) s_part += S;
                }
            }
        }
        __syncthreads();  // the horizontal sums are read
#pragma unroll
        for (int u = 0; u < kPerThreadA; u++) {
            const int item = tid + u * kThreads;
            if (item < kItemsA) {
                const int c = item % kMid, r0 = (item / kMid) * kRunA;
#pragma unroll
                for (int j = 0; j < kRunA; j++) {
                    s.u.d.D[0][r0 + j][c] = dv[u][j][0];
                    s.u.d.D[1][r0 + j][c] = dv[u][j][1];
                    s.u.d.D[2][r0 + j][c] = dv[u][j][2];
                }
            }
        }
        __syncthreads();
        // the next channel's loads, in flight behind the last two passes
        if (ch + 1 < 3) issue(ch + 1);
        // ---- horizontal window sums of the partials: rows of tile and ring,
        // columns of the tile; one map per item (504 items for 256 threads),
        // consecutive lanes on consecutive rows
        constexpr int kItemsB = kMid * (kT / kRunB);  // per map: 168
        for (int item = tid; item < 3 * kItemsB; item += kThreads) {
            const int m = item / kItemsB, rest = item % kItemsB;
            const int r = rest % kMid, c0 = (rest / kMid) * kRunB;
            float row[kRunB + kTaps - 1];
#pragma unroll
            for (int k = 0; k < kRunB + kTaps - 1; k++) row[k] = s.u.d.D[m][r][c0 + k];
#pragma unroll
            for (int j = 0; j < kRunB; j++) {
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < kTaps; k++) acc = __builtin_fmaf(win.g[k], row[j + k], acc);
                s.u.d.E[m][r][c0 + j] = acc;
            }
        }
        __syncthreads();
        // ---- vertical window sums over the tile, the gradient, the L1 term
        static_assert(kT * (kT / kRunC) <= kThreads, "one item per thread");
        if (tid < kT * (kT / kRunC)) {
            const int c = tid % kT, r0 = (tid / kT) * kRunC;
            float ag[3][kRunC];
#pragma unroll
            for (int m = 0; m < 3; m++) {
                float col[kRunC + kTaps - 1];
#pragma unroll
                for (int k = 0; k < kRunC + kTaps - 1; k++) col[k] = s.u.d.E[m][r0 + k][c];
#pragma unroll
                for (int j = 0; j < kRunC; j++) {
                    float acc = 0.f;
#pragma unroll
                    for (int k = 0; k < kTaps; k++) acc = __builtin_fmaf(win.g[k], col[j + k], acc);
                    ag[m][j] = acc;
                }
            }
            const int px = x0 + c;
#pragma unroll
            for (int j = 0; j < kRunC; j++) {
                const int py = y0 + r0 + j;
                if (px >= W || py >= H) continue;
                const float xv = s.X[2 * kR + r0 + j][2 * kR + c];
                const float yv = s.Y[2 * kR + r0 + j][2 * kR + c];
                const float d = xv - yv;
                const float dssim = __builtin_fmaf(2.f * xv, ag[1][j], __builtin_fmaf(yv, ag[2][j], ag[0][j]));
                const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
                l1_part += fabsf(d);
                const int64_t q = poff + (int64_t)py * W + px;
                a.v_rgb[3 * q + ch] = wv * ((1.f - lam) * sg - lam * dssim);
            }
        }
        __syncthreads();  // LDS is reused by the next channel
    }
    // one double atomic per block for each sum, weighted by the view's share
    const float l1s = wave_sum(l1_part), ss = wave_sum(s_part);
    if (__lane_id() == 0) {
        s.red[0][tid / kWave] = l1s;
        s.red[1][tid / kWave] = ss;
    }
    __syncthreads();
    if (tid == 0) {
        double l = 0.0, m = 0.0;
        for (int q = 0; q < kThreads / kWave; q++) {
            l += s.red[0][q];
            m += s.red[1][q];
        }
        // loss = (1 - lambda) L1 + lambda (1 - SSIM); the constant lambda once
        double add = (1.0 - (double)lam) * l * wv - (double)lam * m * wv;
        if (t == 0) add += (double)lam;
        if (add != 0.0) atomicAdd(a.acc, add);
    }
}

}  // namespace

hipError_t launch_photo(Ctx* c, const ViewTable& vt, const float* rgb, const float* target,
                        float lambda, float* v_rgb, float* loss, hipStream_t st) {
    PhotoArgs a;
    a.vt = vt;
    a.rgb = rgb;
    a.target = target;
    a.v_rgb = v_rgb;
    a.acc = c->loss_acc + 2;
    a.lambda = lambda;
    int toff = 0;
    for (int v = 0; v < vt.V; v++) {
        a.tiles_x[v] = (vt.W[v] + kT - 1) / kT;
        a.tile_off[v] = toff;
        toff += a.tiles_x[v] * ((vt.H[v] + kT - 1) / kT);
    }
    a.tile_off[vt.V] = toff;
    // the normalised 1D Gaussian window, std 1.5
    Window win;
    double g[kTaps], sum = 0.0;
    for (int k = 0; k < kTaps; k++) {
        g[k] = exp(-(double)(k - kR) * (k - kR) / (2.0 * 1.5 * 1.5));
        sum += g[k];
    }
    for (int k = 0; k < kTaps; k++) win.g[k] = (float)(g[k] / sum);
    if (toff > 0) {
        hipLaunchKernelGGL(k_photo, dim3((unsigned)toff), dim3(kThreads), 0, st, a, win);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_flush_acc(c->loss_acc + 2, loss, 1, st);
}

}  // namespace gs
