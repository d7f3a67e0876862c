// Host side of the C ABI declared in gs.h: context and workspace, argument
// validation, error codes, and dispatch to the kernel launchers.
#include <math.h>

#include <algorithm>
#include <cmath>
#include <stdlib.h>
#include <string.h>

#include "gs_internal.h"

struct gs_ctx {
    gs::Ctx c;
};

namespace gs {

ViewTable make_view_table(const int32_t* wh, int V, int TW, int TH, const int32_t* index) {
    ViewTable vt;
    memset(&vt, 0, sizeof vt);
    vt.V = V;
    int toff = 0, poff = 0, boff = 0;
    for (int v = 0; v < V; v++) {
        vt.cam[v] = index ? index[v] : v;
        vt.W[v] = wh[2 * v];
        vt.H[v] = wh[2 * v + 1];
        vt.gx[v] = (vt.W[v] + TW - 1) / TW;
        const int gy = (vt.H[v] + TH - 1) / TH;
        vt.bx[v] = (vt.gx[v] + gs::kBlockTiles - 1) / gs::kBlockTiles;
        vt.tile_off[v] = toff;
        vt.pix_off[v] = poff;
        vt.block_off[v] = boff;
        toff += vt.gx[v] * gy;
        poff += vt.W[v] * vt.H[v];
        boff += vt.bx[v] * ((gy + gs::kBlockTiles - 1) / gs::kBlockTiles);
    }
    vt.tile_off[V] = toff;
    vt.pix_off[V] = poff;
    vt.block_off[V] = boff;
    return vt;
}

RasterParams make_raster_params(const gs_settings* s) {
    RasterParams rp;
    rp.alpha_min = s->alpha_min;
    rp.alpha_max = s->alpha_max;
    rp.t_min = s->t_min;
    rp.near_plane = s->near_plane;
    rp.eps2d = s->eps2d;
    rp.fov_pad = s->fov_pad;
    rp.tile_w = s->tile_w;
    rp.tile_h = s->tile_h;
    rp.eval_stats = s->eval_stats;
    rp.tile_order = s->tile_order;
    rp.lazy_lists = s->lazy_lists;
    return rp;
}

}  // namespace gs

namespace {

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

bool tile_ok(int tw, int th) {
    return (tw == 16 && th == 16) || (tw == 16 && th == 8) || (tw == 8 && th == 8) ||
           (tw == 32 && th == 16);
}

gs_status check_settings(const gs_settings* s) {
    if (!s) return GS_ERR_INVALID_ARG;
    if (!tile_ok(s->tile_w, s->tile_h)) return GS_ERR_UNSUPPORTED;
    if (s->tile_order < 0 || s->tile_order > 2) return GS_ERR_INVALID_ARG;
    if (s->lazy_lists != 0 && s->lazy_lists != 1) return GS_ERR_INVALID_ARG;
    if (!(s->alpha_min > 0.f && s->alpha_min < s->alpha_max && s->alpha_max < 1.f) ||
        !(s->t_min > 0.f && s->t_min < 1.f) || !(s->near_plane > 0.f) || !(s->eps2d >= 0.f) ||
        !(s->fov_pad >= 0.f))
        return GS_ERR_INVALID_ARG;
    return GS_OK;
}

gs_status check_cams(const gs::Ctx& c, const gs_cameras* cams, bool need_device) {
    if (!cams || !cams->wh || cams->V <= 0 || cams->V > GS_MAX_VIEWS || cams->V > c.cap.max_views)
        return cams && cams->V > 0 && (cams->V > GS_MAX_VIEWS || cams->V > c.cap.max_views)
                   ? GS_ERR_CAPACITY
                   : GS_ERR_INVALID_ARG;
    if (need_device && (!cams->viewmat || !cams->intr)) return GS_ERR_INVALID_ARG;
    if (cams->index)
        for (int v = 0; v < cams->V; v++)
            if (cams->index[v] < 0) return GS_ERR_INVALID_ARG;
    int64_t P = 0;
    for (int v = 0; v < cams->V; v++) {
        const int W = cams->wh[2 * v], H = cams->wh[2 * v + 1];
        if (W <= 0 || H <= 0 || W > 32768 || H > 32768) return GS_ERR_INVALID_ARG;
        P += (int64_t)W * H;
    }
    if (P >= ((int64_t)1 << 31)) return GS_ERR_CAPACITY;
    return GS_OK;
}

gs_status check_gaussians(const gs_gaussians* g) {
    if (!g) return GS_ERR_INVALID_ARG;
    if (g->sh_degree < 0 || g->sh_degree > 3) return GS_ERR_UNSUPPORTED;
    if (g->N < 0) return GS_ERR_INVALID_ARG;
    if (g->N > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logit || !g->sh))
        return GS_ERR_INVALID_ARG;
    return GS_OK;
}

gs_status from_hip(hipError_t e) { return e == hipSuccess ? GS_OK : GS_ERR_HIP; }

template <typename T>
hipError_t dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void**)p, count * sizeof(T));
}

}  // namespace

extern "C" {

const char* gs_strerror(gs_status s) {
    switch (s) {
        case GS_OK: return "ok";
        case GS_ERR_INVALID_ARG: return "invalid argument";
        case GS_ERR_CAPACITY: return "size exceeds the context's capacity";
        case GS_ERR_HIP: return "HIP runtime error";
        case GS_ERR_UNSUPPORTED: return "unsupported setting";
    }
    return "unknown status";
}

void gs_default_settings(gs_settings* s) {
    if (!s) return;
    s->tile_w = 16;
    s->tile_h = 16;
    s->near_plane = 0.01f;
    s->eps2d = 0.3f;
    s->fov_pad = 0.3f;
    s->alpha_min = 1.f / 255.f;
    s->alpha_max = 0.99f;
    s->t_min = 1e-4f;
    s->grad_accumulate = 0;
    s->tile_order = 0;
    s->eval_stats = 0;
    s->lazy_lists = 0;
}

gs_status gs_ctx_create(gs_ctx** out, const gs_capacity* cap) {
    if (!out) return GS_ERR_INVALID_ARG;
    *out = nullptr;
    if (!cap || cap->max_pairs < 0 || cap->max_isect < 0 || cap->max_tiles < 0 ||
        cap->max_views <= 0 || cap->max_views > GS_MAX_VIEWS || cap->max_cams < 0)
        return GS_ERR_INVALID_ARG;
    // limits of the device scan (16384 blocks of 4096 items) and of the radix
    // histograms (256 digits per 4096-item block go through that scan)
    if (cap->max_pairs > (int64_t)16384 * 4096 || cap->max_isect > ((int64_t)1 << 30) - 65536 ||
        cap->max_tiles > ((int64_t)1 << 24))
        return GS_ERR_CAPACITY;
    gs_ctx* h = (gs_ctx*)calloc(1, sizeof(gs_ctx));
    if (!h) return GS_ERR_HIP;
    gs::Ctx& c = h->c;
    c.cap = *cap;
    hipGetDevice(&c.device);
    const int64_t P = cap->max_pairs, I = cap->max_isect, T = cap->max_tiles;
    const int64_t sortmax = std::max(P, std::max(I, T));
    hipError_t e = hipSuccess;
    auto A = [&](hipError_t r) {
        if (e == hipSuccess) e = r;
    };
    A(dalloc(&c.rec, (size_t)P * GS_RECORD_FLOATS));
    A(dalloc(&c.grad2d, (size_t)P * GS_GRAD2D_FLOATS));
    A(dalloc(&c.cnt, (size_t)P));
    A(dalloc(&c.vmu_dir, (size_t)3 * (P > 0 ? P : 1)));
    A(dalloc(&c.off, (size_t)P));
    for (int k = 0; k < 2; k++) {
        A(dalloc(&c.pk[k], (size_t)P));
        A(dalloc(&c.pv[k], (size_t)P));
        A(dalloc(&c.ik[k], (size_t)I));
        A(dalloc(&c.iv[k], (size_t)I));
    }
    A(dalloc(&c.im[0], (size_t)2 * I));
    A(dalloc(&c.im[1], (size_t)2 * I));
    A(dalloc(&c.ranges, (size_t)2 * T));
    A(dalloc(&c.tcnt, (size_t)T));
    c.nchunks = I / 256 + 1;
    A(dalloc(&c.ccnt, (size_t)16 * (c.nchunks + 1)));
    A(dalloc(&c.cbase, (size_t)16 * c.nchunks));
    A(dalloc(&c.bpre, (size_t)16 * T));
    A(dalloc(&c.bplace, (size_t)T));
    A(dalloc(&c.tbase, (size_t)16 * T));
    A(dalloc(&c.tranges, (size_t)2 * T));
    A(dalloc(&c.tids, (size_t)I));
    A(dalloc(&c.tile_order, (size_t)T));
    A(dalloc(&c.tk[0], (size_t)T));
    A(dalloc(&c.tk[1], (size_t)T));
    A(dalloc(&c.tile_contrib, (size_t)T));
    A(dalloc(&c.tile_entries, (size_t)T));
    A(dalloc(&c.tile_evals, (size_t)T));
    const size_t hw = gs::radix_hist_words(sortmax);
    A(dalloc(&c.hist, hw));
    // the largest scan: radix digit counts, chunk counts, pair counts or tiles
    const int64_t scanmax = std::max<int64_t>(std::max<int64_t>((int64_t)hw, 16 * (c.nchunks + 1)), sortmax);
    A(dalloc(&c.scan_scratch, gs::scan_scratch_words(scanmax)));
    c.scan_max = scanmax;
    A(dalloc(&c.scalars, 16));
    const int nv = cap->max_views;
    const int nc = cap->max_cams > 0 ? cap->max_cams : 1;
    A(dalloc(&c.twist_render, (size_t)6 * nv));
    A(dalloc(&c.twist_track, (size_t)6 * nc));
    // the point-major track pass: per-workgroup twist and loss sums
    c.pm_cams = cap->max_cams > 0 ? std::min(cap->max_cams, GS_TRACK_PM_MAX_CAMS) : 0;
    if (c.pm_cams > 0) {
        A(dalloc(&c.track_part, (size_t)gs::kTrackPmBlocks * 6 * c.pm_cams));
        A(dalloc(&c.track_loss_part, (size_t)gs::kTrackPmBlocks));
    }
    A(dalloc(&c.loss_acc, 4));
    A(dalloc(&c.aux, gs::kAuxFloats));
    A(dalloc(&c.diag, gs::kDiagCount));
    if (e == hipSuccess) A(hipMemset(c.grad2d, 0, sizeof(float) * GS_GRAD2D_FLOATS * (P > 0 ? P : 1)));
    if (e == hipSuccess) A(hipMemset(c.twist_render, 0, sizeof(double) * 6 * nv));
    if (e == hipSuccess) A(hipMemset(c.twist_track, 0, sizeof(double) * 6 * nc));
    if (e == hipSuccess) A(hipMemset(c.loss_acc, 0, sizeof(double) * 4));
    if (e == hipSuccess) A(hipMemset(c.diag, 0, sizeof(uint32_t) * gs::kDiagCount));
    if (e == hipSuccess) A(hipMemset(c.scalars, 0, sizeof(uint32_t) * 16));
    // scans expect a zero workspace and leave it zero
    if (e == hipSuccess) A(hipMemset(c.scan_scratch, 0, sizeof(uint32_t) * gs::scan_scratch_words(scanmax)));
    if (e == hipSuccess) A(hipDeviceSynchronize());
    if (e != hipSuccess) {
        gs_ctx_destroy(h);
        return GS_ERR_HIP;
    }
    *out = h;
    return GS_OK;
}

gs_status gs_ctx_destroy(gs_ctx* h) {
    if (!h) return GS_ERR_INVALID_ARG;
    gs::Ctx& c = h->c;
    void* ptrs[] = {c.rec, c.grad2d, c.vmu_dir, c.cnt, c.off, c.pk[0], c.pk[1], c.pv[0], c.pv[1],
                    c.ik[0], c.ik[1], c.iv[0], c.iv[1], c.im[0], c.im[1], c.tcnt, c.ccnt, c.cbase, c.bpre, c.bplace, c.tbase, c.tranges, c.tids,
                    c.ranges, c.tile_order, c.tk[0], c.tk[1], c.tile_contrib, c.tile_entries, c.tile_evals, c.hist,
                    c.scan_scratch, c.scalars, c.twist_render, c.twist_track, c.track_part,
                    c.track_loss_part, c.loss_acc, c.aux, c.diag};
    hipDeviceSynchronize();
    for (void* p : ptrs)
        if (p) hipFree(p);
    free(h);
    return GS_OK;
}

gs_status gs_ctx_status(gs_ctx* h, gs_diag* out) {
    if (!h || !out) return GS_ERR_INVALID_ARG;
    uint32_t d[gs::kDiagCount];
    if (hipDeviceSynchronize() != hipSuccess) return GS_ERR_HIP;
    if (hipMemcpy(d, h->c.diag, sizeof d, hipMemcpyDeviceToHost) != hipSuccess) return GS_ERR_HIP;
    out->flags = d[gs::kDiagFlags];
    out->n_isect_needed = d[gs::kDiagIsectTotal];
    out->n_isect = d[gs::kDiagIsectUsed];
    out->n_masked_obs = d[gs::kDiagMasked];
    out->n_visible = d[gs::kDiagVisible];
    return GS_OK;
}

gs_status gs_ctx_reset_status(gs_ctx* h, void* stream) {
    if (!h) return GS_ERR_INVALID_ARG;
    return from_hip(gs::launch_fill_u32(h->c.diag, 0u, gs::kDiagCount, (hipStream_t)stream));
}

gs_status gs_ctx_buffers(gs_ctx* h, float** records, int32_t** isect_ids, int32_t** tile_ranges,
                         int64_t* n_tiles) {
    if (!h) return GS_ERR_INVALID_ARG;
    if (records) *records = h->c.rec;
    if (isect_ids) *isect_ids = reinterpret_cast<int32_t*>(h->c.tids);
    if (tile_ranges) *tile_ranges = h->c.tranges;
    if (n_tiles) *n_tiles = h->c.n_tiles;
    return GS_OK;
}

gs_status gs_ctx_generation(gs_ctx* h, int64_t* generation) {
    if (!h || !generation) return GS_ERR_INVALID_ARG;
    *generation = h->c.generation;
    return GS_OK;
}

gs_status gs_ctx_tile_stats(gs_ctx* h, const int32_t** tile_contrib, const int32_t** tile_entries,
                            const int32_t** tile_evals, const uint32_t** tile_order,
                            int32_t* ordered, int64_t* n_tiles) {
    if (!h) return GS_ERR_INVALID_ARG;
    if (tile_contrib) *tile_contrib = h->c.tile_contrib;
    if (tile_entries) *tile_entries = h->c.tile_entries;
    if (tile_evals) *tile_evals = h->c.tile_evals;
    if (tile_order) *tile_order = h->c.tile_order;
    if (ordered) *ordered = h->c.ordered ? 1 : 0;
    if (n_tiles) *n_tiles = h->c.n_tiles;
    return GS_OK;
}

gs_status gs_project(gs_ctx* h, const gs_gaussians* g, const gs_cameras* cams, const gs_settings* s,
                     void* stream) {
    if (!h) return GS_ERR_INVALID_ARG;
    gs_status r;
    if ((r = check_settings(s)) != GS_OK) return r;
    if ((r = check_gaussians(g)) != GS_OK) return r;
    if ((r = check_cams(h->c, cams, true)) != GS_OK) return r;
    if ((int64_t)cams->V * g->N > h->c.cap.max_pairs) return GS_ERR_CAPACITY;
    const gs::ViewTable vt = gs::make_view_table(cams->wh, cams->V, s->tile_w, s->tile_h, cams->index);
    const gs::RasterParams rp = gs::make_raster_params(s);
    return from_hip(gs::launch_project_fwd(&h->c, g, cams, vt, rp, (hipStream_t)stream));
}

gs_status gs_bin_sort(gs_ctx* h, const gs_cameras* cams, int32_t N, const gs_settings* s,
                      const float* records, void* stream) {
    if (!h) return GS_ERR_INVALID_ARG;
    gs_status r;
    if ((r = check_settings(s)) != GS_OK) return r;
    if ((r = check_cams(h->c, cams, false)) != GS_OK) return r;
    if (N < 0) return GS_ERR_INVALID_ARG;
    if (records && !aligned(records, 16)) return GS_ERR_INVALID_ARG;
    if ((int64_t)cams->V * N > h->c.cap.max_pairs) return GS_ERR_CAPACITY;
    const gs::ViewTable vt = gs::make_view_table(cams->wh, cams->V, s->tile_w, s->tile_h, cams->index);
    if (vt.tile_off[vt.V] > h->c.cap.max_tiles) return GS_ERR_CAPACITY;
    const gs::RasterParams rp = gs::make_raster_params(s);
    h->c.generation++;
    // only the heaviest-first order needs a permutation of the tiles
    return from_hip(gs::launch_bin(&h->c, vt, N, rp, records, s->tile_order == 1, (hipStream_t)stream));
}

static gs_status check_bins_match(const gs::Ctx& c, const gs_cameras* cams, const gs_settings* s) {
    if (c.bin_V != cams->V || c.bin_tw != s->tile_w || c.bin_th != s->tile_h) return GS_ERR_INVALID_ARG;
    return GS_OK;
}

gs_status gs_render_fwd(gs_ctx* h, const gs_cameras* cams, const gs_settings* s, const float* bg,
                        float* rgb, float* T_final, int32_t* last, void* stream) {
    if (!h || !rgb || !T_final || !last) return GS_ERR_INVALID_ARG;
    gs_status r;
    if ((r = check_settings(s)) != GS_OK) return r;
    if ((r = check_cams(h->c, cams, false)) != GS_OK) return r;
    if ((r = check_bins_match(h->c, cams, s)) != GS_OK) return r;
    const gs::ViewTable vt = gs::make_view_table(cams->wh, cams->V, s->tile_w, s->tile_h, cams->index);
    const gs::RasterParams rp = gs::make_raster_params(s);
    return from_hip(gs::launch_render_fwd(&h->c, vt, rp, bg, rgb, T_final, last, (hipStream_t)stream));
}

static gs_status check_raster_bwd(gs_ctx* h, const gs_cameras* cams, const gs_settings* s,
                                  const float* T_final, const int32_t* last, const float* v_rgb) {
    if (!h || !T_final || !last || !v_rgb) return GS_ERR_INVALID_ARG;
    gs_status r;
    if ((r = check_settings(s)) != GS_OK) return r;
    if ((r = check_cams(h->c, cams, false)) != GS_OK) return r;
    return check_bins_match(h->c, cams, s);
}

static gs_status check_project_bwd(gs_ctx* h, const gs_gaussians* g, const gs_cameras* cams,
                                   const gs_settings* s, const gs_gaussians_grad* grads,
                                   const float* v_twist) {
    if (!h || !v_twist) return GS_ERR_INVALID_ARG;
    gs_status r;
    if ((r = check_settings(s)) != GS_OK) return r;
    if ((r = check_gaussians(g)) != GS_OK) return r;
    if ((r = check_cams(h->c, cams, true)) != GS_OK) return r;
    if ((r = check_bins_match(h->c, cams, s)) != GS_OK) return r;
    if (h->c.bin_N != g->N) return GS_ERR_INVALID_ARG;
    if (grads && g->N > 0 && (!grads->means || !grads->log_scales || !grads->quats ||
                              !grads->opacity_logit || !grads->sh))
        return GS_ERR_INVALID_ARG;
    return GS_OK;
}

gs_status gs_raster_bwd(gs_ctx* h, const gs_cameras* cams, const gs_settings* s, const float* bg,
                        const float* T_final, const int32_t* last, const float* v_rgb, void* stream) {
    gs_status r;
    if ((r = check_raster_bwd(h, cams, s, T_final, last, v_rgb)) != GS_OK) return r;
    const gs::ViewTable vt = gs::make_view_table(cams->wh, cams->V, s->tile_w, s->tile_h, cams->index);
    const gs::RasterParams rp = gs::make_raster_params(s);
    return from_hip(gs::launch_render_bwd(&h->c, vt, rp, bg, T_final, last, v_rgb, (hipStream_t)stream));
}

gs_status gs_project_bwd(gs_ctx* h, const gs_gaussians* g, const gs_cameras* cams, const gs_settings* s,
                         gs_gaussians_grad* grads, float* v_twist, void* stream) {
    if (!grads) return GS_ERR_INVALID_ARG;
    gs_status r;
    if ((r = check_project_bwd(h, g, cams, s, grads, v_twist)) != GS_OK) return r;
    const gs::ViewTable vt = gs::make_view_table(cams->wh, cams->V, s->tile_w, s->tile_h, cams->index);
    const gs::RasterParams rp = gs::make_raster_params(s);
    return from_hip(gs::launch_project_bwd(&h->c, g, cams, vt, rp, nullptr, grads, s->grad_accumulate,
                                           v_twist, (hipStream_t)stream));
}

gs_status gs_project_bwd_adam(gs_ctx* h, const gs_gaussians* g, const gs_cameras* cams,
                              const gs_settings* s, const gs_gaussian_adam* adam, int32_t step,
                              const int32_t* step_dev, float beta1, float beta2, float eps,
                              float* v_twist, void* stream) {
    if (!adam || (!step_dev && step <= 0)) return GS_ERR_INVALID_ARG;
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f))
        return GS_ERR_INVALID_ARG;
    gs_status r;
    if ((r = check_project_bwd(h, g, cams, s, nullptr, v_twist)) != GS_OK) return r;
    // the parameters stepped are the arrays g points to (updated in place)
    const float* arrays[5] = {g->means, g->log_scales, g->quats, g->opacity_logit, g->sh};
    gs::AdamGauss a{};
    for (int q = 0; q < 5; q++) {
        if (g->N > 0 && (adam->params[q] != arrays[q] || !adam->exp_avg[q] || !adam->exp_avg_sq[q]))
            return GS_ERR_INVALID_ARG;
        a.p[q] = adam->params[q];
        a.m[q] = adam->exp_avg[q];
        a.v[q] = adam->exp_avg_sq[q];
        a.lr[q] = adam->lr[q];
    }
    a.b1 = beta1;
    a.b2 = beta2;
    a.eps = eps;
    a.step_dev = step_dev;
    a.step = step;
    const gs::ViewTable vt = gs::make_view_table(cams->wh, cams->V, s->tile_w, s->tile_h, cams->index);
    const gs::RasterParams rp = gs::make_raster_params(s);
    return from_hip(gs::launch_project_bwd(&h->c, g, cams, vt, rp, &a, nullptr, 0, v_twist,
                                           (hipStream_t)stream));
}

gs_status gs_render_bwd(gs_ctx* h, const gs_gaussians* g, const gs_cameras* cams, const gs_settings* s,
                        const float* bg, const float* T_final, const int32_t* last, const float* v_rgb,
                        gs_gaussians_grad* grads, float* v_twist, void* stream) {
    // every check of both halves before anything is enqueued: a failed check
    // must not leave 2D gradients behind in the context
    if (!grads) return GS_ERR_INVALID_ARG;
    gs_status r;
    if ((r = check_raster_bwd(h, cams, s, T_final, last, v_rgb)) != GS_OK) return r;
    if ((r = check_project_bwd(h, g, cams, s, grads, v_twist)) != GS_OK) return r;
    if ((r = gs_raster_bwd(h, cams, s, bg, T_final, last, v_rgb, stream)) != GS_OK) return r;
    return gs_project_bwd(h, g, cams, s, grads, v_twist, stream);
}

gs_status gs_l1_loss_grad(gs_ctx* h, const gs_cameras* cams, const float* rgb, const float* target,
                          float* v_rgb, float* loss, void* stream) {
    if (!h || !rgb || !target || !v_rgb || !loss) return GS_ERR_INVALID_ARG;
    gs_status r;
    if ((r = check_cams(h->c, cams, false)) != GS_OK) return r;
    const gs::ViewTable vt = gs::make_view_table(cams->wh, cams->V, 16, 16, cams->index);
    return from_hip(gs::launch_l1(&h->c, vt, rgb, target, v_rgb, loss, (hipStream_t)stream));
}

gs_status gs_photo_loss_grad(gs_ctx* h, const gs_cameras* cams, const float* rgb, const float* target,
                             float lambda_ssim, float* v_rgb, float* loss, void* stream) {
    if (!h || !rgb || !target || !v_rgb || !loss) return GS_ERR_INVALID_ARG;
    if (!(lambda_ssim >= 0.f && lambda_ssim <= 1.f)) return GS_ERR_INVALID_ARG;
    gs_status r;
    if ((r = check_cams(h->c, cams, false)) != GS_OK) return r;
    const gs::ViewTable vt = gs::make_view_table(cams->wh, cams->V, 16, 16, cams->index);
    return from_hip(gs::launch_photo(&h->c, vt, rgb, target, lambda_ssim, v_rgb, loss, (hipStream_t)stream));
}

gs_status gs_mcmc_relocate(gs_ctx* h, const gs_gaussian_adam* state, int32_t N, int32_t sh_degree,
                           const float* u, float dead_opacity, int32_t* src, int32_t* n_relocated,
                           void* stream) {
    if (!h || !state || N < 0) return GS_ERR_INVALID_ARG;
    if (sh_degree < 0 || sh_degree > 3) return GS_ERR_UNSUPPORTED;
    if (!(dead_opacity >= 0.f && dead_opacity < 1.f)) return GS_ERR_INVALID_ARG;
    if (N > 0) {
        if (!u) return GS_ERR_INVALID_ARG;
        for (int q = 0; q < 5; q++)
            if (!state->params[q] || !state->exp_avg[q] || !state->exp_avg_sq[q]) return GS_ERR_INVALID_ARG;
    }
    if ((int64_t)N > h->c.cap.max_pairs) return GS_ERR_CAPACITY;
    return from_hip(gs::launch_mcmc_relocate(&h->c, state, N, sh_degree, u, dead_opacity, src, n_relocated,
                                             (hipStream_t)stream));
}

gs_status gs_mcmc_noise(float* means, const float* log_scales, const float* quats,
                        const float* opacity_logit, int32_t N, const float* eta, float scale, float k,
                        float t, void* stream) {
    if (N < 0 || (N > 0 && (!means || !log_scales || !quats || !opacity_logit || !eta)))
        return GS_ERR_INVALID_ARG;
    if (!std::isfinite(scale) || !std::isfinite(k) || !std::isfinite(t)) return GS_ERR_INVALID_ARG;
    return from_hip(gs::launch_mcmc_noise(means, log_scales, quats, opacity_logit, N, eta, scale, k, t,
                                          (hipStream_t)stream));
}

gs_status gs_init_gaussians(gs_ctx* h, const float* points, const float* rgb, int32_t n, int32_t k,
                            float opacity, int32_t sh_degree, float* means, float* log_scales,
                            float* quats, float* opacity_logit, float* sh, void* stream) {
    if (!h || n < 0 || k < 1 || k > GS_INIT_MAX_K) return GS_ERR_INVALID_ARG;
    if (sh_degree < 0 || sh_degree > 3) return GS_ERR_UNSUPPORTED;
    if (!(opacity > 0.f && opacity < 1.f)) return GS_ERR_INVALID_ARG;
    if (n > 0 && (!points || !rgb || !means || !log_scales || !quats || !opacity_logit || !sh))
        return GS_ERR_INVALID_ARG;
    if ((int64_t)n > h->c.cap.max_pairs) return GS_ERR_CAPACITY;
    return from_hip(gs::launch_init_gaussians(&h->c, points, rgb, n, k, opacity, sh_degree, means,
                                              log_scales, quats, opacity_logit, sh,
                                              (hipStream_t)stream));
}

gs_status track_reproj_fwd_bwd(gs_ctx* h, const float* X, int32_t Pt, const float* viewmat,
                               const float* intr, int32_t n_cams, const int32_t* obs_cam,
                               const int32_t* obs_pt, const float* obs_xy, int32_t M, float delta,
                               float lambda, float near_plane, float* residual, float* loss,
                               float* v_X, float* v_twist, float* J_pose, float* J_X,
                               const int32_t* pt_off, const int32_t* pt_obs, const int32_t* pm_cam,
                               const float* pm_xy, void* stream) {
    if (!h || Pt < 0 || n_cams < 0 || M < 0) return GS_ERR_INVALID_ARG;
    if (M > 0 && (!X || !viewmat || !intr || !obs_cam || !obs_pt || !obs_xy)) return GS_ERR_INVALID_ARG;
    if (!(delta > 0.f) || !(near_plane > 0.f) || !isfinite(lambda)) return GS_ERR_INVALID_ARG;
    if (v_twist && n_cams > h->c.cap.max_cams) return GS_ERR_CAPACITY;
    if (!v_twist && M > 0) return GS_ERR_INVALID_ARG;  // the twist accumulator must be drained
    if (!loss && M > 0) return GS_ERR_INVALID_ARG;
    if ((pt_off == nullptr) != (pt_obs == nullptr)) return GS_ERR_INVALID_ARG;  // both or neither
    if ((pm_cam == nullptr) != (pm_xy == nullptr)) return GS_ERR_INVALID_ARG;
    if (pm_cam && !pt_off) return GS_ERR_INVALID_ARG;  // the copies come with their index
    return from_hip(gs::launch_track(&h->c, X, Pt, viewmat, intr, n_cams, obs_cam, obs_pt, obs_xy, M,
                                     delta, lambda, near_plane, residual, loss, v_X, v_twist, J_pose,
                                     J_X, pt_off, pt_obs, pm_cam, pm_xy, (hipStream_t)stream));
}

gs_status track_point_index(gs_ctx* h, const int32_t* obs_pt, int32_t M, int32_t Pt, int32_t* pt_off,
                            int32_t* pt_obs, const int32_t* obs_cam, const float* obs_xy,
                            int32_t* pm_cam, float* pm_xy, void* stream) {
    if (!h || M < 0 || Pt < 0 || !pt_off || (M > 0 && (!obs_pt || !pt_obs))) return GS_ERR_INVALID_ARG;
    // the point-major copies: all four arrays or none (no observations: nothing
    // to copy, any pointers); pixels read as float2
    const int ncopy = (obs_cam != nullptr) + (obs_xy != nullptr) + (pm_cam != nullptr) + (pm_xy != nullptr);
    if (M > 0 && ncopy != 0 && ncopy != 4) return GS_ERR_INVALID_ARG;
    if (M > 0 && ncopy == 4 &&
        (reinterpret_cast<uintptr_t>(obs_xy) % 8 != 0 || reinterpret_cast<uintptr_t>(pm_xy) % 8 != 0))
        return GS_ERR_INVALID_ARG;
    if (ncopy != 4) obs_cam = nullptr, obs_xy = nullptr, pm_cam = nullptr, pm_xy = nullptr;
    // the scan reads pt_off as 16-byte vectors
    if (reinterpret_cast<uintptr_t>(pt_off) % 16 != 0) return GS_ERR_INVALID_ARG;
    // cursors live in the pair-count buffer, the scan in the context's scratch
    if ((int64_t)Pt > h->c.cap.max_pairs || (int64_t)Pt + 1 > h->c.scan_max) return GS_ERR_CAPACITY;
    return from_hip(gs::launch_track_index(&h->c, obs_pt, M, Pt, pt_off, pt_obs, obs_cam, obs_xy, pm_cam,
                                           pm_xy, (hipStream_t)stream));
}

gs_status gs_pose_compose(int32_t V, const float* twist, const float* base, float* out, void* stream) {
    if (V < 0 || (V > 0 && (!twist || !base || !out))) return GS_ERR_INVALID_ARG;
    return from_hip(gs::launch_pose_compose(V, twist, base, out, (hipStream_t)stream));
}

gs_status gs_pose_compose_bwd(int32_t V, const float* twist, const float* g, float* out, void* stream) {
    if (V < 0 || (V > 0 && (!twist || !g || !out))) return GS_ERR_INVALID_ARG;
    return from_hip(gs::launch_pose_compose_bwd(V, twist, g, out, (hipStream_t)stream));
}

gs_status gs_adam_step(const gs_adam_group* groups, int32_t n_groups, int32_t step,
                       const int32_t* step_dev, float beta1, float beta2, float eps, void* stream) {
    if (!groups || n_groups <= 0 || n_groups > GS_ADAM_MAX_GROUPS || (!step_dev && step <= 0))
        return GS_ERR_INVALID_ARG;
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f))
        return GS_ERR_INVALID_ARG;
    for (int q = 0; q < n_groups; q++) {
        const gs_adam_group& g = groups[q];
        if (g.n < 0) return GS_ERR_INVALID_ARG;
        if (g.n > 0 && (!g.param || !g.grad || !g.exp_avg || !g.exp_avg_sq)) return GS_ERR_INVALID_ARG;
    }
    return from_hip(gs::launch_adam(groups, n_groups, step, step_dev, beta1, beta2, eps,
                                    (hipStream_t)stream));
}

gs_status gs_step_advance(int32_t* step_dev, void* stream) {
    if (!step_dev) return GS_ERR_INVALID_ARG;
    return from_hip(gs::launch_step_advance(step_dev, (hipStream_t)stream));
}

}  // extern "C"
