/*
 * gs.h -- C ABI of the MI355X (gfx950) splatting hot path of GloSplat's joint
 * pose-appearance step: differentiable tile-based 3D Gaussian splatting
 * (projection, tile binning and key sort, front-to-back compositing, and its
 * backward to the Gaussian parameters and to each camera's SE(3) pose), the
 * track reprojection residual with its Jacobian, the photometric L1 term,
 * pose composition and the Adam update.
 *
 * Paper: GloSplat (arXiv 2603.04847).  The calls follow its statement of the
 * problem:
 *   Rasterize(G, T_i, K_i) -> I_i                 Algorithm 1 (render step),
 *                                                 Sec. 3.3 "Implementation";
 *   pi(K, T, X) = proj(K (R X + t))               Sec. 3.2 "Bundle Adjustment",
 *                                                 Appendix E (projection function);
 *   rho_Huber(||pi_i(X_k) - x_ip||^2; delta)      Sec. 3.3 eq. L_BA^joint;
 *   L = L_photo + lambda_BA L_BA, poses get both  Sec. 3.3, Algorithm 1
 *   gradients                                     (backward and update steps);
 *   T_i = T_i^(0) (+) dT_i                        Algorithm 1 (pose adjustment).
 *
 * Conventions shared by every call
 * --------------------------------
 * - All buffers are DEVICE pointers (hipMalloc'd or torch CUDA tensors) unless
 *   marked HOST.  The caller owns every buffer it passes; the library owns only
 *   the workspace inside a gs_ctx, allocated once by gs_ctx_create.  No call
 *   allocates, frees, or synchronises the host (except gs_ctx_create/destroy/
 *   status), so a sequence of calls can be captured in a HIP graph.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *   work of a call is enqueued on it, in order.
 * - Floats are IEEE binary32.  Gaussian parameters are planar (SoA):
 *     means[3][N], log_scales[3][N], quats[4][N] (w,x,y,z; need not be unit),
 *     opacity_logit[N], sh[K][3][N] with K = (deg+1)^2, coefficient index
 *     l*l + l + m (m = -l..l), real SH with the Condon-Shortley phase.
 * - Cameras: viewmat[V][12] = world->camera [R|t], 3x4 row-major; camera axes
 *   x right, y down, z forward.  intr[V][4] = fx, fy, cx, cy (pinhole, no
 *   skew, no distortion).  wh[V][2] = width, height (HOST).  Pixel (u,v) is
 *   sampled at (u+0.5, v+0.5).
 * - Images: views packed view-major, rows y-major, RGB interleaved:
 *   rgb[sum_v W_v H_v][3].
 * - Pair index of (view v, Gaussian g) in one call is v*N + g.
 * - Gradients of the twist are with respect to a LEFT perturbation of the
 *   current world->camera pose, T <- Exp(xi) T, xi = (rho, phi), translation
 *   first.  Every twist output ACCUMULATES (+=) so the photometric and the
 *   reprojection gradients of a pose land in one buffer; the caller zeroes it.
 * - Errors: host-detectable problems return at once with no work enqueued:
 *   GS_ERR_INVALID_ARG (null or misaligned pointer, bad size), GS_ERR_CAPACITY
 *   (a size beyond the context's capacity), GS_ERR_UNSUPPORTED (sh_degree > 3,
 *   tile shape not offered), GS_ERR_HIP (a launch failed).  Conditions only the
 *   device sees (too many tile intersections, non-finite inputs, track points
 *   behind their camera) set flags in the context's status word, read with
 *   gs_ctx_status after the stream is done; a step that overflowed has
 *   undefined outputs and must be re-run with a larger capacity.
 *
 * Rendering definition (the paper delegates rasterization to an external 3DGS
 * library and gives no formula; this is the standard EWA-splatting definition):
 *   p = R mu + t; cull if p_z < near.  Sigma = Rq S S^T Rq^T (S = diag(exp(s))),
 *   Sigma_c = R Sigma R^T, J = [[fx/z, 0, -fx tx/z], [0, fy/z, -fy ty/z]] with
 *   tx = x/z clamped to [-(cx/fx + pad W/(2fx)), (W-cx)/fx + pad W/(2fx)] (ty
 *   alike), Sigma2D = J Sigma_c J^T + eps2d I, conic = Sigma2D^-1,
 *   mean2d = (fx x/z + cx, fy y/z + cy), o = sigmoid(logit) (cull if
 *   o <= alpha_min), colour = max(0, sum_lm Y_lm(d) sh_lm + 0.5) with d the unit
 *   direction from the camera centre -R^T t to mu.
 *   Per pixel, splats in ascending (float32 depth, pair index) order:
 *   sigma = 0.5 (A dx^2 + C dy^2) + B dx dy with d = mean2d - pixel centre;
 *   alpha = min(alpha_max, o exp(-sigma)); skip if alpha < alpha_min; stop
 *   (excluding this splat) once T (1 - alpha) < T_min; otherwise
 *   C += colour alpha T, T *= 1 - alpha.  Output C + T bg.
 */
#ifndef GLOSPLAT_GS_H
#define GLOSPLAT_GS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GS_OK = 0,
    GS_ERR_INVALID_ARG = -1,
    GS_ERR_CAPACITY = -2,
    GS_ERR_HIP = -3,
    GS_ERR_UNSUPPORTED = -4,
} gs_status;

/* Device status flags (gs_diag.flags). */
#define GS_FLAG_ISECT_OVERFLOW 1u   /* tile-list entries exceeded max_isect */
#define GS_FLAG_NONFINITE 2u        /* a Gaussian with a non-finite parameter, or a pair whose
                                       projected record was not finite, was culled (it
                                       contributes nothing and receives no gradient) */
#define GS_FLAG_SCAN_STALLED 4u     /* a device-wide scan stopped waiting for a preceding
                                       workgroup (bounded wait); that step counts as overflowed:
                                       its lists are empty, and no write leaves its buffer */
#define GS_FLAG_COUNT_BOUND 8u      /* internal check: a pair met more blocks than the bound its
                                       slots were sized by; that step's lists are incomplete */

/* Most views one render call takes. */
#define GS_MAX_VIEWS 64

typedef struct gs_ctx gs_ctx;

/* Workspace sizes, fixed at creation. */
typedef struct {
    int64_t max_pairs;   /* views x Gaussians per gs_project call */
    int64_t max_isect;   /* tile-list entries (tile, splat) per gs_bin_sort call */
    int64_t max_tiles;   /* tiles summed over the views of one call */
    int32_t max_views;   /* views per call (<= GS_MAX_VIEWS) for twist accumulators */
    int32_t max_cams;    /* cameras of track_reproj_fwd_bwd (twist accumulators) */
} gs_capacity;

/* Rendering settings; gs_default_settings fills the reference values. */
typedef struct {
    int32_t tile_w, tile_h;   /* 16x16 (default), 16x8, 8x8, 32x16 */
    float near_plane;         /* 0.01 */
    float eps2d;              /* 0.3 px^2 dilation of Sigma2D */
    float fov_pad;            /* 0.3: J clamp at 1.3x the half field of view */
    float alpha_min;          /* 1/255 */
    float alpha_max;          /* 0.99 */
    float t_min;              /* 1e-4 */
    int32_t grad_accumulate;  /* 0: gs_render_bwd overwrites Gaussian grads; 1: adds */
    int32_t tile_order;       /* 0: natural tile order; 1: launch the raster kernels on
                                 the tiles heaviest first: by decreasing bucket of the
                                 list length, 16 buckets per octave (bucket of n > 0:
                                 1 + 16 floor(log2 n) + the 4 bits after n's leading
                                 bit; 0 for an empty list), any order inside a bucket;
                                 2: tiles walked by 4x4 blocks, each block's 16 tiles on
                                 consecutive workgroups of one XCD (workgroups are dealt
                                 round-robin over the 8 XCDs), so neighbouring tiles read
                                 their shared splats through one L2.  The image does not
                                 depend on the order */
    int32_t eval_stats;       /* 0; 1: gs_render_fwd also counts per tile the contributing
                                 pairs, list entries read and (pixel, splat) evaluations
                                 (gs_ctx_tile_stats), a slower variant */
    int32_t lazy_lists;       /* 0: gs_bin_sort writes every tile list in full;
                                 1: it stops at the per-block lists and the tile list
                                 lengths, and gs_render_fwd draws each tile's list from
                                 its block's list, writing the part it reads (up to the
                                 batch of 64 in which the tile's last pixel stopped) to
                                 the tile lists.  The backward reads no further than that
                                 part; run without a forward since the bin step, it first
                                 writes the lists in full.  Images and gradients are the
                                 same bit for bit; only the unread list tails are left
                                 unwritten */
} gs_settings;

typedef struct {
    const float* means;          /* [3][N] */
    const float* log_scales;     /* [3][N] */
    const float* quats;          /* [4][N] w,x,y,z */
    const float* opacity_logit;  /* [N] */
    const float* sh;             /* [K][3][N] */
    int32_t N;
    int32_t sh_degree;           /* 0..3 */
} gs_gaussians;

typedef struct {
    float* means;
    float* log_scales;
    float* quats;
    float* opacity_logit;
    float* sh;
} gs_gaussians_grad;

typedef struct {
    const float* viewmat;   /* [n_rows][12] */
    const float* intr;      /* [n_rows][4] */
    const int32_t* wh;      /* HOST [V][2]: size of each view of the call */
    int32_t V;              /* views in this call */
    const int32_t* index;   /* HOST [V] or NULL: view v of the call uses row index[v] of
                               viewmat, intr and v_twist (a sampled batch of a larger
                               camera set); NULL means row v */
} gs_cameras;

/* Diagnostics read by gs_ctx_status. */
typedef struct {
    uint32_t flags;          /* GS_FLAG_* */
    int64_t n_isect;         /* tile-list entries of the last gs_bin_sort */
    int64_t n_isect_needed;  /* entries that call needed (> max_isect on overflow) */
    int64_t n_masked_obs;    /* observations masked (behind the camera) since reset */
    int64_t n_visible;       /* pairs listed in at least one tile in the last gs_bin_sort */
} gs_diag;

/* A per-step record of the projected splat of each pair, 12 floats (48 B,
 * 16-B aligned) per pair v*N+g:
 *   [0] mean2d.x [1] mean2d.y [2] depth (camera z) [3] opacity (<= 0: culled)
 *   [4] conic A  [5] conic B  [6] conic C          [7] red
 *   [8] green    [9] blue     [10],[11] unused
 * gs_project writes it into the context; gs_bin_sort may also be given a
 * caller-built record array in this layout. */
#define GS_RECORD_FLOATS 12

/* Per-pair 2D gradient, 9 floats per pair, accumulated by the raster backward
 * into the context:
 *   d/d(mean2d.x, mean2d.y, conic A, B, C, opacity, red, green, blue).
 * They are held in two planes: the first six of every pair, then (after
 * max_pairs such groups) the last three of every pair. */
#define GS_GRAD2D_FLOATS 9

const char* gs_strerror(gs_status s);
void gs_default_settings(gs_settings* s);

/* Create a context: allocates the whole workspace once (device memory of about
 * 48+36+24 B per pair + 36 B per list entry + 40 B per tile, and 12 KB per
 * camera up to GS_TRACK_PM_MAX_CAMS).  *out is NULL on failure. */
gs_status gs_ctx_create(gs_ctx** out, const gs_capacity* cap);
gs_status gs_ctx_destroy(gs_ctx* ctx);
/* Synchronise the device and read the status word. */
gs_status gs_ctx_status(gs_ctx* ctx, gs_diag* out);
/* Number of gs_bin_sort calls enqueued on the context so far (HOST value, no
 * synchronisation).  The tile lists and projected records a backward reads
 * are those of the latest gs_project / gs_bin_sort; a caller holding several
 * forwards compares this number to the one it saw at its forward and
 * re-projects and re-bins before a backward whose lists were replaced. */
gs_status gs_ctx_generation(gs_ctx* ctx, int64_t* generation);
/* Clear the status flags and counters (enqueued on stream). */
gs_status gs_ctx_reset_status(gs_ctx* ctx, void* stream);
/* Device pointers into the workspace (valid for the context's lifetime):
 * records [max_pairs][12], the tile lists [max_isect] (pair index in the low
 * 28 bits, the 4-bit quadrant mask in the top 4), tile ranges [max_tiles][2]
 * (start, end) int32, and the tile count of the last gs_bin_sort (HOST
 * value).  After a gs_bin_sort with lazy_lists = 1 a tile list holds only the
 * entries a forward (or backward) has written since. */
gs_status gs_ctx_buffers(gs_ctx* ctx, float** records, int32_t** isect_ids,
                         int32_t** tile_ranges, int64_t* n_tiles);

/* Workload statistics of the last gs_render_fwd run with settings
 * eval_stats = 1 (device pointers, valid for the context's lifetime; the
 * plain forward leaves them as they were): tile_contrib[t] = number of (pixel, splat) pairs
 * that contributed to tile t; tile_entries[t] = entries of tile t's list the
 * forward read (up to the batch in which its last pixel stopped);
 * tile_evals[t] = sum over tile t's pixels of the entries of its list, up to
 * the pixel's last contributor, whose mask covers the pixel's quadrant (the
 * (pixel, splat) evaluations the definition makes, forward or backward);
 * tile_order = launch order of the tiles when the last gs_bin_sort ran with
 * tile_order = 1 (*ordered = 1), heaviest first as gs_settings.tile_order
 * describes; n_tiles = tiles of
 * the last gs_bin_sort (HOST value). */
gs_status gs_ctx_tile_stats(gs_ctx* ctx, const int32_t** tile_contrib,
                            const int32_t** tile_entries, const int32_t** tile_evals,
                            const uint32_t** tile_order, int32_t* ordered, int64_t* n_tiles);

/* Project every (view, Gaussian) pair (render step of Algorithm 1; the
 * definition above).  Reads each Gaussian's parameters once for all V views and
 * writes the V*N records into the context.  Requires V*N <= max_pairs,
 * V <= max_views, 0 <= sh_degree <= 3. */
gs_status gs_project(gs_ctx* ctx, const gs_gaussians* g, const gs_cameras* cams,
                     const gs_settings* s, void* stream);

/* Bin and sort (the Rasterize step of the Appendix E algorithm goes through the
 * tile rasterizer Sec. 3.3 names; this is its binning and key sort).  A tile
 * (tile_w x tile_h) has four quadrants (tile_w/2 x tile_h/2); a splat meets a
 * quadrant when its alpha >= alpha_min ellipse meets the rectangle of the
 * quadrant's pixel centres.  Tile t's list holds every pair meeting one of its
 * quadrants, in ascending (float32 depth, pair) order, each entry the pair
 * index with the 4-bit mask of the quadrants met (bit qx + 2 qy) in its top 4
 * bits; tile ranges index the lists.  Tiles of view v are numbered after those
 * of views < v, row-major inside a view.  `records` = NULL uses the context's
 * records (from gs_project); otherwise a caller array of V*N records in the
 * layout above.  max_isect bounds the total list length; overflow sets
 * GS_FLAG_ISECT_OVERFLOW, leaves every list empty, and n_isect_needed reports
 * the need (or, when even the 4x4-tile blocks the lists are built from
 * overflowed, a lower bound of it).  With s->lazy_lists = 1 the tile ranges
 * are the same but the entries are left to the forward (gs_settings); the
 * render calls follow the mode of the last gs_bin_sort, whatever their own
 * settings say. */
gs_status gs_bin_sort(gs_ctx* ctx, const gs_cameras* cams, int32_t N,
                      const gs_settings* s, const float* records, void* stream);

/* The projected records and the tile lists live in the context: gs_project
 * writes the records, gs_bin_sort the lists, and the render calls read the
 * latest ones (they are not passed as arguments).
 *
 * Forward compositing (the Rasterize step of Algorithm 1, render step; the
 * per-pixel definition above) over the tile lists of the last gs_bin_sort.
 * bg[3] (device, may be NULL = black).  Outputs rgb[P][3], T_final[P] and
 * last[P] = 1 + position, within its tile's list, of the pixel's final
 * contributor (0 if none); P = sum_v W_v H_v.  T_final and last are what the
 * backward needs (it recomputes the blending state per pixel instead of
 * storing it). */
gs_status gs_render_fwd(gs_ctx* ctx, const gs_cameras* cams, const gs_settings* s,
                        const float* bg, float* rgb, float* T_final, int32_t* last,
                        void* stream);

/* Backward of gs_project + gs_render_fwd (Algorithm 1, backward step: the
 * gradient of the photometric loss to the Gaussians and, through the dual
 * gradient flow, to each pose) for the image gradient v_rgb[P][3]:
 * walks each pixel's list back to front from `last`, recovering T by division,
 * reduces per splat over the wave before any global atomic, then chains the
 * per-pair 2D gradients to the Gaussian parameters (summed over views; written
 * or added per s->grad_accumulate) and adds each view's twist gradient into
 * row index[v] (or v) of v_twist.  `g` and `cams` must be those of the forward.
 * Every argument check of both halves runs before any work is enqueued. */
gs_status gs_render_bwd(gs_ctx* ctx, const gs_gaussians* g, const gs_cameras* cams,
                        const gs_settings* s, const float* bg, const float* T_final,
                        const int32_t* last, const float* v_rgb, gs_gaussians_grad* grads,
                        float* v_twist, void* stream);

/* The two halves of gs_render_bwd, for callers that time or schedule them
 * separately.  gs_raster_bwd: the per-pixel walk, adding the per-pair 2D
 * gradients into the context.  gs_project_bwd: consumes (and clears) them,
 * writing the Gaussian gradients and adding the twists.  gs_render_bwd is
 * gs_raster_bwd followed by gs_project_bwd. */
gs_status gs_raster_bwd(gs_ctx* ctx, const gs_cameras* cams, const gs_settings* s,
                        const float* bg, const float* T_final, const int32_t* last,
                        const float* v_rgb, void* stream);
gs_status gs_project_bwd(gs_ctx* ctx, const gs_gaussians* g, const gs_cameras* cams,
                         const gs_settings* s, gs_gaussians_grad* grads, float* v_twist,
                         void* stream);

/* Photometric L1 term (Sec. 3.3 eq. L_photo, its l1 part): loss += mean over
 * views of the mean over pixels and channels of |rgb - target|; v_rgb =
 * sign(rgb - target) / (3 P_v V) (sign(0) = 0), overwritten.  loss[1] is a
 * device float, accumulated. */
gs_status gs_l1_loss_grad(gs_ctx* ctx, const gs_cameras* cams, const float* rgb,
                          const float* target, float* v_rgb, float* loss, void* stream);

/* The whole photometric loss (Sec. 3.3 eq. L_photo; Algorithm 1, photometric
 * loss): loss += (1 - lambda_ssim) L1 + lambda_ssim (1 - SSIM), lambda_ssim =
 * 0.2 in the paper, each term the mean over views of the mean over the view's
 * pixels and channels; v_rgb[P][3] = its gradient, overwritten.  SSIM per
 * channel with an 11 x 11 Gaussian window of standard deviation 1.5 (the outer
 * product of the normalised 1D window), c1 = 0.01^2, c2 = 0.03^2 (data range
 * 1), and zeros beyond each view's border; the L1 gradient is sign(d) with
 * sign(0) = 0.  lambda_ssim in [0, 1] (0 gives gs_l1_loss_grad's result).
 * loss[1] is a device float, accumulated. */
gs_status gs_photo_loss_grad(gs_ctx* ctx, const gs_cameras* cams, const float* rgb,
                             const float* target, float lambda_ssim, float* v_rgb, float* loss,
                             void* stream);

/* Gaussians from SfM points (Sec. 3.3, initialisation; Algorithm 1,
 * initialise G from the SfM points): for each point i of points[n][3] (with
 * colour rgb[n][3] in [0, 1]): mean = the point; an isotropic scale s = the
 * mean Euclidean distance to its k nearest other points (k = 4 in the paper;
 * all other points when there are fewer; s raised to 1e-7 when smaller),
 * log_scales = log s on all three axes; identity rotation (1, 0, 0, 0);
 * opacity_logit = log(opacity / (1 - opacity)) (opacity = 0.1 in the paper);
 * sh degree-0 band = (rgb - 0.5) 2 sqrt(pi), so the renderer's colour rule
 * gives back rgb; the other bands zero.  Outputs in the planar layout of
 * gs_gaussians (caller-owned device arrays).  The neighbours are exact (a
 * bounding-volume hierarchy over the points in Morton order, searched depth
 * first and pruned by the k-th distance found so far); any of several
 * equidistant neighbours may be taken, which leaves s unchanged.  Points must
 * be finite (a non-finite point is never taken as a neighbour and gets an
 * undefined scale).  1 <= k <= GS_INIT_MAX_K; n <= the context's max_pairs
 * (it uses the pair-sized workspace). */
#define GS_INIT_MAX_K 8
gs_status gs_init_gaussians(gs_ctx* ctx, const float* points, const float* rgb, int32_t n,
                            int32_t k, float opacity, int32_t sh_degree, float* means,
                            float* log_scales, float* quats, float* opacity_logit, float* sh,
                            void* stream);

/* One Levenberg-Marquardt step of bundle adjustment (Sec. 3.2 "Bundle
 * Adjustment", eq. L_BA^SfM: Huber on the squared reprojection error, poses on
 * SE(3), Levenberg-Marquardt), iteratively reweighted: for each observation
 * (camera obs_cam, point obs_pt, pixel obs_xy) with residual r = pi_i(X_k) -
 * x, s = |r|^2, weight w = 1 (s <= delta^2) or delta / sqrt(s), and Jacobian
 * J = dr/d(xi_i, X_k) (xi the left twist at the current pose, translation
 * first, as everywhere in this library), the step d = (d_twist, d_X) solves
 *   (H + lm_lambda diag(H)) d = -g,   H = sum w J^T J,   g = sum w J^T r.
 * Observations with p_z < near_plane are left out; a camera or a point with
 * no observation is held fixed (d = 0).  The points are eliminated (Schur
 * complement) and the 6 n_cams camera system is solved by conjugate
 * gradients preconditioned with its inverse 6x6 diagonal blocks, in double,
 * for max_iter iterations or until the residual is below tol times the
 * right-hand side (a device flag ends the iteration: the call stays
 * graph-capturable).  The step is to be applied as T_i <- Exp(d_twist_i) T_i
 * (gs_pose_compose) and X_k <- X_k + d_X_k.
 * X[Pt][3], viewmat[n_cams][12], intr[n_cams][4]; observations SORTED BY
 * CAMERA (otherwise stats[4] = 1 and the step is zero); pt_off / pt_obs: the
 * point-major index of the observations from track_point_index; pm_cam /
 * pm_xy (both NULL, or both set): its point-major copies of obs_cam and
 * obs_xy, which the passes over the points then read in order.
 * Outputs: d_twist[n_cams][6], d_X[Pt][3] (device floats, overwritten); stats
 * (device float[5], may be NULL): iterations run, final relative residual,
 * the robust cost sum rho before the step, masked observations, unsorted
 * flag.  lm_lambda > 0. */
#define GS_BA_MAX_CAMS 65536
typedef struct gs_ba gs_ba;
/* BA workspace: 96 B per point and 676 B per camera of device memory,
 * allocated once. */
gs_status gs_ba_create(gs_ba** out, int64_t max_points, int32_t max_cams);
gs_status gs_ba_destroy(gs_ba* ba);
gs_status gs_ba_lm_step(gs_ba* ba, const float* X, int32_t Pt, const float* viewmat,
                        const float* intr, int32_t n_cams, const int32_t* obs_cam,
                        const int32_t* obs_pt, const float* obs_xy, int32_t M,
                        const int32_t* pt_off, const int32_t* pt_obs, const int32_t* pm_cam,
                        const float* pm_xy, float delta, float lm_lambda, float near_plane,
                        int32_t max_iter, float tol, float* d_twist, float* d_X, float* stats,
                        void* stream);

/* Track reprojection (Sec. 3.3 eq. L_BA^joint; Algorithm 1, joint BA loss):
 * for each observation o = (camera obs_cam[o], point obs_pt[o], pixel
 * obs_xy[o][2]):  p = R X + t; masked (no loss, no gradient, counted) if
 * p_z < near; r = (fx px/pz + cx, fy py/pz + cy) - x; s = |r|^2;
 * rho(s) = s if s <= delta^2 else 2 delta sqrt(s) - delta^2.
 *   loss[1]            += lambda sum rho                      (device float)
 *   v_X[Pt][3]         += d(lambda sum rho)/dX
 *   v_twist[n_cams][6] += d(lambda sum rho)/dxi               (left twist)
 *   residual[M][2]      = r                    (may be NULL)
 *   J_pose[M][2][6]     = dr/dxi, J_X[M][2][3] = dr/dX        (may be NULL)
 * X[Pt][3] (points, kept separate from the Gaussian means), viewmat[n_cams][12],
 * intr[n_cams][4].  Observations must be sorted by camera (any order works,
 * sorted is faster).  pt_off / pt_obs (both NULL, or both set): a point-major
 * index of the observations built by track_point_index for these obs_pt, M and
 * Pt; with it v_X is summed per point (no atomics, a fixed order) instead of
 * scattered with atomics per observation; the results agree up to rounding.
 * pm_cam / pm_xy (both NULL, or both set, and then the index too): the
 * observations' cameras and pixels in that point-major order (track_point_index
 * writes them); with them, and with n_cams <= GS_TRACK_PM_MAX_CAMS, no
 * residual or Jacobian asked for and v_X given, the whole term is one pass
 * over the points reading every array in order (per-workgroup twist sums in
 * LDS, then summed over the workgroups in a fixed order): no global atomics,
 * the same results up to rounding.  Otherwise they are not read. */
#define GS_TRACK_PM_MAX_CAMS 2048
gs_status track_reproj_fwd_bwd(gs_ctx* ctx, const float* X, int32_t Pt,
                               const float* viewmat, const float* intr, int32_t n_cams,
                               const int32_t* obs_cam, const int32_t* obs_pt,
                               const float* obs_xy, int32_t M, float delta, float lambda,
                               float near_plane, float* residual, float* loss, float* v_X,
                               float* v_twist, float* J_pose, float* J_X,
                               const int32_t* pt_off, const int32_t* pt_obs,
                               const int32_t* pm_cam, const float* pm_xy, void* stream);

/* track_reproj_fwd_bwd without a context, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors as
 * track_reproj_fwd_bwd minus the context; it allocates nothing and
 * synchronises nothing (it takes no point-major copies: pm_cam / pm_xy of
 * track_reproj_fwd_bwd are not among its arguments).  Its accumulators (per-camera twist sums and the loss
 * in double, status words) live in one fixed array of device memory inside
 * the library, 6 x GS_NOALLOC_MAX_CAMS doubles plus a few words (about 197
 * KB), one copy per GPU, held until the process ends; each call clears the
 * part it uses first.  n_cams > GS_NOALLOC_MAX_CAMS returns GS_ERR_CAPACITY;
 * a device index >= GS_NOALLOC_MAX_DEVICES returns GS_ERR_HIP.  The count of
 * masked observations is not reported (track_reproj_fwd_bwd reports it).
 * Calls that overlap on one GPU (on different streams, or from different
 * threads without ordering) share that array and race: order them. */
#define GS_NOALLOC_MAX_CAMS 4096
#define GS_NOALLOC_MAX_DEVICES 64
gs_status track_reproj_fwd_bwd_noalloc(const float* X, int32_t Pt, const float* viewmat,
                                       const float* intr, int32_t n_cams, const int32_t* obs_cam,
                                       const int32_t* obs_pt, const float* obs_xy, int32_t M,
                                       float delta, float lambda, float near_plane,
                                       float* residual, float* loss, float* v_X, float* v_twist,
                                       float* J_pose, float* J_X, const int32_t* pt_off,
                                       const int32_t* pt_obs, void* stream);

/* The point-major index of track observations that track_reproj_fwd_bwd can
 * take (it depends on obs_pt only, so a scene builds it once):
 * pt_off[Pt + 1] (device, 16-byte aligned): point k's observations are
 * pt_obs[pt_off[k] .. pt_off[k + 1]), ascending; pt_obs[M] (device) receives
 * pt_off[Pt] <= M indices (observations whose point is outside [0, Pt) are left
 * out).  Both caller-owned.  obs_cam[M], obs_xy[M][2] and pm_cam[M],
 * pm_xy[M][2] (all four NULL, or all set, unless M = 0; device,
 * caller-owned): the
 * observations' cameras and pixels copied into pm_* in the index's order
 * (pm_cam[j] = obs_cam[pt_obs[j]], j < pt_off[Pt]), for track_reproj_fwd_bwd's
 * point-major pass; obs_xy and pm_xy 8-byte aligned.  GS_ERR_CAPACITY if Pt
 * exceeds the context's max_pairs or its scan workspace. */
gs_status track_point_index(gs_ctx* ctx, const int32_t* obs_pt, int32_t M, int32_t Pt,
                            int32_t* pt_off, int32_t* pt_obs, const int32_t* obs_cam,
                            const float* obs_xy, int32_t* pm_cam, float* pm_xy, void* stream);

/* Pose composition T_i = Exp(dxi_i) T_i^(0) (Algorithm 1, pose adjustment,
 * with (+) read as left composition): twist[V][6] = (rho, phi), base[V][12],
 * out[V][12]. */
gs_status gs_pose_compose(int32_t V, const float* twist, const float* base, float* out,
                          void* stream);

/* Its backward: out[V][6] = J_l(twist)^T g, with g[V][6] the left-twist
 * gradient at the composed pose and J_l the SE(3) left Jacobian. */
gs_status gs_pose_compose_bwd(int32_t V, const float* twist, const float* g, float* out,
                              void* stream);

/* One Adam step (Algorithm 1, update step) on up to GS_ADAM_MAX_GROUPS
 * parameter groups in one launch: p -= lr m_hat / (sqrt(v_hat) + eps) with
 * bias-corrected moments; m, v updated in place.  The step number t of the
 * bias corrections 1 / (1 - beta^t) is *step_dev (a device int32 read when the
 * kernel runs; values below 1 count as 1) when step_dev is not NULL, else
 * `step` (>= 1).  With the device counter a captured HIP graph takes a new
 * step number on every replay (see gs_step_advance). */
#define GS_ADAM_MAX_GROUPS 16
typedef struct {
    float* param;
    const float* grad;
    float* exp_avg;
    float* exp_avg_sq;
    int64_t n;
    float lr;
} gs_adam_group;

gs_status gs_adam_step(const gs_adam_group* groups, int32_t n_groups, int32_t step,
                       const int32_t* step_dev, float beta1, float beta2, float eps,
                       void* stream);

/* *step_dev += 1 on the device (enqueued on stream): the step counter a
 * training step advances once before its Adam calls read it. */
gs_status gs_step_advance(int32_t* step_dev, void* stream);

/* Adam state of the five Gaussian arrays for gs_project_bwd_adam: params[q] is
 * the array of gs_gaussians it steps (means, log_scales, quats, opacity_logit,
 * sh, in that order; the same pointers), exp_avg / exp_avg_sq its moments in
 * the same layout, lr[q] its learning rate. */
typedef struct {
    float* params[5];
    float* exp_avg[5];
    float* exp_avg_sq[5];
    float lr[5];
} gs_gaussian_adam;

/* gs_project_bwd followed by gs_adam_step on the five Gaussian arrays, in one
 * pass (the backward and update steps of Algorithm 1): each Gaussian's
 * gradient, summed over the views, is spent on its Adam step in place instead
 * of being written, so the gradients never reach memory.  Same results as the
 * two calls (the element update is the same code); the twists are added into
 * v_twist as gs_project_bwd does.  The arrays of `adam->params` must be those
 * of `g`; the step number is *step_dev when step_dev is not NULL, else step
 * (>= 1), as in gs_adam_step. */
gs_status gs_project_bwd_adam(gs_ctx* ctx, const gs_gaussians* g, const gs_cameras* cams,
                              const gs_settings* s, const gs_gaussian_adam* adam, int32_t step,
                              const int32_t* step_dev, float beta1, float beta2, float eps,
                              float* v_twist, void* stream);

/* MCMC densification (Sec. 3.3, stochastic density control; Algorithm 1,
 * MCMCDensify), relocation: every Gaussian whose opacity sigmoid(logit) is
 * at most dead_opacity (0.005) moves onto a live one drawn with probability
 * proportional to opacity; a source drawn c times ends as n = c + 1 copies
 * with opacity 1 - (1 - o)^(1/n) and scale multiplied by
 * o / sum_{i=1..n} sum_{k=0..i-1} C(i-1, k) (-1)^k o'^(k+1) / sqrt(k+1)
 * (n capped at 51 in both rules); copies take the source's mean, rotation and
 * SH; the Adam moments of sources and copies are zeroed.  The draw is exact
 * integer arithmetic: weight floor(o 2^24) (o in double), Gaussian j (dead)
 * takes the first index whose inclusive weight prefix exceeds floor(u[j] W),
 * W the total, u[N] device floats in [0, 1) supplied by the caller (the
 * library draws no random numbers).  state: the five planar parameter arrays
 * of N Gaussians and their moments (lr unused), updated in place.  src[N]
 * (device, may be NULL) receives each Gaussian's source or -1; n_relocated
 * (device int32, may be NULL) the count.  To grow the set, enlarge the
 * arrays with dead slots (opacity logit far below the threshold, zero
 * moments) and relocate.  N <= the context's max_pairs. */
gs_status gs_mcmc_relocate(gs_ctx* ctx, const gs_gaussian_adam* state, int32_t N,
                           int32_t sh_degree, const float* u, float dead_opacity, int32_t* src,
                           int32_t* n_relocated, void* stream);

/* MCMC densification, noise on the means after an update:
 * mu += scale sigmoid(-k (o - t)) Sigma eta, Sigma = R diag(exp(2 s)) R^T the
 * Gaussian's covariance, eta[3][N] standard normal draws supplied by the
 * caller, scale = the noise weight times the position learning rate (the
 * adopted method uses k = 100, t = 0.005). */
gs_status gs_mcmc_noise(float* means, const float* log_scales, const float* quats,
                        const float* opacity_logit, int32_t N, const float* eta, float scale,
                        float k, float t, void* stream);

#ifdef __cplusplus
}
#endif
#endif
