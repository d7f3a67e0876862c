/*
 * FP64 CPU oracle for the splatting hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct definitions of what the GPU path computes.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library; the product path never does.  It shares no code with the
 * HIP library (no headers, no helpers, no constants).
 *
 * Inputs are double (callers widen the FP32 values the GPU gets, which is
 * exact); all arithmetic is double.  Layouts match the GPU library's:
 *   Gaussians (planar): means[3][N], log_scales[3][N], quats[4][N] (w,x,y,z),
 *     opacity_logit[N], sh[K][3][N], K = (deg+1)^2 (l-major, m = -l..l).
 *   Cameras: viewmat[V][12] world->camera [R|t] row-major 3x4,
 *     intr[V][4] = fx, fy, cx, cy, wh[V][2] = W, H.
 *   Pixels: views packed view-major, rows y-major, pixel (u,v) sampled at
 *     (u+0.5, v+0.5).
 *
 * cfg[] (OR_CFG_N doubles):
 *   0 near plane            1 eps2d (dilation)        2 frustum pad for J
 *   3 alpha_min (1/255)     4 alpha_max (0.99)        5 T_min (1e-4)
 *   6 band: float32 position error of mean2d, relative to its magnitude
 *   7 band: T stop, relative  8 band: float32 relative error of sigma
 *   9 band: depth key, relative distance of the FP64 depth from a midpoint
 *     between two adjacent float32 values
 * A pixel is flagged ambiguous when a decision that shapes it (alpha gate,
 * alpha clamp, transmittance stop, depth order) lies within these bands.  The
 * depth order is the order of the float32-rounded depth (ties by pair index),
 * so it is in doubt only where two neighbours' rounded depths are equal or
 * adjacent and one FP64 depth sits within the band of a rounding midpoint.
 */
#ifndef GLOSPLAT_ORACLE_H
#define GLOSPLAT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define OR_CFG_N 10

/* Projection of every (view, Gaussian) pair (EWA splatting of 3D Gaussians,
 * colour from SH at the view direction).  Outputs are [V*N] (x k) arrays.
 * valid = 0 for pairs culled by the near plane, a non-positive 2D
 * determinant, or opacity <= alpha_min. */
int or_project(int N, int sh_degree, const double* means, const double* log_scales,
               const double* quats, const double* opacity_logit, const double* sh,
               int V, const double* viewmat, const double* intr, const int* wh,
               const double* cfg,
               int* valid, double* depth, double* mean2d, double* cov2d,
               double* conic, double* opacity, double* rgb, double* ext);

/* Brute-force per-pixel compositing over all valid splats of the pixel's view,
 * in ascending (float32 rounding of the depth, Gaussian index) order, with the
 * 1/255 alpha gate, the 0.99 alpha clamp and the 1e-4 transmittance stop, then
 * C + T bg.  npix/pix select global pixel indices (pix == NULL: all pixels).
 * out_ngate = number of splats passing the alpha gate at the pixel;
 * out_nclamp = number of contributors whose alpha was clamped (any output
 * pointer may be NULL).
 * If v_rgb != NULL the exact derivative of the image is pulled back from the
 * stored per-pixel list into v2d[V*N][9] (accumulated):
 *   (d/d mean2d.x, mean2d.y, conic A, B, C, opacity, r, g, b),
 * with sigma = 0.5*(A dx^2 + C dy^2) + B dx dy and d = mean2d - pixel. */
int or_render(int V, const int* wh, int N, const int* valid, const double* depth,
              const double* mean2d, const double* conic, const double* opacity,
              const double* rgb, const double* bg, const double* cfg,
              long long npix, const long long* pix,
              double* out_rgb, double* out_T, int* out_ncontrib, int* out_ngate, int* out_nclamp,
              int* ambiguous, const double* v_rgb, double* v2d);

/* Chain rule from the per-pair 2D gradients to the Gaussian parameters (summed
 * over views, overwriting the outputs) and to each view's left-perturbation
 * twist (rho, phi) (overwriting v_twist[V][6]). */
int or_project_bwd(int N, int sh_degree, const double* means, const double* log_scales,
                   const double* quats, const double* opacity_logit, const double* sh,
                   int V, const double* viewmat, const double* intr, const int* wh,
                   const double* cfg, const double* v2d,
                   double* v_means, double* v_log_scales, double* v_quats,
                   double* v_opacity_logit, double* v_sh, double* v_twist);

/* Track reprojection: residual pi_i(X_k) - x, Huber on the squared norm with
 * threshold delta, scaled by lambda.  Outputs overwrite: residual[M][2],
 * loss[1], v_X[Pt][3], v_twist[ncam][6], J_pose[M][2][6], J_X[M][2][3],
 * masked[M]. Any output pointer may be NULL. */
int or_track(int Pt, const double* X, int ncam, const double* viewmat, const double* intr,
             int M, const int* obs_cam, const int* obs_pt, const double* obs_xy,
             double delta, double lambda, double near_plane,
             double* residual, double* loss, double* v_X, double* v_twist,
             double* J_pose, double* J_X, int* masked);

/* T = Exp(xi) * T0 for xi = (rho, phi), by the power series of the 4x4
 * matrix exponential.  out[V][12]. */
void or_se3_exp_compose(int V, const double* xi, const double* base, double* out);

/* out = J_l(xi)^T g, J_l = sum_n ad_xi^n / (n+1)!  (SE(3) left Jacobian). */
void or_se3_jl_transpose(int V, const double* xi, const double* g, double* out);

/* Adam (bias-corrected), in place. */
void or_adam(long long n, double* p, const double* g, double* m, double* v,
             double lr, double beta1, double beta2, double eps, int step);

/* Tile lists: pair (v,g) is listed in tile t of view v iff, for some quadrant
 * (tile_w/2 x tile_h/2 block) of t, the minimum of sigma over the rectangle
 * spanned by that quadrant's pixel centres is <= ln(o/alpha_min) + margin; the
 * quadrants that pass form the entry's 4-bit mask (bit qx + 2 qy).  Lists are
 * ordered by (float32 depth bits, pair index).  ranges[T_total][2] (start,
 * end) into ids[] / masks[] (masks may be NULL); returns the total count, or
 * -(needed) if it exceeds cap. */
long long or_bin_sort(int V, const int* wh, int tile_w, int tile_h, int N,
                      const int* valid, const float* mean2d, const float* conic,
                      const float* opacity, const float* depth, double alpha_min,
                      double margin, long long cap, long long* ranges, int* ids, int* masks);

/* Photometric L1 term: loss = mean over views of the mean over the view's
 * pixels and channels of |rgb - target|; v_rgb[P][3] (may be NULL) =
 * sign(rgb - target) / (3 P_v V), with sign(0) = 0. */
int or_l1(int V, const int* wh, const double* rgb, const double* target, double* loss,
          double* v_rgb);

/* SSIM with a win x win Gaussian window (std wsig), constants c1, c2 and zeros
 * beyond the image border: ssim = mean over views of the mean over the view's
 * pixels and channels of the SSIM map; ssim_map[P][3] and v_rgb[P][3] =
 * d ssim / d rgb may be NULL. */
int or_ssim(int V, const int* wh, const double* rgb, const double* target, int win,
            double wsig, double c1, double c2, double* ssim, double* ssim_map, double* v_rgb);

/* Mean Euclidean distance of points (pts[n][3]) to their k nearest other
 * points (all of them when fewer), by brute force: for the nq points q_idx[]
 * (q_idx == NULL: all n) into out[nq]. */
int or_knn_mean_dist(long long n, const double* pts, int k, long long nq, const long long* q_idx,
                     double* out);

/* Gaussians from SfM points: means = pts, isotropic log-scale = log(max(mean
 * distance to the k nearest other points, s_min)), identity rotation, opacity
 * logit = logit(opacity), SH degree-0 band = (rgb - 0.5) / C0, other bands 0.
 * Outputs in the planar layout of the Gaussians. */
int or_init_gaussians(long long n, const double* pts, const double* rgb, int k, double opacity,
                      double s_min, int sh_degree, double* means, double* log_scales,
                      double* quats, double* opacity_logit, double* sh);

/* Bundle adjustment, one Levenberg-Marquardt step (iteratively reweighted
 * Gauss-Newton on the Huber cost): the dense undamped normal equations
 * H [n][n], g [n] (n = 6 ncam + 3 Pt; cameras first, left twists (rho, phi),
 * then points) and the robust cost; returns the masked-observation count. */
int or_ba_normal(int Pt, const double* X, int ncam, const double* viewmat, const double* intr,
                 int M, const int* obs_cam, const int* obs_pt, const double* obs_xy, double delta,
                 double near_plane, double* H, double* g, double* cost);

/* out[n] = (H + lambda diag(H)) d + g, accumulated per observation (any size). */
int or_ba_normal_residual(int Pt, const double* X, int ncam, const double* viewmat,
                          const double* intr, int M, const int* obs_cam, const int* obs_pt,
                          const double* obs_xy, double delta, double near_plane, double lambda,
                          const double* d, double* out);

/* MCMC relocation of dead Gaussians (opacity <= t_dead) onto live ones drawn
 * with probability proportional to opacity (integer weights floor(o 2^24),
 * draws floor(u_j W) given by u[N]); the n copies of a source take opacity
 * 1 - (1 - o)^(1/n) and their scale is multiplied by o / sum_i sum_k
 * C(i-1,k) (-1)^k o'^(k+1) / sqrt(k+1), with n capped at 51 in both rules;
 * moments of sources and copies reset.
 * In place on the planar arrays; exp_avg / exp_avg_sq: the five moment arrays
 * of each.  src[N] = source of each relocated Gaussian, -1 otherwise. */
int or_mcmc_relocate(long long N, int sh_degree, double* means, double* log_scales, double* quats,
                     double* opacity_logit, double* sh, double* const* exp_avg,
                     double* const* exp_avg_sq, const double* u, double t_dead, long long* src,
                     long long* n_relocated);

/* MCMC noise on the means: mu += scale sigmoid(-k (o - t)) Sigma eta. */
void or_mcmc_noise(long long N, double* means, const double* log_scales, const double* quats,
                   const double* opacity_logit, const double* eta, double scale, double k, double t);

/* Real spherical-harmonic basis (Condon-Shortley phase) at unit direction d,
 * K = (deg+1)^2 values; dY[K][3] = gradient of the polynomial form, may be
 * NULL. */
void or_sh_basis(int deg, const double* d, double* Y, double* dY);

int or_num_threads(void);
void or_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
