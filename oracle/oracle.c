/*
 * FP64 CPU oracle for the splatting hot path -- TEST INFRASTRUCTURE ONLY.
 * See oracle.h for layouts.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg use this file.
 *
 * What it follows:
 *  - pinhole projection pi(X) = proj(K (R X + t)), world->camera [R|t]
 *    (GloSplat Sec. 3.2, "Bundle Adjustment"; Appendix E, projection function);
 *  - pose composition T = T0 (+) dT with (+) read as Exp(dT) * T0
 *    (Appendix E, Algorithm 1, pose adjustment);
 *  - joint BA loss: Huber on the squared reprojection error, delta = 1 px,
 *    weighted by lambda_BA (Sec. 3.3, eq. L_BA^joint and the total objective);
 *  - rasterization Rasterize(G, T_i, K_i) (Sec. 3.3 "Implementation",
 *    Algorithm 1): the paper delegates it to an external 3DGS rasterizer and
 *    states no formula, so the standard EWA-splatting definition is written
 *    out here (projected covariance J W Sigma W^T J^T with a 0.3 px^2
 *    dilation, the 1/255 alpha gate, the 0.99 alpha clamp and the 1e-4
 *    transmittance stop);
 *  - Adam with the bias-corrected moments (Algorithm 1, update step).
 *
 * Everything is computed per pixel by brute force over all splats: no tiles,
 * no sorting of intersections.  The backward walks the forward's stored list.
 */
#include "oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (timing runs only). */
void or_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------ small linear algebra */

static void mat3_mul(const double* A, const double* B, double* C) {
    double T[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += A[3 * i + k] * B[3 * k + j];
            T[3 * i + j] = s;
        }
    memcpy(C, T, sizeof T);
}

static void mat3_transpose(const double* A, double* B) {
    double T[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) T[3 * i + j] = A[3 * j + i];
    memcpy(B, T, sizeof T);
}

static void mat3_vec(const double* A, const double* x, double* y) {
    double t[3];
    for (int i = 0; i < 3; i++) t[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
    memcpy(y, t, sizeof t);
}

static void mat3T_vec(const double* A, const double* x, double* y) {
    double t[3];
    for (int i = 0; i < 3; i++) t[i] = A[i] * x[0] + A[3 + i] * x[1] + A[6 + i] * x[2];
    memcpy(y, t, sizeof t);
}

static void cross3(const double* a, const double* b, double* c) {
    double t[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    memcpy(c, t, sizeof t);
}

/* Rotation of a unit quaternion (w,x,y,z): the standard matrix of v -> q v q*. */
static void quat_to_rot(const double* q, double* R) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* d R_ij / d q_c for the matrix above, dR[c][9]. */
static void quat_to_rot_jac(const double* q, double dR[4][9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double J[4][9] = {
        /* d/dw */ {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0},
        /* d/dx */ {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x},
        /* d/dy */ {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y},
        /* d/dz */ {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0},
    };
    memcpy(dR, J, sizeof J);
}

/* ------------------------------------------------------------ spherical harmonics */
/*
 * Real SH with the Condon-Shortley phase kept, written from the
 * associated-Legendre closed form:
 *   Y_l0  = K_l^0 P_l(z)
 *   Y_lm  = sqrt(2) K_l^m (-1)^m P_l^(m)(z) Re((x+iy)^m)      m > 0
 *   Y_l-m = sqrt(2) K_l^m (-1)^m P_l^(m)(z) Im((x+iy)^m)      m > 0
 * with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), P_l^(m) the m-th derivative
 * of the Legendre polynomial P_l, and (x+iy)^m = sin^m(theta) e^{i m phi} on
 * the unit sphere.  Each Y is a polynomial in (x,y,z), so its gradient is
 * exact.  Index of (l,m) is l*l + l + m.
 */
static double factorial(int n) {
    double f = 1;
    for (int i = 2; i <= n; i++) f *= i;
    return f;
}

static double binom(int n, int k) { return factorial(n) / (factorial(k) * factorial(n - k)); }

/* m-th derivative of P_l at z: P_l(z) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k,l) z^(l-2k). */
static double legendre_deriv(int l, int m, double z) {
    double s = 0;
    for (int k = 0; 2 * k <= l; k++) {
        int p = l - 2 * k;
        if (p < m) continue;
        double c = ((k & 1) ? -1.0 : 1.0) * binom(l, k) * binom(2 * l - 2 * k, l);
        s += c * factorial(p) / factorial(p - m) * pow(z, p - m);
    }
    return s / pow(2.0, l);
}

void or_sh_basis(int deg, const double* d, double* Y, double* dY) {
    double x = d[0], y = d[1], z = d[2];
    /* a[m] + i b[m] = (x + i y)^m */
    double a[8], b[8];
    a[0] = 1; b[0] = 0;
    for (int m = 1; m <= deg; m++) {
        a[m] = a[m - 1] * x - b[m - 1] * y;
        b[m] = a[m - 1] * y + b[m - 1] * x;
    }
    for (int l = 0; l <= deg; l++) {
        for (int m = 0; m <= l; m++) {
            double K = sqrt((2 * l + 1) / (4 * PI) * factorial(l - m) / factorial(l + m));
            double P = legendre_deriv(l, m, z);
            double dP = legendre_deriv(l, m + 1, z);
            if (m == 0) {
                int i = l * l + l;
                Y[i] = K * P;
                if (dY) { dY[3 * i] = 0; dY[3 * i + 1] = 0; dY[3 * i + 2] = K * dP; }
                continue;
            }
            double s = sqrt(2.0) * K * ((m & 1) ? -1.0 : 1.0);
            int ip = l * l + l + m, in = l * l + l - m;
            Y[ip] = s * P * a[m];
            Y[in] = s * P * b[m];
            if (dY) {
                /* d a_m/dx = m a_{m-1}, d a_m/dy = -m b_{m-1};
                   d b_m/dx = m b_{m-1}, d b_m/dy =  m a_{m-1} */
                dY[3 * ip + 0] = s * P * m * a[m - 1];
                dY[3 * ip + 1] = s * P * (-m * b[m - 1]);
                dY[3 * ip + 2] = s * dP * a[m];
                dY[3 * in + 0] = s * P * m * b[m - 1];
                dY[3 * in + 1] = s * P * m * a[m - 1];
                dY[3 * in + 2] = s * dP * b[m];
            }
        }
    }
}

/* ------------------------------------------------------------ per-pair projection */

typedef struct {
    double R[9], t[3], fx, fy, cx, cy;
    int W, H;
} cam_t;

static void load_cam(const double* viewmat, const double* intr, const int* wh, int v, cam_t* c) {
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) c->R[3 * i + j] = viewmat[12 * v + 4 * i + j];
        c->t[i] = viewmat[12 * v + 4 * i + 3];
    }
    c->fx = intr[4 * v]; c->fy = intr[4 * v + 1]; c->cx = intr[4 * v + 2]; c->cy = intr[4 * v + 3];
    c->W = wh[2 * v]; c->H = wh[2 * v + 1];
}

typedef struct {
    int valid;
    double mu[3], p[3];         /* world mean, camera-space mean */
    double qn[4], qnorm;        /* normalised quaternion and |q| */
    double Rq[9], s[3];         /* rotation of the Gaussian, scales exp(log_scale) */
    double Sig[9], Sigc[9];     /* world and camera covariance */
    double J[6];                /* 2x3 projection Jacobian (with the off-screen clamp) */
    int clampx, clampy;         /* clamp active; then limx/limy hold the clamp value */
    double limx, limy;
    double cov2d[3];            /* a, b, c of the dilated 2D covariance */
    double conic[3];            /* A, B, C of its inverse */
    double mean2d[2], depth, opacity;
    double dir[3], dist, camc[3];
    double shsum[3], rgb[3];
    double ext[2];
} pair_t;

static void project_pair(int N, int deg, const double* means, const double* log_scales,
                         const double* quats, const double* opacity_logit, const double* sh,
                         const cam_t* c, int g, const double* cfg, pair_t* P) {
    const double near_plane = cfg[0], eps2d = cfg[1], pad = cfg[2], amin = cfg[3];
    memset(P, 0, sizeof *P);
    for (int i = 0; i < 3; i++) P->mu[i] = means[(size_t)i * N + g];
    mat3_vec(c->R, P->mu, P->p);
    for (int i = 0; i < 3; i++) P->p[i] += c->t[i];
    P->depth = P->p[2];
    double q[4];
    for (int i = 0; i < 4; i++) q[i] = quats[(size_t)i * N + g];
    P->qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int i = 0; i < 4; i++) P->qn[i] = q[i] / P->qnorm;
    quat_to_rot(P->qn, P->Rq);
    for (int i = 0; i < 3; i++) P->s[i] = exp((double)log_scales[(size_t)i * N + g]);
    /* Sigma = Rq S S^T Rq^T */
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double v = 0;
            for (int k = 0; k < 3; k++) v += P->Rq[3 * i + k] * P->s[k] * P->s[k] * P->Rq[3 * j + k];
            P->Sig[3 * i + j] = v;
        }
    double RS[9], Rt[9];
    mat3_mul(c->R, P->Sig, RS);
    mat3_transpose(c->R, Rt);
    mat3_mul(RS, Rt, P->Sigc);
    P->opacity = 1.0 / (1.0 + exp(-(double)opacity_logit[g]));
    /* colour: view direction from the camera centre c = -R^T t */
    double mt[3] = {-c->t[0], -c->t[1], -c->t[2]};
    mat3T_vec(c->R, mt, P->camc);
    double dv[3] = {P->mu[0] - P->camc[0], P->mu[1] - P->camc[1], P->mu[2] - P->camc[2]};
    P->dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    for (int i = 0; i < 3; i++) P->dir[i] = dv[i] / P->dist;
    int K = (deg + 1) * (deg + 1);
    double Y[16];
    or_sh_basis(deg, P->dir, Y, NULL);
    for (int ch = 0; ch < 3; ch++) {
        double s = 0;
        for (int k = 0; k < K; k++) s += Y[k] * sh[((size_t)k * 3 + ch) * N + g];
        P->shsum[ch] = s;
        P->rgb[ch] = s + 0.5 > 0 ? s + 0.5 : 0.0;
    }
    if (P->p[2] < near_plane) return;
    double x = P->p[0], y = P->p[1], z = P->p[2];
    /* Jacobian of the perspective map, with x/z and y/z clamped to the view
       frustum widened by pad * (half the field of view) on each side */
    double lxp = (c->W - c->cx) / c->fx + pad * 0.5 * c->W / c->fx;
    double lxn = c->cx / c->fx + pad * 0.5 * c->W / c->fx;
    double lyp = (c->H - c->cy) / c->fy + pad * 0.5 * c->H / c->fy;
    double lyn = c->cy / c->fy + pad * 0.5 * c->H / c->fy;
    double tx = x / z, ty = y / z;
    P->clampx = 0; P->clampy = 0;
    if (tx > lxp) { tx = lxp; P->clampx = 1; }
    if (tx < -lxn) { tx = -lxn; P->clampx = 1; }
    if (ty > lyp) { ty = lyp; P->clampy = 1; }
    if (ty < -lyn) { ty = -lyn; P->clampy = 1; }
    P->limx = tx; P->limy = ty;
    P->J[0] = c->fx / z; P->J[1] = 0; P->J[2] = -c->fx * tx / z;
    P->J[3] = 0; P->J[4] = c->fy / z; P->J[5] = -c->fy * ty / z;
    /* cov2d = J Sigc J^T + eps2d I */
    double JS[6];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 3; j++) {
            double v = 0;
            for (int k = 0; k < 3; k++) v += P->J[3 * i + k] * P->Sigc[3 * k + j];
            JS[3 * i + j] = v;
        }
    double M2[4];
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            double v = 0;
            for (int k = 0; k < 3; k++) v += JS[3 * i + k] * P->J[3 * j + k];
            M2[2 * i + j] = v;
        }
    double a = M2[0] + eps2d, b = M2[1], cc = M2[3] + eps2d;
    P->cov2d[0] = a; P->cov2d[1] = b; P->cov2d[2] = cc;
    double det = a * cc - b * b;
    if (!(det > 0)) return;
    P->conic[0] = cc / det; P->conic[1] = -b / det; P->conic[2] = a / det;
    P->mean2d[0] = c->fx * x / z + c->cx;
    P->mean2d[1] = c->fy * y / z + c->cy;
    if (!(P->opacity > amin)) return;
    double kk = 2.0 * log(P->opacity / amin);
    P->ext[0] = sqrt(kk * a);
    P->ext[1] = sqrt(kk * cc);
    P->valid = 1;
}

int or_project(int N, int sh_degree, const double* means, const double* log_scales,
               const double* quats, const double* opacity_logit, const double* sh,
               int V, const double* viewmat, const double* intr, const int* wh,
               const double* cfg,
               int* valid, double* depth, double* mean2d, double* cov2d,
               double* conic, double* opacity, double* rgb, double* ext) {
    if (sh_degree < 0 || sh_degree > 3) return -1;
    for (int v = 0; v < V; v++) {
        cam_t c;
        load_cam(viewmat, intr, wh, v, &c);
#pragma omp parallel for schedule(static)
        for (int g = 0; g < N; g++) {
            pair_t P;
            project_pair(N, sh_degree, means, log_scales, quats, opacity_logit, sh, &c, g, cfg, &P);
            size_t i = (size_t)v * N + g;
            if (valid) valid[i] = P.valid;
            if (depth) depth[i] = P.depth;
            if (mean2d) { mean2d[2 * i] = P.mean2d[0]; mean2d[2 * i + 1] = P.mean2d[1]; }
            if (cov2d) for (int k = 0; k < 3; k++) cov2d[3 * i + k] = P.cov2d[k];
            if (conic) for (int k = 0; k < 3; k++) conic[3 * i + k] = P.conic[k];
            if (opacity) opacity[i] = P.opacity;
            if (rgb) for (int k = 0; k < 3; k++) rgb[3 * i + k] = P.rgb[k];
            if (ext) { ext[2 * i] = P.ext[0]; ext[2 * i + 1] = P.ext[1]; }
        }
    }
    return 0;
}

/* ------------------------------------------------------------ per-pixel compositing */

typedef struct {
    int g;
    uint32_t dkey;  /* bits of the float32 rounding of the FP64 camera depth */
    int dmid;       /* FP64 depth within the band of a float32 rounding midpoint */
    double alpha, araw, sigma, dx, dy, T;
} hit_t;

/* The compositing order is ascending (float32 depth, pair index): depths are
 * > near > 0, so the raw bits of the rounded depth order like the numbers.
 * Within one view the pair index v*N + g orders like g. */
static int hit_cmp(const void* pa, const void* pb) {
    const hit_t* a = (const hit_t*)pa;
    const hit_t* b = (const hit_t*)pb;
    if (a->dkey != b->dkey) return a->dkey < b->dkey ? -1 : 1;
    return (a->g > b->g) - (a->g < b->g);
}

static uint32_t depth_key(double d) {
    float f = (float)d;
    uint32_t b;
    memcpy(&b, &f, 4);
    return b;
}

/* Could another FP64 evaluation of the same depth (differing in its last
 * bits) round to a different float32?  Only when the FP64 value lies within
 * `band` (relative) of a midpoint between two adjacent float32 values. */
static int near_rounding_midpoint(double d, double band) {
    float f = (float)d;
    double lo = 0.5 * ((double)f + (double)nextafterf(f, -INFINITY));
    double hi = 0.5 * ((double)f + (double)nextafterf(f, INFINITY));
    double tol = band * fabs(d);
    return fabs(d - lo) <= tol || fabs(d - hi) <= tol;
}

int or_render(int V, const int* wh, int N, const int* valid, const double* depth,
              const double* mean2d, const double* conic, const double* opacity,
              const double* rgb, const double* bg, const double* cfg,
              long long npix, const long long* pix,
              double* out_rgb, double* out_T, int* out_ncontrib, int* out_ngate, int* out_nclamp,
              int* ambiguous, const double* v_rgb, double* v2d) {
    const double amin = cfg[3], amax = cfg[4], tmin = cfg[5];
    const double band_pos = cfg[6], band_t = cfg[7], band_sig = cfg[8], band_mid = cfg[9];
    long long* voff = (long long*)malloc(sizeof(long long) * (V + 1));
    voff[0] = 0;
    for (int v = 0; v < V; v++) voff[v + 1] = voff[v] + (long long)wh[2 * v] * wh[2 * v + 1];
    if (pix == NULL) npix = voff[V];
    int fail = 0;
#pragma omp parallel
    {
        hit_t* hits = (hit_t*)malloc(sizeof(hit_t) * (size_t)(N > 0 ? N : 1));
        uint32_t* gate_key = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(N > 0 ? N : 1));
        int* gate_g = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
#pragma omp for schedule(dynamic, 64)
        for (long long s = 0; s < npix; s++) {
            long long gp = pix ? pix[s] : s;
            int v = 0;
            while (v < V && gp >= voff[v + 1]) v++;
            if (v >= V) { fail = 1; continue; }
            long long local = gp - voff[v];
            int W = wh[2 * v];
            double px = (double)(local % W) + 0.5, py = (double)(local / W) + 0.5;
            int nh = 0, ng = 0;
            for (int g = 0; g < N; g++) {
                size_t i = (size_t)v * N + g;
                if (!valid[i]) continue;
                double mx = mean2d[2 * i], my = mean2d[2 * i + 1];
                double dx = mx - px, dy = my - py;
                double A = conic[3 * i], B = conic[3 * i + 1], C = conic[3 * i + 2];
                double sigma = 0.5 * (A * dx * dx + C * dy * dy) + B * dx * dy;
                if (sigma < 0) continue;
                double araw = opacity[i] * exp(-sigma);
                double alpha = araw < amax ? araw : amax;
                /* how far a float32 evaluation of sigma may stray: position error
                   (relative to the coordinate's magnitude) times |grad sigma|,
                   plus a relative error of sigma itself */
                double gsx = A * dx + B * dy, gsy = B * dx + C * dy;
                double mag = fabs(mx) > fabs(my) ? fabs(mx) : fabs(my);
                if (mag < 1.0) mag = 1.0;
                double err = sqrt(gsx * gsx + gsy * gsy) * band_pos * mag + band_sig * sigma;
                if (fabs(sigma - log(opacity[i] / amin)) <= err) {
                    gate_key[ng] = depth_key(depth[i]); gate_g[ng] = g; ng++;
                }
                if (opacity[i] > amax && fabs(sigma - log(opacity[i] / amax)) <= err) {
                    gate_key[ng] = depth_key(depth[i]); gate_g[ng] = g; ng++;
                }
                if (alpha < amin) continue;
                hit_t h = {g, depth_key(depth[i]), near_rounding_midpoint(depth[i], band_mid),
                           alpha, araw, sigma, dx, dy, 0};
                hits[nh++] = h;
            }
            qsort(hits, nh, sizeof(hit_t), hit_cmp);
            double T = 1.0, Cp[3] = {0, 0, 0};
            int amb = 0, n = 0, stop = -1, nclamp = 0;
            for (int k = 0; k < nh; k++) {
                double Tn = T * (1.0 - hits[k].alpha);
                if (fabs(Tn - tmin) <= band_t * tmin) amb = 1;
                /* two neighbours whose float32 depths are equal or adjacent
                   could swap if either depth's rounding is not certain */
                if (k + 1 < nh && hits[k + 1].dkey - hits[k].dkey <= 1u &&
                    (hits[k].dmid || hits[k + 1].dmid))
                    amb = 1;
                if (Tn < tmin) { stop = k; break; }
                if (!(hits[k].araw < amax)) nclamp++;
                hits[k].T = T;
                size_t i = (size_t)v * N + hits[k].g;
                for (int ch = 0; ch < 3; ch++) Cp[ch] += rgb[3 * i + ch] * hits[k].alpha * T;
                T = Tn;
                n = k + 1;
            }
            /* a splat at the alpha gate or the clamp matters only if it lies
               before the stop */
            for (int j = 0; j < ng && !amb; j++) {
                if (stop < 0) { amb = 1; break; }
                hit_t key = {gate_g[j], gate_key[j], 0, 0, 0, 0, 0, 0, 0};
                if (hit_cmp(&key, &hits[stop]) < 0) amb = 1;
            }
            for (int ch = 0; ch < 3; ch++) {
                double bgc = bg ? bg[ch] : 0.0;
                if (out_rgb) out_rgb[3 * s + ch] = Cp[ch] + T * bgc;
            }
            if (out_T) out_T[s] = T;
            if (out_ncontrib) out_ncontrib[s] = n;
            if (out_ngate) out_ngate[s] = nh;
            if (out_nclamp) out_nclamp[s] = nclamp;
            if (ambiguous) ambiguous[s] = amb;
            if (v_rgb && v2d) {
                /* dC/d alpha_k = c_k T_k - (sum_{j>k} c_j alpha_j T_j + T_N bg) / (1 - alpha_k) */
                const double* vc = v_rgb + 3 * s;
                double Bsum[3] = {0, 0, 0};
                double Tfin = T;
                for (int k = n - 1; k >= 0; k--) {
                    hit_t* h = &hits[k];
                    size_t i = (size_t)v * N + h->g;
                    double* o = v2d + 9 * i;
                    double va = 0;
                    for (int ch = 0; ch < 3; ch++) {
                        double c = rgb[3 * i + ch];
                        double bgc = bg ? bg[ch] : 0.0;
                        double wgt = h->alpha * h->T;
#pragma omp atomic
                        o[6 + ch] += wgt * vc[ch];
                        va += vc[ch] * (c * h->T - (Bsum[ch] + Tfin * bgc) / (1.0 - h->alpha));
                        Bsum[ch] += c * wgt;
                    }
                    if (h->araw < amax) {
                        double vo = va * exp(-h->sigma);
                        double vs = -h->alpha * va;
                        double A = conic[3 * i], B = conic[3 * i + 1], C = conic[3 * i + 2];
                        double gx = vs * (A * h->dx + B * h->dy);
                        double gy = vs * (B * h->dx + C * h->dy);
#pragma omp atomic
                        o[0] += gx;
#pragma omp atomic
                        o[1] += gy;
#pragma omp atomic
                        o[2] += vs * 0.5 * h->dx * h->dx;
#pragma omp atomic
                        o[3] += vs * h->dx * h->dy;
#pragma omp atomic
                        o[4] += vs * 0.5 * h->dy * h->dy;
#pragma omp atomic
                        o[5] += vo;
                    }
                }
            }
        }
        free(hits);
        free(gate_key);
        free(gate_g);
    }
    free(voff);
    return fail ? -1 : 0;
}

/* ------------------------------------------------------------ projection backward */

int or_project_bwd(int N, int sh_degree, const double* means, const double* log_scales,
                   const double* quats, const double* opacity_logit, const double* sh,
                   int V, const double* viewmat, const double* intr, const int* wh,
                   const double* cfg, const double* v2d,
                   double* v_means, double* v_log_scales, double* v_quats,
                   double* v_opacity_logit, double* v_sh, double* v_twist) {
    if (sh_degree < 0 || sh_degree > 3) return -1;
    int K = (sh_degree + 1) * (sh_degree + 1);
    memset(v_means, 0, sizeof(double) * 3 * N);
    memset(v_log_scales, 0, sizeof(double) * 3 * N);
    memset(v_quats, 0, sizeof(double) * 4 * N);
    memset(v_opacity_logit, 0, sizeof(double) * N);
    memset(v_sh, 0, sizeof(double) * (size_t)K * 3 * N);
    memset(v_twist, 0, sizeof(double) * 6 * V);
    for (int v = 0; v < V; v++) {
        cam_t c;
        load_cam(viewmat, intr, wh, v, &c);
        double tw[6] = {0, 0, 0, 0, 0, 0};
#pragma omp parallel
        {
            double twl[6] = {0, 0, 0, 0, 0, 0};
#pragma omp for schedule(static)
            for (int g = 0; g < N; g++) {
                pair_t P;
                project_pair(N, sh_degree, means, log_scales, quats, opacity_logit, sh, &c, g, cfg, &P);
                if (!P.valid) continue;
                const double* G9 = v2d + 9 * ((size_t)v * N + g);
                double vp[3] = {0, 0, 0};
                double vmu[3] = {0, 0, 0};
                /* opacity */
                double o = P.opacity;
                v_opacity_logit[g] += G9[5] * o * (1 - o);
                /* colour and SH */
                double Y[16], dY[48];
                or_sh_basis(sh_degree, P.dir, Y, dY);
                double vdir[3] = {0, 0, 0};
                for (int ch = 0; ch < 3; ch++) {
                    if (!(P.shsum[ch] + 0.5 > 0)) continue;
                    double vr = G9[6 + ch];
                    for (int k = 0; k < K; k++) {
                        v_sh[((size_t)k * 3 + ch) * N + g] += Y[k] * vr;
                        double co = sh[((size_t)k * 3 + ch) * N + g];
                        for (int e = 0; e < 3; e++) vdir[e] += vr * co * dY[3 * k + e];
                    }
                }
                /* dir = (mu - c)/|mu - c|: tangential projection */
                double dd = P.dir[0] * vdir[0] + P.dir[1] * vdir[1] + P.dir[2] * vdir[2];
                double vmud[3];
                for (int e = 0; e < 3; e++) vmud[e] = (vdir[e] - P.dir[e] * dd) / P.dist;
                for (int e = 0; e < 3; e++) vmu[e] += vmud[e];
                /* camera centre moves by -R^T rho under the left twist */
                double Rvm[3];
                mat3_vec(c.R, vmud, Rvm);
                for (int e = 0; e < 3; e++) twl[e] += Rvm[e];
                /* mean2d */
                double x = P.p[0], y = P.p[1], z = P.p[2];
                double vmx = G9[0], vmy = G9[1];
                vp[0] += c.fx / z * vmx;
                vp[1] += c.fy / z * vmy;
                vp[2] += -(c.fx * x * vmx + c.fy * y * vmy) / (z * z);
                /* conic -> cov2d: G2 = -M Gc M, Gc = [[vA, vB/2],[vB/2, vC]] */
                double A = P.conic[0], B = P.conic[1], C = P.conic[2];
                double gA = G9[2], gB = 0.5 * G9[3], gC = G9[4];
                double M[4] = {A, B, B, C}, Gc[4] = {gA, gB, gB, gC}, T1[4], G2[4];
                for (int i = 0; i < 2; i++)
                    for (int j = 0; j < 2; j++)
                        T1[2 * i + j] = M[2 * i] * Gc[j] + M[2 * i + 1] * Gc[2 + j];
                for (int i = 0; i < 2; i++)
                    for (int j = 0; j < 2; j++)
                        G2[2 * i + j] = -(T1[2 * i] * M[j] + T1[2 * i + 1] * M[2 + j]);
                /* v_J = 2 G2 J Sigc ; v_Sigc = J^T G2 J */
                double JS[6];
                for (int i = 0; i < 2; i++)
                    for (int j = 0; j < 3; j++) {
                        double s = 0;
                        for (int k = 0; k < 3; k++) s += P.J[3 * i + k] * P.Sigc[3 * k + j];
                        JS[3 * i + j] = s;
                    }
                double vJ[6];
                for (int i = 0; i < 2; i++)
                    for (int j = 0; j < 3; j++)
                        vJ[3 * i + j] = 2 * (G2[2 * i] * JS[j] + G2[2 * i + 1] * JS[3 + j]);
                double vSc[9];
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) {
                        double s = 0;
                        for (int a = 0; a < 2; a++)
                            for (int b = 0; b < 2; b++) s += P.J[3 * a + i] * G2[2 * a + b] * P.J[3 * b + j];
                        vSc[3 * i + j] = s;
                    }
                /* J = [[fx/z, 0, -fx tx/z], [0, fy/z, -fy ty/z]], tx = x/z unless clamped */
                vp[2] += -c.fx / (z * z) * vJ[0] - c.fy / (z * z) * vJ[4];
                if (!P.clampx) {
                    vp[0] += -c.fx / (z * z) * vJ[2];
                    vp[2] += 2 * c.fx * x / (z * z * z) * vJ[2];
                } else {
                    vp[2] += c.fx * P.limx / (z * z) * vJ[2];
                }
                if (!P.clampy) {
                    vp[1] += -c.fy / (z * z) * vJ[5];
                    vp[2] += 2 * c.fy * y / (z * z * z) * vJ[5];
                } else {
                    vp[2] += c.fy * P.limy / (z * z) * vJ[5];
                }
                /* p = R mu + t */
                double vmp[3];
                mat3T_vec(c.R, vp, vmp);
                for (int e = 0; e < 3; e++) vmu[e] += vmp[e];
                /* twist: rho gets v_p, phi gets p x v_p + 2 axial(Sigc vSigc) */
                double pxv[3];
                cross3(P.p, vp, pxv);
                double W9[9];
                mat3_mul(P.Sigc, vSc, W9);
                twl[0] += vp[0]; twl[1] += vp[1]; twl[2] += vp[2];
                twl[3] += pxv[0] + 2 * (W9[5] - W9[7]);
                twl[4] += pxv[1] + 2 * (W9[6] - W9[2]);
                twl[5] += pxv[2] + 2 * (W9[1] - W9[3]);
                /* Sigc = R Sig R^T -> vSig = R^T vSc R */
                double Rt[9], T9[9], vS[9];
                mat3_transpose(c.R, Rt);
                mat3_mul(Rt, vSc, T9);
                mat3_mul(T9, c.R, vS);
                /* Sig = Mm Mm^T, Mm = Rq S -> vMm = 2 vS Mm */
                double Mm[9];
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) Mm[3 * i + j] = P.Rq[3 * i + j] * P.s[j];
                double vM[9];
                mat3_mul(vS, Mm, vM);
                for (int k = 0; k < 9; k++) vM[k] *= 2;
                /* scales: vs_j = (Rq^T vM)_jj, then through exp */
                for (int j = 0; j < 3; j++) {
                    double s = 0;
                    for (int i = 0; i < 3; i++) s += P.Rq[3 * i + j] * vM[3 * i + j];
                    v_log_scales[(size_t)j * N + g] += s * P.s[j];
                }
                /* rotation: vRq = vM S, then dRq/dq, then normalisation */
                double vRq[9];
                for (int i = 0; i < 3; i++)
                    for (int j = 0; j < 3; j++) vRq[3 * i + j] = vM[3 * i + j] * P.s[j];
                double dR[4][9];
                quat_to_rot_jac(P.qn, dR);
                double vqn[4];
                for (int a = 0; a < 4; a++) {
                    double s = 0;
                    for (int k = 0; k < 9; k++) s += dR[a][k] * vRq[k];
                    vqn[a] = s;
                }
                double qd = 0;
                for (int a = 0; a < 4; a++) qd += P.qn[a] * vqn[a];
                for (int a = 0; a < 4; a++)
                    v_quats[(size_t)a * N + g] += (vqn[a] - P.qn[a] * qd) / P.qnorm;
                for (int e = 0; e < 3; e++) v_means[(size_t)e * N + g] += vmu[e];
            }
#pragma omp critical
            for (int k = 0; k < 6; k++) tw[k] += twl[k];
        }
        for (int k = 0; k < 6; k++) v_twist[6 * v + k] = tw[k];
    }
    return 0;
}

/* ------------------------------------------------------------ track reprojection */

int or_track(int Pt, const double* X, int ncam, const double* viewmat, const double* intr,
             int M, const int* obs_cam, const int* obs_pt, const double* obs_xy,
             double delta, double lambda, double near_plane,
             double* residual, double* loss, double* v_X, double* v_twist,
             double* J_pose, double* J_X, int* masked) {
    if (v_X) memset(v_X, 0, sizeof(double) * 3 * (size_t)Pt);
    if (v_twist) memset(v_twist, 0, sizeof(double) * 6 * (size_t)ncam);
    double L = 0;
    for (int o = 0; o < M; o++) {
        int ci = obs_cam[o], k = obs_pt[o];
        if (ci < 0 || ci >= ncam || k < 0 || k >= Pt) return -1;
        double R[9], t[3], Xk[3], p[3];
        for (int i = 0; i < 3; i++) {
            for (int j = 0; j < 3; j++) R[3 * i + j] = viewmat[12 * ci + 4 * i + j];
            t[i] = viewmat[12 * ci + 4 * i + 3];
            Xk[i] = X[3 * (size_t)k + i];
        }
        mat3_vec(R, Xk, p);
        for (int i = 0; i < 3; i++) p[i] += t[i];
        double fx = intr[4 * ci], fy = intr[4 * ci + 1], cx = intr[4 * ci + 2], cy = intr[4 * ci + 3];
        int msk = !(p[2] >= near_plane);
        if (masked) masked[o] = msk;
        if (msk) {
            if (residual) { residual[2 * o] = 0; residual[2 * o + 1] = 0; }
            if (J_pose) memset(J_pose + 12 * (size_t)o, 0, sizeof(double) * 12);
            if (J_X) memset(J_X + 6 * (size_t)o, 0, sizeof(double) * 6);
            continue;
        }
        double z = p[2];
        double r[2] = {fx * p[0] / z + cx - obs_xy[2 * o], fy * p[1] / z + cy - obs_xy[2 * o + 1]};
        if (residual) { residual[2 * o] = r[0]; residual[2 * o + 1] = r[1]; }
        double s = r[0] * r[0] + r[1] * r[1];
        double rho, drho;
        if (s <= delta * delta) { rho = s; drho = 1.0; }
        else { rho = 2 * delta * sqrt(s) - delta * delta; drho = delta / sqrt(s); }
        L += lambda * rho;
        /* J_pi (2x3) at p */
        double Jp[6] = {fx / z, 0, -fx * p[0] / (z * z), 0, fy / z, -fy * p[1] / (z * z)};
        double vr[2] = {lambda * 2 * drho * r[0], lambda * 2 * drho * r[1]};
        double vp[3];
        for (int j = 0; j < 3; j++) vp[j] = Jp[j] * vr[0] + Jp[3 + j] * vr[1];
        if (v_X) {
            double vx[3];
            mat3T_vec(R, vp, vx);
            for (int j = 0; j < 3; j++) v_X[3 * (size_t)k + j] += vx[j];
        }
        if (v_twist) {
            double pxv[3];
            cross3(p, vp, pxv);
            for (int j = 0; j < 3; j++) {
                v_twist[6 * ci + j] += vp[j];
                v_twist[6 * ci + 3 + j] += pxv[j];
            }
        }
        if (J_pose) {
            /* d p / d(rho, phi) = [I | -[p]x] */
            double D[18] = {1, 0, 0, 0, p[2], -p[1],
                            0, 1, 0, -p[2], 0, p[0],
                            0, 0, 1, p[1], -p[0], 0};
            for (int a = 0; a < 2; a++)
                for (int b = 0; b < 6; b++) {
                    double v = 0;
                    for (int e = 0; e < 3; e++) v += Jp[3 * a + e] * D[6 * e + b];
                    J_pose[12 * (size_t)o + 6 * a + b] = v;
                }
        }
        if (J_X) {
            for (int a = 0; a < 2; a++)
                for (int b = 0; b < 3; b++) {
                    double v = 0;
                    for (int e = 0; e < 3; e++) v += Jp[3 * a + e] * R[3 * e + b];
                    J_X[6 * (size_t)o + 3 * a + b] = v;
                }
        }
    }
    if (loss) *loss = L;
    return 0;
}

/* ------------------------------------------------------------ SE(3) by power series */

static void mat_mul_n(int n, const double* A, const double* B, double* C) {
    double T[36];
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            double s = 0;
            for (int k = 0; k < n; k++) s += A[n * i + k] * B[n * k + j];
            T[n * i + j] = s;
        }
    memcpy(C, T, sizeof(double) * n * n);
}

void or_se3_exp_compose(int V, const double* xi, const double* base, double* out) {
    for (int v = 0; v < V; v++) {
        const double* x = xi + 6 * v;
        /* twist matrix [[phi]x, rho; 0 0] */
        double A[16] = {0, -x[5], x[4], x[0],
                        x[5], 0, -x[3], x[1],
                        -x[4], x[3], 0, x[2],
                        0, 0, 0, 0};
        double E[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
        double P[16];
        memcpy(P, E, sizeof P);
        for (int n = 1; n < 80; n++) {
            mat_mul_n(4, P, A, P);
            double mx = 0;
            for (int k = 0; k < 16; k++) { P[k] /= n; E[k] += P[k]; if (fabs(P[k]) > mx) mx = fabs(P[k]); }
            if (mx < 1e-300) break;
        }
        double B[16] = {0};
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 4; j++) B[4 * i + j] = base[12 * v + 4 * i + j];
        B[15] = 1;
        double T[16];
        mat_mul_n(4, E, B, T);
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 4; j++) out[12 * v + 4 * i + j] = T[4 * i + j];
    }
}

void or_se3_jl_transpose(int V, const double* xi, const double* g, double* out) {
    for (int v = 0; v < V; v++) {
        const double* x = xi + 6 * v;
        const double *r = x, *f = x + 3;
        /* ad = [[phi]x, [rho]x; 0, [phi]x] */
        double ad[36] = {0};
        double fx[9] = {0, -f[2], f[1], f[2], 0, -f[0], -f[1], f[0], 0};
        double rx[9] = {0, -r[2], r[1], r[2], 0, -r[0], -r[1], r[0], 0};
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) {
                ad[6 * i + j] = fx[3 * i + j];
                ad[6 * i + 3 + j] = rx[3 * i + j];
                ad[6 * (3 + i) + 3 + j] = fx[3 * i + j];
            }
        double J[36] = {0}, P[36] = {0};
        for (int i = 0; i < 6; i++) { J[7 * i] = 1; P[7 * i] = 1; }
        for (int n = 1; n < 80; n++) {
            mat_mul_n(6, P, ad, P);
            double mx = 0;
            for (int k = 0; k < 36; k++) { P[k] /= (n + 1); J[k] += P[k]; if (fabs(P[k]) > mx) mx = fabs(P[k]); }
            if (mx < 1e-300) break;
        }
        for (int j = 0; j < 6; j++) {
            double s = 0;
            for (int i = 0; i < 6; i++) s += J[6 * i + j] * g[6 * v + i];
            out[6 * v + j] = s;
        }
    }
}

/* ------------------------------------------------------------ Adam */

void or_adam(long long n, double* p, const double* g, double* m, double* v,
             double lr, double beta1, double beta2, double eps, int step) {
    double bc1 = 1 - pow(beta1, step), bc2 = 1 - pow(beta2, step);
    for (long long i = 0; i < n; i++) {
        m[i] = beta1 * m[i] + (1 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1 - beta2) * g[i] * g[i];
        double mh = m[i] / bc1, vh = v[i] / bc2;
        p[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------ tile lists */

/* minimum over the rectangle [x0,x1]x[y0,y1] of q(d) = 0.5(A dx^2 + C dy^2) + B dx dy,
   d = point - m.  q is convex, so off-centre the minimum lies on an edge. */
static double edge_min(double A, double B, double C, double fixed, int fixed_is_x,
                       double lo, double hi) {
    /* along an edge one coordinate is fixed (f), the other (u) runs over [lo,hi]:
       q(u) = 0.5 P f^2 + Q f u + 0.5 S u^2 */
    double Pc = fixed_is_x ? A : C, Sc = fixed_is_x ? C : A;
    double u = -B * fixed / Sc;
    if (u < lo) u = lo;
    if (u > hi) u = hi;
    return 0.5 * Pc * fixed * fixed + B * fixed * u + 0.5 * Sc * u * u;
}

static double rect_min(double A, double B, double C, double mx, double my,
                       double x0, double x1, double y0, double y1) {
    if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return 0.0;
    double lx = x0 - mx, hx = x1 - mx, ly = y0 - my, hy = y1 - my;
    double q = edge_min(A, B, C, lx, 1, ly, hy);
    double t = edge_min(A, B, C, hx, 1, ly, hy); if (t < q) q = t;
    t = edge_min(A, B, C, ly, 0, lx, hx); if (t < q) q = t;
    t = edge_min(A, B, C, hy, 0, lx, hx); if (t < q) q = t;
    return q;
}

typedef struct {
    uint32_t dbits;
    int id;
} key_t;

static int key_cmp(const void* pa, const void* pb) {
    const key_t* a = (const key_t*)pa;
    const key_t* b = (const key_t*)pb;
    if (a->dbits != b->dbits) return a->dbits < b->dbits ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

long long or_bin_sort(int V, const int* wh, int tile_w, int tile_h, int N,
                      const int* valid, const float* mean2d, const float* conic,
                      const float* opacity, const float* depth, double alpha_min,
                      double margin, long long cap, long long* ranges, int* ids, int* masks) {
    long long total = 0, tcount = 0;
    key_t* buf = (key_t*)malloc(sizeof(key_t) * (size_t)(N > 0 ? N : 1));
    int* mbuf = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    const int hw = tile_w / 2, hh = tile_h / 2;
    for (int v = 0; v < V; v++) {
        int W = wh[2 * v], H = wh[2 * v + 1];
        int gx = (W + tile_w - 1) / tile_w, gy = (H + tile_h - 1) / tile_h;
        for (int ty = 0; ty < gy; ty++)
            for (int tx = 0; tx < gx; tx++) {
                int n = 0;
                for (int g = 0; g < N; g++) {
                    size_t i = (size_t)v * N + g;
                    if (!valid[i]) continue;
                    double o = opacity[i];
                    if (!(o > alpha_min)) continue;
                    int m = 0;
                    for (int q = 0; q < 4; q++) {
                        int xs = tx * tile_w + (q & 1) * hw, ys = ty * tile_h + (q >> 1) * hh;
                        if (xs >= W || ys >= H) continue;
                        double x0 = xs + 0.5, y0 = ys + 0.5;
                        double x1 = (xs + hw < W ? xs + hw : W) - 0.5;
                        double y1 = (ys + hh < H ? ys + hh : H) - 0.5;
                        double qm = rect_min(conic[3 * i], conic[3 * i + 1], conic[3 * i + 2],
                                             mean2d[2 * i], mean2d[2 * i + 1], x0, x1, y0, y1);
                        if (qm <= log(o / alpha_min) + margin) m |= 1 << q;
                    }
                    if (m) {
                        uint32_t b;
                        memcpy(&b, &depth[i], 4);
                        buf[n].dbits = b;
                        buf[n].id = (int)i;
                        n++;
                    }
                }
                qsort(buf, n, sizeof(key_t), key_cmp);
                if (ranges) { ranges[2 * tcount] = total; ranges[2 * tcount + 1] = total + n; }
                for (int k = 0; k < n; k++) {
                    if (total + k >= cap) continue;
                    if (ids) ids[total + k] = buf[k].id;
                    if (masks) {
                        /* recompute the mask of the sorted entry */
                        size_t i = (size_t)buf[k].id;
                        double o = opacity[i];
                        int m = 0;
                        for (int q = 0; q < 4; q++) {
                            int xs = tx * tile_w + (q & 1) * hw, ys = ty * tile_h + (q >> 1) * hh;
                            if (xs >= W || ys >= H) continue;
                            double x0 = xs + 0.5, y0 = ys + 0.5;
                            double x1 = (xs + hw < W ? xs + hw : W) - 0.5;
                            double y1 = (ys + hh < H ? ys + hh : H) - 0.5;
                            double qm = rect_min(conic[3 * i], conic[3 * i + 1], conic[3 * i + 2],
                                                 mean2d[2 * i], mean2d[2 * i + 1], x0, x1, y0, y1);
                            if (qm <= log(o / alpha_min) + margin) m |= 1 << q;
                        }
                        masks[total + k] = m;
                    }
                }
                total += n;
                tcount++;
            }
    }
    free(buf);
    free(mbuf);
    return total <= cap ? total : -total;
}

/* ------------------------------------------------------------ photometric loss */
/*
 * L_photo = (1 - lambda) L1 + lambda (1 - SSIM), lambda = 0.2 (Sec. 3.3,
 * eq. L_photo; Algorithm 1, photometric loss).  Both terms are means over the
 * pixels and channels of one view, then over the views of the batch (the
 * algorithm's per-view loss read as a mean).
 */

static long long view_offsets(int V, const int* wh, long long* off) {
    off[0] = 0;
    for (int v = 0; v < V; v++) off[v + 1] = off[v] + (long long)wh[2 * v] * wh[2 * v + 1];
    return off[V];
}

int or_l1(int V, const int* wh, const double* rgb, const double* target, double* loss,
          double* v_rgb) {
    if (V <= 0) return -1;
    long long* off = (long long*)malloc(sizeof(long long) * (V + 1));
    view_offsets(V, wh, off);
    double L = 0;
    for (int v = 0; v < V; v++) {
        long long n = off[v + 1] - off[v];
        if (n <= 0) { free(off); return -1; }
        double s = 0, w = 1.0 / (3.0 * (double)n * V);
        for (long long i = 3 * off[v]; i < 3 * off[v + 1]; i++) {
            double d = rgb[i] - target[i];
            s += fabs(d);
            /* |d| has derivative sign(d), taken as 0 at d = 0 */
            if (v_rgb) v_rgb[i] = d > 0 ? w : (d < 0 ? -w : 0.0);
        }
        L += s * w;
    }
    if (loss) *loss = L;
    free(off);
    return 0;
}

/*
 * SSIM (Wang et al. 2004) per channel with a win x win Gaussian window of
 * standard deviation wsig (the outer product of the normalised 1D window),
 * constants c1, c2, and the image extended by zeros beyond its border (the
 * window keeps its weights there):
 *   mu_x = w * x,  s_xx = w * x^2 - mu_x^2,  s_xy = w * (x y) - mu_x mu_y,
 *   S = (2 mu_x mu_y + c1)(2 s_xy + c2) / ((mu_x^2 + mu_y^2 + c1)(s_xx + s_yy + c2)).
 * ssim = mean over views of the mean of S over the view's pixels and channels.
 * ssim_map[P][3] (may be NULL) receives S.  v_rgb[P][3] (may be NULL) receives
 * d ssim / d rgb: S at p depends on x through mu_x(p), E_xx(p) = w * x^2 and
 * E_xy(p) = w * (x y), so
 *   d ssim / d x(q) = sum_p w(p - q) [dS/dmu_x(p) + 2 x(q) dS/dE_xx(p)
 *                                      + y(q) dS/dE_xy(p)] / (3 P_v V).
 */
int or_ssim(int V, const int* wh, const double* rgb, const double* target, int win,
            double wsig, double c1, double c2, double* ssim, double* ssim_map, double* v_rgb) {
    if (V <= 0 || win <= 0 || (win & 1) == 0) return -1;
    const int r = win / 2;
    double* g = (double*)malloc(sizeof(double) * win);
    double gs = 0;
    for (int i = 0; i < win; i++) {
        g[i] = exp(-(double)(i - r) * (i - r) / (2.0 * wsig * wsig));
        gs += g[i];
    }
    for (int i = 0; i < win; i++) g[i] /= gs;
    long long* off = (long long*)malloc(sizeof(long long) * (V + 1));
    long long P = view_offsets(V, wh, off);
    /* per pixel and channel: dS/dmu_x, dS/dE_xx, dS/dE_xy */
    double* dS = v_rgb ? (double*)malloc(sizeof(double) * 9 * (size_t)(P > 0 ? P : 1)) : NULL;
    double total = 0;
    for (int v = 0; v < V; v++) {
        const int W = wh[2 * v], H = wh[2 * v + 1];
        const long long base = off[v];
        double vsum = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : vsum)
        for (int py = 0; py < H; py++)
            for (int px = 0; px < W; px++) {
                const long long p = base + (long long)py * W + px;
                for (int ch = 0; ch < 3; ch++) {
                    double mx = 0, my = 0, exx = 0, eyy = 0, exy = 0;
                    for (int j = -r; j <= r; j++) {
                        const int qy = py + j;
                        if (qy < 0 || qy >= H) continue;
                        for (int i = -r; i <= r; i++) {
                            const int qx = px + i;
                            if (qx < 0 || qx >= W) continue;
                            const double w = g[j + r] * g[i + r];
                            const long long q = base + (long long)qy * W + qx;
                            const double x = rgb[3 * q + ch], y = target[3 * q + ch];
                            mx += w * x;
                            my += w * y;
                            exx += w * x * x;
                            eyy += w * y * y;
                            exy += w * x * y;
                        }
                    }
                    const double sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
                    const double A1 = 2 * mx * my + c1, A2 = 2 * sxy + c2;
                    const double B1 = mx * mx + my * my + c1, B2 = sxx + syy + c2;
                    const double S = A1 * A2 / (B1 * B2);
                    vsum += S;
                    if (ssim_map) ssim_map[3 * p + ch] = S;
                    if (dS) {
                        /* S = A1 A2 / (B1 B2) with s_xx = E_xx - mu_x^2 and
                           s_xy = E_xy - mu_x mu_y */
                        const double D = B1 * B2;
                        const double dN = 2 * my * A2 + A1 * (-2 * my);
                        const double dD = 2 * mx * B2 + B1 * (-2 * mx);
                        dS[9 * p + 3 * ch + 0] = (dN * D - A1 * A2 * dD) / (D * D);
                        dS[9 * p + 3 * ch + 1] = -S / B2;
                        dS[9 * p + 3 * ch + 2] = 2 * A1 / D;
                    }
                }
            }
        total += vsum / (3.0 * (double)(off[v + 1] - off[v]));
        if (v_rgb) {
            const double sc = 1.0 / (3.0 * (double)(off[v + 1] - off[v]) * V);
#pragma omp parallel for schedule(dynamic, 4)
            for (int qy = 0; qy < H; qy++)
                for (int qx = 0; qx < W; qx++) {
                    const long long q = base + (long long)qy * W + qx;
                    for (int ch = 0; ch < 3; ch++) {
                        const double x = rgb[3 * q + ch], y = target[3 * q + ch];
                        double s = 0;
                        for (int j = -r; j <= r; j++) {
                            const int py = qy + j;
                            if (py < 0 || py >= H) continue;
                            for (int i = -r; i <= r; i++) {
                                const int px = qx + i;
                                if (px < 0 || px >= W) continue;
                                const double w = g[j + r] * g[i + r];
                                const long long p = base + (long long)py * W + px;
                                const double* d = dS + 9 * p + 3 * ch;
                                s += w * (d[0] + 2 * x * d[1] + y * d[2]);
                            }
                        }
                        v_rgb[3 * q + ch] = s * sc;
                    }
                }
        }
    }
    if (ssim) *ssim = total / V;
    free(dS);
    free(off);
    free(g);
    return 0;
}

/* ------------------------------------------------------------ Gaussian initialisation */
/*
 * Each SfM point starts one Gaussian (Sec. 3.3, first paragraph; Algorithm 1,
 * initialisation): mean = the point, an isotropic scale equal to the mean
 * Euclidean distance to its k = 4 nearest other points (found here by brute
 * force over all points), opacity 0.1, and spherical harmonics holding the
 * point's colour in the degree-0 band (rgb = 0.5 + C0 sh_0, C0 = 1/(2 sqrt(pi)),
 * the colour rule of the renderer), higher bands zero, identity rotation.
 * With fewer than k other points all of them are used; a scale below s_min
 * (coincident points) is raised to s_min.
 */
int or_knn_mean_dist(long long n, const double* pts, int k, long long nq, const long long* q_idx,
                     double* out) {
    if (n < 0 || k <= 0 || k > 64) return -1;
    if (!q_idx) nq = n;
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (long long qi = 0; qi < nq; qi++) {
        const long long i = q_idx ? q_idx[qi] : qi;
        if (i < 0 || i >= n) { fail = 1; continue; }
        double best[64];
        int nb = 0;
        for (long long j = 0; j < n; j++) {
            if (j == i) continue;
            double dx = pts[3 * j] - pts[3 * i], dy = pts[3 * j + 1] - pts[3 * i + 1],
                   dz = pts[3 * j + 2] - pts[3 * i + 2];
            double d = sqrt(dx * dx + dy * dy + dz * dz);
            /* keep the k smallest distances, ascending */
            if (nb < k) {
                int p = nb++;
                while (p > 0 && best[p - 1] > d) { best[p] = best[p - 1]; p--; }
                best[p] = d;
            } else if (d < best[k - 1]) {
                int p = k - 1;
                while (p > 0 && best[p - 1] > d) { best[p] = best[p - 1]; p--; }
                best[p] = d;
            }
        }
        double s = 0;
        for (int q = 0; q < nb; q++) s += best[q];
        out[qi] = nb > 0 ? s / nb : 0.0;
    }
    return fail ? -1 : 0;
}

int or_init_gaussians(long long n, const double* pts, const double* rgb, int k, double opacity,
                      double s_min, int sh_degree, double* means, double* log_scales,
                      double* quats, double* opacity_logit, double* sh) {
    if (sh_degree < 0 || sh_degree > 3 || !(opacity > 0 && opacity < 1)) return -1;
    double* d = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (or_knn_mean_dist(n, pts, k, n, NULL, d) != 0) { free(d); return -1; }
    const int K = (sh_degree + 1) * (sh_degree + 1);
    const double C0 = 1.0 / (2.0 * sqrt(PI));
    for (long long i = 0; i < n; i++) {
        double s = d[i] > s_min ? d[i] : s_min;
        for (int a = 0; a < 3; a++) {
            means[(size_t)a * n + i] = pts[3 * i + a];
            log_scales[(size_t)a * n + i] = log(s);
        }
        quats[i] = 1.0;
        quats[(size_t)n + i] = quats[2 * (size_t)n + i] = quats[3 * (size_t)n + i] = 0.0;
        opacity_logit[i] = log(opacity / (1.0 - opacity));
        for (int c = 0; c < K; c++)
            for (int ch = 0; ch < 3; ch++)
                sh[((size_t)c * 3 + ch) * n + i] = c == 0 ? (rgb[3 * i + ch] - 0.5) / C0 : 0.0;
    }
    free(d);
    return 0;
}

/* ------------------------------------------------------------ one LM step of bundle adjustment */
/*
 * Bundle adjustment minimises sum_obs rho_Huber(|pi_i(X_k) - x|^2) over the
 * poses (SE(3), here left twists xi_i at the current pose) and the points X_k
 * (Sec. 3.2 "Bundle Adjustment", eq. L_BA^SfM), by Levenberg-Marquardt.  One
 * step, iteratively reweighted: with r the residual, s = |r|^2 and the weight
 * w = rho'(s) (1 for an inlier s <= delta^2, delta / sqrt(s) otherwise), the
 * Gauss-Newton normal equations of the robust cost are
 *   H = sum_obs w J^T J,   g = sum_obs w J^T r,   J = dr/d(xi, X),
 * and the step solves (H + lambda diag(H)) d = -g.  Masked observations
 * (p_z < near) are left out.  Unknowns whose diagonal is zero (a camera or a
 * point with no observation) are held fixed (d = 0).
 * Unknowns are ordered cameras first (6 each: rho, phi), then points (3).
 */
typedef struct {
    int ok;
    double r[2], w, Jp[12], Jx[6], rho;
} obs_lin_t;

static void ba_linearise(const double* X, const double* viewmat, const double* intr, int ci, int k,
                         const double* xy, double delta, double near_plane, obs_lin_t* L) {
    double R[9], t[3], p[3];
    for (int a = 0; a < 3; a++) {
        for (int b = 0; b < 3; b++) R[3 * a + b] = viewmat[12 * ci + 4 * a + b];
        t[a] = viewmat[12 * ci + 4 * a + 3];
    }
    mat3_vec(R, X + 3 * (size_t)k, p);
    for (int a = 0; a < 3; a++) p[a] += t[a];
    L->ok = p[2] >= near_plane;
    if (!L->ok) return;
    double fx = intr[4 * ci], fy = intr[4 * ci + 1], cx = intr[4 * ci + 2], cy = intr[4 * ci + 3];
    double z = p[2];
    L->r[0] = fx * p[0] / z + cx - xy[0];
    L->r[1] = fy * p[1] / z + cy - xy[1];
    double s = L->r[0] * L->r[0] + L->r[1] * L->r[1];
    L->w = s <= delta * delta ? 1.0 : delta / sqrt(s);
    L->rho = s <= delta * delta ? s : 2 * delta * sqrt(s) - delta * delta;
    double Jpi[6] = {fx / z, 0, -fx * p[0] / (z * z), 0, fy / z, -fy * p[1] / (z * z)};
    double D[18] = {1, 0, 0, 0, p[2], -p[1],
                    0, 1, 0, -p[2], 0, p[0],
                    0, 0, 1, p[1], -p[0], 0};
    for (int a = 0; a < 2; a++) {
        for (int b = 0; b < 6; b++) {
            double v = 0;
            for (int e = 0; e < 3; e++) v += Jpi[3 * a + e] * D[6 * e + b];
            L->Jp[6 * a + b] = v;
        }
        for (int b = 0; b < 3; b++) {
            double v = 0;
            for (int e = 0; e < 3; e++) v += Jpi[3 * a + e] * R[3 * e + b];
            L->Jx[3 * a + b] = v;
        }
    }
}

/* Dense undamped H [n][n] and g [n] (n = 6 ncam + 3 Pt) and the robust cost
 * sum rho; returns the number of masked observations, -1 on a bad index. */
int or_ba_normal(int Pt, const double* X, int ncam, const double* viewmat, const double* intr,
                 int M, const int* obs_cam, const int* obs_pt, const double* obs_xy, double delta,
                 double near_plane, double* H, double* g, double* cost) {
    const long long n = 6LL * ncam + 3LL * Pt;
    memset(H, 0, sizeof(double) * (size_t)(n * n));
    memset(g, 0, sizeof(double) * (size_t)n);
    double C = 0;
    int masked = 0;
    for (int o = 0; o < M; o++) {
        int ci = obs_cam[o], k = obs_pt[o];
        if (ci < 0 || ci >= ncam || k < 0 || k >= Pt) return -1;
        obs_lin_t L;
        ba_linearise(X, viewmat, intr, ci, k, obs_xy + 2 * (size_t)o, delta, near_plane, &L);
        if (!L.ok) { masked++; continue; }
        C += L.rho;
        /* this observation's row block J = [.. Jp at camera ci .. Jx at point k ..] */
        long long idx[9];
        double J[2][9];
        for (int b = 0; b < 6; b++) idx[b] = 6LL * ci + b;
        for (int b = 0; b < 3; b++) idx[6 + b] = 6LL * ncam + 3LL * k + b;
        for (int a = 0; a < 2; a++) {
            for (int b = 0; b < 6; b++) J[a][b] = L.Jp[6 * a + b];
            for (int b = 0; b < 3; b++) J[a][6 + b] = L.Jx[3 * a + b];
        }
        for (int u = 0; u < 9; u++) {
            g[idx[u]] += L.w * (J[0][u] * L.r[0] + J[1][u] * L.r[1]);
            for (int v = 0; v < 9; v++)
                H[idx[u] * n + idx[v]] += L.w * (J[0][u] * J[0][v] + J[1][u] * J[1][v]);
        }
    }
    if (cost) *cost = C;
    return masked;
}

/* out = (H + lambda diag(H)) d + g, accumulated observation by observation
 * (no dense matrix: any size).  Fixed unknowns (zero diagonal) contribute
 * nothing because their columns are zero. */
int or_ba_normal_residual(int Pt, const double* X, int ncam, const double* viewmat,
                          const double* intr, int M, const int* obs_cam, const int* obs_pt,
                          const double* obs_xy, double delta, double near_plane, double lambda,
                          const double* d, double* out) {
    const long long n = 6LL * ncam + 3LL * Pt;
    double* diag = (double*)calloc((size_t)n, sizeof(double));
    memset(out, 0, sizeof(double) * (size_t)n);
    for (int o = 0; o < M; o++) {
        int ci = obs_cam[o], k = obs_pt[o];
        if (ci < 0 || ci >= ncam || k < 0 || k >= Pt) { free(diag); return -1; }
        obs_lin_t L;
        ba_linearise(X, viewmat, intr, ci, k, obs_xy + 2 * (size_t)o, delta, near_plane, &L);
        if (!L.ok) continue;
        long long idx[9];
        double J[2][9];
        for (int b = 0; b < 6; b++) idx[b] = 6LL * ci + b;
        for (int b = 0; b < 3; b++) idx[6 + b] = 6LL * ncam + 3LL * k + b;
        for (int a = 0; a < 2; a++) {
            for (int b = 0; b < 6; b++) J[a][b] = L.Jp[6 * a + b];
            for (int b = 0; b < 3; b++) J[a][6 + b] = L.Jx[3 * a + b];
        }
        /* J d for this observation */
        double Jd[2] = {0, 0};
        for (int u = 0; u < 9; u++) {
            Jd[0] += J[0][u] * d[idx[u]];
            Jd[1] += J[1][u] * d[idx[u]];
        }
        for (int u = 0; u < 9; u++) {
            out[idx[u]] += L.w * (J[0][u] * (Jd[0] + L.r[0]) + J[1][u] * (Jd[1] + L.r[1]));
            diag[idx[u]] += L.w * (J[0][u] * J[0][u] + J[1][u] * J[1][u]);
        }
    }
    for (long long i = 0; i < n; i++) out[i] += lambda * diag[i] * d[i];
    free(diag);
    return 0;
}

/* ------------------------------------------------------------ MCMC densification */
/*
 * The stochastic density control the paper adopts (Sec. 3.3, first paragraph;
 * Algorithm 1, MCMC densification): Gaussians whose opacity is at most
 * t_dead are "dead" and are moved onto live ones, each dead Gaussian taking a
 * source drawn from the live ones with probability proportional to opacity;
 * a source chosen by c dead Gaussians ends as n = c + 1 identical copies
 * whose opacity o' = 1 - (1 - o)^(1/n) keeps the combined opacity at the
 * centre, and whose scale is multiplied by o / sum_{i=1..n} sum_{k=0..i-1}
 * C(i-1, k) (-1)^k o'^(k+1) / sqrt(k+1), which keeps the integral of the
 * combined opacity along an axis.  Copies take the source's mean, rotation and
 * colour; the Adam moments of sources and copies restart at zero.  As in the
 * adopted method, n is capped at 51 in these two rules (a source drawn more
 * often still gives every draw a copy).
 *
 * Sampling is exact in integers: the weight of a live Gaussian is
 * floor(o 2^24) with o = sigmoid(logit) in double, the draw for dead Gaussian
 * j is the first live index whose inclusive weight prefix exceeds
 * floor(u_j W) (u_j in [0, 1) given, W the total weight, the product taken in
 * double).
 */
static double mcmc_scale_factor(double o, double op, int n) {
    double denom = 0;
    for (int i = 1; i <= n; i++) {
        double binom_c = 1;  /* C(i-1, k), built up in k */
        for (int k = 0; k <= i - 1; k++) {
            denom += binom_c * ((k & 1) ? -1.0 : 1.0) * pow(op, k + 1) / sqrt((double)(k + 1));
            binom_c = binom_c * (i - 1 - k) / (k + 1);
        }
    }
    return o / denom;
}

int or_mcmc_relocate(long long N, int sh_degree, double* means, double* log_scales, double* quats,
                     double* opacity_logit, double* sh, double* const* exp_avg,
                     double* const* exp_avg_sq, const double* u, double t_dead, long long* src,
                     long long* n_relocated) {
    if (N < 0 || sh_degree < 0 || sh_degree > 3) return -1;
    const int K = (sh_degree + 1) * (sh_degree + 1);
    const long long rows[5] = {3, 3, 4, 1, 3LL * K};
    double* P[5] = {means, log_scales, quats, opacity_logit, sh};
    unsigned long long* cdf = (unsigned long long*)malloc(sizeof(unsigned long long) * (size_t)(N > 0 ? N : 1));
    long long* count = (long long*)calloc((size_t)(N > 0 ? N : 1), sizeof(long long));
    double* o = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    unsigned long long W = 0;
    for (long long i = 0; i < N; i++) {
        o[i] = 1.0 / (1.0 + exp(-opacity_logit[i]));
        if (o[i] > t_dead) W += (unsigned long long)floor(o[i] * 16777216.0);
        cdf[i] = W;
    }
    long long moved = 0;
    for (long long j = 0; j < N; j++) {
        src[j] = -1;
        if (o[j] > t_dead || W == 0) continue;
        unsigned long long tv = (unsigned long long)floor(u[j] * (double)W);
        /* first index with cdf > tv */
        long long lo = 0, hi = N;
        while (lo < hi) {
            long long mid = (lo + hi) / 2;
            if (cdf[mid] > tv) hi = mid; else lo = mid + 1;
        }
        src[j] = lo;
        count[lo]++;
        moved++;
    }
    /* sources: opacity and scale of their n copies */
    for (long long s = 0; s < N; s++) {
        if (count[s] == 0) continue;
        int n = count[s] + 1 < 51 ? (int)count[s] + 1 : 51;
        double op = 1.0 - pow(1.0 - o[s], 1.0 / n);
        double f = mcmc_scale_factor(o[s], op, n);
        opacity_logit[s] = log(op / (1.0 - op));
        for (int a = 0; a < 3; a++) log_scales[(size_t)a * N + s] += log(f);
        for (int q = 0; q < 5; q++)
            for (long long r = 0; r < rows[q]; r++) {
                exp_avg[q][(size_t)r * N + s] = 0;
                exp_avg_sq[q][(size_t)r * N + s] = 0;
            }
    }
    /* targets: copies of their (updated) source */
    for (long long j = 0; j < N; j++) {
        long long s = src[j];
        if (s < 0) continue;
        for (int q = 0; q < 5; q++)
            for (long long r = 0; r < rows[q]; r++) {
                P[q][(size_t)r * N + j] = P[q][(size_t)r * N + s];
                exp_avg[q][(size_t)r * N + j] = 0;
                exp_avg_sq[q][(size_t)r * N + j] = 0;
            }
    }
    if (n_relocated) *n_relocated = moved;
    free(cdf);
    free(count);
    free(o);
    return 0;
}

/* Noise on the means after an update (the same adopted method): mu += scale *
 * sigmoid(-k (o - t)) * Sigma eta, Sigma = Rq diag(exp(2 s)) Rq^T the
 * Gaussian's covariance (normalised quaternion), eta [3][N] given normal
 * draws, scale = the noise weight times the position learning rate. */
void or_mcmc_noise(long long N, double* means, const double* log_scales, const double* quats,
                   const double* opacity_logit, const double* eta, double scale, double k, double t) {
    for (long long i = 0; i < N; i++) {
        double q[4], qn = 0;
        for (int a = 0; a < 4; a++) { q[a] = quats[(size_t)a * N + i]; qn += q[a] * q[a]; }
        qn = sqrt(qn);
        for (int a = 0; a < 4; a++) q[a] /= qn;
        double R[9];
        quat_to_rot(q, R);
        double s2[3];
        for (int a = 0; a < 3; a++) s2[a] = exp(2 * log_scales[(size_t)a * N + i]);
        double o = 1.0 / (1.0 + exp(-opacity_logit[i]));
        double gate = 1.0 / (1.0 + exp(k * (o - t)));
        double e[3] = {eta[i], eta[(size_t)N + i], eta[2 * (size_t)N + i]};
        for (int a = 0; a < 3; a++) {
            double v = 0;
            for (int b = 0; b < 3; b++) {
                double S = 0;
                for (int c = 0; c < 3; c++) S += R[3 * a + c] * s2[c] * R[3 * b + c];
                v += S * e[b];
            }
            means[(size_t)a * N + i] += scale * gate * v;
        }
    }
}
