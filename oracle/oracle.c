/*
 * oracle.c -- plain, slow FP64 reference for point-based ray tracing of 3D
 * Gaussians. TEST INFRASTRUCTURE ONLY: nothing in the product path may link,
 * load or call this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do. It shares no code, header or constant table with the
 * HIP library.
 *
 * What it computes (all FP64, brute force over every Gaussian, no BVH, no
 * early exit):
 *
 *  - Gaussian density, Eq. (1): G(x) = exp(-1/2 (x-mu)^T Sigma^-1 (x-mu)),
 *    Sigma = R(q) S S^T R(q)^T with S = diag(exp(log_scale)), q a unit
 *    quaternion (w,x,y,z) (Sec. 3.1).
 *  - The equivalent intersection point of a ray with a Gaussian, Eq. (13), at
 *    the parameter t_j where the Gaussian's response along the ray peaks,
 *    Eq. (14). Eq. (14) as printed uses Sigma; the peak of Eq. (1) along the
 *    ray needs Sigma^-1, which is what is used here (reading of a misprint).
 *  - alpha_j = o_j * G_j(r_x) (Sec. 4.1 takes the Gaussian's contribution at
 *    the equivalent intersection point), cut to the 3-sigma support (q <= 9),
 *    kept only if alpha >= 1/255, clamped to 0.99.
 *  - Transmittance T = prod_j (1 - alpha_j) over every Gaussian the ray crosses
 *    (Sec. 4.1: all-hit, order independent; the recurrence is Eq. (15)).
 *  - Rays start at each Gaussian mean, skip the source Gaussian, and count a
 *    Gaussian only if its peak lies at t >= t_min = 3 * max scale of the source.
 *  - Directions: a table of unit vectors, used in world frame (sphere mode) or
 *    rotated into the frame of the source normal (hemisphere mode, Sec. 4.2,
 *    hemisphere about n) with the orthonormal basis of Duff et al., "Building
 *    an Orthonormal Basis, Revisited" (JCGT 2017).
 *  - The LBVH reference (Sec. 4.1 builds a binary radix tree after Karras
 *    2012): FP32 Morton codes, and a TOP-DOWN radix-tree construction that is
 *    independent of the bottom-up per-node construction it is compared with.
 *  - The analytic gradient of sum_r w_r T_r with respect to opacity, mean and
 *    log-scale.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no -ffast-math).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define U32 (5.9604644775390625e-08) /* 2^-24: unit roundoff of binary32 */

/* ------------------------------------------------------------------------ */
/* Gaussian geometry                                                        */
/* ------------------------------------------------------------------------ */

/* Rotation matrix of the normalised quaternion q = (w, x, y, z). */
static void quat_to_rot(const double q_in[4], double R[9])
{
    double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] + q_in[3] * q_in[3]);
    double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Whitening matrix W = S^-1 R^T, so that (x-mu)^T Sigma^-1 (x-mu) = |W (x-mu)|^2. */
static void whitening(const double *quat, const double *log_scale, double W[9])
{
    double R[9];
    quat_to_rot(quat, R);
    for (int a = 0; a < 3; ++a) {
        double inv_s = exp(-log_scale[a]);
        for (int c = 0; c < 3; ++c)
            W[a * 3 + c] = inv_s * R[c * 3 + a]; /* row a = column a of R, scaled */
    }
}

/* Exposed for the tests: W for one Gaussian. */
void or_whitening(const double *quat, const double *log_scale, double *W) { whitening(quat, log_scale, W); }

/* Duff et al. 2017 orthonormal basis (b1, b2) completing the unit vector n. */
static void onb_duff(const double n[3], double b1[3], double b2[3])
{
    double sign = copysign(1.0, n[2]);
    double a = -1.0 / (sign + n[2]);
    double b = n[0] * n[1] * a;
    b1[0] = 1.0 + sign * n[0] * n[0] * a;
    b1[1] = sign * b;
    b1[2] = -sign * n[0];
    b2[0] = b;
    b2[1] = sign + n[1] * n[1] * a;
    b2[2] = -n[1];
}

void or_onb(const double *n, double *b1, double *b2) { onb_duff(n, b1, b2); }

/* Ray r = i*K + k: origin mu_i, unit direction, and t_min of the source. */
static void make_ray(const double *mean, const double *normal, const double *log_scale, int32_t K,
                     const double *dirs, int32_t dir_mode, double tmin_scale, int64_t r,
                     double o[3], double d[3], double *tmin, int64_t *src)
{
    int64_t i = r / K, k = r % K;
    const double *dk = dirs + 3 * k;
    for (int a = 0; a < 3; ++a) o[a] = mean[3 * i + a];
    if (dir_mode == 0) {
        for (int a = 0; a < 3; ++a) d[a] = dk[a];
    } else {
        double n[3], b1[3], b2[3];
        double nl = sqrt(normal[3 * i] * normal[3 * i] + normal[3 * i + 1] * normal[3 * i + 1] +
                         normal[3 * i + 2] * normal[3 * i + 2]);
        for (int a = 0; a < 3; ++a) n[a] = normal[3 * i + a] / nl;
        onb_duff(n, b1, b2);
        for (int a = 0; a < 3; ++a) d[a] = dk[0] * b1[a] + dk[1] * b2[a] + dk[2] * n[a];
    }
    double dl = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int a = 0; a < 3; ++a) d[a] /= dl;
    double ms = log_scale[3 * i];
    if (log_scale[3 * i + 1] > ms) ms = log_scale[3 * i + 1];
    if (log_scale[3 * i + 2] > ms) ms = log_scale[3 * i + 2];
    *tmin = tmin_scale * exp(ms);
    *src = i;
}

void or_make_ray(const double *mean, const double *normal, const double *log_scale, int32_t K,
                 const double *dirs, int32_t dir_mode, double tmin_scale, int64_t r,
                 double *o, double *d, double *tmin)
{
    int64_t src;
    make_ray(mean, normal, log_scale, K, dirs, dir_mode, tmin_scale, r, o, d, tmin, &src);
}

/*
 * Peak of one Gaussian along one ray (Eq. (13)-(14), Sigma^-1 reading).
 * With p = W (o - mu) and v = W d the exponent of Eq. (1) along the ray is
 * |p + t v|^2, minimised at t* = -(p.v)/(v.v); its minimum value is
 * q = |p x v|^2 / (v.v) (Lagrange's identity). Also returns e = p + t* v.
 */
static void peak(const double W[9], const double *mu, const double o[3], const double d[3],
                 double *t_out, double *q_out, double e[3], double *pn, double *vn)
{
    double x[3] = {o[0] - mu[0], o[1] - mu[1], o[2] - mu[2]};
    double p[3], v[3];
    for (int a = 0; a < 3; ++a) {
        p[a] = W[a * 3] * x[0] + W[a * 3 + 1] * x[1] + W[a * 3 + 2] * x[2];
        v[a] = W[a * 3] * d[0] + W[a * 3 + 1] * d[1] + W[a * 3 + 2] * d[2];
    }
    double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double pv = p[0] * v[0] + p[1] * v[1] + p[2] * v[2];
    double t = -pv / vv;
    double c0 = p[1] * v[2] - p[2] * v[1];
    double c1 = p[2] * v[0] - p[0] * v[2];
    double c2 = p[0] * v[1] - p[1] * v[0];
    *t_out = t;
    *q_out = (c0 * c0 + c1 * c1 + c2 * c2) / vv;
    for (int a = 0; a < 3; ++a) e[a] = p[a] + t * v[a];
    *pn = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    *vn = sqrt(vv);
}

void or_peak(const double *quat, const double *log_scale, const double *mu, const double *o,
             const double *d, double *t_out, double *q_out)
{
    double W[9], e[3], pn, vn;
    whitening(quat, log_scale, W);
    peak(W, mu, o, d, t_out, q_out, e, &pn, &vn);
}

/* Per-Gaussian tables: W (9 per Gaussian) and the Frobenius norm of W. */
static void tables(int64_t n, const double *quat, const double *log_scale, double *W, double *Wn)
{
    for (int64_t j = 0; j < n; ++j) {
        whitening(quat + 4 * j, log_scale + 3 * j, W + 9 * j);
        double s = 0.0;
        for (int a = 0; a < 9; ++a) s += W[9 * j + a] * W[9 * j + a];
        Wn[j] = sqrt(s);
    }
}

/* ------------------------------------------------------------------------ */
/* Forward: brute-force transmittance with ambiguity bounds                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    double alpha_min, alpha_max, sigma_cut, tmin_scale, kappa;
} or_params;

/*
 * For each requested ray: P = prod over included Gaussians of (1 - alpha), the
 * plain definition. A Gaussian whose inclusion could flip under binary32
 * evaluation of the same cuts (its t*, q or alpha lies within an error bound
 * of a cut, the bound being kappa * 2^-24 times the magnitudes that enter the
 * computation) is "ambiguous": V_lo multiplies in every possibly included
 * Gaussian, V_hi only the surely included ones. Unambiguous rays have
 * V_lo = P = V_hi.
 */
void or_trace_rays(int64_t n, const double *mean, const double *quat, const double *log_scale,
                   const double *opacity, const double *normal, int32_t K, const double *dirs,
                   int32_t dir_mode, const or_params *prm, int64_t n_rays, const int64_t *rays,
                   double *P, double *V_lo, double *V_hi, int32_t *n_incl, int32_t *n_amb, int32_t *n_clamp,
                   int32_t *n_near_clamp)
{
    double *W = (double *)malloc(sizeof(double) * 9 * (n > 0 ? n : 1));
    double *Wn = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    tables(n, quat, log_scale, W, Wn);
    const double qcut = prm->sigma_cut * prm->sigma_cut;
    const double ln_amin = log(prm->alpha_min);
    const double c = prm->kappa * U32;

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < n_rays; ++s) {
        double o[3], d[3], tmin;
        int64_t src;
        make_ray(mean, normal, log_scale, K, dirs, dir_mode, prm->tmin_scale, rays[s], o, d, &tmin, &src);
        double prod = 1.0, lo = 1.0, hi = 1.0;
        int32_t cnt = 0, amb = 0, ncl = 0, nnc = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == src) continue;
            double t, q, e[3], pn, vn;
            peak(W + 9 * j, mean + 3 * j, o, d, &t, &q, e, &pn, &vn);
            const double *mu = mean + 3 * j;
            double dist = sqrt((o[0] - mu[0]) * (o[0] - mu[0]) + (o[1] - mu[1]) * (o[1] - mu[1]) +
                               (o[2] - mu[2]) * (o[2] - mu[2]));
            double Pabs = Wn[j] * dist + pn, Vabs = Wn[j];
            double err_q = 2.0 * sqrt(q) * c * (Pabs + fabs(t) * Vabs) + c * (q + 1.0);
            double err_t = c * (Pabs / vn + pn * Vabs / (vn * vn) + 2.0 * fabs(t) * Vabs / vn + tmin + fabs(t));
            /* far outside every band: excluded and not ambiguous */
            if (t < tmin - err_t || q > qcut + err_q) continue;
            double alpha = opacity[j] * exp(-0.5 * q);
            double lna = log(opacity[j]) - 0.5 * q;
            double err_a = 0.5 * err_q + c * (2.0 + 0.5 * q + fabs(log(opacity[j])));
            int inc = (t >= tmin) && (q <= qcut) && (alpha >= prm->alpha_min);
            int maybe = (t >= tmin - err_t) && (q <= qcut + err_q) && (lna >= ln_amin - err_a);
            int sure = (t >= tmin + err_t) && (q <= qcut - err_q) && (lna >= ln_amin + err_a);
            double ac = alpha < prm->alpha_max ? alpha : prm->alpha_max;
            if (inc) {
                prod *= 1.0 - ac;
                ++cnt;
                ncl += alpha >= prm->alpha_max;
                /* T is continuous at the clamp but its derivative is not */
                nnc += fabs(lna - log(prm->alpha_max)) <= err_a;
            }
            if (maybe) lo *= 1.0 - ac;
            if (sure) hi *= 1.0 - ac;
            if (maybe && !sure) ++amb;
        }
        P[s] = prod;
        if (V_lo) V_lo[s] = lo;
        if (V_hi) V_hi[s] = hi;
        if (n_incl) n_incl[s] = cnt;
        if (n_amb) n_amb[s] = amb;
        if (n_clamp) n_clamp[s] = ncl;
        if (n_near_clamp) n_near_clamp[s] = nnc;
    }
    free(W);
    free(Wn);
}

/*
 * Analytic gradient of F = sum_s w_s P_s (P_s as in or_trace_rays, no early
 * exit) with respect to opacity, mean and log-scale, ACCUMULATED into the
 * output arrays. For an included Gaussian j with unclamped alpha:
 *   dP/dalpha_j = -P / (1 - alpha_j)
 *   dalpha/do_j = alpha / o_j
 *   dalpha/dmu_j = alpha W^T e           (e = p + t* v; envelope theorem)
 *   dalpha/dls_{j,a} = alpha e_a^2
 *   dalpha/d(origin) = -alpha W^T e      (the origin is the source mean)
 * A clamped alpha (0.99) has zero derivative. The cuts are not differentiated.
 * With absolute == 1 the magnitudes |term| are accumulated instead; with
 * absolute == 2, each term's first-order sensitivity to binary32 rounding of
 * the ray and of W (the scale of a binary32 evaluation's deviation).
 */
void or_grad_rays(int64_t n, const double *mean, const double *quat, const double *log_scale,
                  const double *opacity, const double *normal, int32_t K, const double *dirs,
                  int32_t dir_mode, const or_params *prm, int64_t n_rays, const int64_t *rays,
                  const double *w, double *g_opacity, double *g_mean, double *g_log_scale, int32_t absolute)
{
    double *W = (double *)malloc(sizeof(double) * 9 * (n > 0 ? n : 1));
    double *Wn = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    tables(n, quat, log_scale, W, Wn);
    const double qcut = prm->sigma_cut * prm->sigma_cut;
    /* serial over rays: accumulation order fixed, no races */
    int64_t *hit = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    double *hit_alpha = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *hit_e = (double *)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    double *hit_t = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    double *hit_q = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int64_t s = 0; s < n_rays; ++s) {
        double o[3], d[3], tmin;
        int64_t src;
        make_ray(mean, normal, log_scale, K, dirs, dir_mode, prm->tmin_scale, rays[s], o, d, &tmin, &src);
        double prod = 1.0;
        int64_t nh = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == src) continue;
            double t, q, e[3], pn, vn;
            peak(W + 9 * j, mean + 3 * j, o, d, &t, &q, e, &pn, &vn);
            if (!(t >= tmin) || !(q <= qcut)) continue;
            double alpha = opacity[j] * exp(-0.5 * q);
            if (!(alpha >= prm->alpha_min)) continue;
            double ac = alpha < prm->alpha_max ? alpha : prm->alpha_max;
            prod *= 1.0 - ac;
            hit[nh] = (alpha < prm->alpha_max) ? j : -1 - j;
            hit_alpha[nh] = alpha;
            hit_e[3 * nh] = e[0];
            hit_e[3 * nh + 1] = e[1];
            hit_e[3 * nh + 2] = e[2];
            hit_t[nh] = t;
            hit_q[nh] = q;
            ++nh;
        }
        for (int64_t h = 0; h < nh; ++h) {
            if (hit[h] < 0) continue; /* clamped: no derivative */
            int64_t j = hit[h];
            double alpha = hit_alpha[h];
            const double *e = hit_e + 3 * h;
            double g = w[s] * (-prod / (1.0 - alpha)); /* dF/dalpha_j */
            const double *Wj = W + 9 * j;
            double wte[3];
            for (int c = 0; c < 3; ++c) wte[c] = Wj[c] * e[0] + Wj[3 + c] * e[1] + Wj[6 + c] * e[2];
            if (absolute == 2) {
                /* sensitivity of each term to binary32 rounding of the ray (origin
                 * difference x and direction d, ~u |x| in world units) and of W:
                 * the whitened closest-approach vector e moves by de */
                const double *mu = mean + 3 * j;
                double xn = sqrt((o[0] - mu[0]) * (o[0] - mu[0]) + (o[1] - mu[1]) * (o[1] - mu[1]) +
                                 (o[2] - mu[2]) * (o[2] - mu[2]));
                double tj = hit_t[h];
                double en = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
                double de = Wn[j] * (xn + fabs(tj) + 1.0) * U32;
                double ga = fabs(g) * alpha;
                g_opacity[j] += ga / opacity[j] * (en * de + U32 * (2.0 + hit_q[h]));
                for (int c = 0; c < 3; ++c) {
                    double sm = ga * (Wn[j] * de + fabs(wte[c]) * en * de);
                    g_mean[3 * j + c] += sm;
                    g_mean[3 * src + c] += sm;
                    g_log_scale[3 * j + c] += ga * (2.0 * fabs(e[c]) * de + e[c] * e[c] * en * de);
                }
            } else if (!absolute) {
                g_opacity[j] += g * alpha / opacity[j];
                for (int c = 0; c < 3; ++c) {
                    g_mean[3 * j + c] += g * alpha * wte[c];
                    g_mean[3 * src + c] -= g * alpha * wte[c];
                    g_log_scale[3 * j + c] += g * alpha * e[c] * e[c];
                }
            } else { /* sum of |term|: the scale of the summation's rounding error */
                g_opacity[j] += fabs(g * alpha / opacity[j]);
                for (int c = 0; c < 3; ++c) {
                    g_mean[3 * j + c] += fabs(g * alpha * wte[c]);
                    g_mean[3 * src + c] += fabs(g * alpha * wte[c]);
                    g_log_scale[3 * j + c] += fabs(g * alpha * e[c] * e[c]);
                }
            }
        }
    }
    free(hit);
    free(hit_alpha);
    free(hit_e);
    free(hit_t);
    free(hit_q);
    free(W);
    free(Wn);
}

/*
 * Rays (i, k) with i in [0, n) whose half-line [0, inf) meets the axis-aligned
 * box [lo, hi], plus every ray whose source is `always_src` (>= 0). Writes up
 * to cap ray ids and returns the total count. Used to restrict finite
 * differences to the rays a single Gaussian can influence.
 */
int64_t or_rays_meeting_box(int64_t n, const double *mean, const double *normal, const double *log_scale,
                            int32_t K, const double *dirs, int32_t dir_mode, double tmin_scale,
                            const double *lo, const double *hi, int64_t always_src, int64_t cap,
                            int64_t *out)
{
    int64_t count = 0;
    for (int64_t r = 0; r < n * (int64_t)K; ++r) {
        double o[3], d[3], tmin;
        int64_t src;
        make_ray(mean, normal, log_scale, K, dirs, dir_mode, tmin_scale, r, o, d, &tmin, &src);
        int hit = (src == always_src);
        if (!hit) {
            double t0 = 0.0, t1 = INFINITY;
            int ok = 1;
            for (int a = 0; a < 3 && ok; ++a) {
                if (d[a] == 0.0) {
                    if (o[a] < lo[a] || o[a] > hi[a]) ok = 0;
                } else {
                    double ta = (lo[a] - o[a]) / d[a], tb = (hi[a] - o[a]) / d[a];
                    if (ta > tb) { double tt = ta; ta = tb; tb = tt; }
                    if (ta > t0) t0 = ta;
                    if (tb < t1) t1 = tb;
                    if (t0 > t1) ok = 0;
                }
            }
            hit = ok;
        }
        if (hit) {
            if (count < cap) out[count] = r;
            ++count;
        }
    }
    return count;
}

/*
 * One Gaussian's terms on a list of rays: for the Gaussian with parameters
 * (mu, quat, log_scale, opacity) -- passed explicitly so that callers can
 * perturb them -- and each ray s: its peak parameter t*, the squared
 * Mahalanobis distance q at the peak, the unclamped alpha, whether it is
 * included under the cuts, and whether that decision is ambiguous under
 * binary32 rounding (same error model as or_trace_rays). Rays whose source
 * index equals `self` get inc = 0 (a Gaussian never occludes its own rays).
 */
void or_pair_terms(const double *mean, const double *normal, const double *log_scale, int32_t K,
                   const double *dirs, int32_t dir_mode, const or_params *prm, int64_t n_rays, const int64_t *rays,
                   int64_t self, const double *mu_j, const double *quat_j, const double *ls_j, double o_j,
                   double *t_out, double *q_out, double *alpha_out, int32_t *inc_out, int32_t *amb_out,
                   int32_t *near_clamp_out)
{
    double W[9];
    whitening(quat_j, ls_j, W);
    double Wn = 0.0;
    for (int a = 0; a < 9; ++a) Wn += W[a] * W[a];
    Wn = sqrt(Wn);
    const double qcut = prm->sigma_cut * prm->sigma_cut;
    const double ln_amin = log(prm->alpha_min);
    const double c = prm->kappa * U32;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n_rays; ++s) {
        double o[3], d[3], tmin;
        int64_t src;
        make_ray(mean, normal, log_scale, K, dirs, dir_mode, prm->tmin_scale, rays[s], o, d, &tmin, &src);
        double t, q, e[3], pn, vn;
        peak(W, mu_j, o, d, &t, &q, e, &pn, &vn);
        double dist = sqrt((o[0] - mu_j[0]) * (o[0] - mu_j[0]) + (o[1] - mu_j[1]) * (o[1] - mu_j[1]) +
                           (o[2] - mu_j[2]) * (o[2] - mu_j[2]));
        double Pabs = Wn * dist + pn, Vabs = Wn;
        double err_q = 2.0 * sqrt(q) * c * (Pabs + fabs(t) * Vabs) + c * (q + 1.0);
        double err_t = c * (Pabs / vn + pn * Vabs / (vn * vn) + 2.0 * fabs(t) * Vabs / vn + tmin + fabs(t));
        double alpha = o_j * exp(-0.5 * q);
        double lna = log(o_j) - 0.5 * q;
        double err_a = 0.5 * err_q + c * (2.0 + 0.5 * q + fabs(log(o_j)));
        int inc = (src != self) && (t >= tmin) && (q <= qcut) && (alpha >= prm->alpha_min);
        int maybe = (src != self) && (t >= tmin - err_t) && (q <= qcut + err_q) && (lna >= ln_amin - err_a);
        int sure = (src != self) && (t >= tmin + err_t) && (q <= qcut - err_q) && (lna >= ln_amin + err_a);
        t_out[s] = t;
        q_out[s] = q;
        alpha_out[s] = alpha;
        inc_out[s] = inc;
        amb_out[s] = maybe && !sure;
        near_clamp_out[s] = inc && fabs(lna - log(prm->alpha_max)) <= err_a;
    }
}

/*
 * For every ray r < n*K and each of nb boxes, bit b of mask[r] is set iff the
 * half-line of ray r meets box b (slab test in FP64, boxes given as lo/hi).
 * nb <= 64.
 */
void or_rays_meeting_boxes(int64_t n, const double *mean, const double *normal, const double *log_scale,
                           int32_t K, const double *dirs, int32_t dir_mode, double tmin_scale, int32_t nb,
                           const double *lo, const double *hi, uint64_t *mask)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n * (int64_t)K; ++r) {
        double o[3], d[3], tmin;
        int64_t src;
        make_ray(mean, normal, log_scale, K, dirs, dir_mode, tmin_scale, r, o, d, &tmin, &src);
        double inv[3];
        for (int a = 0; a < 3; ++a) inv[a] = 1.0 / d[a];
        uint64_t bits = 0;
        for (int b = 0; b < nb; ++b) {
            double t0 = 0.0, t1 = INFINITY;
            for (int a = 0; a < 3; ++a) {
                double ta = (lo[3 * b + a] - o[a]) * inv[a], tb = (hi[3 * b + a] - o[a]) * inv[a];
                if (ta > tb) { double tt = ta; ta = tb; tb = tt; }
                if (ta > t0) t0 = ta;
                if (tb < t1) t1 = tb;
            }
            if (t0 <= t1) bits |= 1ull << b;
        }
        mask[r] = bits;
    }
}

/* ------------------------------------------------------------------------ */
/* LBVH reference                                                           */
/* ------------------------------------------------------------------------ */

/* Spread the low 21 bits of v so that bit b lands at bit 3b. */
static uint64_t spread3(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

/*
 * 63-bit Morton keys in binary32 arithmetic (the quantisation is an integer
 * decision, so it is replayed in the precision the builder uses): per axis
 * u = (x - lo) / (hi - lo) (u = 0 when hi == lo), c = floor(u * 2^21) clamped
 * to [0, 2^21 - 1]; x bits take the most significant place of each triplet.
 * lo/hi are the min/max of the means over all Gaussians.
 */
void or_morton63(int64_t n, const float *mean, float *lo_out, float *hi_out, uint64_t *keys)
{
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            float x = mean[3 * i + a];
            if (x < lo[a]) lo[a] = x;
            if (x > hi[a]) hi[a] = x;
        }
    for (int a = 0; a < 3; ++a) {
        if (lo_out) lo_out[a] = lo[a];
        if (hi_out) hi_out[a] = hi[a];
    }
    for (int64_t i = 0; i < n; ++i) {
        uint64_t c[3];
        for (int a = 0; a < 3; ++a) {
            volatile float num = mean[3 * i + a] - lo[a];
            volatile float den = hi[a] - lo[a];
            volatile float u = (den > 0.0f) ? num / den : 0.0f;
            volatile float sc = u * 2097152.0f;
            float f = floorf(sc);
            if (f < 0.0f) f = 0.0f;
            if (f > 2097151.0f) f = 2097151.0f;
            c[a] = (uint64_t)f;
        }
        keys[i] = (spread3(c[0]) << 2) | (spread3(c[1]) << 1) | spread3(c[2]);
    }
}

/* Highest set bit index of x (x != 0). */
static int top_bit64(uint64_t x)
{
    int b = 63;
    while (!((x >> b) & 1ull)) --b;
    return b;
}

/*
 * Binary radix tree over the sorted keys, built TOP-DOWN: a node covering the
 * sorted range [f, l] (f < l) is split after the last position whose
 * augmented key (key, then the 32-bit position as a tie-break) has a 0 at the
 * most significant bit where the augmented keys at f and l differ. Node ids
 * follow Karras 2012: the root is internal node 0; a child range [f, g] with
 * f < g is internal node g, a child range [g, l] with g < l is internal node
 * g, and a single-element range m is leaf m. Children are written as the
 * internal id, or as ~m (negative) for leaf m. parent[] indexes internal nodes
 * as 0..n-2 and leaf m as n-1+m; the root's parent is -1. For n == 1 there are
 * no internal nodes and parent[0] = -1.
 */
int32_t or_radix_tree(int64_t n, const uint64_t *keys, int32_t *left, int32_t *right, int32_t *parent)
{
    if (n <= 0) return -1;
    if (n == 1) {
        parent[0] = -1;
        return 0;
    }
    int64_t *st_f = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * n));
    int64_t *st_l = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * n));
    int64_t *st_id = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * n));
    int64_t sp = 0;
    st_f[0] = 0;
    st_l[0] = n - 1;
    st_id[0] = 0;
    sp = 1;
    parent[0] = -1;
    while (sp > 0) {
        --sp;
        int64_t f = st_f[sp], l = st_l[sp], id = st_id[sp];
        int64_t split_first; /* first position of the right child */
        if (keys[f] != keys[l]) {
            int b = top_bit64(keys[f] ^ keys[l]);
            int64_t a = f, c = l; /* bit b: 0 at a, 1 at c; find first 1 */
            while (c - a > 1) {
                int64_t m = a + (c - a) / 2;
                if ((keys[m] >> b) & 1ull) c = m; else a = m;
            }
            split_first = c;
        } else {
            uint32_t x = (uint32_t)f ^ (uint32_t)l;
            int b = 31;
            while (!((x >> b) & 1u)) --b;
            split_first = (int64_t)(((uint64_t)l >> b) << b);
        }
        int64_t g = split_first - 1;
        /* left child covers [f, g] */
        if (g == f) {
            left[id] = ~(int32_t)g;
            parent[n - 1 + g] = (int32_t)id;
        } else {
            left[id] = (int32_t)g;
            parent[g] = (int32_t)id;
            st_f[sp] = f; st_l[sp] = g; st_id[sp] = g; ++sp;
        }
        /* right child covers [g+1, l] */
        if (g + 1 == l) {
            right[id] = ~(int32_t)(g + 1);
            parent[n - 1 + g + 1] = (int32_t)id;
        } else {
            right[id] = (int32_t)(g + 1);
            parent[g + 1] = (int32_t)id;
            st_f[sp] = g + 1; st_l[sp] = l; st_id[sp] = g + 1; ++sp;
        }
    }
    free(st_f);
    free(st_l);
    free(st_id);
    return 0;
}

/* Tree depth statistics: max number of internal nodes on a root-leaf path. */
int32_t or_tree_depth(int64_t n, const int32_t *left, const int32_t *right)
{
    if (n <= 1) return 0;
    int32_t *st = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * n));
    int32_t *dp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * n));
    int64_t sp = 0;
    int32_t best = 0;
    st[sp] = 0; dp[sp] = 1; ++sp;
    while (sp > 0) {
        --sp;
        int32_t id = st[sp], depth = dp[sp];
        if (depth > best) best = depth;
        int32_t ch[2] = {left[id], right[id]};
        for (int c = 0; c < 2; ++c)
            if (ch[c] >= 0) { st[sp] = ch[c]; dp[sp] = depth + 1; ++sp; }
    }
    free(st);
    free(dp);
    return best;
}

/* 3-sigma AABB of each Gaussian: mu_a +- sigma_cut * sqrt(sum_m (R_am s_m)^2). */
void or_leaf_boxes(int64_t n, const double *mean, const double *quat, const double *log_scale,
                   double sigma_cut, double *lo, double *hi)
{
    for (int64_t i = 0; i < n; ++i) {
        double R[9];
        quat_to_rot(quat + 4 * i, R);
        for (int a = 0; a < 3; ++a) {
            double s2 = 0.0;
            for (int m = 0; m < 3; ++m) {
                double v = R[a * 3 + m] * exp(log_scale[3 * i + m]);
                s2 += v * v;
            }
            double h = sigma_cut * sqrt(s2);
            lo[3 * i + a] = mean[3 * i + a] - h;
            hi[3 * i + a] = mean[3 * i + a] + h;
        }
    }
}

/* Internal-node boxes as the union of child boxes (leaf boxes indexed by
 * sorted position), computed by a post-order walk from the root. */
void or_refit(int64_t n, const int32_t *left, const int32_t *right, const double *leaf_lo,
              const double *leaf_hi, double *node_lo, double *node_hi)
{
    if (n <= 1) return;
    int32_t *st = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * n));
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    int64_t sp = 0;
    st[sp++] = 0;
    while (sp > 0) {
        int32_t id = st[sp - 1];
        if (!seen[id]) {
            seen[id] = 1;
            if (left[id] >= 0) st[sp++] = left[id];
            if (right[id] >= 0) st[sp++] = right[id];
            continue;
        }
        --sp;
        int32_t ch[2] = {left[id], right[id]};
        for (int a = 0; a < 3; ++a) {
            node_lo[3 * id + a] = INFINITY;
            node_hi[3 * id + a] = -INFINITY;
        }
        for (int c = 0; c < 2; ++c) {
            const double *cl, *chh;
            if (ch[c] >= 0) { cl = node_lo + 3 * ch[c]; chh = node_hi + 3 * ch[c]; }
            else { cl = leaf_lo + 3 * (int64_t)(~ch[c]); chh = leaf_hi + 3 * (int64_t)(~ch[c]); }
            for (int a = 0; a < 3; ++a) {
                if (cl[a] < node_lo[3 * id + a]) node_lo[3 * id + a] = cl[a];
                if (chh[a] > node_hi[3 * id + a]) node_hi[3 * id + a] = chh[a];
            }
        }
    }
    free(st);
    free(seen);
}

/* Threads the parallel loops use, and a way to set them (the CPU baseline is
 * timed on all host cores and on one). */
int32_t or_max_threads(void) { return (int32_t)omp_get_max_threads(); }
void or_set_threads(int32_t t) { omp_set_num_threads(t > 0 ? t : 1); }
