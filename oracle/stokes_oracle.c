/*
 * FP64 CPU oracle for the free-space 2D Stokes layer potentials of the
 * periodic-channel method (Marple, Barnett, Gillman, Veerapaneni,
 * arXiv 1510.05616).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition of the discrete sums the GPU library computes.  It shares no code
 * with the GPU path and is called only by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark.
 *
 * Every sum is written as its definition: a double loop over targets and
 * (image, source node) pairs, each term evaluated in IEEE double with the C
 * library's log, accumulated per target with Neumaier's compensated sum.
 * OpenMP splits the target loop only.
 *
 * Single layer (Section 2.1, Eq. (S); imposed flow Section 3.1, Eq. (utotrep)):
 *   u(x) = 1/(4 pi mu) sum_{n=img_lo..img_hi} sum_j
 *          [ -1/2 log|r|^2 g_j + r (r . g_j) / |r|^2 ],
 *   r = x - y_j - n d e1,  g_j = w_j f_j,
 * where, when x is node i of source curve c and n = 0, the pairs with curve c
 * are replaced by Kress's product quadrature on that curve (Section 3.2 cites
 * it for the log-singular self interaction; the rule is Kress's periodic
 * logarithmic quadrature on 2n equispaced nodes).
 *
 * Double layer (Section 2.1, Eq. (D); near-image sum Eq. (Dnr)):
 *   u(x) = 1/pi sum_n sum_j r (r . nu_j)(r . tau_j) / |r|^4,  nu_j = w_j n_j,
 * where, when x is source node j and n = 0, that one term is replaced by the
 * Nystrom diagonal limit -(kappa_j / 2 pi) t_j t_j^T tau_j w_j
 * (Section 2.3).  The result is the principal-value operator; no -1/2 jump
 * term is added.
 *
 * Kress's weights for N = 2m nodes t_k = 2 pi k / N (LIE, Sec. 12.3):
 *   R_j = -(2 pi / m) sum_{p=1}^{m-1} cos(p j pi / m) / p - (pi / m^2) cos(j pi),
 * so that sum_k R_{|i-k|} phi(t_k) integrates log(4 sin^2((t_i - t)/2)) phi(t)
 * exactly for trigonometric polynomials of degree < m, and the remaining
 * smooth factor log(|r|^2 / (4 sin^2((t_i - t_k)/2))) tends to 2 log|x'(t_i)|
 * on the diagonal, with |x'(t_k)| = w_k N / (2 pi); the diagonal of
 * r r^T / |r|^2 tends to the tangent dyad t t^T = I - n n^T.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct { double s, c; } nsum;   /* Neumaier running sum */

static inline void nadd(nsum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->c; }

/* Kress weight R_j for N = 2m nodes, straight from the cosine sum. */
static double kress_R(int N, int j) {
    int m = N / 2;
    double acc = 0.0;
    for (int p = 1; p <= m - 1; ++p)
        acc += cos((double)p * (double)j * M_PI / (double)m) / (double)p;
    return -(2.0 * M_PI / (double)m) * acc - (M_PI / ((double)m * (double)m)) * cos((double)j * M_PI);
}

/*
 * Single-layer potential at n_trg targets.  All arrays are host FP64 (int32
 * for indices).  on_curve/on_node may be NULL.  Returns 0, or -1 on bad
 * arguments (odd curve size with a self target, inconsistent on_node).
 */
int oracle_slp(int64_t n_src, int32_t n_curves, const int32_t *curve_off,
               const double *x, const double *y, const double *nx, const double *ny,
               const double *w, const double *fx, const double *fy,
               int64_t n_trg, const double *tx, const double *ty,
               const int32_t *on_curve, const int32_t *on_node,
               double d, int32_t img_lo, int32_t img_hi, double mu,
               double *out_u, double *out_v)
{
    if (n_trg > 0 && on_curve) {
        for (int64_t i = 0; i < n_trg; ++i) {
            int c = on_curve[i];
            if (c < 0) continue;
            if (c >= n_curves) return -1;
            int N = curve_off[c + 1] - curve_off[c];
            if (N % 2 != 0 || N < 2) return -1;
            if (!on_node || on_node[i] < curve_off[c] || on_node[i] >= curve_off[c + 1]) return -1;
            if (!nx || !ny) return -1;
        }
    }
    (void)n_src;
    const double pref = 1.0 / (4.0 * M_PI * mu);
    int rc = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_trg; ++i) {
        nsum su = {0, 0}, sv = {0, 0};
        int own = (on_curve && on_curve[i] >= 0) ? on_curve[i] : -1;
        int64_t own_lo = own >= 0 ? curve_off[own] : 0, own_hi = own >= 0 ? curve_off[own + 1] : 0;
        for (int n = img_lo; n <= img_hi; ++n) {
            double px = tx[i] - (double)n * d, py = ty[i];
            for (int64_t j = 0; j < n_src; ++j) {
                if (n == 0 && j >= own_lo && j < own_hi) continue;
                double rx = px - x[j], ry = py - y[j];
                double q = rx * rx + ry * ry;
                double gx = w[j] * fx[j], gy = w[j] * fy[j];
                double lq = log(q);
                double rg = rx * gx + ry * gy;
                nadd(&su, -0.5 * lq * gx);
                nadd(&su, rx * rg / q);
                nadd(&sv, -0.5 * lq * gy);
                nadd(&sv, ry * rg / q);
            }
        }
        if (own >= 0 && img_lo <= 0 && img_hi >= 0) {
            int N = (int)(own_hi - own_lo);
            int64_t gi = on_node[i];
            int ii = (int)(gi - own_lo);
            for (int k = 0; k < N; ++k) {
                int64_t gk = own_lo + k;
                int mm = ((ii - k) % N + N) % N;
                double R = kress_R(N, mm);
                double gx = w[gk] * fx[gk], gy = w[gk] * fy[gk];
                double logpart, rrx, rry;   /* smooth log factor; (r r^T / q) g */
                if (k == ii) {
                    double sp = w[gk] * (double)N / (2.0 * M_PI);
                    logpart = -log(sp);
                    /* t t^T g = g - n (n . g) */
                    double ng = nx[gk] * gx + ny[gk] * gy;
                    rrx = gx - nx[gk] * ng;
                    rry = gy - ny[gk] * ng;
                } else {
                    double rx = x[gi] - x[gk], ry = y[gi] - y[gk];
                    double q = rx * rx + ry * ry;
                    double sn = sin(M_PI * (double)mm / (double)N);
                    logpart = -0.5 * log(q / (4.0 * sn * sn));
                    double rg = rx * gx + ry * gy;
                    rrx = rx * rg / q;
                    rry = ry * rg / q;
                }
                double coef = -0.5 * R * (double)N / (2.0 * M_PI) + logpart;
                nadd(&su, coef * gx);
                nadd(&su, rrx);
                nadd(&sv, coef * gy);
                nadd(&sv, rry);
            }
        }
        out_u[i] = pref * nval(&su);
        out_v[i] = pref * nval(&sv);
    }
    return rc;
}

/*
 * Double-layer potential (principal value on the source curves).  kappa may be
 * NULL only when no target sits on a source node.
 */
int oracle_dlp(int64_t n_src, int32_t n_curves, const int32_t *curve_off,
               const double *x, const double *y, const double *nx, const double *ny,
               const double *w, const double *kappa, const double *tx_d, const double *ty_d,
               int64_t n_trg, const double *tx, const double *ty,
               const int32_t *on_curve, const int32_t *on_node,
               double d, int32_t img_lo, int32_t img_hi,
               double *out_u, double *out_v)
{
    if (n_trg > 0 && on_curve) {
        for (int64_t i = 0; i < n_trg; ++i) {
            int c = on_curve[i];
            if (c < 0) continue;
            if (c >= n_curves || !on_node || !kappa) return -1;
            if (on_node[i] < curve_off[c] || on_node[i] >= curve_off[c + 1]) return -1;
        }
    }
    const double pref = 1.0 / M_PI;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_trg; ++i) {
        nsum su = {0, 0}, sv = {0, 0};
        int64_t self = (on_curve && on_curve[i] >= 0) ? on_node[i] : -1;
        for (int n = img_lo; n <= img_hi; ++n) {
            double px = tx[i] - (double)n * d, py = ty[i];
            for (int64_t j = 0; j < n_src; ++j) {
                if (n == 0 && j == self) {
                    /* -(kappa/2pi) t t^T tau w, written with the 1/pi prefactor outside */
                    double tg = nx[j] * tx_d[j] + ny[j] * ty_d[j];
                    double ttx = tx_d[j] - nx[j] * tg, tty = ty_d[j] - ny[j] * tg;
                    nadd(&su, -0.5 * kappa[j] * w[j] * ttx);
                    nadd(&sv, -0.5 * kappa[j] * w[j] * tty);
                    continue;
                }
                double rx = px - x[j], ry = py - y[j];
                double q = rx * rx + ry * ry;
                double rn = w[j] * (rx * nx[j] + ry * ny[j]);
                double rt = rx * tx_d[j] + ry * ty_d[j];
                double s = rn * rt / (q * q);
                nadd(&su, rx * s);
                nadd(&sv, ry * s);
            }
        }
        out_u[i] = pref * nval(&su);
        out_v[i] = pref * nval(&sv);
    }
    return 0;
}

/*
 * Pressures and traction at free targets (no target coincides with a source
 * node; a coincident pair gives an infinite or NaN term, as the kernels are
 * singular there).  Sums over the images n = img_lo..img_hi as above.
 *
 * Single-layer pressure (Section 2.1, Eq. (Q)):
 *   p(x) = 1/(2 pi) sum_n sum_j (r . g_j) / |r|^2,  g_j = w_j f_j.
 * Double-layer pressure (Section 2.1, Eq. (P)):
 *   p(x) = mu/pi sum_n sum_j [ -(nu_j . tau_j) / |r|^2
 *                              + 2 (r . nu_j)(r . tau_j) / |r|^4 ],  nu_j = w_j n_j.
 * Single-layer traction at a target with unit normal m (Section 2.1, Eq. (K)):
 *   t(x) = -1/pi sum_n sum_j r (r . g_j)(r . m) / |r|^4.
 */
int oracle_slp_pressure(int64_t n_src, const double *x, const double *y, const double *w,
                        const double *fx, const double *fy, int64_t n_trg,
                        const double *tx, const double *ty, double d, int32_t img_lo,
                        int32_t img_hi, double *out_p)
{
    if (img_lo > img_hi) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_trg; ++i) {
        nsum sp = {0, 0};
        for (int n = img_lo; n <= img_hi; ++n) {
            double px = tx[i] - (double)n * d, py = ty[i];
            for (int64_t j = 0; j < n_src; ++j) {
                double rx = px - x[j], ry = py - y[j];
                double q = rx * rx + ry * ry;
                double rg = rx * (w[j] * fx[j]) + ry * (w[j] * fy[j]);
                nadd(&sp, rg / q);
            }
        }
        out_p[i] = nval(&sp) / (2.0 * M_PI);
    }
    return 0;
}

int oracle_dlp_pressure(int64_t n_src, const double *x, const double *y, const double *nx,
                        const double *ny, const double *w, const double *tx_d,
                        const double *ty_d, int64_t n_trg, const double *tx, const double *ty,
                        double d, int32_t img_lo, int32_t img_hi, double mu, double *out_p)
{
    if (img_lo > img_hi) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_trg; ++i) {
        nsum sp = {0, 0};
        for (int n = img_lo; n <= img_hi; ++n) {
            double px = tx[i] - (double)n * d, py = ty[i];
            for (int64_t j = 0; j < n_src; ++j) {
                double rx = px - x[j], ry = py - y[j];
                double q = rx * rx + ry * ry;
                double vx = w[j] * nx[j], vy = w[j] * ny[j];
                double rn = rx * vx + ry * vy;
                double rt = rx * tx_d[j] + ry * ty_d[j];
                double nt = vx * tx_d[j] + vy * ty_d[j];
                nadd(&sp, -nt / q);
                nadd(&sp, 2.0 * rn * rt / (q * q));
            }
        }
        out_p[i] = mu / M_PI * nval(&sp);
    }
    return 0;
}

int oracle_slp_traction(int64_t n_src, const double *x, const double *y, const double *w,
                        const double *fx, const double *fy, int64_t n_trg,
                        const double *tx, const double *ty, const double *mx, const double *my,
                        double d, int32_t img_lo, int32_t img_hi, double *out_x, double *out_y)
{
    if (img_lo > img_hi) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_trg; ++i) {
        nsum sx = {0, 0}, sy = {0, 0};
        for (int n = img_lo; n <= img_hi; ++n) {
            double px = tx[i] - (double)n * d, py = ty[i];
            for (int64_t j = 0; j < n_src; ++j) {
                double rx = px - x[j], ry = py - y[j];
                double q = rx * rx + ry * ry;
                double rg = rx * (w[j] * fx[j]) + ry * (w[j] * fy[j]);
                double rm = rx * mx[i] + ry * my[i];
                double s = rg * rm / (q * q);
                nadd(&sx, rx * s);
                nadd(&sy, ry * s);
            }
        }
        out_x[i] = -nval(&sx) / M_PI;
        out_y[i] = -nval(&sy) / M_PI;
    }
    return 0;
}

/* Kress weights for a curve of N nodes (exposed for the tests' pins). */
int oracle_kress_weights(int N, double *R) {
    if (N < 2 || N % 2) return -1;
    for (int j = 0; j < N; ++j) R[j] = kress_R(N, j);
    return 0;
}

/* Threads the OpenMP runtime would use for the target loop. */
int oracle_num_threads(void) {
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
