#pragma once
// Own-curve terms and the final reduction.
//
// Single layer: a target that is node i of a closed source curve with
// N = 2m equispaced-parameter nodes gets its n = 0 own-curve interaction from
// Kress's product quadrature for the logarithmic singularity (the paper's
// Section 3.2 discretises the single-layer operator with periodic Kress
// corrections).  Splitting log|r|^2 = log(4 sin^2((t_i - t)/2)) + smooth part
// and writing Kress's weights R_j for the first factor, the own-curve sum is
//
//   sum_k [ T_{(i-k) mod N} - 1/2 log|r_ik|^2 ] g_k + r r^T/|r|^2 g_k   (k != i)
//   + [ T_0 - log|x'(t_i)| ] g_i + t_i t_i^T g_i                       (k == i)
//
// with g = w f, |x'(t_k)| = w_k N / (2 pi), t t^T = I - n n^T, and the table
//   T_0 = -(N / 4 pi) R_0,
//   T_j = -(N / 4 pi) R_j + log(2 |sin(pi j / N)|)   (j != 0),
//   -(N / 4 pi) R_j = sum_{p=1}^{m-1} cos(2 pi p j / N) / p + (-1)^j / N.
// The table is built per curve (one workgroup each, cosines staged in LDS);
// the sum runs one thread per target, in FP64 in every mode, with the pair
// kernels' table log and one-step reciprocal (absolute error below 1e-15 and
// about 2e-15 relative).
//
// Double layer: the n = 0 term of a target's own node is the diagonal limit
// -(kappa / 2 pi) t t^T tau w (Section 2.3), added in the final reduction.
#include "pair_impl.h"

namespace s2d {

constexpr int kCosTab = 4096;

// Kress table T[lo .. lo+N) of curve c; called by a whole workgroup with the
// LDS array ctab[kCosTab].
__device__ __forceinline__ void kress_table_curve(const int32_t *__restrict__ off, int32_t c,
                                                  int64_t n_src, double *__restrict__ T, double *ctab) {
    const int lo = off[c], N = off[c + 1] - lo;
    // odd, empty or out-of-range curves get NaN in kress_self
    if (N < 2 || (N & 1) || lo < 0 || (int64_t)lo + N > n_src) return;
    const bool tab = N <= kCosTab;
    if (tab)
        for (int k = threadIdx.x; k < N; k += blockDim.x) ctab[k] = cospi(2.0 * (double)k / (double)N);
    __syncthreads();
    const int m = N / 2;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        double acc = 0.0;
        int idx = (int)(((int64_t)(m - 1) * j) % N);        // p j mod N, stepped down with p
        for (int p = m - 1; p >= 1; --p) {
            const double cs = tab ? ctab[idx] : cospi(2.0 * (double)idx / (double)N);
            acc += cs / (double)p;
            idx -= j;
            idx += idx < 0 ? N : 0;
        }
        acc += ((j & 1) ? -1.0 : 1.0) / (double)N;
        if (j != 0) acc += log(2.0 * fabs(sinpi((double)j / (double)N)));
        T[lo + j] = acc;
    }
}

// Own-curve Kress sum for target i (0 when the target is free); ltab: the
// LDS log table (fill_log_table).
__device__ __forceinline__ void kress_self_one(int64_t i, int64_t n_src, const int32_t *__restrict__ on_curve,
                                               const int32_t *__restrict__ on_node,
                                               const int32_t *__restrict__ off, int32_t n_curves,
                                               const double *__restrict__ x, const double *__restrict__ y,
                                               const double *__restrict__ nx, const double *__restrict__ ny,
                                               const double *__restrict__ w,
                                               const double *__restrict__ fx, const double *__restrict__ fy,
                                               const double *__restrict__ T, const double *ltab, double &sx,
                                               double &sy) {
    const int c = on_curve[i];
    sx = 0.0;
    sy = 0.0;
    if (c < 0) return;
    int lo = 0, N = 0, gi = -1;
    if (c < n_curves) {
        lo = off[c];
        N = off[c + 1] - lo;
        gi = on_node[i];
    }
    if (c >= n_curves || N < 2 || (N & 1) || lo < 0 || (int64_t)lo + N > n_src || gi < lo || gi >= lo + N) {
        sx = sy = __builtin_nan("");
        return;
    }
    const int ii = gi - lo;
    const double xi = x[gi], yi = y[gi];
    for (int k = 0; k < N; ++k) {
        const int gk = lo + k;
        const double gx = w[gk] * fx[gk], gy = w[gk] * fy[gk];
        double coef, rrx, rry;
        if (k == ii) {
            const double sp = w[gk] * (double)N * 0.15915494309189535;   // N / (2 pi)
            coef = T[lo] - log(sp);
            const double ng = nx[gk] * gx + ny[gk] * gy;
            rrx = gx - nx[gk] * ng;
            rry = gy - ny[gk] * ng;
        } else {
            int m = ii - k;
            if (m < 0) m += N;
            const double rx = xi - x[gk], ry = yi - y[gk];
            const double q = rx * rx + ry * ry;
            coef = T[lo + m] - 0.5 * log64_tab(q, ltab);
            const double t = (rx * gx + ry * gy) * rcp64(q);
            rrx = rx * t;
            rry = ry * t;
        }
        sx += coef * gx + rrx;
        sy += coef * gy + rry;
    }
}

// Double-layer diagonal limit for target i (times pi), added to (sx, sy).
__device__ __forceinline__ void dlp_diag_one(int64_t i, int64_t n_src, const int32_t *__restrict__ on_curve,
                                             const int32_t *__restrict__ on_node,
                                             const int32_t *__restrict__ off, int32_t n_curves,
                                             const double *__restrict__ nx, const double *__restrict__ ny,
                                             const double *__restrict__ w, const double *__restrict__ kappa,
                                             const double *__restrict__ fx, const double *__restrict__ fy,
                                             double &sx, double &sy) {
    const int c = on_curve[i];
    if (c < 0) return;
    const int j = on_node[i];
    if (c >= n_curves || j < 0 || j >= n_src || j < off[c] || j >= off[c + 1]) {
        sx = sy = __builtin_nan("");
        return;
    }
    // pi * (-(kappa / 2 pi) t t^T tau w) = -(1/2) kappa w (tau - n (n . tau))
    const double tn = nx[j] * fx[j] + ny[j] * fy[j];
    const double cc = -0.5 * kappa[j] * w[j];
    sx += cc * (fx[j] - nx[j] * tn);
    sy += cc * (fy[j] - ny[j] * tn);
}

// Last step for target i, given its pair sum (sx, sy) without prefactor: the
// own-curve Kress sums, the double layer's diagonal limit, the prefactor and
// the accumulate flag (fixed order).
__device__ __forceinline__ void final_one(const FinalArgs &a, int64_t i, double sx, double sy) {
    if (a.self) {
        sx += a.self[i];
        sy += a.self[a.n_trg + i];
    }
    if (a.dlp_diag)
        dlp_diag_one(i, a.n_src, a.on_curve, a.on_node, a.curve_off, a.n_curves, a.nx, a.ny, a.w, a.kappa,
                     a.fx, a.fy, sx, sy);
    const double ux = a.pref * sx, uy = a.pref * sy;
    a.u[i] = a.accumulate ? a.u[i] + ux : ux;
    if (a.ncomp == 2) a.v[i] = a.accumulate ? a.v[i] + uy : uy;
}

}  // namespace s2d
