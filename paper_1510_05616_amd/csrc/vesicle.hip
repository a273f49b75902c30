// The vesicle time step (Section 3.2; Algorithm 1, steps 2 and 6-9;
// Appendices A-C): membrane forces, the semi-implicit step system with the
// arc-length correction solved by restarted GMRES, the update, the area
// correction and the reparameterization.
//
// Per-curve work runs one workgroup per curve with the curve in LDS (N <= 512
// nodes).  The spectral derivative is the even-N Fourier differentiation
// circulant, (D v)_m = sum_{j != m} 1/2 (-1)^(m-j) cot(pi (m-j)/N) v_j, which
// is the derivative of the trigonometric interpolant at the nodes (Nyquist
// mode: zero derivative); D_s = D / |x_alpha|.  The single-layer sums of the
// step operator are the library's on-curve single-layer evaluation (Kress's
// product quadrature on the own curve).  GMRES runs on the host with device
// vectors: classical Gram-Schmidt applied twice, dot products reduced in a
// fixed order (reproducible bit for bit), the small Hessenberg least-squares
// problem by Givens rotations on the host.
#include "self_impl.h"
#include "s2d_near.h"
#include "../../include/stokes2d_vesicle.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace s2d {

namespace {

constexpr int kVesMaxN = 512;
constexpr int kVesBlock = 256;
constexpr int kMaxRestart = 128;

// ---------------------------------------------------------------------------
// per-curve helpers (block-cooperative; every thread of the block calls them)
// ---------------------------------------------------------------------------
struct CurveRange {
    int64_t lo, hi;
    int N;
    bool ok;
};

__device__ __forceinline__ CurveRange curve_range(const int32_t *off, int64_t n) {
    const int c = blockIdx.x;
    CurveRange r;
    r.lo = off[c];
    r.hi = off[c + 1];
    r.N = (int)(r.hi - r.lo);
    r.ok = r.lo >= 0 && r.hi <= n && r.N >= 4 && r.N <= kVesMaxN && (r.N & 1) == 0;
    return r;
}

// NaN over the valid part of the curve's node range
__device__ void curve_nan(const CurveRange &r, int64_t n, double *a, double *b = nullptr, double *c = nullptr) {
    const int64_t lo = max(r.lo, (int64_t)0), hi = min(r.hi, n);
    const double nan = __builtin_nan("");
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        if (a) a[i] = nan;
        if (b) b[i] = nan;
        if (c) c[i] = nan;
    }
}

// dtab[l] = 1/2 (-1)^l cot(pi l / N), l = 1..N-1
__device__ void fill_dtab(double *dtab, int N) {
    for (int l = threadIdx.x; l < N; l += blockDim.x) {
        if (l == 0) {
            dtab[0] = 0.0;
        } else {
            double s, c;
            sincospi((double)l / (double)N, &s, &c);
            dtab[l] = ((l & 1) ? -0.5 : 0.5) * c / s;
        }
    }
}

// out = D v (spectral derivative in alpha); v, out in LDS, distinct
__device__ void dalpha(const double *v, double *out, const double *dtab, int N) {
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        double acc = 0.0;
        for (int l = 1; l <= m; ++l) acc = __builtin_fma(dtab[l], v[m - l], acc);
        for (int l = m + 1; l < N; ++l) acc = __builtin_fma(dtab[l], v[m - l + N], acc);
        out[m] = acc;
    }
}

// out = D v / sp (arc-length derivative)
__device__ void dsv(const double *v, double *out, const double *dtab, const double *sp, int N) {
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        double acc = 0.0;
        for (int l = 1; l <= m; ++l) acc = __builtin_fma(dtab[l], v[m - l], acc);
        for (int l = m + 1; l < N; ++l) acc = __builtin_fma(dtab[l], v[m - l + N], acc);
        out[m] = acc / sp[m];
    }
}

// sum over the block of one value per thread, fixed order (tree in LDS);
// every thread gets the result
__device__ double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// x, y of the curve into LDS relative to its first node (derivatives and
// the area do not depend on the origin, and small coordinates keep the
// rounding that D_s^4 amplifies small), then xa, ya, speed and unit tangent
__device__ void load_geometry(const CurveRange &r, const double *x, const double *y, double *lx, double *ly,
                              double *xa, double *ya, double *sp, double *tx, double *ty, const double *dtab) {
    const double x0 = x[r.lo], y0 = y[r.lo];
    for (int m = threadIdx.x; m < r.N; m += blockDim.x) {
        lx[m] = x[r.lo + m] - x0;
        ly[m] = y[r.lo + m] - y0;
    }
    __syncthreads();
    dalpha(lx, xa, dtab, r.N);
    dalpha(ly, ya, dtab, r.N);
    __syncthreads();
    for (int m = threadIdx.x; m < r.N; m += blockDim.x) {
        sp[m] = sqrt(xa[m] * xa[m] + ya[m] * ya[m]);
        if (tx) {
            tx[m] = xa[m] / sp[m];
            ty[m] = ya[m] / sp[m];
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
struct GeomOut {
    double *sp, *w, *nx, *ny, *tx, *ty;
};

__global__ __launch_bounds__(kVesBlock) void ves_geom_kernel(int64_t n, const int32_t *off, const double *x,
                                                             const double *y, GeomOut o) {
    __shared__ double dtab[kVesMaxN], lx[kVesMaxN], ly[kVesMaxN], xa[kVesMaxN], ya[kVesMaxN], sp[kVesMaxN];
    const CurveRange r = curve_range(off, n);
    if (!r.ok) {
        curve_nan(r, n, o.sp, o.w, o.nx);
        curve_nan(r, n, o.ny, o.tx, o.ty);
        return;
    }
    fill_dtab(dtab, r.N);
    __syncthreads();
    load_geometry(r, x, y, lx, ly, xa, ya, sp, nullptr, nullptr, dtab);
    const double h = 2.0 * M_PI / (double)r.N;
    for (int m = threadIdx.x; m < r.N; m += blockDim.x) {
        const int64_t i = r.lo + m;
        if (o.sp) o.sp[i] = sp[m];
        if (o.w) o.w[i] = h * sp[m];
        if (o.nx) o.nx[i] = ya[m] / sp[m];
        if (o.ny) o.ny[i] = -xa[m] / sp[m];
        if (o.tx) o.tx[i] = xa[m] / sp[m];
        if (o.ty) o.ty[i] = ya[m] / sp[m];
    }
}

// f_b = -kappa_B D_s^4 x, f_sigma = D_s(sigma x_s); total: fb receives f_b + f_sigma
__global__ __launch_bounds__(kVesBlock) void ves_forces_kernel(int64_t n, const int32_t *off, const double *x,
                                                               const double *y, const double *sigma, double kb,
                                                               double *fbx, double *fby, double *fsx,
                                                               double *fsy, int total) {
    __shared__ double dtab[kVesMaxN], lx[kVesMaxN], ly[kVesMaxN], xa[kVesMaxN], ya[kVesMaxN], sp[kVesMaxN],
        tx[kVesMaxN], ty[kVesMaxN];
    const CurveRange r = curve_range(off, n);
    if (!r.ok) {
        curve_nan(r, n, fbx, fby, fsx);
        curve_nan(r, n, fsy);
        return;
    }
    fill_dtab(dtab, r.N);
    __syncthreads();
    load_geometry(r, x, y, lx, ly, xa, ya, sp, tx, ty, dtab);
    if (fbx) {
        // lx, ly -> D_s^4 (xa, ya and lx, ly alternate as scratch)
        double *a = lx, *b = ly, *ta = xa, *tb = ya;
        for (int k = 0; k < 4; ++k) {
            dsv(a, ta, dtab, sp, r.N);
            dsv(b, tb, dtab, sp, r.N);
            __syncthreads();
            double *t = a; a = ta; ta = t;
            t = b; b = tb; tb = t;
        }
        for (int m = threadIdx.x; m < r.N; m += blockDim.x) {
            fbx[r.lo + m] = -kb * a[m];
            fby[r.lo + m] = -kb * b[m];
        }
        __syncthreads();
    }
    if (fsx || total) {
        // xa, ya <- sigma x_s; lx, ly <- D_s of it
        for (int m = threadIdx.x; m < r.N; m += blockDim.x) {
            const double s = sigma ? sigma[r.lo + m] : 0.0;
            xa[m] = s * tx[m];
            ya[m] = s * ty[m];
        }
        __syncthreads();
        dsv(xa, lx, dtab, sp, r.N);
        dsv(ya, ly, dtab, sp, r.N);
        __syncthreads();
        for (int m = threadIdx.x; m < r.N; m += blockDim.x) {
            if (total) {
                fbx[r.lo + m] += lx[m];
                fby[r.lo + m] += ly[m];
            } else {
                fsx[r.lo + m] = lx[m];
                fsy[r.lo + m] = ly[m];
            }
        }
    }
}

// perimeter and area per curve
__global__ __launch_bounds__(kVesBlock) void ves_measure_kernel(int64_t n, const int32_t *off, const double *x,
                                                                const double *y, double *len, double *area) {
    __shared__ double dtab[kVesMaxN], lx[kVesMaxN], ly[kVesMaxN], xa[kVesMaxN], ya[kVesMaxN], sp[kVesMaxN];
    __shared__ double red[kVesBlock];
    const CurveRange r = curve_range(off, n);
    const int c = blockIdx.x;
    if (!r.ok) {
        if (threadIdx.x == 0) {
            if (len) len[c] = __builtin_nan("");
            if (area) area[c] = __builtin_nan("");
        }
        return;
    }
    fill_dtab(dtab, r.N);
    __syncthreads();
    load_geometry(r, x, y, lx, ly, xa, ya, sp, nullptr, nullptr, dtab);
    double sl = 0.0, sa = 0.0;
    for (int m = threadIdx.x; m < r.N; m += blockDim.x) {
        sl += sp[m];
        sa += lx[m] * ya[m];
    }
    const double h = 2.0 * M_PI / (double)r.N;
    sl = block_sum(sl, red);
    sa = block_sum(sa, red);
    if (threadIdx.x == 0) {
        if (len) len[c] = h * sl;
        if (area) area[c] = h * sa;
    }
}

// Pre-pass of the step operator.  From z = [u_x; u_y; sigma] (OP) or the
// shape (RHS), per curve:
//   OP:  density f = dt kappa_B D_s^4 u - D_s(sigma x_s), out rows 1-2 = u,
//        out row 3 = x_s . D_s u
//   RHS: density f = -kappa_B D_s^4 x, out rows 1-2 = u_resp (or 0),
//        out row 3 = (L0 - L) / (dt L) (or 0)
// The single layer of f is added to rows 1-2 afterwards.
struct OpArgs {
    int64_t n;
    const int32_t *off;
    const double *x, *y;
    const double *z;                 // OP input [3n]
    double dt, kb;
    const double *L0, *urx, *ury;    // RHS inputs
    double *fx, *fy;                 // density out [n]
    double *out;                     // [3n]
};

template <bool RHS>
__global__ __launch_bounds__(kVesBlock) void ves_op_kernel(OpArgs a) {
    __shared__ double dtab[kVesMaxN], lx[kVesMaxN], ly[kVesMaxN], xa[kVesMaxN], ya[kVesMaxN], sp[kVesMaxN],
        tx[kVesMaxN], ty[kVesMaxN], ua[kVesMaxN], ub[kVesMaxN], va[kVesMaxN], vb[kVesMaxN];
    __shared__ double red[kVesBlock];
    const int64_t n = a.n;
    const CurveRange r = curve_range(a.off, n);
    if (!r.ok) {
        curve_nan(r, n, a.fx, a.fy);
        curve_nan(r, n, a.out, a.out + n, a.out + 2 * n);
        return;
    }
    fill_dtab(dtab, r.N);
    __syncthreads();
    load_geometry(r, a.x, a.y, lx, ly, xa, ya, sp, tx, ty, dtab);
    const int N = r.N;
    // ua, va <- the field to differentiate four times
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        if (RHS) {
            ua[m] = lx[m];
            va[m] = ly[m];
        } else {
            ua[m] = a.z[r.lo + m];
            va[m] = a.z[n + r.lo + m];
        }
    }
    __syncthreads();
    double *p = ua, *q = va, *tp = ub, *tq = vb;
    for (int k = 0; k < 4; ++k) {
        dsv(p, tp, dtab, sp, N);
        dsv(q, tq, dtab, sp, N);
        __syncthreads();
        if (!RHS && k == 0) {
            // constraint row x_s . D_s u
            for (int m = threadIdx.x; m < N; m += blockDim.x)
                a.out[2 * n + r.lo + m] = tx[m] * tp[m] + ty[m] * tq[m];
        }
        double *t = p; p = tp; tp = t;
        t = q; q = tq; tq = t;
    }
    // p, q = D_s^4 of the field; tp, tq are free
    if (RHS) {
        double sl = 0.0;
        for (int m = threadIdx.x; m < N; m += blockDim.x) sl += sp[m];
        const double L = (2.0 * M_PI / (double)N) * block_sum(sl, red);
        const double alc = a.L0 ? (a.L0[blockIdx.x] - L) / (a.dt * L) : 0.0;
        for (int m = threadIdx.x; m < N; m += blockDim.x) {
            const int64_t i = r.lo + m;
            a.fx[i] = -a.kb * p[m];
            a.fy[i] = -a.kb * q[m];
            a.out[i] = a.urx ? a.urx[i] : 0.0;
            a.out[n + i] = a.ury ? a.ury[i] : 0.0;
            a.out[2 * n + i] = alc;
        }
    } else {
        // tension part: D_s(sigma x_s)
        for (int m = threadIdx.x; m < N; m += blockDim.x) {
            const double s = a.z[2 * n + r.lo + m];
            xa[m] = s * tx[m];
            ya[m] = s * ty[m];
        }
        __syncthreads();
        dsv(xa, tp, dtab, sp, N);
        dsv(ya, tq, dtab, sp, N);
        __syncthreads();
        const double c = a.dt * a.kb;
        for (int m = threadIdx.x; m < N; m += blockDim.x) {
            const int64_t i = r.lo + m;
            a.fx[i] = c * p[m] - tp[m];
            a.fy[i] = c * q[m] - tq[m];
            a.out[i] = a.z[i];
            a.out[n + i] = a.z[n + i];
        }
    }
}

// Appendix B, in place
__global__ __launch_bounds__(kVesBlock) void ves_area_kernel(int64_t n, const int32_t *off, double *x, double *y,
                                                             const double *A0) {
    __shared__ double dtab[kVesMaxN], lx[kVesMaxN], ly[kVesMaxN], xa[kVesMaxN], ya[kVesMaxN], xaa[kVesMaxN];
    __shared__ double red[kVesBlock];
    const CurveRange r = curve_range(off, n);
    if (!r.ok) {
        curve_nan(r, n, x, y);
        return;
    }
    const int N = r.N;
    fill_dtab(dtab, N);
    // coordinates relative to the first node (the integrals do not change)
    const double x0 = x[r.lo], y0 = y[r.lo];
    __syncthreads();
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        lx[m] = x[r.lo + m] - x0;
        ly[m] = y[r.lo + m] - y0;
    }
    __syncthreads();
    dalpha(lx, xa, dtab, N);
    dalpha(ly, ya, dtab, N);
    __syncthreads();
    dalpha(xa, xaa, dtab, N);
    __syncthreads();
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        s1 += ya[m] * xaa[m];
        s2 += ya[m] * ya[m] - lx[m] * xaa[m];
        s3 += lx[m] * ya[m];
    }
    const double h = 2.0 * M_PI / (double)N;
    const double qa = -h * block_sum(s1, red);
    const double qb = h * block_sum(s2, red);
    const double qc = h * block_sum(s3, red) - A0[blockIdx.x];
    // the root nearest zero of qa c^2 + qb c + qc = 0
    double c;
    if (qa == 0.0) {
        c = -qc / qb;
    } else {
        const double disc = sqrt(qb * qb - 4.0 * qa * qc);
        const double r1 = (-qb + disc) / (2.0 * qa), r2 = (-qb - disc) / (2.0 * qa);
        c = fabs(r1) <= fabs(r2) ? r1 : r2;
    }
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        x[r.lo + m] = x0 + (lx[m] + c * ya[m]);
        y[r.lo + m] = y0 + (ly[m] - c * xa[m]);
    }
}

// Appendix C, Algorithm 2, in place
__global__ __launch_bounds__(kVesBlock) void ves_reparam_kernel(int64_t n, const int32_t *off, double *x,
                                                                double *y, double *sigma) {
    __shared__ double dtab[kVesMaxN], lx[kVesMaxN], ly[kVesMaxN], ls[kVesMaxN], xa[kVesMaxN], ya[kVesMaxN];
    __shared__ double cw[kVesMaxN], sw[kVesMaxN], stab[kVesMaxN + 1], ast[kVesMaxN];
    __shared__ double Cr[kVesMaxN / 2 + 1], Ci[kVesMaxN / 2 + 1];
    const CurveRange r = curve_range(off, n);
    if (!r.ok) {
        curve_nan(r, n, x, y, sigma);
        return;
    }
    const int N = r.N, h = N / 2;
    fill_dtab(dtab, N);
    for (int l = threadIdx.x; l < N; l += blockDim.x) sincospi(2.0 * (double)l / (double)N, &sw[l], &cw[l]);
    // coordinates relative to the first node, restored on output
    const double x0 = x[r.lo], y0 = y[r.lo];
    __syncthreads();
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        lx[m] = x[r.lo + m] - x0;
        ly[m] = y[r.lo + m] - y0;
        ls[m] = sigma ? sigma[r.lo + m] : 0.0;
    }
    __syncthreads();
    dalpha(lx, xa, dtab, N);
    dalpha(ly, ya, dtab, N);
    __syncthreads();
    // speed into xa; C_k = (1/N) sum_j sp_j e^{-2 pi i j k / N}, k = 0..h
    for (int m = threadIdx.x; m < N; m += blockDim.x) xa[m] = sqrt(xa[m] * xa[m] + ya[m] * ya[m]);
    __syncthreads();
    for (int k = threadIdx.x; k <= h; k += blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int j = 0; j < N; ++j) {
            const int l = (j * k) % N;
            re = __builtin_fma(xa[j], cw[l], re);
            im = __builtin_fma(-xa[j], sw[l], im);
        }
        Cr[k] = re / (double)N;
        Ci[k] = im / (double)N;
    }
    __syncthreads();
    // s_m = C_0 alpha_m + sum_{k=1}^{h-1} 2 (Ci_k (cos k alpha_m - 1) + Cr_k sin k alpha_m) / k
    for (int m = threadIdx.x; m <= N; m += blockDim.x) {
        double s = 0.0;
        for (int k = 1; k < h; ++k) {
            const int l = (k * m) % N;
            s += 2.0 * (Ci[k] * (cw[l] - 1.0) + Cr[k] * sw[l]) / (double)k;
        }
        stab[m] = Cr[0] * (2.0 * M_PI * (double)m / (double)N) + s;
    }
    __syncthreads();
    // alpha*_k: s_j <= k L / N < s_{j+1} (binary search; s increasing)
    const double L = stab[N];
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        if (k == 0) {
            ast[0] = 0.0;
            continue;
        }
        const double t = L * (double)k / (double)N;
        int lo = 0, hi = N;                          // invariant: s_lo <= t < s_hi
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (stab[mid] <= t) lo = mid; else hi = mid;
        }
        ast[k] = 2.0 * M_PI / (double)N * ((double)lo + (t - stab[lo]) / (stab[lo + 1] - stab[lo]));
    }
    __syncthreads();
    // trigonometric interpolants of x, y, sigma at alpha*, one series at a
    // time: coefficients V_k = sum_j v_j e^{-2 pi i j k / N}, k = 0..h, into
    // xa (re) and ya (im), then the interpolant at every alpha*_m
    for (int q = 0; q < (sigma ? 3 : 2); ++q) {
        const double *v = q == 0 ? lx : (q == 1 ? ly : ls);
        __syncthreads();
        for (int k = threadIdx.x; k <= h; k += blockDim.x) {
            double re = 0.0, im = 0.0;
            for (int j = 0; j < N; ++j) {
                const int l = (j * k) % N;
                re = __builtin_fma(v[j], cw[l], re);
                im = __builtin_fma(-v[j], sw[l], im);
            }
            xa[k] = re;
            ya[k] = im;
        }
        __syncthreads();
        double *dst = q == 0 ? x : (q == 1 ? y : sigma);
        const double base = q == 0 ? x0 : (q == 1 ? y0 : 0.0);
        for (int m = threadIdx.x; m < N; m += blockDim.x) {
            const double al = ast[m];
            double ws, wc;
            sincos(al, &ws, &wc);
            double acc = 0.0;
            for (int k0 = 1; k0 < h; k0 += 32) {
                // e^{i k alpha*} by rotation, re-anchored every 32 modes
                double zs, zc;
                sincos((double)k0 * al, &zs, &zc);
                const int k1 = min(k0 + 32, h);
                for (int k = k0; k < k1; ++k) {
                    acc += xa[k] * zc - ya[k] * zs;
                    const double t = zc * wc - zs * ws;
                    zs = zc * ws + zs * wc;
                    zc = t;
                }
            }
            dst[r.lo + m] = base + (xa[0] + 2.0 * acc + xa[h] * cos((double)h * al)) / (double)N;
        }
    }
}

// x += dt u, y += dt v, sigma = z row 3, optional copies of u, v
__global__ __launch_bounds__(256) void ves_update_kernel(int64_t n, const double *z, double dt, double *x, double *y,
                                                         double *sigma, double *u, double *v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    x[i] += dt * z[i];
    y[i] += dt * z[n + i];
    sigma[i] = z[2 * n + i];
    if (u) u[i] = z[i];
    if (v) v[i] = z[n + i];
}

__global__ __launch_bounds__(256) void ves_targets_kernel(int64_t n, int n_curves, const int32_t *off,
                                                          int32_t *on_curve, int32_t *on_node) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = n_curves;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    on_curve[i] = lo;
    on_node[i] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// the block-diagonal preconditioner: per curve c (N nodes, padded to Nm),
//   P_c = [ I + dt kappa_B S_cc D_s^4      -S_cc D_s(x_s .) ]
//         [ x_s . D_s                       0               ]
// with S_cc the curve's own single layer at image 0 (Kress), stored
// column-major with rows and columns [x block; y block; sigma block], each
// block Nm long; padding rows and columns hold the identity.
// ---------------------------------------------------------------------------
struct PcArgs {
    int64_t n;
    const int32_t *off;
    int Nm;
    const double *x, *y, *sp, *w, *nx, *ny, *tx, *ty;
    double dtk, pref;
    double *T, *Dm, *D4, *Sm, *Bm, *Top, *Pm;
};

// Kress table, D_s (Nm x Nm) and S_cc (2Nm x 2Nm) of curve blockIdx.x
__global__ __launch_bounds__(kVesBlock) void pc_fill_ds(PcArgs a) {
    __shared__ double ctab[kCosTab];
    __shared__ double dtab[kVesMaxN];
    const int c = blockIdx.x, Nm = a.Nm;
    const CurveRange r = curve_range(a.off, a.n);
    double *Dm = a.Dm + (int64_t)c * Nm * Nm, *Sm = a.Sm + (int64_t)c * 4 * Nm * Nm;
    const int N = r.ok ? r.N : 0;
    if (r.ok) {
        kress_table_curve(a.off, c, a.n, a.T, ctab);
        fill_dtab(dtab, N);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < Nm * Nm; idx += blockDim.x) {
        const int j = idx % Nm, k = idx / Nm;
        double v = 0.0;
        if (j < N && k < N && j != k) v = dtab[(j - k + N) % N] / a.sp[r.lo + j];
        Dm[idx] = v;
    }
    const int M2 = 2 * Nm;
    for (int idx = threadIdx.x; idx < M2 * M2; idx += blockDim.x) {
        const int row = idx % M2, col = idx / M2;
        const int ra = row / Nm, i = row % Nm, cb = col / Nm, k = col % Nm;
        double v = 0.0;
        if (i < N && k < N) {
            const int64_t gi = r.lo + i, gk = r.lo + k;
            double coef, R;
            if (i == k) {
                coef = a.T[r.lo] - log(a.w[gk] * (double)N * 0.15915494309189535);
                const double na = ra == 0 ? a.nx[gk] : a.ny[gk], nb = cb == 0 ? a.nx[gk] : a.ny[gk];
                R = (ra == cb ? 1.0 : 0.0) - na * nb;
            } else {
                const double rx = a.x[gi] - a.x[gk], ry = a.y[gi] - a.y[gk];
                const double q = rx * rx + ry * ry;
                coef = a.T[r.lo + (i - k + N) % N] - 0.5 * log(q);
                R = (ra == 0 ? rx : ry) * (cb == 0 ? rx : ry) / q;
            }
            v = a.pref * a.w[gk] * ((ra == cb ? coef : 0.0) + R);
        }
        Sm[idx] = v;
    }
}

// B_c (2Nm x 3Nm) = [ dt kappa_B D_s^4  0  -D_s diag(t_x) ;  0  dt kappa_B D_s^4  -D_s diag(t_y) ]
__global__ __launch_bounds__(kVesBlock) void pc_fill_b(PcArgs a) {
    const int c = blockIdx.x, Nm = a.Nm, M2 = 2 * Nm;
    const CurveRange r = curve_range(a.off, a.n);
    const int N = r.ok ? r.N : 0;
    const double *Dm = a.Dm + (int64_t)c * Nm * Nm, *D4 = a.D4 + (int64_t)c * Nm * Nm;
    double *B = a.Bm + (int64_t)c * 6 * Nm * Nm;
    for (int idx = threadIdx.x; idx < M2 * 3 * Nm; idx += blockDim.x) {
        const int row = idx % M2, col = idx / M2;
        const int ra = row / Nm, j = row % Nm, cb = col / Nm, k = col % Nm;
        double v = 0.0;
        if (j < N && k < N) {
            if (cb < 2)
                v = ra == cb ? a.dtk * D4[j + k * Nm] : 0.0;
            else
                v = -Dm[j + k * Nm] * (ra == 0 ? a.tx[r.lo + k] : a.ty[r.lo + k]);
        }
        B[idx] = v;
    }
}

// P_c (3Nm x 3Nm) from Top_c = S_cc B_c
__global__ __launch_bounds__(kVesBlock) void pc_fill_p(PcArgs a) {
    const int c = blockIdx.x, Nm = a.Nm, M2 = 2 * Nm, M3 = 3 * Nm;
    const CurveRange r = curve_range(a.off, a.n);
    const int N = r.ok ? r.N : 0;
    const double *Dm = a.Dm + (int64_t)c * Nm * Nm, *Top = a.Top + (int64_t)c * 6 * Nm * Nm;
    double *P = a.Pm + (int64_t)c * 9 * Nm * Nm;
    for (int idx = threadIdx.x; idx < M3 * M3; idx += blockDim.x) {
        const int row = idx % M3, col = idx / M3;
        const int ra = row / Nm, i = row % Nm, cb = col / Nm, k = col % Nm;
        double v;
        if (i >= N || k >= N) {
            v = row == col ? 1.0 : 0.0;
        } else if (ra < 2) {
            v = Top[row + (int64_t)col * M2] + (row == col ? 1.0 : 0.0);
        } else {
            v = cb < 2 ? (cb == 0 ? a.tx[r.lo + i] : a.ty[r.lo + i]) * Dm[i + k * Nm] : 0.0;
        }
        P[idx] = v;
    }
}

// padded per-curve right-hand sides from a [3n] vector, and back
__global__ __launch_bounds__(256) void pc_gather(int64_t n, const int32_t *off, int Nm, const double *v,
                                                 double *rhs) {
    const int c = blockIdx.x;
    const int64_t lo = off[c];
    const int N = (int)(off[c + 1] - lo);
    double *o = rhs + (int64_t)c * 3 * Nm;
    for (int idx = threadIdx.x; idx < 3 * Nm; idx += blockDim.x) {
        const int ab = idx / Nm, m = idx % Nm;
        o[idx] = m < N ? v[ab * n + lo + m] : 0.0;
    }
}

__global__ __launch_bounds__(256) void pc_scatter(int64_t n, const int32_t *off, int Nm, const double *rhs,
                                                  double *v) {
    const int c = blockIdx.x;
    const int64_t lo = off[c];
    const int N = (int)(off[c + 1] - lo);
    const double *o = rhs + (int64_t)c * 3 * Nm;
    for (int idx = threadIdx.x; idx < 3 * Nm; idx += blockDim.x) {
        const int ab = idx / Nm, m = idx % Nm;
        if (m < N) v[ab * n + lo + m] = o[idx];
    }
}

// ---------------------------------------------------------------------------
// device vectors for GMRES
// ---------------------------------------------------------------------------
constexpr int kDotBlocks = 240;

// partial[b * k1 + j] = sum over block b's chunk of V_j . w (j < k1)
__global__ __launch_bounds__(256) void vec_dots_kernel(int64_t len, int k1, const double *V, int64_t ldv,
                                                       const double *w, double *partial) {
    __shared__ double red[256];
    const int64_t chunk = (len + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = (int64_t)blockIdx.x * chunk, b1 = min(b0 + chunk, len);
    for (int j = 0; j < k1; ++j) {
        const double *vj = V + j * ldv;
        double s = 0.0;
        for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) s = __builtin_fma(vj[i], w[i], s);
        red[threadIdx.x] = s;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * k1 + j] = red[0];
        __syncthreads();
    }
}

__global__ void vec_dots_final(int nb, int k1, const double *partial, double *out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k1) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[(int64_t)b * k1 + j];
    out[j] = s;
}

struct Coefs {
    double c[kMaxRestart + 2];
};

// w = sw * w + sum_j c_j V_j (j < k1)
__global__ __launch_bounds__(256) void vec_combo_kernel(int64_t len, int k1, const double *V, int64_t ldv, Coefs c,
                                                        double sw, double *w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    double acc = sw == 0.0 ? 0.0 : sw * w[i];
    for (int j = 0; j < k1; ++j) acc = __builtin_fma(c.c[j], V[j * ldv + i], acc);
    w[i] = acc;
}

// out = a * x + b * y
__global__ __launch_bounds__(256) void vec_axpby_kernel(int64_t len, double a, const double *x, double b,
                                                        const double *y, double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    out[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}

// ---------------------------------------------------------------------------
// close evaluation between vesicles (Section 3.2): a node closer than
// band h_c to another vesicle c, or to an image of one (h_c the largest
// trapezoid weight of c), gets the difference between the upsampled
// quadrature of c's single layer and its trapezoid rule at that node
// ---------------------------------------------------------------------------
// per curve: box[5 c ..] = x min, x max, y min, y max, h_c; NaN for a curve
// of invalid size (never near)
__global__ __launch_bounds__(256) void ves_near_box(int64_t n, const int32_t *off, const double *x, const double *y,
                                                    const double *w, double *box) {
    __shared__ double red[5][256];
    const CurveRange r = curve_range(off, n);
    const double inf = __builtin_inf();
    double v[5] = {inf, -inf, inf, -inf, 0.0};
    if (r.ok)
        for (int64_t i = r.lo + threadIdx.x; i < r.hi; i += blockDim.x) {
            v[0] = fmin(v[0], x[i]);
            v[1] = fmax(v[1], x[i]);
            v[2] = fmin(v[2], y[i]);
            v[3] = fmax(v[3], y[i]);
            v[4] = fmax(v[4], w[i]);
        }
    for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            const int o = threadIdx.x + h;
            red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][o]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][o]);
            red[2][threadIdx.x] = fmin(red[2][threadIdx.x], red[2][o]);
            red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][o]);
            red[4][threadIdx.x] = fmax(red[4][threadIdx.x], red[4][o]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) box[5 * blockIdx.x + threadIdx.x] = r.ok ? red[threadIdx.x][0] : __builtin_nan("");
}

// The near test of the point (tx, ty) against curve c: the squared distance
// to c's nearest node below (band h_c)^2, every product and sum rounded on
// its own (no fused multiply-add), as the host-side reference computes it.
__device__ bool ves_near_hit(double tx, double ty, const double *x, const double *y, int64_t lo, int64_t hi,
                             double R2) {
#pragma clang fp contract(off)
    double q = __builtin_inf();
    for (int64_t j = lo; j < hi; ++j) {
        const double dx = tx - x[j], dy = ty - y[j];
        q = fmin(q, dx * dx + dy * dy);
    }
    return q < R2;
}

// Per node i (on curve ci), the (curve c, image k) pairs with c != ci or
// k != 0 for which the node, shifted by -k d, is near c: counted (WRITE
// false, cnt[i]) or written from pos[i] on in the order c, then k (WRITE
// true): the node, the curve and the shifted coordinates.
template <bool WRITE>
__global__ __launch_bounds__(256) void ves_near_pairs(int64_t n, int32_t nc, const int32_t *off, const int32_t *oc,
                                                      const double *x, const double *y, const double *box, double d,
                                                      int img_lo, int img_hi, double band, int32_t *cnt,
                                                      const int64_t *pos, int32_t *pnode, int32_t *pcurve,
                                                      double *px, double *py) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ci = oc[i];
    const double xi = x[i], yi = y[i];
    int32_t m = 0;
    int64_t at = WRITE ? pos[i] : 0;
    for (int c = 0; c < nc; ++c) {
        const double *b = box + 5 * c;
        const double R = band * b[4], R2 = R * R, Rb = 1.01 * R;   // the box test only pre-selects
        for (int k = img_lo; k <= img_hi; ++k) {
            if (c == ci && k == 0) continue;
            const double tx = xi - (double)k * d;
            if (!(tx >= b[0] - Rb && tx <= b[1] + Rb && yi >= b[2] - Rb && yi <= b[3] + Rb)) continue;
            if (!ves_near_hit(tx, yi, x, y, off[c], off[c + 1], R2)) continue;
            if (WRITE) {
                pnode[at] = (int32_t)i;
                pcurve[at] = c;
                px[at] = tx;
                py[at] = yi;
                ++at;
            } else {
                ++m;
            }
        }
    }
    if (!WRITE) cnt[i] = m;
}

// exclusive scan of cnt[0 .. n) into pos[0 .. n], pos[n] the total; one
// workgroup, each thread over a contiguous segment
__global__ __launch_bounds__(1024) void ves_near_scan(int64_t n, const int32_t *cnt, int64_t *pos) {
    __shared__ int64_t part[1024];
    const int64_t seg = (n + 1023) / 1024;
    const int64_t b0 = min((int64_t)threadIdx.x * seg, n), b1 = min(b0 + seg, n);
    int64_t s = 0;
    for (int64_t i = b0; i < b1; ++i) s += cnt[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int t = 0; t < 1024; ++t) {
            const int64_t v = part[t];
            part[t] = acc;
            acc += v;
        }
        pos[n] = acc;
    }
    __syncthreads();
    int64_t acc = part[threadIdx.x];
    for (int64_t i = b0; i < b1; ++i) {
        pos[i] = acc;
        acc += cnt[i];
    }
}

// out[i] += the node's corrections, out[n + i] likewise, summed in list order
__global__ __launch_bounds__(256) void ves_near_add(int64_t n, const int64_t *pos, const double *du, const double *dv,
                                                    double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t a = pos[i], b = pos[i + 1];
    if (b <= a) return;
    double su = 0.0, sv = 0.0;
    for (int64_t p = a; p < b; ++p) {
        su += du[p];
        sv += dv[p];
    }
    out[i] += su;
    out[n + i] += sv;
}

unsigned g256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct StepLayout {
    size_t geo, dens, tgt, b, r, w, dz, ri, V, z, part, dots, slp, slp_bytes;
    // preconditioner (precond != 0): Kress table, per-curve D_s, D_s^2, D_s^4,
    // S_cc, B, S_cc B, P (LU), pivots, info, padded right-hand sides, two
    // [3n] vectors
    size_t T, Dm, D2, D4, Sm, Bm, Top, Pm, ipiv, info, rhs, t1, t2;
    // close evaluation (near != 0): curve boxes, per-node counts and list
    // offsets, the near pairs (node, curve, shifted coordinates, corrections),
    // the upsampled records
    size_t nbox, ncnt, npos, pnode, pcurve, px, py, pdu, pdv, up;
    size_t total;
};

s2d_curves ves_curves(int64_t n, int32_t nc, const int32_t *off, const double *x, const double *y) {
    s2d_curves c{};
    c.n_nodes = n;
    c.n_curves = nc;
    c.curve_off = off;
    c.x = x;
    c.y = y;
    return c;
}

StepLayout step_layout(int64_t n, int32_t nc, const ves_step_params *p) {
    StepLayout L{};
    const size_t d = sizeof(double);
    const size_t n3 = 3 * (size_t)n;
    const int m = std::max(1, std::min(p->restart, kMaxRestart));
    size_t o = 0;
    L.geo = o;
    o += al256(6 * (size_t)n * d);       // speed, w, nx, ny, tx, ty
    L.dens = o;
    o += al256(2 * (size_t)n * d);
    L.tgt = o;
    o += al256(2 * (size_t)n * sizeof(int32_t));
    L.b = o;
    o += al256(n3 * d);
    L.r = o;
    o += al256(n3 * d);
    L.w = o;
    o += al256(n3 * d);
    L.dz = o;
    o += al256(n3 * d);
    L.ri = o;
    o += al256(n3 * d);
    L.V = o;
    o += al256((size_t)(m + 1) * n3 * d);
    L.z = o;
    o += al256(n3 * d);
    L.part = o;
    o += al256((size_t)kDotBlocks * (m + 2) * d);
    L.dots = o;
    o += al256((size_t)(m + 2) * d);
    // the single-layer workspace for n on-curve targets
    // pointers stand in for the arrays: only the sizes are read
    s2d_curves c = ves_curves(n, nc, (const int32_t *)1, (const double *)1, (const double *)1);
    c.nx = c.ny = c.w = c.fx = c.fy = (const double *)1;
    s2d_targets t{};
    t.n = n;
    t.x = t.y = (const double *)1;
    t.on_curve = t.on_node = (const int32_t *)1;
    // FP64 sums always run (right-hand side and residuals); FP32C ones too in that mode
    const size_t sz = std::max(stokes2d_workspace_size(S2D_OP_SLP, S2D_FP64, &c, &t),
                               p->mode == S2D_FP32C ? stokes2d_workspace_size(S2D_OP_SLP, S2D_FP32C, &c, &t) : 0);
    L.slp = o;
    L.slp_bytes = std::max<size_t>(sz, 256);
    o += al256(L.slp_bytes);
    if (p->precond) {
        const size_t Nm = (size_t)p->nmax, q = (size_t)nc * Nm * Nm * d;
        L.T = o;
        o += al256((size_t)n * d);
        L.Dm = o;
        o += al256(q);
        L.D2 = o;
        o += al256(q);
        L.D4 = o;
        o += al256(q);
        L.Sm = o;
        o += al256(4 * q);
        L.Bm = o;
        o += al256(6 * q);
        L.Top = o;
        o += al256(6 * q);
        L.Pm = o;
        o += al256(9 * q);
        L.ipiv = o;
        o += al256((size_t)nc * 3 * Nm * sizeof(int32_t));
        L.info = o;
        o += al256((size_t)nc * sizeof(int32_t));
        L.rhs = o;
        o += al256((size_t)nc * 3 * Nm * d);
        L.t1 = o;
        o += al256(n3 * d);
        L.t2 = o;
        o += al256(n3 * d);
    }
    if (p->near) {
        const size_t cap = (size_t)std::max(p->near_max, 1);
        L.nbox = o;
        o += al256((size_t)nc * 5 * d);
        L.ncnt = o;
        o += al256((size_t)n * sizeof(int32_t));
        L.npos = o;
        o += al256(((size_t)n + 1) * sizeof(int64_t));
        L.pnode = o;
        o += al256(cap * sizeof(int32_t));
        L.pcurve = o;
        o += al256(cap * sizeof(int32_t));
        L.px = o;
        o += al256(cap * d);
        L.py = o;
        o += al256(cap * d);
        L.pdu = o;
        o += al256(cap * d);
        L.pdv = o;
        o += al256(cap * d);
        L.up = o;
        o += al256(4 * ((size_t)p->near_P + 1) * (size_t)n * d);
    }
    L.total = o;
    return L;
}

// the step operator's context
struct StepCtx {
    int64_t n;
    int32_t nc;
    const int32_t *off;
    const double *x, *y;
    const ves_step_params *p;
    char *ws;
    StepLayout L;
    hipStream_t st;
    s2d_curves src;
    s2d_targets trg;
    double *geo;
    bool pc;
    rocblas_handle h;        // set while the preconditioner is in use (blas_mutex held)
    int64_t nm;              // near pairs (close evaluation)
};

int ves_fail(int code, const std::string &m) { return set_error(code, m); }

int check_set(int64_t n, int32_t nc, const int32_t *off, const void *x, const void *y) {
    if (n < 0 || nc < 0 || n > INT32_MAX / 4) return ves_fail(S2D_EINVAL, "vesicle sizes out of range");
    if (nc > 0 && !off) return ves_fail(S2D_EINVAL, "curve_off must not be NULL");
    if (n > 0 && (nc < 1 || !x || !y)) return ves_fail(S2D_EINVAL, "vesicles with nodes need curves, x and y");
    return S2D_OK;
}

int check_params(const ves_step_params *p) {
    if (!p) return ves_fail(S2D_EINVAL, "params must not be NULL");
    if (p->mode != S2D_FP64 && p->mode != S2D_FP32C) return ves_fail(S2D_EINVAL, "mode must be an s2d_mode");
    if (!(std::isfinite(p->dt) && p->dt > 0.0)) return ves_fail(S2D_EINVAL, "dt must be finite and > 0");
    if (!(std::isfinite(p->kappa_b) && p->kappa_b >= 0.0)) return ves_fail(S2D_EINVAL, "kappa_b must be >= 0");
    if (!(std::isfinite(p->mu) && p->mu > 0.0)) return ves_fail(S2D_EINVAL, "mu must be finite and > 0");
    if (p->img_lo > p->img_hi || p->img_lo < -64 || p->img_hi > 64) return ves_fail(S2D_EINVAL, "bad image range");
    if ((p->img_lo != 0 || p->img_hi != 0) && !(std::isfinite(p->d) && p->d > 0.0))
        return ves_fail(S2D_EINVAL, "period d must be > 0 when images are used");
    if ((p->u_resp_x == nullptr) != (p->u_resp_y == nullptr))
        return ves_fail(S2D_EINVAL, "u_resp_x and u_resp_y must both be NULL or both be set");
    if (p->restart < 1 || p->restart > kMaxRestart) return ves_fail(S2D_EINVAL, "restart must be in 1..128");
    if (p->precond && (p->nmax < 4 || p->nmax > kVesMaxN))
        return ves_fail(S2D_EINVAL, "the preconditioner needs nmax in 4..512");
    if (!p->precond && p->nmax != 0 && (p->nmax < 4 || p->nmax > kVesMaxN))
        return ves_fail(S2D_EINVAL, "nmax must be 0 or in 4..512");
    if (p->near != 0 && p->near != 1) return ves_fail(S2D_EINVAL, "near must be 0 or 1");
    if (p->near) {
        if (p->nmax < 4 || p->nmax > kUpMaxN)
            return ves_fail(S2D_EINVAL, "close evaluation needs nmax in 4..256");
        if (p->near_P < 2 || (int64_t)p->near_P * p->nmax > kUpMaxM)
            return ves_fail(S2D_EINVAL, "close evaluation needs near_P >= 2 and near_P * nmax <= 2048");
        if (!(std::isfinite(p->near_band) && p->near_band > 0.0))
            return ves_fail(S2D_EINVAL, "near_band must be finite and > 0");
        if (p->near_max < 1) return ves_fail(S2D_EINVAL, "near_max must be >= 1");
    }
    if (p->max_iter < 1) return ves_fail(S2D_EINVAL, "max_iter must be >= 1");
    if (!(p->tol >= 0.0)) return ves_fail(S2D_EINVAL, "tol must be >= 0");
    if (p->warm != 0 && p->warm != 1) return ves_fail(S2D_EINVAL, "warm must be 0 or 1");
    return S2D_OK;
}

int hipf(hipError_t e, const char *what) {
    return ves_fail(S2D_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int setup_ctx(StepCtx &C, int64_t n, int32_t nc, const int32_t *off, const double *x, const double *y,
              const ves_step_params *p, void *ws, size_t ws_bytes, void *stream) {
    C.n = n;
    C.nc = nc;
    C.off = off;
    C.x = x;
    C.y = y;
    C.p = p;
    C.L = step_layout(n, nc, p);
    if (!ws || ws_bytes < C.L.total)
        return ves_fail(S2D_EWORKSPACE, "vesicle step workspace too small: need " + std::to_string(C.L.total));
    if (((uintptr_t)ws & 255) != 0) return ves_fail(S2D_EWORKSPACE, "workspace must be 256-byte aligned");
    C.ws = (char *)ws;
    C.st = (hipStream_t)stream;
    C.geo = (double *)(C.ws + C.L.geo);
    GeomOut g{C.geo, C.geo + n, C.geo + 2 * n, C.geo + 3 * n, C.geo + 4 * n, C.geo + 5 * n};
    hipLaunchKernelGGL(ves_geom_kernel, dim3(nc), dim3(kVesBlock), 0, C.st, n, off, x, y, g);
    int32_t *oc = (int32_t *)(C.ws + C.L.tgt), *on = oc + n;
    hipLaunchKernelGGL(ves_targets_kernel, dim3(g256(n)), dim3(256), 0, C.st, n, nc, off, oc, on);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipf(e, "vesicle geometry launch");
    double *dens = (double *)(C.ws + C.L.dens);
    C.src = ves_curves(n, nc, off, x, y);
    C.src.nx = g.nx;
    C.src.ny = g.ny;
    C.src.w = g.w;
    C.src.fx = dens;
    C.src.fy = dens + n;
    C.trg = s2d_targets{};
    C.trg.n = n;
    C.trg.x = x;
    C.trg.y = y;
    C.trg.on_curve = oc;
    C.trg.on_node = on;
    C.nm = 0;
    if (p->near && n > 0) {
        char *b = C.ws;
        double *box = (double *)(b + C.L.nbox);
        int32_t *cnt = (int32_t *)(b + C.L.ncnt);
        int64_t *pos = (int64_t *)(b + C.L.npos);
        int32_t *pn = (int32_t *)(b + C.L.pnode), *pc = (int32_t *)(b + C.L.pcurve);
        double *px = (double *)(b + C.L.px), *py = (double *)(b + C.L.py);
        hipLaunchKernelGGL(ves_near_box, dim3(nc), dim3(256), 0, C.st, n, off, x, y, g.w, box);
        hipLaunchKernelGGL(ves_near_pairs<false>, dim3(g256(n)), dim3(256), 0, C.st, n, nc, off, oc, x, y, box, p->d,
                           p->img_lo, p->img_hi, p->near_band, cnt, pos, pn, pc, px, py);
        hipLaunchKernelGGL(ves_near_scan, dim3(1), dim3(1024), 0, C.st, n, cnt, pos);
        int64_t total = 0;
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&total, pos + n, sizeof(int64_t), hipMemcpyDeviceToHost, C.st);
        if (e == hipSuccess) e = hipStreamSynchronize(C.st);
        if (e != hipSuccess) return hipf(e, "near pairs");
        if (total > p->near_max)
            return ves_fail(S2D_EINVAL, std::to_string(total) + " near pairs exceed near_max = " +
                                            std::to_string(p->near_max));
        if (total > 0) {
            hipLaunchKernelGGL(ves_near_pairs<true>, dim3(g256(n)), dim3(256), 0, C.st, n, nc, off, oc, x, y, box,
                               p->d, p->img_lo, p->img_hi, p->near_band, cnt, pos, pn, pc, px, py);
            e = hipGetLastError();
            if (e != hipSuccess) return hipf(e, "near pairs");
        }
        C.nm = total;
    }
    return S2D_OK;
}

#define S2D_TRY(x)                          \
    do {                                    \
        const int rc_ = (x);                \
        if (rc_ != S2D_OK) return rc_;      \
    } while (0)

// out = A z (RHS = false) or out = b (RHS = true, z unused), single-layer
// sums in `mode`
template <bool RHS>
int apply(StepCtx &C, const double *z, double *out, int mode) {
    OpArgs a{};
    a.n = C.n;
    a.off = C.off;
    a.x = C.x;
    a.y = C.y;
    a.z = z;
    a.dt = C.p->dt;
    a.kb = C.p->kappa_b;
    a.L0 = C.p->L0;
    a.urx = C.p->u_resp_x;
    a.ury = C.p->u_resp_y;
    a.fx = (double *)C.src.fx;
    a.fy = (double *)C.src.fy;
    a.out = out;
    hipLaunchKernelGGL(ves_op_kernel<RHS>, dim3(C.nc), dim3(kVesBlock), 0, C.st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipf(e, "vesicle operator launch");
    S2D_TRY(stokes2d_slp_eval(mode, &C.src, &C.trg, C.p->d, C.p->img_lo, C.p->img_hi, C.p->mu, out, out + C.n, 1,
                              C.ws + C.L.slp, C.L.slp_bytes, C.st));
    if (C.nm > 0) {
        // close evaluation: the upsampled records of every vesicle's layer
        // for this density, the corrections at the near pairs, summed per node
        char *b = C.ws;
        double *up = (double *)(b + C.L.up), *du = (double *)(b + C.L.pdu), *dv = (double *)(b + C.L.pdv);
        s2d_targets nt{};
        nt.n = C.nm;
        nt.x = (const double *)(b + C.L.px);
        nt.y = (const double *)(b + C.L.py);
        e = near_launch_upsample(&C.src, C.p->near_P, up, C.st);
        if (e == hipSuccess)
            e = near_launch_quad(&C.src, &nt, (const int32_t *)(b + C.L.pcurve), nullptr, nullptr, C.p->near_P, up,
                                 C.p->mu, du, dv, C.st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(ves_near_add, dim3(g256(C.n)), dim3(256), 0, C.st, C.n,
                               (const int64_t *)(b + C.L.npos), du, dv, out);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return hipf(e, "close evaluation");
    }
    return S2D_OK;
}

// dots[j] = V_j . w, j < k1, read back to the host
int dots(StepCtx &C, int k1, const double *V, const double *w, double *host) {
    const int64_t len = 3 * C.n;
    double *part = (double *)(C.ws + C.L.part), *d = (double *)(C.ws + C.L.dots);
    hipLaunchKernelGGL(vec_dots_kernel, dim3(kDotBlocks), dim3(256), 0, C.st, len, k1, V, len, w, part);
    hipLaunchKernelGGL(vec_dots_final, dim3((k1 + 63) / 64), dim3(64), 0, C.st, kDotBlocks, k1, part, d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(host, d, k1 * sizeof(double), hipMemcpyDeviceToHost, C.st);
    if (e == hipSuccess) e = hipStreamSynchronize(C.st);
    return e == hipSuccess ? S2D_OK : hipf(e, "GMRES dot products");
}

int combo(StepCtx &C, int k1, const double *V, const double *c, double sw, double *w) {
    Coefs k{};
    for (int j = 0; j < k1; ++j) k.c[j] = c[j];
    const int64_t len = 3 * C.n;
    hipLaunchKernelGGL(vec_combo_kernel, dim3(g256(len)), dim3(256), 0, C.st, len, k1, V, len, k, sw, w);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? S2D_OK : hipf(e, "GMRES vector update");
}

int axpby(StepCtx &C, double a, const double *x, double b, const double *y, double *out) {
    const int64_t len = 3 * C.n;
    hipLaunchKernelGGL(vec_axpby_kernel, dim3(g256(len)), dim3(256), 0, C.st, len, a, x, b, y, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? S2D_OK : hipf(e, "GMRES vector update");
}

int rbf(rocblas_status s, const char *what) {
    return s == rocblas_status_success ? S2D_OK
                                       : ves_fail(S2D_EHIP, std::string(what) + ": " + rocblas_status_to_string(s));
}

// Checks the curve table on the host (the preconditioner pads every curve
// to nmax) and builds and factors the blocks.  The caller holds blas_mutex.
int pc_build(StepCtx &C) {
    const int nc = C.nc, Nm = C.p->nmax;
    std::vector<int32_t> off(nc + 1);
    hipError_t e = hipMemcpyAsync(off.data(), C.off, (nc + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, C.st);
    if (e == hipSuccess) e = hipStreamSynchronize(C.st);
    if (e != hipSuccess) return hipf(e, "reading curve_off");
    if (off[0] != 0 || off[nc] != C.n) return ves_fail(S2D_EINVAL, "curve_off must run from 0 to n_nodes");
    for (int c = 0; c < nc; ++c) {
        const int N = off[c + 1] - off[c];
        if (N < 4 || N > Nm || (N & 1))
            return ves_fail(S2D_EINVAL, "curve " + std::to_string(c) + " has " + std::to_string(N) +
                                            " nodes; the preconditioner needs even sizes in 4..nmax");
    }
    char *b = C.ws;
    const double *g = C.geo;
    const int64_t n = C.n;
    PcArgs a{};
    a.n = n;
    a.off = C.off;
    a.Nm = Nm;
    a.x = C.x;
    a.y = C.y;
    a.sp = g;
    a.w = g + n;
    a.nx = g + 2 * n;
    a.ny = g + 3 * n;
    a.tx = g + 4 * n;
    a.ty = g + 5 * n;
    a.dtk = C.p->dt * C.p->kappa_b;
    a.pref = 1.0 / (4.0 * M_PI * C.p->mu);
    a.T = (double *)(b + C.L.T);
    a.Dm = (double *)(b + C.L.Dm);
    a.D4 = (double *)(b + C.L.D4);
    a.Sm = (double *)(b + C.L.Sm);
    a.Bm = (double *)(b + C.L.Bm);
    a.Top = (double *)(b + C.L.Top);
    a.Pm = (double *)(b + C.L.Pm);
    double *D2 = (double *)(b + C.L.D2);
    hipLaunchKernelGGL(pc_fill_ds, dim3(nc), dim3(kVesBlock), 0, C.st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return hipf(e, "preconditioner fill");
    const double one = 1.0, zero = 0.0;
    const rocblas_stride s1 = (rocblas_stride)Nm * Nm;
    // D_s^2 = D_s D_s, D_s^4 = D_s^2 D_s^2
    S2D_TRY(rbf(rocblas_dgemm_strided_batched(C.h, rocblas_operation_none, rocblas_operation_none, Nm, Nm, Nm, &one,
                                              a.Dm, Nm, s1, a.Dm, Nm, s1, &zero, D2, Nm, s1, nc),
                "preconditioner D_s^2"));
    S2D_TRY(rbf(rocblas_dgemm_strided_batched(C.h, rocblas_operation_none, rocblas_operation_none, Nm, Nm, Nm, &one,
                                              D2, Nm, s1, D2, Nm, s1, &zero, a.D4, Nm, s1, nc),
                "preconditioner D_s^4"));
    hipLaunchKernelGGL(pc_fill_b, dim3(nc), dim3(kVesBlock), 0, C.st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return hipf(e, "preconditioner fill");
    S2D_TRY(rbf(rocblas_dgemm_strided_batched(C.h, rocblas_operation_none, rocblas_operation_none, 2 * Nm, 3 * Nm,
                                              2 * Nm, &one, a.Sm, 2 * Nm, 4 * s1, a.Bm, 2 * Nm, 6 * s1, &zero, a.Top,
                                              2 * Nm, 6 * s1, nc),
                "preconditioner S_cc B"));
    hipLaunchKernelGGL(pc_fill_p, dim3(nc), dim3(kVesBlock), 0, C.st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return hipf(e, "preconditioner fill");
    rocblas_int *ipiv = (rocblas_int *)(b + C.L.ipiv), *info = (rocblas_int *)(b + C.L.info);
    S2D_TRY(rbf(rocsolver_dgetrf_strided_batched(C.h, 3 * Nm, 3 * Nm, a.Pm, 3 * Nm, 9 * s1, ipiv, 3 * Nm, info, nc),
                "preconditioner LU"));
    std::vector<rocblas_int> inf(nc);
    e = hipMemcpyAsync(inf.data(), info, nc * sizeof(rocblas_int), hipMemcpyDeviceToHost, C.st);
    if (e == hipSuccess) e = hipStreamSynchronize(C.st);
    if (e != hipSuccess) return hipf(e, "preconditioner LU info");
    for (int c = 0; c < nc; ++c)
        if (inf[c] != 0)
            return ves_fail(S2D_EINVAL, "the preconditioner block of curve " + std::to_string(c) +
                                            " is singular (a circular vesicle leaves the tension's constant "
                                            "mode undetermined)");
    return S2D_OK;
}

// out = P^-1 v
int pc_apply(StepCtx &C, const double *v, double *out) {
    const int nc = C.nc, Nm = C.p->nmax;
    double *rhs = (double *)(C.ws + C.L.rhs);
    hipLaunchKernelGGL(pc_gather, dim3(nc), dim3(256), 0, C.st, C.n, C.off, Nm, v, rhs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipf(e, "preconditioner gather");
    const rocblas_stride s1 = (rocblas_stride)Nm * Nm;
    S2D_TRY(rbf(rocsolver_dgetrs_strided_batched(C.h, rocblas_operation_none, 3 * Nm, 1,
                                                 (double *)(C.ws + C.L.Pm), 3 * Nm, 9 * s1,
                                                 (rocblas_int *)(C.ws + C.L.ipiv), 3 * Nm, rhs, 3 * Nm, 3 * Nm, nc),
                "preconditioner solve"));
    hipLaunchKernelGGL(pc_scatter, dim3(nc), dim3(256), 0, C.st, C.n, C.off, Nm, rhs, out);
    e = hipGetLastError();
    return e == hipSuccess ? S2D_OK : hipf(e, "preconditioner scatter");
}

// Restarted GMRES on A x = rhs from x = 0 (single-layer sums in `mode`),
// right-preconditioned when C.pc; stops at ||rhs - A x|| <= tol ||rhs||
// (explicit residual at every restart) or after max_iter iterations.
int krylov(StepCtx &C, const double *rhs, double rhs_norm, double *x, double tol, int mode, int max_iter,
           int &iters, double &rel) {
    const int64_t len = 3 * C.n;
    const int m = C.p->restart;
    double *r = (double *)(C.ws + C.L.ri), *w = (double *)(C.ws + C.L.w);
    double *V = (double *)(C.ws + C.L.V);
    S2D_TRY(axpby(C, 0.0, rhs, 0.0, nullptr, x));
    iters = 0;
    rel = 0.0;
    if (rhs_norm == 0.0 || !std::isfinite(rhs_norm)) {
        rel = rhs_norm == 0.0 ? 0.0 : rhs_norm;
        return S2D_OK;
    }
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hc(m + 2), h2(m + 2), y(m);
    S2D_TRY(axpby(C, 1.0, rhs, 0.0, nullptr, r));
    double beta = rhs_norm;
    while (true) {
        rel = beta / rhs_norm;
        if (rel <= tol || iters >= max_iter) break;
        S2D_TRY(axpby(C, 1.0 / beta, r, 0.0, nullptr, V));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;          // columns built this cycle
        for (int j = 0; j < m; ++j) {
            double *vj = V + (int64_t)j * len, *vn = V + (int64_t)(j + 1) * len;
            if (C.pc) {
                double *t1 = (double *)(C.ws + C.L.t1);
                S2D_TRY(pc_apply(C, vj, t1));
                S2D_TRY(apply<false>(C, t1, w, mode));
            } else {
                S2D_TRY(apply<false>(C, vj, w, mode));
            }
            // classical Gram-Schmidt, twice
            S2D_TRY(dots(C, j + 1, V, w, hc.data()));
            for (int i = 0; i <= j; ++i) h2[i] = -hc[i];
            S2D_TRY(combo(C, j + 1, V, h2.data(), 1.0, w));
            S2D_TRY(dots(C, j + 1, V, w, h2.data()));
            for (int i = 0; i <= j; ++i) hc[i] += h2[i];
            for (int i = 0; i <= j; ++i) h2[i] = -h2[i];
            S2D_TRY(combo(C, j + 1, V, h2.data(), 1.0, w));
            double ww = 0.0;
            S2D_TRY(dots(C, 1, w, w, &ww));
            const double hn = std::sqrt(ww);
            // Hessenberg column j, previous rotations, a new one
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hc[i];
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            const double a = H[(size_t)j * m + j];
            const double rr = std::hypot(a, hn);
            cs[j] = rr == 0.0 ? 1.0 : a / rr;
            sn[j] = rr == 0.0 ? 0.0 : hn / rr;
            H[(size_t)j * m + j] = rr;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++iters;
            k = j + 1;
            const double res = std::fabs(g[j + 1]) / rhs_norm;
            if (hn == 0.0 || res <= tol || iters >= max_iter) break;
            S2D_TRY(axpby(C, 1.0 / hn, w, 0.0, nullptr, vn));
        }
        // y = H^-1 g (upper triangular k x k), x += V y
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < k; ++l) s -= H[(size_t)i * m + l] * y[l];
            y[i] = s / H[(size_t)i * m + i];
        }
        if (C.pc) {
            // x += P^-1 (V y)
            double *t1 = (double *)(C.ws + C.L.t1), *t2 = (double *)(C.ws + C.L.t2);
            S2D_TRY(combo(C, k, V, y.data(), 0.0, t2));
            S2D_TRY(pc_apply(C, t2, t1));
            S2D_TRY(axpby(C, 1.0, x, 1.0, t1, x));
        } else {
            S2D_TRY(combo(C, k, V, y.data(), 1.0, x));
        }
        // explicit residual r = rhs - A x
        S2D_TRY(apply<false>(C, x, w, mode));
        S2D_TRY(axpby(C, 1.0, rhs, -1.0, w, r));
        double rr2 = 0.0;
        S2D_TRY(dots(C, 1, r, r, &rr2));
        beta = std::sqrt(rr2);
        if (!std::isfinite(beta)) break;
    }
    rel = beta / rhs_norm;
    return S2D_OK;
}

// a correction solve of the refinement needs to gain at least this factor
constexpr double kInnerTol = 1e-4;
constexpr int kMaxRefine = 30;

// The step system A z = b.  FP64: GMRES with FP64 single-layer sums.
// FP32C: iterative refinement; b and every residual b - A z in FP64, each
// correction A dz = r solved by GMRES with FP32C sums to a relative
// kInnerTol (or to what the tolerance still asks), z += dz.
// The solve from z = 0, or (warm) from the z passed in: then GMRES works on
// the residual r = b - A z (FP64) and adds its correction.
int gmres_run(StepCtx &C, double *z, bool warm, int32_t *iters_out, double *res_out) {
    double *b = (double *)(C.ws + C.L.b), *r = (double *)(C.ws + C.L.r), *w = (double *)(C.ws + C.L.w);
    double *dz = (double *)(C.ws + C.L.dz);
    S2D_TRY(apply<true>(C, nullptr, b, S2D_FP64));
    double nb2 = 0.0;
    S2D_TRY(dots(C, 1, b, b, &nb2));
    const double bnorm = std::sqrt(nb2);
    int iters = 0;
    double rel = 0.0;
    // the starting residual and its norm
    double rnorm = bnorm;
    if (warm) {
        S2D_TRY(apply<false>(C, z, w, S2D_FP64));
        S2D_TRY(axpby(C, 1.0, b, -1.0, w, r));
        double rr2 = 0.0;
        S2D_TRY(dots(C, 1, r, r, &rr2));
        rnorm = std::sqrt(rr2);
    }
    if (C.p->mode == S2D_FP64 && !warm) {
        S2D_TRY(krylov(C, b, bnorm, z, C.p->tol, S2D_FP64, C.p->max_iter, iters, rel));
    } else if (C.p->mode == S2D_FP64) {
        rel = bnorm == 0.0 ? 0.0 : rnorm / bnorm;
        if (bnorm > 0.0 && std::isfinite(rnorm) && rel > C.p->tol) {
            double irel = 0.0;
            S2D_TRY(krylov(C, r, rnorm, dz, C.p->tol * bnorm / rnorm, S2D_FP64, C.p->max_iter, iters, irel));
            S2D_TRY(axpby(C, 1.0, z, 1.0, dz, z));
            rel = irel * rnorm / bnorm;
        }
    } else {
        if (!warm) {
            S2D_TRY(axpby(C, 0.0, b, 0.0, nullptr, z));
            S2D_TRY(axpby(C, 1.0, b, 0.0, nullptr, r));
        }
        rel = bnorm == 0.0 ? 0.0 : rnorm / bnorm;
        for (int o = 0; o < kMaxRefine && bnorm > 0.0 && std::isfinite(rnorm); ++o) {
            if (rel <= C.p->tol || iters >= C.p->max_iter) break;
            const double itol = std::max(C.p->tol * bnorm / rnorm, kInnerTol);
            int it = 0;
            double irel = 0.0;
            S2D_TRY(krylov(C, r, rnorm, dz, itol, S2D_FP32C, C.p->max_iter - iters, it, irel));
            iters += it;
            S2D_TRY(axpby(C, 1.0, z, 1.0, dz, z));
            S2D_TRY(apply<false>(C, z, w, S2D_FP64));
            S2D_TRY(axpby(C, 1.0, b, -1.0, w, r));
            double rr2 = 0.0;
            S2D_TRY(dots(C, 1, r, r, &rr2));
            const double next = std::sqrt(rr2);
            const bool stalled = !(next < 0.5 * rnorm);
            rnorm = next;
            rel = rnorm / bnorm;
            if (stalled) break;
        }
    }
    if (iters_out) *iters_out = iters;
    if (res_out) *res_out = rel;
    return S2D_OK;
}

// the step system, right-preconditioned when asked
int gmres(StepCtx &C, double *z, int32_t *iters_out, double *res_out) {
    C.pc = C.p->precond != 0;
    const bool warm = C.p->warm != 0;
    if (!C.pc) return gmres_run(C, z, warm, iters_out, res_out);
    std::lock_guard<std::mutex> lk(blas_mutex());
    std::string err;
    C.h = (rocblas_handle)blas_handle(C.st, err);
    if (!C.h) return ves_fail(S2D_EHIP, err);
    S2D_TRY(pc_build(C));
    return gmres_run(C, z, warm, iters_out, res_out);
}

}  // namespace

}  // namespace s2d

using namespace s2d;

extern "C" {

S2D_API int ves_geometry(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off, const double *x,
                         const double *y, double *speed, double *w, double *nx, double *ny, double *tx, double *ty,
                         void *stream) {
    int rc = check_set(n_nodes, n_curves, curve_off, x, y);
    if (rc != S2D_OK) return rc;
    int dev = 0;
    rc = device_ready(&dev);
    if (rc != S2D_OK || n_nodes == 0) return rc;
    GeomOut g{speed, w, nx, ny, tx, ty};
    hipLaunchKernelGGL(ves_geom_kernel, dim3(n_curves), dim3(kVesBlock), 0, (hipStream_t)stream, n_nodes,
                       curve_off, x, y, g);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? S2D_OK : hipf(e, "ves_geometry launch");
}

S2D_API int ves_forces(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off, const double *x,
                       const double *y, const double *sigma, double kappa_b, double *fbx, double *fby, double *fsx,
                       double *fsy, void *stream) {
    int rc = check_set(n_nodes, n_curves, curve_off, x, y);
    if (rc != S2D_OK) return rc;
    if ((fbx == nullptr) != (fby == nullptr) || (fsx == nullptr) != (fsy == nullptr))
        return ves_fail(S2D_EINVAL, "force outputs come in pairs");
    if (!std::isfinite(kappa_b)) return ves_fail(S2D_EINVAL, "kappa_b must be finite");
    int dev = 0;
    rc = device_ready(&dev);
    if (rc != S2D_OK || n_nodes == 0) return rc;
    hipLaunchKernelGGL(ves_forces_kernel, dim3(n_curves), dim3(kVesBlock), 0, (hipStream_t)stream, n_nodes,
                       curve_off, x, y, sigma, kappa_b, fbx, fby, fsx, fsy, 0);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? S2D_OK : hipf(e, "ves_forces launch");
}

S2D_API int ves_total_force(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off, const double *x,
                            const double *y, const double *sigma, double kappa_b, double *fx, double *fy,
                            void *stream) {
    int rc = check_set(n_nodes, n_curves, curve_off, x, y);
    if (rc != S2D_OK) return rc;
    if (n_nodes > 0 && (!fx || !fy)) return ves_fail(S2D_EINVAL, "fx and fy must not be NULL");
    if (!std::isfinite(kappa_b)) return ves_fail(S2D_EINVAL, "kappa_b must be finite");
    int dev = 0;
    rc = device_ready(&dev);
    if (rc != S2D_OK || n_nodes == 0) return rc;
    hipLaunchKernelGGL(ves_forces_kernel, dim3(n_curves), dim3(kVesBlock), 0, (hipStream_t)stream, n_nodes,
                       curve_off, x, y, sigma, kappa_b, fx, fy, nullptr, nullptr, 1);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? S2D_OK : hipf(e, "ves_total_force launch");
}

S2D_API int ves_measure(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off, const double *x,
                        const double *y, double *length, double *area, void *stream) {
    int rc = check_set(n_nodes, n_curves, curve_off, x, y);
    if (rc != S2D_OK) return rc;
    int dev = 0;
    rc = device_ready(&dev);
    if (rc != S2D_OK || n_curves == 0) return rc;
    hipLaunchKernelGGL(ves_measure_kernel, dim3(n_curves), dim3(kVesBlock), 0, (hipStream_t)stream, n_nodes,
                       curve_off, x, y, length, area);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? S2D_OK : hipf(e, "ves_measure launch");
}

S2D_API size_t ves_step_workspace_size(int64_t n_nodes, int32_t n_curves, const ves_step_params *p) {
    if (!p || n_nodes < 0 || n_curves < 0 || n_nodes > INT32_MAX / 4 || p->restart < 1 || p->restart > kMaxRestart ||
        (p->mode != S2D_FP64 && p->mode != S2D_FP32C))
        return 0;
    return step_layout(n_nodes, n_curves, p).total;
}

S2D_API int ves_step_apply(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off, const double *x,
                           const double *y, const ves_step_params *p, const double *z, double *out, double *b,
                           void *ws, size_t ws_bytes, void *stream) {
    int rc = check_set(n_nodes, n_curves, curve_off, x, y);
    if (rc == S2D_OK) rc = check_params(p);
    if (rc != S2D_OK) return rc;
    if (n_nodes > 0 && (!z || !out)) return ves_fail(S2D_EINVAL, "z and out must not be NULL");
    int dev = 0;
    rc = device_ready(&dev);
    if (rc != S2D_OK || n_nodes == 0) return rc;
    StepCtx C{};
    S2D_TRY(setup_ctx(C, n_nodes, n_curves, curve_off, x, y, p, ws, ws_bytes, stream));
    S2D_TRY(apply<false>(C, z, out, p->mode));
    if (b) S2D_TRY(apply<true>(C, nullptr, b, p->mode));
    return S2D_OK;
}

S2D_API int ves_step_solve(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off, const double *x,
                           const double *y, const ves_step_params *p, double *z, int32_t *iters, double *rel_res,
                           void *ws, size_t ws_bytes, void *stream) {
    int rc = check_set(n_nodes, n_curves, curve_off, x, y);
    if (rc == S2D_OK) rc = check_params(p);
    if (rc != S2D_OK) return rc;
    if (n_nodes > 0 && !z) return ves_fail(S2D_EINVAL, "z must not be NULL");
    int dev = 0;
    rc = device_ready(&dev);
    if (rc != S2D_OK) return rc;
    if (n_nodes == 0) {
        if (iters) *iters = 0;
        if (rel_res) *rel_res = 0.0;
        return S2D_OK;
    }
    StepCtx C{};
    S2D_TRY(setup_ctx(C, n_nodes, n_curves, curve_off, x, y, p, ws, ws_bytes, stream));
    return gmres(C, z, iters, rel_res);
}

S2D_API int ves_area_correct(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off, double *x, double *y,
                             const double *A0, void *stream) {
    int rc = check_set(n_nodes, n_curves, curve_off, x, y);
    if (rc != S2D_OK) return rc;
    if (n_curves > 0 && !A0) return ves_fail(S2D_EINVAL, "A0 must not be NULL");
    int dev = 0;
    rc = device_ready(&dev);
    if (rc != S2D_OK || n_nodes == 0) return rc;
    hipLaunchKernelGGL(ves_area_kernel, dim3(n_curves), dim3(kVesBlock), 0, (hipStream_t)stream, n_nodes,
                       curve_off, x, y, A0);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? S2D_OK : hipf(e, "ves_area_correct launch");
}

S2D_API int ves_reparameterize(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off, double *x, double *y,
                               double *sigma, void *stream) {
    int rc = check_set(n_nodes, n_curves, curve_off, x, y);
    if (rc != S2D_OK) return rc;
    int dev = 0;
    rc = device_ready(&dev);
    if (rc != S2D_OK || n_nodes == 0) return rc;
    hipLaunchKernelGGL(ves_reparam_kernel, dim3(n_curves), dim3(kVesBlock), 0, (hipStream_t)stream, n_nodes,
                       curve_off, x, y, sigma);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? S2D_OK : hipf(e, "ves_reparameterize launch");
}

S2D_API int ves_time_step(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off, double *x, double *y,
                          double *sigma, const ves_step_params *p, const double *A0, int reparam, double *u,
                          double *v, int32_t *iters, double *rel_res, void *ws, size_t ws_bytes, void *stream) {
    int rc = check_set(n_nodes, n_curves, curve_off, x, y);
    if (rc == S2D_OK) rc = check_params(p);
    if (rc != S2D_OK) return rc;
    if (n_nodes > 0 && !sigma) return ves_fail(S2D_EINVAL, "sigma must not be NULL");
    int dev = 0;
    rc = device_ready(&dev);
    if (rc != S2D_OK) return rc;
    if (n_nodes == 0) {
        if (iters) *iters = 0;
        if (rel_res) *rel_res = 0.0;
        return S2D_OK;
    }
    if (p->warm && (!u || !v)) return ves_fail(S2D_EINVAL, "a warm start needs u and v (the previous velocity)");
    StepCtx C{};
    S2D_TRY(setup_ctx(C, n_nodes, n_curves, curve_off, x, y, p, ws, ws_bytes, stream));
    double *z = (double *)(C.ws + C.L.z);
    if (p->warm) {
        // the starting guess (u, v, sigma): the previous step's velocity and
        // the current tension
        const size_t nb = (size_t)n_nodes * sizeof(double);
        hipError_t e = hipMemcpyAsync(z, u, nb, hipMemcpyDeviceToDevice, C.st);
        if (e == hipSuccess) e = hipMemcpyAsync(z + n_nodes, v, nb, hipMemcpyDeviceToDevice, C.st);
        if (e == hipSuccess) e = hipMemcpyAsync(z + 2 * n_nodes, sigma, nb, hipMemcpyDeviceToDevice, C.st);
        if (e != hipSuccess) return hipf(e, "warm start copy");
    }
    S2D_TRY(gmres(C, z, iters, rel_res));
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(ves_update_kernel, dim3(g256(n_nodes)), dim3(256), 0, st, n_nodes, z, p->dt, x, y, sigma, u,
                       v);
    if (A0)
        hipLaunchKernelGGL(ves_area_kernel, dim3(n_curves), dim3(kVesBlock), 0, st, n_nodes, curve_off, x, y, A0);
    if (reparam)
        hipLaunchKernelGGL(ves_reparam_kernel, dim3(n_curves), dim3(kVesBlock), 0, st, n_nodes, curve_off, x, y,
                           sigma);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? S2D_OK : hipf(e, "ves_time_step launch");
}

}  // extern "C"
