#pragma once
// Pair-sum kernels: Stokeslet single layer (Section 2.1 Eq. (S), summed over
// the near images of Section 3.1 Eq. (utotrep)) and stresslet double layer
// (Eq. (D), summed as Eq. (Dnr)), for every target against every source node
// of a curve set and its images n = img_lo..img_hi; and, at free targets, the
// pressures of both layers (Section 2.1 Eqs. (Q), (P)) and the single-layer
// traction (Eq. (K)), which share the double layer's rational-term paths.
//
// Work decomposition.  A wavefront owns kWave * TPT targets (TPT per lane,
// lane-strided so target loads are coalesced) and one source split (a run of
// superblocks of kSuperBlock sources).  Every lane of a wave walks the same
// sources in the same order, so each source record is wave-uniform: it is
// fetched through the scalar data path into SGPRs (no LDS staging, no
// barriers) and used as the SGPR operand of the vector ALU instructions.
// pair_sum() returns a wave's sum over its split; the single-call kernel
// (pair.hip) adds the splits of one target tile held by the waves of a
// workgroup, and the batched kernel writes one partial per split.  Both
// reduce in a fixed order (deterministic, no atomics).
//
// Images.  The images of a call are taken in groups of NI consecutive ones
// (NI = 3 when the image count is a multiple of 3, as for the n = -1, 0, 1
// sum of Eq. (utotrep); else NI = 1).  Within a group each source record is
// used for all NI images at once: the y offset, its square and its products
// with the source data are shared, and the single layer's log term, whose
// density factor is the same for every image, takes one logarithm of the
// product of the NI squared distances (sum_n g log q_n = g log prod_n q_n).
//
// Exclusions.  For a target that is node i of source curve c, the single
// layer skips curve c at n = 0 (Kress's rule covers it elsewhere) and the
// double layer skips node i at n = 0 (the diagonal limit covers it).  A wave
// folds its targets' excluded index ranges into one hull; a superblock that
// meets the hull in a group holding n = 0 takes a masked path that goes
// image by image with a per-pair select (it also skips the padding records
// past the last source).  All other superblocks, the ragged last one
// included, take the unmasked path.
//
// Precision.  FP64 mode evaluates each term in double.  FP32C mode evaluates
// each term in float with the hardware log2 and reciprocal, sums a sub-block
// of kSubBlock sources in float (single-layer log and rational parts and odd
// and even sources in separate accumulators, halving the length of each
// float sum) and merges it into double accumulators.  The
// difference r is formed, per sub-block and wave, either from FP32 offsets to
// the sub-block's FP64 origin (when every target of the wave is at least
// kFarRadii sub-block radii away from it at every image of the group, so r
// keeps a relative error of a few roundings) or in double and rounded once
// (near sub-blocks, so near pairs keep one-rounding relative accuracy).  For
// the single-layer log term a per-(target, superblock, image group)
// reference factor, the power of two nearest below the product of the
// images' squared distances to the superblock's first source, is divided out
// (exactly) before the float log2, and its log, an integer times ln 2, is
// added back in double against the superblock's FP64 density sum, so the
// float logs stay O(1) in magnitude.
#include "s2d_internal.h"
#include <type_traits>

#include <climits>

namespace s2d {

// Read-only view of a workspace array that the reading kernel never writes
// (source records, sub-block descriptors, superblock sums; all written by an
// earlier launch).  Reads through the constant address space are invariant
// for the kernel, so wave-uniform ones use scalar loads also where they
// follow the kernel's own stores (the persistent batched loop), not only
// before them.
template <class T>
using cview = const __attribute__((address_space(4))) T *;

// Element i of an array of T (trivially copyable, a whole number of dwords)
// read through such a view, one dword at a time (adjacent scalar loads are
// merged into wide ones) and reassembled.
template <class T>
__device__ __forceinline__ T load_ro(const void *base, int64_t i) {
    static_assert(sizeof(T) % 4 == 0, "whole dwords only");
    constexpr int n = (int)(sizeof(T) / 4);
    const cview<uint32_t> p = (cview<uint32_t>)((const char *)base + i * (int64_t)sizeof(T));
    struct Words {
        uint32_t w[n];
    } t;
#pragma unroll
    for (int k = 0; k < n; ++k) t.w[k] = p[k];
    return __builtin_bit_cast(T, t);
}


// 1/q: the hardware seed (measured relative error below 5e-8) and one
// Newton step, relative error about 2e-15.
__device__ __forceinline__ double rcp64(double q) {
    double y = __builtin_amdgcn_rcp(q);
    double e = __builtin_fma(-q, y, 1.0);
    return __builtin_fma(y, e, y);
}

// Natural log of a positive, finite, normal double (q = |r|^2 here), from
// the reduction x = 2^e m with m in [sqrt(1/2), sqrt(2)) and
// log m = 2 atanh(s), s = (m - 1) / (m + 1), |s| <= 0.1716, summed as the
// odd series 2 (s + s^3/3 + ... + s^23/23): the first omitted term is below
// 1e-18 relative.  Error: a few ulp, from the rounding of m + 1 and of the
// reciprocal.  Zero or negative input gives a finite meaningless value (the
// callers mask those pairs out).
__device__ __forceinline__ double log64(double x) {
    int e = __builtin_amdgcn_frexp_exp(x);             // x = m 2^e, m in [0.5, 1)
    double m = __builtin_amdgcn_frexp_mant(x);
    const bool lo = m < 0.70710678118654752440;
    m = lo ? m + m : m;
    e = lo ? e - 1 : e;
    const double f = m - 1.0;
    const double s = f * rcp64(2.0 + f);
    const double z = s * s;
    double p = 2.0 / 23.0;
    p = __builtin_fma(p, z, 2.0 / 21.0);
    p = __builtin_fma(p, z, 2.0 / 19.0);
    p = __builtin_fma(p, z, 2.0 / 17.0);
    p = __builtin_fma(p, z, 2.0 / 15.0);
    p = __builtin_fma(p, z, 2.0 / 13.0);
    p = __builtin_fma(p, z, 2.0 / 11.0);
    p = __builtin_fma(p, z, 2.0 / 9.0);
    p = __builtin_fma(p, z, 2.0 / 7.0);
    p = __builtin_fma(p, z, 2.0 / 5.0);
    p = __builtin_fma(p, z, 2.0 / 3.0);
    const double lm = __builtin_fma(s * z, p, s + s);  // log m
    const double de = (double)e;
    // ln 2 split so that de * kLn2Hi is exact for |e| < 2^11
    constexpr double kLn2Hi = 6.93147180369123816490e-01;
    constexpr double kLn2Lo = 1.90821492927058770002e-10;
    return __builtin_fma(de, kLn2Hi, __builtin_fma(de, kLn2Lo, lm));
}

// Table-driven natural log (Tang's method) of a positive, finite, normal
// double: x = 2^e m, m in [1/2, 1); the top 9 mantissa bits pick the
// breakpoint F_k = 1/2 + (k + 1/2) / 1024, and
// log x = e ln 2 + log F_k + log1p(u), u = m / F_k - 1, |u| <= 2^-10.
// u is formed as one FMA m (1/F_k) - 1 (error below 2^-52 from the rounding
// of 1/F_k), log1p is summed to u^4 (first omitted term below 1.8e-16), and
// e ln 2 is one rounded product: absolute error below 1e-15 for the |e| of
// squared distances, far inside the FP64 path's 1e-12 budget.  tab holds the
// pairs {1/F_k, log F_k} (2 x kLogTab doubles, staged in LDS by
// fill_log_table; one 16-byte LDS read per call).
constexpr int kLogTab = 512;
constexpr int kLogTabWords = 2 * kLogTab;

__device__ __forceinline__ double log64_tab(double x, const double *tab) {
    const int e = __builtin_amdgcn_frexp_exp(x);
    const double m = __builtin_amdgcn_frexp_mant(x);
    const uint32_t hi = (uint32_t)(__builtin_bit_cast(uint64_t, x) >> 32);
    const int k = (hi >> 11) & (kLogTab - 1);
    typedef double double2_t __attribute__((ext_vector_type(2)));
    const double2_t t = ((const double2_t *)tab)[k];     // {1/F_k, log F_k}
    const double u = __builtin_fma(m, t.x, -1.0);
    // log1p(u) = u + u^2 (-1/2 + u/3 - u^2/4): each FMA takes at most one
    // non-inline constant
    const double v = u * u;
    double c = __builtin_fma(u, 1.0 / 3.0, -0.5);
    c = __builtin_fma(v, -0.25, c);
    const double l1p = __builtin_fma(v, c, u);
    constexpr double kLn2 = 6.93147180559945286227e-01;
    return __builtin_fma((double)e, kLn2, t.y + l1p);
}

// Called by every thread of a workgroup before any of them uses the table
// (a __shared__ array of kLogTabWords doubles, 16-byte aligned).
__device__ __forceinline__ void fill_log_table(double *tab) {
    for (int k = threadIdx.x; k < kLogTab; k += blockDim.x) {
        const double F = 0.5 + ((double)k + 0.5) / (2.0 * kLogTab);
        tab[2 * k] = 1.0 / F;
        tab[2 * k + 1] = log64(F);
    }
    __syncthreads();
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m, kWave));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m, kWave));
    return v;
}




// ---------------------------------------------------------------------------
// per-source terms over a group of NI images
// ---------------------------------------------------------------------------
// ln 2 / 2: FP32C single-layer log sums are taken in log2 and scaled once per
// sub-block, -1/2 ln q = -(ln 2 / 2) log2 q
constexpr double kHalfLn2 = 0.34657359027997265471;
#ifndef SLP32_UNROLL
#define SLP32_UNROLL 8
#endif

// FP64 single layer of one source at the NI target positions px[m] (the
// target minus image m's shift) and height py: accumulates A += g log q
// (one log of the product of the NI squared distances) and B += r (r.g)/q.
template <int NI>
__device__ __forceinline__ void slp64_src(const double (&px)[NI], double py, const RecSlp64 &s, const double *ltab,
                                          double &ax, double &ay, double &bx, double &by) {
    const double ry = py - s.y;
    const double ry2 = ry * ry, rgy = ry * s.gy;
    double P = 1.0, ts = 0.0;
#pragma unroll
    for (int m = 0; m < NI; ++m) {
        const double rx = px[m] - s.x;
        const double q = __builtin_fma(rx, rx, ry2);
        const double t = __builtin_fma(rx, s.gx, rgy) * rcp64(q);
        bx = __builtin_fma(rx, t, bx);
        ts = m == 0 ? t : ts + t;
        P = m == 0 ? q : P * q;
    }
    by = __builtin_fma(ry, ts, by);
    const double lq = log64_tab(P, ltab);
    ax = __builtin_fma(s.gx, lq, ax);
    ay = __builtin_fma(s.gy, lq, ay);
}

// FP32 single layer of one source (density g) for the differences
// (rx[m], ry): a = {sum g_x log2(P), sum g_y log2(P), rat x, rat y} with
// P = iqr prod_m q_m (iqr: the power-of-two reference factor, see the file
// comment).  The rational term is taken in the form
//   r (r.g)/q = (g_x (1 - ry^2/q) + g_y rx ry/q,  g_x rx ry/q + g_y ry^2/q),
// so the images enter only through S0 = sum_m 1/q_m and S1 = sum_m rx_m/q_m
// (ry is the same for every image): with C = ry S1 and D = ry^2 S0 the
// accumulators take (-D g_x + C g_y, C g_x + D g_y), and the constant NI g_x
// of the x component is added per superblock from its FP64 density sum.
// With NI = 1 the term is taken directly (a[2], a[3] then hold the whole
// rational term).
template <int NI>
__device__ __forceinline__ void slp32_src(const float (&rx)[NI], float ry, float gx, float gy, float iqr,
                                          float (&a)[4]) {
    const float ry2 = ry * ry;
    if constexpr (NI == 1) {
        // one image: r (r.g)/q directly (cheaper than the shared form, and
        // no constant to add back)
        const float q = __builtin_fmaf(rx[0], rx[0], ry2);
        const float t = __builtin_fmaf(rx[0], gx, ry * gy) * __builtin_amdgcn_rcpf(q);
        a[2] = __builtin_fmaf(rx[0], t, a[2]);
        a[3] = __builtin_fmaf(ry, t, a[3]);
        const float lq = __builtin_amdgcn_logf(q * iqr);
        a[0] = __builtin_fmaf(gx, lq, a[0]);
        a[1] = __builtin_fmaf(gy, lq, a[1]);
        return;
    }
    float P = 1.f, s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int m = NI - 1; m >= 0; --m) {
        const float q = __builtin_fmaf(rx[m], rx[m], ry2);
        const float iq = __builtin_amdgcn_rcpf(q);
        s0 = m == NI - 1 ? iq : s0 + iq;
        s1 = m == NI - 1 ? rx[m] * iq : __builtin_fmaf(rx[m], iq, s1);
        P = m == NI - 1 ? q * iqr : P * q;     // the scaled factor first
    }
    const float C = ry * s1, D = ry2 * s0;
    a[2] = __builtin_fmaf(gy, C, __builtin_fmaf(-gx, D, a[2]));
    a[3] = __builtin_fmaf(gx, C, __builtin_fmaf(gy, D, a[3]));
    const float lq = __builtin_amdgcn_logf(P);     // log2
    a[0] = __builtin_fmaf(gx, lq, a[0]);
    a[1] = __builtin_fmaf(gy, lq, a[1]);
}

// FP64 double layer of one source over NI images: u += r (r.nu)(r.tau)/q^2
template <int NI>
__device__ __forceinline__ void dlp64_src(const double (&px)[NI], double py, const RecDlp64 &s, double &ux,
                                          double &uy) {
    const double ry = py - s.y;
    const double ry2 = ry * ry, rny = ry * s.ny, rty = ry * s.ty;
    double fs = 0.0;
#pragma unroll
    for (int m = 0; m < NI; ++m) {
        const double rx = px[m] - s.x;
        const double q = __builtin_fma(rx, rx, ry2);
        const double iq = rcp64(q);
        const double rn = __builtin_fma(rx, s.nx, rny);
        const double rt = __builtin_fma(rx, s.tx, rty);
        const double f = (rn * rt) * (iq * iq);
        ux = __builtin_fma(rx, f, ux);
        fs = m == 0 ? f : fs + f;
    }
    uy = __builtin_fma(ry, fs, uy);
}

// FP32 double layer of one source for the differences (rx[m], ry),
// accumulators a = {x, y}
template <int NI>
__device__ __forceinline__ void dlp32_src(const float (&rx)[NI], float ry, const RecDlp32 &s, float (&a)[2]) {
    const float ry2 = ry * ry, rny = ry * s.ny, rty = ry * s.ty;
    float fs = 0.f;
#pragma unroll
    for (int m = 0; m < NI; ++m) {
        const float q = __builtin_fmaf(rx[m], rx[m], ry2);
        const float iq = __builtin_amdgcn_rcpf(q);
        const float rn = __builtin_fmaf(rx[m], s.nx, rny);
        const float rt = __builtin_fmaf(rx[m], s.tx, rty);
        const float f = (rn * rt) * (iq * iq);
        a[0] = __builtin_fmaf(rx[m], f, a[0]);
        fs = m == 0 ? f : fs + f;
    }
    a[1] = __builtin_fmaf(ry, fs, a[1]);
}

// ---------------------------------------------------------------------------
// rational operators (no logarithm), one image at a time: the double-layer
// velocity, the pressures of both layers and the single-layer traction.
// Each adds its term for r = (rx, ry) to the accumulators (ax, ay); the
// pressures use ax only.  m = (mx, my) is the target normal (traction only).
// ---------------------------------------------------------------------------
template <int OP>
using Rec64Of = typename std::conditional<slp_sources(OP), RecSlp64, RecDlp64>::type;
template <int OP>
using Rec32Of = typename std::conditional<slp_sources(OP), RecSlp32, RecDlp32>::type;

template <int OP>
__device__ __forceinline__ void rat64(double px, double py, const Rec64Of<OP> &s, double mx, double my,
                                      double &ax, double &ay) {
    if constexpr (OP == S2D_OP_DLP) {
        const double p1[1] = {px};
        dlp64_src<1>(p1, py, s, ax, ay);
    } else {
        const double rx = px - s.x, ry = py - s.y;
        const double q = __builtin_fma(rx, rx, ry * ry);
        const double iq = rcp64(q);
        if constexpr (OP == S2D_OP_DLP_PRESSURE) {
            // -(nu . tau) / q + 2 (r . nu)(r . tau) / q^2
            const double rn = __builtin_fma(rx, s.nx, ry * s.ny);
            const double rt = __builtin_fma(rx, s.tx, ry * s.ty);
            const double nt = __builtin_fma(s.nx, s.tx, s.ny * s.ty);
            ax = __builtin_fma(iq, __builtin_fma(2.0 * rn * rt, iq, -nt), ax);
        } else if constexpr (OP == S2D_OP_SLP_PRESSURE) {
            // (r . g) / q
            ax = __builtin_fma(__builtin_fma(rx, s.gx, ry * s.gy), iq, ax);
        } else {
            // traction: r (r . g)(r . m) / q^2
            const double rg = __builtin_fma(rx, s.gx, ry * s.gy);
            const double rm = __builtin_fma(rx, mx, ry * my);
            const double f = (rg * rm) * (iq * iq);
            ax = __builtin_fma(rx, f, ax);
            ay = __builtin_fma(ry, f, ay);
        }
    }
}

template <int OP>
__device__ __forceinline__ void rat32(float rx, float ry, const Rec32Of<OP> &s, float mx, float my,
                                      float (&a)[2]) {
    if constexpr (OP == S2D_OP_DLP) {
        const float r1[1] = {rx};
        dlp32_src<1>(r1, ry, s, a);
    } else {
        const float q = __builtin_fmaf(rx, rx, ry * ry);
        const float iq = __builtin_amdgcn_rcpf(q);
        if constexpr (OP == S2D_OP_DLP_PRESSURE) {
            const float rn = __builtin_fmaf(rx, s.nx, ry * s.ny);
            const float rt = __builtin_fmaf(rx, s.tx, ry * s.ty);
            const float nt = __builtin_fmaf(s.nx, s.tx, s.ny * s.ty);
            a[0] = __builtin_fmaf(iq, __builtin_fmaf(2.0f * rn * rt, iq, -nt), a[0]);
        } else if constexpr (OP == S2D_OP_SLP_PRESSURE) {
            a[0] = __builtin_fmaf(__builtin_fmaf(rx, s.gx, ry * s.gy), iq, a[0]);
        } else {
            const float rg = __builtin_fmaf(rx, s.gx, ry * s.gy);
            const float rm = __builtin_fmaf(rx, mx, ry * my);
            const float f = (rg * rm) * (iq * iq);
            a[0] = __builtin_fmaf(rx, f, a[0]);
            a[1] = __builtin_fmaf(ry, f, a[1]);
        }
    }
}

// Offsets of the targets from sub-block origin si in FP32 at each image of
// the group, and whether every active target of the wave is at least
// kFarRadii sub-block radii away at every image (then r = offset - local
// source offset has a relative error of a few roundings).
template <int TPT, int NI>
__device__ __forceinline__ bool far_offsets(const SubInfo &si, const double (&px)[TPT][NI], const double (&py)[TPT],
                                            const bool (&act)[TPT], float (&dx)[TPT][NI], float (&dy)[TPT]) {
    bool far = true;
    const float r2 = (float)si.r2;
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        dy[k] = (float)(py[k] - si.oy);
        const float dy2 = dy[k] * dy[k];
#pragma unroll
        for (int m = 0; m < NI; ++m) {
            dx[k][m] = (float)(px[k][m] - si.ox);
            far = far && (!act[k] || __builtin_fmaf(dx[k][m], dx[k][m], dy2) >= r2);
        }
    }
    return __all(far);
}

// ---------------------------------------------------------------------------
// one wave: targets [tile * kWave * TPT, +kWave * TPT) against source split
// `split` (empty past the last superblock), images img_lo..img_hi in groups
// of NI (the image count must be a multiple of NI); returns the FP64 sums
// (ox, oy) of its targets, without the operator's prefactor
// ---------------------------------------------------------------------------
template <int OP, int PREC, int TPT, int NI>
__device__ __forceinline__ void pair_sum(const PairArgs &a, int64_t tile, int split, int lane, const double *ltab,
                                         double (&ox)[TPT], double (&oy)[TPT]) {

    double tx[TPT], ty[TPT];
    int lo[TPT], hi[TPT];
    int64_t ti[TPT];
    bool act[TPT];
    int hlo = INT_MAX, hhi = INT_MIN;
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        ti[k] = tile * (int64_t)(kWave * TPT) + k * kWave + lane;
        act[k] = ti[k] < a.n_trg;
        tx[k] = act[k] ? a.tx[ti[k]] : 0.0;
        ty[k] = act[k] ? a.ty[ti[k]] : 0.0;
        lo[k] = 0;
        hi[k] = 0;
        if (act[k] && a.on_curve) {
            const int c = a.on_curve[ti[k]];
            if (c >= 0 && c < a.n_curves) {
                if (OP == S2D_OP_SLP) {
                    lo[k] = a.curve_off[c];
                    hi[k] = a.curve_off[c + 1];
                } else {
                    const int j = a.on_node[ti[k]];
                    if (j >= a.curve_off[c] && j < a.curve_off[c + 1]) { lo[k] = j; hi[k] = j + 1; }
                }
            }
        }
        if (lo[k] < hi[k]) { hlo = min(hlo, lo[k]); hhi = max(hhi, hi[k]); }
    }
    hlo = __builtin_amdgcn_readfirstlane(wave_min(hlo));
    hhi = __builtin_amdgcn_readfirstlane(wave_max(hhi));
    double mx[TPT], my[TPT];                        // target normals (traction only)
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const bool tr = OP == S2D_OP_SLP_TRACTION && act[k];
        mx[k] = tr ? a.tnx[ti[k]] : 0.0;
        my[k] = tr ? a.tny[ti[k]] : 0.0;
    }

    // superblock range of the split, wave-uniform: the loop runs on the scalar
    // unit and the record addresses it forms stay scalar (n_sb < 2^31)
    const int sb0 = __builtin_amdgcn_readfirstlane((int)min((int64_t)split * a.sb_per_split, a.n_sb));
    const int sb1 = __builtin_amdgcn_readfirstlane((int)min((int64_t)sb0 + a.sb_per_split, a.n_sb));

    double ux[TPT], uy[TPT], vx[TPT], vy[TPT];     // vx, vy: FP64 single-layer log accumulators
#pragma unroll
    for (int k = 0; k < TPT; ++k) { ux[k] = uy[k] = vx[k] = vy[k] = 0.0; }

    for (int n0 = a.img_lo; n0 <= a.img_hi; n0 += NI) {
        double px[TPT][NI], py[TPT];
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
            py[k] = ty[k];
#pragma unroll
            for (int m = 0; m < NI; ++m) px[k][m] = tx[k] - (double)(n0 + m) * a.d;
        }
        const bool has0 = n0 <= 0 && 0 < n0 + NI;

        for (int sb = sb0; sb < sb1; ++sb) {
            const int64_t j0 = (int64_t)sb * kSuperBlock;
            const int64_t j1 = min(j0 + (int64_t)kSuperBlock, a.n_src);
            // padding records are zero-density copies of the last source: a ragged
            // superblock needs no mask
            const bool masked = has0 && hlo < hhi && j0 < hhi && (int64_t)hlo < j0 + kSuperBlock;
            if (!masked) {
                // ---------------- unmasked superblock ----------------
                if (PREC == S2D_FP64) {
                    if (OP == S2D_OP_SLP) {
                        const RecSlp64 *rec = (const RecSlp64 *)a.rec + j0;
                        for (int u = 0; u < kSuperBlock; u += 4) {
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const RecSlp64 s = load_ro<RecSlp64>(rec, u + q);
#pragma unroll
                                for (int k = 0; k < TPT; ++k)
                                    slp64_src<NI>(px[k], py[k], s, ltab, vx[k], vy[k], ux[k], uy[k]);
                            }
                        }
                    } else if (OP == S2D_OP_DLP) {
                        const RecDlp64 *rec = (const RecDlp64 *)a.rec + j0;
                        for (int u = 0; u < kSuperBlock; u += 4) {
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const RecDlp64 s = load_ro<RecDlp64>(rec, u + q);
#pragma unroll
                                for (int k = 0; k < TPT; ++k) dlp64_src<NI>(px[k], py[k], s, ux[k], uy[k]);
                            }
                        }
                    } else {
                        using R = Rec64Of<OP>;
                        const R *rec = (const R *)a.rec + j0;
                        for (int u = 0; u < kSuperBlock; u += 4) {
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const R s = load_ro<R>(rec, u + q);
#pragma unroll
                                for (int k = 0; k < TPT; ++k)
#pragma unroll
                                    for (int m = 0; m < NI; ++m)
                                        rat64<OP>(px[k][m], py[k], s, mx[k], my[k], ux[k], uy[k]);
                            }
                        }
                    }
                } else {
                    if (OP == S2D_OP_SLP) {
                        const RecSlp32 *rec = (const RecSlp32 *)a.rec + j0;
                        // log reference: the superblock's first source at every image of the group
                        float iqr[TPT];
                        const double gsx = load_ro<double>(a.sbsum, 2 * sb), gsy = load_ro<double>(a.sbsum, 2 * sb + 1);
                        const RecSlp32 r0 = load_ro<RecSlp32>(rec, 0);
#pragma unroll
                        for (int k = 0; k < TPT; ++k) {
                            const double ry0 = py[k] - r0.y;
                            double qp = 1.0;
#pragma unroll
                            for (int m = 0; m < NI; ++m) {
                                const double rx0 = px[k][m] - r0.x;
                                qp *= __builtin_fma(rx0, rx0, ry0 * ry0);
                            }
                            // iqr = 2^-e with qp = m 2^e, m in [1/2, 1): scaling by it is exact in
                            // float, and -1/2 sum g ln prod q = -(ln2/2) sum g log2(iqr prod q)
                            // - (ln2/2) e sum g
                            const int e = min(max(__builtin_amdgcn_frexp_exp(qp), -100), 100);
                            iqr[k] = __builtin_bit_cast(float, (uint32_t)(127 - e) << 23);
                            const double c = -kHalfLn2 * (double)e;
                            // and, for grouped images, the rational term's constant NI g_x (see slp32_src)
                            ux[k] = __builtin_fma(c, gsx, NI > 1 ? __builtin_fma((double)NI, gsx, ux[k]) : ux[k]);
                            uy[k] = __builtin_fma(c, gsy, uy[k]);
                        }
                        for (int u = 0; u < kSuperBlock; u += kSubBlock) {
                            // per target: [source parity][log x, log y, rat x, rat y]
                            float ac[TPT][2][4], dx[TPT][NI], dy[TPT];
#pragma unroll
                            for (int k = 0; k < TPT; ++k)
#pragma unroll
                                for (int e = 0; e < 8; ++e) ac[k][e / 4][e % 4] = 0.f;
                            const SubInfo si = load_ro<SubInfo>(a.sub, (j0 + u) / kSubBlock);
                            if (far_offsets<TPT, NI>(si, px, py, act, dx, dy)) {
#pragma unroll SLP32_UNROLL
                                for (int q2 = 0; q2 < kSubBlock; q2 += 2) {
#pragma unroll
                                    for (int par = 0; par < 2; ++par) {
                                        const RecSlp32 s = load_ro<RecSlp32>(rec, u + q2 + par);
#pragma unroll
                                        for (int k = 0; k < TPT; ++k) {
                                            float rx[NI];
#pragma unroll
                                            for (int m = 0; m < NI; ++m) rx[m] = dx[k][m] - s.xl;
                                            slp32_src<NI>(rx, dy[k] - s.yl, s.gx, s.gy, iqr[k], ac[k][par]);
                                        }
                                    }
                                }
                            } else {
#pragma unroll 4
                                for (int q = 0; q < kSubBlock; ++q) {
                                    const RecSlp32 s = load_ro<RecSlp32>(rec, u + q);
#pragma unroll
                                    for (int k = 0; k < TPT; ++k) {
                                        float rx[NI];
#pragma unroll
                                        for (int m = 0; m < NI; ++m) rx[m] = (float)(px[k][m] - s.x);
                                        slp32_src<NI>(rx, (float)(py[k] - s.y), s.gx, s.gy, iqr[k], ac[k][q & 1]);
                                    }
                                }
                            }
#pragma unroll
                            for (int k = 0; k < TPT; ++k) {
                                // -1/2 ln = -(ln 2 / 2) log2
                                ux[k] = __builtin_fma(-kHalfLn2, (double)(ac[k][0][0] + ac[k][1][0]),
                                                      ux[k] + (double)(ac[k][0][2] + ac[k][1][2]));
                                uy[k] = __builtin_fma(-kHalfLn2, (double)(ac[k][0][1] + ac[k][1][1]),
                                                      uy[k] + (double)(ac[k][0][3] + ac[k][1][3]));
                            }
                        }
                    } else if (OP == S2D_OP_DLP) {
                        const RecDlp32 *rec = (const RecDlp32 *)a.rec + j0;
                        for (int u = 0; u < kSuperBlock; u += kSubBlock) {
                            float ac[TPT][2][2], dx[TPT][NI], dy[TPT];     // [source parity][x, y]
#pragma unroll
                            for (int k = 0; k < TPT; ++k)
#pragma unroll
                                for (int e = 0; e < 4; ++e) ac[k][e / 2][e % 2] = 0.f;
                            const SubInfo si = load_ro<SubInfo>(a.sub, (j0 + u) / kSubBlock);
                            if (far_offsets<TPT, NI>(si, px, py, act, dx, dy)) {
#pragma unroll
                                for (int q = 0; q < kSubBlock; ++q) {
                                    const RecDlp32 s = load_ro<RecDlp32>(rec, u + q);
#pragma unroll
                                    for (int k = 0; k < TPT; ++k) {
                                        float rx[NI];
#pragma unroll
                                        for (int m = 0; m < NI; ++m) rx[m] = dx[k][m] - s.xl;
                                        dlp32_src<NI>(rx, dy[k] - s.yl, s, ac[k][q & 1]);
                                    }
                                }
                            } else {
#pragma unroll 4
                                for (int q = 0; q < kSubBlock; ++q) {
                                    const RecDlp32 s = load_ro<RecDlp32>(rec, u + q);
#pragma unroll
                                    for (int k = 0; k < TPT; ++k) {
                                        float rx[NI];
#pragma unroll
                                        for (int m = 0; m < NI; ++m) rx[m] = (float)(px[k][m] - s.x);
                                        dlp32_src<NI>(rx, (float)(py[k] - s.y), s, ac[k][q & 1]);
                                    }
                                }
                            }
#pragma unroll
                            for (int k = 0; k < TPT; ++k) {
                                ux[k] += (double)(ac[k][0][0] + ac[k][1][0]);
                                uy[k] += (double)(ac[k][0][1] + ac[k][1][1]);
                            }
                        }
                    } else {
                        // pressures and traction, FP32C
                        using R = Rec32Of<OP>;
                        const R *rec = (const R *)a.rec + j0;
                        for (int u = 0; u < kSuperBlock; u += kSubBlock) {
                            float ac[TPT][2][2], dx[TPT][NI], dy[TPT];     // [source parity][x, y]
#pragma unroll
                            for (int k = 0; k < TPT; ++k)
#pragma unroll
                                for (int e = 0; e < 4; ++e) ac[k][e / 2][e % 2] = 0.f;
                            const SubInfo si = load_ro<SubInfo>(a.sub, (j0 + u) / kSubBlock);
                            if (far_offsets<TPT, NI>(si, px, py, act, dx, dy)) {
#pragma unroll
                                for (int q = 0; q < kSubBlock; ++q) {
                                    const R s = load_ro<R>(rec, u + q);
#pragma unroll
                                    for (int k = 0; k < TPT; ++k)
#pragma unroll
                                        for (int m = 0; m < NI; ++m)
                                            rat32<OP>(dx[k][m] - s.xl, dy[k] - s.yl, s, (float)mx[k], (float)my[k],
                                                      ac[k][q & 1]);
                                }
                            } else {
                                // near terms in FP64 (their sum can be much smaller than the
                                // terms, so FP32 terms would lose digits)
                                using R64 = Rec64Of<OP>;
                                const R64 *rec64 = (const R64 *)a.rec64 + j0;
#pragma unroll 4
                                for (int q = 0; q < kSubBlock; ++q) {
                                    const R64 s = load_ro<R64>(rec64, u + q);
#pragma unroll
                                    for (int k = 0; k < TPT; ++k)
#pragma unroll
                                        for (int m = 0; m < NI; ++m)
                                            rat64<OP>(px[k][m], py[k], s, mx[k], my[k], ux[k], uy[k]);
                                }
                            }
#pragma unroll
                            for (int k = 0; k < TPT; ++k) {
                                ux[k] += (double)(ac[k][0][0] + ac[k][1][0]);
                                uy[k] += (double)(ac[k][0][1] + ac[k][1][1]);
                            }
                        }
                    }
                }
            } else {
                // ---------------- masked superblock (rare): image by image ----------------
                for (int m = 0; m < NI; ++m) {
                    const int n = n0 + m;
                    for (int64_t j = j0; j < j0 + kSuperBlock; ++j) {
                        const bool inrange = j < j1;
#pragma unroll
                        for (int k = 0; k < TPT; ++k) {
                            const bool ok = inrange && (n != 0 || j < lo[k] || j >= hi[k]);
                            const double p1[1] = {px[k][m]};
                            if (PREC == S2D_FP64) {
                                if (OP == S2D_OP_SLP) {
                                    const RecSlp64 s = load_ro<RecSlp64>(a.rec, j);
                                    double ax = 0, ay = 0, bx = 0, by = 0;
                                    slp64_src<1>(p1, py[k], s, ltab, ax, ay, bx, by);
                                    vx[k] += ok ? ax : 0.0; vy[k] += ok ? ay : 0.0;
                                    ux[k] += ok ? bx : 0.0; uy[k] += ok ? by : 0.0;
                                } else {
                                    const Rec64Of<OP> s = load_ro<Rec64Of<OP>>(a.rec, j);
                                    double ax = 0, ay = 0;
                                    rat64<OP>(px[k][m], py[k], s, mx[k], my[k], ax, ay);
                                    ux[k] += ok ? ax : 0.0; uy[k] += ok ? ay : 0.0;
                                }
                            } else {
                                if (OP == S2D_OP_SLP) {
                                    const RecSlp32 s = load_ro<RecSlp32>(a.rec, j);
                                    float t4[4] = {0.f, 0.f, 0.f, 0.f};
                                    const float r1[1] = {(float)(px[k][m] - s.x)};
                                    slp32_src<1>(r1, (float)(py[k] - s.y), s.gx, s.gy, 1.0f, t4);
                                    ux[k] += ok ? __builtin_fma(-kHalfLn2, (double)t4[0], (double)t4[2]) : 0.0;
                                    uy[k] += ok ? __builtin_fma(-kHalfLn2, (double)t4[1], (double)t4[3]) : 0.0;
                                } else if constexpr (near_fp64(OP)) {
                                    const Rec64Of<OP> s = load_ro<Rec64Of<OP>>(a.rec64, j);
                                    double ax = 0, ay = 0;
                                    rat64<OP>(px[k][m], py[k], s, mx[k], my[k], ax, ay);
                                    ux[k] += ok ? ax : 0.0;
                                    uy[k] += ok ? ay : 0.0;
                                } else {
                                    const Rec32Of<OP> s = load_ro<Rec32Of<OP>>(a.rec, j);
                                    float t2[2] = {0.f, 0.f};
                                    rat32<OP>((float)(px[k][m] - s.x), (float)(py[k] - s.y), s, (float)mx[k],
                                              (float)my[k], t2);
                                    ux[k] += ok ? (double)t2[0] : 0.0;
                                    uy[k] += ok ? (double)t2[1] : 0.0;
                                }
                            }
                        }
                    }
                }
            }
        }
    }

#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        ox[k] = ux[k];
        oy[k] = uy[k];
        if (OP == S2D_OP_SLP && PREC == S2D_FP64) {
            // -1/2 sum g ln q (FP32C folds its log2 sums into (ux, uy) per sub-block)
            ox[k] = __builtin_fma(-0.5, vx[k], ox[k]);
            oy[k] = __builtin_fma(-0.5, vy[k], oy[k]);
        }
    }
}

// pair_sum() for one wave, written as the split's FP64 partial
// part[split][2][n_trg] (the batched path's per-item slots).
template <int OP, int PREC, int TPT, int NI>
__device__ __forceinline__ void pair_tile(const PairArgs &a, int64_t tile, int split, int lane, const double *ltab) {
    double ox[TPT], oy[TPT];
    pair_sum<OP, PREC, TPT, NI>(a, tile, split, lane, ltab, ox, oy);
    const int64_t plane = a.n_trg;
    double *out = a.part + (int64_t)split * 2 * plane;
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        const int64_t i = tile * (int64_t)(kWave * TPT) + k * kWave + lane;
        if (i < a.n_trg) {
            out[i] = ox[k];
            out[plane + i] = oy[k];
        }
    }
}

}  // namespace s2d
