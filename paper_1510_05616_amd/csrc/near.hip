// Near-field correction of the single layer for targets within a few node
// spacings of a closed curve.
//
// The periodic trapezoid rule loses accuracy for targets close to a curve
// (the paper notes this for the channel walls in a footnote of Section 5 and
// in the error band of its serpentine-channel figure, Section 5.1, and uses a
// dedicated close evaluation scheme for near vesicle pairs, Section 3.2).  Here the
// correction Delta = u_P(x) - u_1(x) of one curve's single layer is computed
// either by FFT-upsampled quadrature (the reference and fallback) or by a
// small MLP that predicts it from local features.
//
//  * upsample: per curve (one workgroup), the N-node samples of x, y, f are
//    expanded in their discrete Fourier coefficients and evaluated at P*N
//    equispaced parameter nodes (Nyquist mode split evenly); the speed comes
//    from the spectral derivative, weights (2 pi / (P N)) |x'|.  FP64.
//  * quadrature: per target, the fine trapezoid sum minus the coarse one,
//    FP64, over the target's own curve.
//  * features: per target, nearest node k* by a scan of the curve, k0 = k* or
//    k* - 1 so that the target lies over [k0, k0+1), the local frame of k0,
//    offsets in units of h = (sum w) / N, ln(distance / h), kappa h, and the
//    densities of nodes k0-3..k0+4 rotated into the frame and divided by
//    their largest norm F.
//  * MLP inference: 20 -> 64 -> 64 -> 64 -> 2, tanh-form GELU; weights and
//    activations rounded to BF16, products accumulated in FP32 on the matrix
//    cores (v_mfma_f32_32x32x8_bf16, 32 targets per wave).  The output is the
//    correction in the local frame in units of h F / (4 pi mu).  A per-bin
//    error bound (bins in the normal offset) calibrated on validation data
//    decides the fallback to the upsampled quadrature.
//  * training (FP32 master weights): forward and backward deltas with a wave
//    per sample and a lane per neuron, per-weight gradient sums over the batch
//    in fixed order, and an Adam update; all deterministic.
#include "pair_impl.h"
#include "s2d_near.h"

#include <algorithm>
#include <climits>

namespace s2d {

// ---------------------------------------------------------------------------
// a8: upsampling and FP64 quadrature
// ---------------------------------------------------------------------------
// Output: the fine curve as records {x, y, w fx, w fy} at up[4 (P lo + j)],
// j < P N, with the fine trapezoid weight w = (2 pi / (P N)) |x'|, then the
// given nodes as records {x, y, w fx, w fy} at up[4 (P n_src + lo + k)].
//
// With v(t) = sum_{m=0}^{H} (a_m cos m t + b_m sin m t) (H = N/2, the weights
// 2/N and 1/N folded into a, b), the fine nodes j, M - j, M/2 + j and M/2 - j
// see the same cos and sin of m t_j up to signs: the sign of sin flips under
// reflection and both flip with (-1)^m under the half turn.  One thread sums
// the even-m and odd-m parts of the cosine and sine series separately for
// t_j, 0 <= j <= M/4, and forms all four values from them.  The analysis sums
// pair node k with node N - k (same cosine, opposite sine).  Both stages step
// cos and sin of the multiple angles by rotation through the base angle (at
// most 128 steps; the rounding error grows at most linearly, and the fine
// nodes stay within about 1e-14 of the exact interpolant), so no table is
// kept in LDS.
constexpr int kUpThreads = 320;   // >= M/4 + 1 and >= 4 (H + 1) at N = 128, P = 8

__device__ __forceinline__ void up_acc(const double *__restrict__ c, double co, double sn, double (&C)[4],
                                       double (&S)[4], double (&Dc)[2], double (&Ds)[2]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        C[s] = __builtin_fma(c[s], co, C[s]);
        S[s] = __builtin_fma(c[4 + s], sn, S[s]);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        Dc[s] = __builtin_fma(c[8 + s], co, Dc[s]);
        Ds[s] = __builtin_fma(c[10 + s], sn, Ds[s]);
    }
}

__global__ __launch_bounds__(kUpThreads) void near_upsample(const int32_t *__restrict__ off, int32_t n_curves,
                                                            int64_t n_src, const double *__restrict__ x,
                                                            const double *__restrict__ y,
                                                            const double *__restrict__ w,
                                                            const double *__restrict__ fx,
                                                            const double *__restrict__ fy, int P,
                                                            double *__restrict__ up /* [4 (P + 1) n_src] */) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    const int c = blockIdx.x;
    if (c >= n_curves) return;
    const int lo = off[c], N = off[c + 1] - lo;
    if (N < 4 || (N & 1) || N > kUpMaxN || lo < 0 || (int64_t)lo + N > n_src || P * N > kUpMaxM) return;
    const int M = P * N, H = N / 2;
    double *eo = lds;                 // [4][H] pairs: {v_0, v_H}, then {v_k + v_{N-k}, v_k - v_{N-k}}
    double *cf = eo + 8 * H;          // [H + 1][12]: a_0..3, b_0..3, m b_0..1, m a_0..1
    const double *sig[4] = {x + lo, y + lo, fx + lo, fy + lo};
    for (int q = threadIdx.x; q < 4 * H; q += blockDim.x) {
        const int s = q / H, k = q % H;
        const double *v = sig[s];
        const double p = v[k], r = k ? v[N - k] : v[H];
        eo[2 * q] = k ? p + r : p;
        eo[2 * q + 1] = k ? p - r : r;
    }
    double *coarse = up + 4 * ((int64_t)n_src * P + lo);
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        coarse[4 * k] = x[lo + k];
        coarse[4 * k + 1] = y[lo + k];
        coarse[4 * k + 2] = w[lo + k] * fx[lo + k];
        coarse[4 * k + 3] = w[lo + k] * fy[lo + k];
    }
    __syncthreads();
    const double inv = 1.0 / (double)N;
    for (int q = threadIdx.x; q < 4 * (H + 1); q += blockDim.x) {
        const int s = q / (H + 1), m = q % (H + 1);
        const double *e = eo + 2 * H * s;
        // (cos, sin)(2 pi m k / N) by rotation through 2 pi m / N
        double c1, s1;
        sincospi(2.0 * (double)m / (double)N, &s1, &c1);
        double a = (m & 1) ? e[0] - e[1] : e[0] + e[1];          // k = 0 and k = H
        double b = 0.0, co = c1, sn = s1;
        for (int k = 1; k < H; ++k) {
            a = __builtin_fma(e[2 * k], co, a);
            b = __builtin_fma(e[2 * k + 1], sn, b);
            const double r = __builtin_fma(co, c1, -sn * s1);
            sn = __builtin_fma(sn, c1, co * s1);
            co = r;
        }
        const bool edge = m == 0 || m == H;                      // no sine term, weight 1 / N
        const double wgt = edge ? inv : 2.0 * inv;
        a *= wgt;
        b = edge ? 0.0 : b * wgt;
        double *cm = cf + 12 * m;
        cm[s] = a;
        cm[4 + s] = b;
        if (s < 2) {
            cm[8 + s] = (double)m * b;
            cm[10 + s] = (double)m * a;
        }
    }
    __syncthreads();
    const int64_t base = (int64_t)lo * P;
    const double hw = 2.0 * M_PI / (double)M;
    const int G = M / 4 + 1;
    for (int j = threadIdx.x; j < G; j += blockDim.x) {
        double Ce[4] = {0, 0, 0, 0}, Co[4] = {0, 0, 0, 0}, Se[4] = {0, 0, 0, 0}, So[4] = {0, 0, 0, 0};
        double Dce[2] = {0, 0}, Dco[2] = {0, 0}, Dse[2] = {0, 0}, Dso[2] = {0, 0};
        // (cos, sin)(m t_j) by rotation through t_j: no lane-varying table reads
        double c1, s1;
        sincospi(2.0 * (double)j / (double)M, &s1, &c1);
        double co = 1.0, sn = 0.0;
        int m = 0;
        for (; m < H; m += 2) {
            up_acc(cf + 12 * m, co, sn, Ce, Se, Dce, Dse);
            double t = __builtin_fma(co, c1, -sn * s1);
            sn = __builtin_fma(sn, c1, co * s1);
            co = t;
            up_acc(cf + 12 * (m + 1), co, sn, Co, So, Dco, Dso);
            t = __builtin_fma(co, c1, -sn * s1);
            sn = __builtin_fma(sn, c1, co * s1);
            co = t;
        }
        if (m == H) up_acc(cf + 12 * m, co, sn, Ce, Se, Dce, Dse);
        // sign of the odd-m part (half turn) and of the sine part (reflection)
        const int pts[4] = {j, j ? M - j : 0, M / 2 + j, M / 2 - j};
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const double ho = (o & 2) ? -1.0 : 1.0, rs = (o & 1) ? -1.0 : 1.0;
            double v[4], dv[2];
#pragma unroll
            for (int s = 0; s < 4; ++s) v[s] = (Ce[s] + ho * Co[s]) + rs * (Se[s] + ho * So[s]);
#pragma unroll
            for (int s = 0; s < 2; ++s) dv[s] = (Dce[s] + ho * Dco[s]) - rs * (Dse[s] + ho * Dso[s]);
            const double ww = hw * sqrt(dv[0] * dv[0] + dv[1] * dv[1]);
            double *rec = up + 4 * (base + pts[o]);
            rec[0] = v[0];
            rec[1] = v[1];
            rec[2] = ww * v[2];
            rec[3] = ww * v[3];
        }
    }
}

__device__ __forceinline__ void slp64_acc(double px, double py, double sx, double sy, double gx, double gy,
                                          const double *ltab, double &ax, double &ay, double &bx, double &by) {
    const double rx = px - sx, ry = py - sy;
    const double q = __builtin_fma(rx, rx, ry * ry);
    const double lq = log64_tab(q, ltab);
    const double t = __builtin_fma(rx, gx, ry * gy) * rcp64(q);
    ax = __builtin_fma(gx, lq, ax);
    ay = __builtin_fma(gy, lq, ay);
    bx = __builtin_fma(rx, t, bx);
    by = __builtin_fma(ry, t, by);
}

// Part `part` of `parts` of the coarse (N nodes) and fine (P N nodes)
// single-layer sums of one curve, from the records {x, y, g_x, g_y} written
// by near_upsample: the sources are taken as one list, the N coarse records
// then the P N fine ones, cut into `parts` contiguous pieces; coarse sources
// go to s[0..3], fine ones to s[4..7].
template <bool UNIFORM>
__device__ __forceinline__ void near_sums(double px, double py, int lo, int N, int P, int64_t n_src, int part,
                                          int parts, const double *__restrict__ up, const double *ltab,
                                          double (&s)[8]) {
    if (UNIFORM) {
        lo = __builtin_amdgcn_readfirstlane(lo);
        N = __builtin_amdgcn_readfirstlane(N);
    }
    const int L = (P + 1) * N;
    const int a = L * part / parts, b = L * (part + 1) / parts;
    const double *cr = up + 4 * ((int64_t)n_src * P + lo);
    const int ce = min(b, N);
#pragma unroll 4
    for (int k = a; k < ce; ++k)
        slp64_acc(px, py, cr[4 * k], cr[4 * k + 1], cr[4 * k + 2], cr[4 * k + 3], ltab, s[0], s[1], s[2], s[3]);
    const double *fr = up + 4 * (int64_t)lo * P;
    const int fb = b - N;
#pragma unroll 4
    for (int k = max(a, N) - N; k < fb; ++k)
        slp64_acc(px, py, fr[4 * k], fr[4 * k + 1], fr[4 * k + 2], fr[4 * k + 3], ltab, s[4], s[5], s[6], s[7]);
}

// Delta for the 64 targets q = 64 blk + lane, or, with an index list, for
// targets list[q], q < *list_len (the list keeps the targets' order, so its
// waves stay on one curve).  The four waves of the workgroup take the
// same targets and a quarter of the sources each; wave 0 adds the other
// three's partial sums in fixed order.  Short workgroups keep the launch
// balanced across curves of different sizes.  When every live target of the
// wave lies on the same curve (targets sorted by curve), the source loops are
// wave-uniform and their loads go through the scalar path.
constexpr int kQuadParts = 4;

__global__ __launch_bounds__(64 * kQuadParts) void near_quad(int64_t n_trg, const int32_t *__restrict__ list,
                                                             const int32_t *__restrict__ list_len,
                                                             const double *__restrict__ tx,
                                                             const double *__restrict__ ty,
                                                             const int32_t *__restrict__ tc,
                                                             const int32_t *__restrict__ off, int32_t n_curves,
                                                             int64_t n_src, int P, const double *__restrict__ up,
                                                             double pref, double *__restrict__ du,
                                                             double *__restrict__ dv, double *__restrict__ uf,
                                                             double *__restrict__ vf, double *__restrict__ uc,
                                                             double *__restrict__ vc) {
    __shared__ __attribute__((aligned(16))) double ltab[kLogTabWords];
    __shared__ double partial[kQuadParts - 1][8][kWave];
    // targets to process (the list's length is known on the device only;
    // workgroups past it leave before any barrier)
    const int64_t n = list ? (int64_t)*list_len : n_trg;
    const unsigned nb = (unsigned)((n + kWave - 1) / kWave);
    if (blockIdx.x >= nb) return;
    fill_log_table(ltab);
    const int lane = threadIdx.x & (kWave - 1);
    const int part = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    // workgroups are dispatched round-robin over the 8 XCDs; XCD r takes a
    // contiguous run of target groups, so the 3-4 workgroups of one curve
    // share that XCD's L2 copy of the curve's records
    const unsigned r = blockIdx.x % 8, per = nb / 8, rem = nb % 8;
    const unsigned blk = (r < rem ? r * (per + 1) : rem * (per + 1) + (r - rem) * per) + blockIdx.x / 8;
    const int64_t q = (int64_t)blk * kWave + lane;
    const bool live = q < n;
    const int64_t i = live ? (list ? (int64_t)list[q] : q) : 0;
    const int c = live ? tc[i] : -1;
    const int lo = (c >= 0 && c < n_curves) ? off[c] : 0;
    const int N = (c >= 0 && c < n_curves) ? off[c + 1] - lo : 0;
    const bool ok = c >= 0 && c < n_curves && N >= 4 && !(N & 1) && N <= kUpMaxN && P * N <= kUpMaxM &&
                    lo >= 0 && (int64_t)lo + N <= n_src;
    // a wave is uniform when all its live lanes share one valid curve
    const int cl = ok ? c : INT_MAX;
    const int cmin = wave_min(cl);
    const bool any_ok = cmin != INT_MAX;
    const bool uniform = any_ok && __all(!live || (ok && c == cmin));
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (uniform) {
        // idle lanes follow the wave's curve (their results are dropped)
        const int cu = __builtin_amdgcn_readfirstlane(cmin);
        const int lou = off[cu], Nu = off[cu + 1] - lou;
        near_sums<true>(live ? tx[i] : tx[0], live ? ty[i] : ty[0], lou, Nu, P, n_src, part, kQuadParts, up, ltab,
                        s);
    } else if (ok) {
        near_sums<false>(tx[i], ty[i], lo, N, P, n_src, part, kQuadParts, up, ltab, s);
    }
    if (part > 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) partial[part - 1][k][lane] = s[k];
    }
    __syncthreads();
    if (part > 0 || !live) return;
#pragma unroll
    for (int p = 0; p < kQuadParts - 1; ++p) {
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] += partial[p][k][lane];
    }
    if (!ok) {
        du[i] = dv[i] = __builtin_nan("");
        if (uf) uf[i] = vf[i] = uc[i] = vc[i] = __builtin_nan("");
        return;
    }
    du[i] = pref * ((-0.5 * s[4] + s[6]) - (-0.5 * s[0] + s[2]));
    dv[i] = pref * ((-0.5 * s[5] + s[7]) - (-0.5 * s[1] + s[3]));
    if (uf) {
        uf[i] = pref * (-0.5 * s[4] + s[6]);
        vf[i] = pref * (-0.5 * s[5] + s[7]);
        uc[i] = pref * (-0.5 * s[0] + s[2]);
        vc[i] = pref * (-0.5 * s[1] + s[3]);
    }
}

// Order-keeping compaction of the targets with flag == 1 (AUTO's fallback):
// per-workgroup counts, one exclusive scan, then each workgroup writes its
// targets' indices at its offset in target order.
constexpr int kCompactBlock = 256;

__device__ __forceinline__ uint64_t flag_ballot(int64_t n, const int32_t *__restrict__ flag, int64_t i) {
    return __ballot(i < n && flag[i] == 1);
}

__global__ __launch_bounds__(kCompactBlock) void near_compact_count(int64_t n, const int32_t *__restrict__ flag,
                                                                    int32_t *__restrict__ cnt) {
    __shared__ int wsum[kCompactBlock / kWave];
    const int64_t i = (int64_t)blockIdx.x * kCompactBlock + threadIdx.x;
    const uint64_t b = flag_ballot(n, flag, i);
    if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < kCompactBlock / kWave; ++w) s += wsum[w];
        cnt[blockIdx.x] = s;
    }
}

// exclusive scan of cnt[0 .. nb) in place, total in cnt[nb]; one workgroup
// of 1024 threads, each over a contiguous segment
__global__ __launch_bounds__(1024) void near_compact_scan(int64_t nb, int32_t *__restrict__ cnt) {
    __shared__ int64_t part[1024];
    const int64_t seg = (nb + 1023) / 1024;
    const int64_t b0 = min((int64_t)threadIdx.x * seg, nb), b1 = min(b0 + seg, nb);
    int64_t s = 0;
    for (int64_t b = b0; b < b1; ++b) s += cnt[b];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int k = 0; k < 1024; ++k) {
            const int64_t v = part[k];
            part[k] = run;
            run += v;
        }
        cnt[nb] = (int32_t)run;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t b = b0; b < b1; ++b) {
        const int32_t v = cnt[b];
        cnt[b] = (int32_t)run;
        run += v;
    }
}

__global__ __launch_bounds__(kCompactBlock) void near_compact_scatter(int64_t n, const int32_t *__restrict__ flag,
                                                                      const int32_t *__restrict__ cnt,
                                                                      int32_t *__restrict__ list) {
    __shared__ int wsum[kCompactBlock / kWave];
    const int64_t i = (int64_t)blockIdx.x * kCompactBlock + threadIdx.x;
    const uint64_t b = flag_ballot(n, flag, i);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) wsum[w] = __popcll(b);
    __syncthreads();
    int base = cnt[blockIdx.x];
    for (int k = 0; k < w; ++k) base += wsum[k];
    if ((b >> lane) & 1) list[base + __popcll(b & ((1ull << lane) - 1))] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// a9: features
// ---------------------------------------------------------------------------
// nearest node k* of the curve at [lo, lo + N) and the curve's weight sum;
// UNIFORM: lo and N are the same in every lane (loads take the scalar path)
template <bool UNIFORM>
__device__ __forceinline__ int near_scan(double px, double py, int lo, int N, const double *__restrict__ x,
                                         const double *__restrict__ y, const double *__restrict__ w, double &best,
                                         double &wsum) {
    if (UNIFORM) {
        lo = __builtin_amdgcn_readfirstlane(lo);
        N = __builtin_amdgcn_readfirstlane(N);
    }
    best = 1e300;
    wsum = 0.0;
    int ks = 0;
#pragma unroll 4
    for (int k = 0; k < N; ++k) {
        const double dx = px - x[lo + k], dy = py - y[lo + k];
        const double d2 = dx * dx + dy * dy;
        if (d2 < best) { best = d2; ks = k; }
        wsum += w[lo + k];
    }
    return ks;
}

__global__ __launch_bounds__(256) void near_features(int64_t n_trg, const double *__restrict__ tx,
                                                     const double *__restrict__ ty, const int32_t *__restrict__ tc,
                                                     const int32_t *__restrict__ off, int32_t n_curves, int64_t n_src,
                                                     const double *__restrict__ x, const double *__restrict__ y,
                                                     const double *__restrict__ nx, const double *__restrict__ ny,
                                                     const double *__restrict__ kap, const double *__restrict__ w,
                                                     const double *__restrict__ fx, const double *__restrict__ fy,
                                                     float *__restrict__ X, double *__restrict__ frame) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = q < n_trg;
    const int64_t i = live ? q : 0;
    const int c = live ? tc[i] : -1;
    const int lo = (c >= 0 && c < n_curves) ? off[c] : 0;
    const int N = (c >= 0 && c < n_curves) ? off[c + 1] - lo : 0;
    const bool ok = c >= 0 && c < n_curves && N >= 8 && lo >= 0 && (int64_t)lo + N <= n_src;
    // a wave is uniform when all its live lanes share one valid curve (every
    // lane of the wave reaches this vote)
    const int cl = ok ? c : INT_MAX;
    const int cmin = wave_min(cl);
    const bool uniform = cmin != INT_MAX && __all(!live || (ok && c == cmin));
    const double px = live ? tx[i] : 0.0, py = live ? ty[i] : 0.0;
    double best = 0.0, wsum = 0.0;
    int ks = 0;
    if (uniform) {
        const int cu = __builtin_amdgcn_readfirstlane(cmin);
        const int lou = off[cu];
        ks = near_scan<true>(px, py, lou, off[cu + 1] - lou, x, y, w, best, wsum);
    } else if (ok) {
        ks = near_scan<false>(px, py, lo, N, x, y, w, best, wsum);
    }
    if (!live) return;
    float *xi = X + i * kNearFeat;
    double *fr = frame + i * 6;
    if (!ok) {
        for (int k = 0; k < kNearFeat; ++k) xi[k] = __builtin_nanf("");
        for (int k = 0; k < 6; ++k) fr[k] = __builtin_nan("");
        return;
    }
    const double h = wsum / (double)N;
    const double ts0 = -ny[lo + ks], ts1 = nx[lo + ks];
    const int k0 = ((px - x[lo + ks]) * ts0 + (py - y[lo + ks]) * ts1 >= 0.0) ? ks : (ks + N - 1) % N;
    const double t0 = -ny[lo + k0], t1 = nx[lo + k0];
    const double n0 = nx[lo + k0], n1 = ny[lo + k0];
    const double ox = px - x[lo + k0], oy = py - y[lo + k0];
    double ft[8], fn[8], F = 0.0;
    for (int j = 0; j < 8; ++j) {
        const int k = lo + (k0 + j - 3 + N) % N;
        ft[j] = fx[k] * t0 + fy[k] * t1;
        fn[j] = fx[k] * n0 + fy[k] * n1;
        F = fmax(F, sqrt(ft[j] * ft[j] + fn[j] * fn[j]));
    }
    if (F == 0.0) F = 1.0;
    xi[0] = (float)((ox * t0 + oy * t1) / h);
    xi[1] = (float)((ox * n0 + oy * n1) / h);
    xi[2] = (float)log(sqrt(best) / h);
    xi[3] = (float)(kap[lo + k0] * h);
    for (int j = 0; j < 8; ++j) {
        xi[4 + j] = (float)(ft[j] / F);
        xi[12 + j] = (float)(fn[j] / F);
    }
    fr[0] = t0;
    fr[1] = t1;
    fr[2] = n0;
    fr[3] = n1;
    fr[4] = h;
    fr[5] = F;
}

// a9 for the walls: target i near one period of wall curve tc[i] (N >= 8
// nodes advancing by sg d in x), the wall unrolled over three periods (node
// K in [-N, 2N) at (x_{K mod N} + sg d floor(K / N), y_{K mod N})); nearest
// unrolled node with the smallest K on ties, then the same features as for
// closed curves; frame (t0, n0, 1, F): the double layer's correction scales
// with F alone
// Nearest-node search over the three periods of a wall.  Nodes are grouped in
// cells of kWallCell consecutive nodes; a cell's centre is its middle node and
// its radius the largest distance of its nodes from that centre.  The search is
// exact: a cell can hold a node closer than B only if |p - centre| <= B +
// radius.  Pass 1 takes B from the cell centres (actual nodes); pass 2 scans,
// in ascending (period, cell) order, every cell that passes the test, node by
// node in ascending order with a strict comparison.  So the smallest unrolled
// index among equal distances wins, as in a plain scan.  Each lane collects
// its own list of cells to scan (up to kWallScan; a lane with more scans every
// passing cell in order instead), so the lanes of a wave do not scan each
// other's cells.
constexpr int kWallCell = 128;
constexpr int kWallMaxCells = 1024;
constexpr int kWallMaxCurves = 64;
constexpr int kWallScan = 10;            // two words of five 12-bit cell codes

struct WallCells {
    double cx[kWallMaxCells], cy[kWallMaxCells], rad[kWallMaxCells];
    double h[kWallMaxCurves];            // mean weight of each curve
    int coff[kWallMaxCurves + 1];
    int ok;
};

__device__ __forceinline__ int wall_curve_nodes(const int32_t *off, int c, int64_t n_src) {
    const int lo = off[c], hi = off[c + 1];
    return (lo >= 0 && hi >= lo + 8 && (int64_t)hi <= n_src) ? hi - lo : 0;
}

// every thread of the block calls this (it synchronises)
__device__ void wall_cells_build(WallCells &W, const int32_t *off, int n_curves, int64_t n_src, const double *x,
                                 const double *y, const double *w) {
    __shared__ double red[256];
    if (threadIdx.x == 0) {
        int acc = 0;
        bool ok = n_curves <= kWallMaxCurves;
        for (int c = 0; ok && c < n_curves; ++c) {
            W.coff[c] = acc;
            acc += (wall_curve_nodes(off, c, n_src) + kWallCell - 1) / kWallCell;
            ok = acc <= kWallMaxCells;
        }
        if (ok) W.coff[n_curves] = acc;
        W.ok = ok ? 1 : 0;
    }
    __syncthreads();
    if (!W.ok) return;                  // block-uniform
    const int total = W.coff[n_curves];
    for (int cell = threadIdx.x; cell < total; cell += blockDim.x) {
        int c = 0;
        while (W.coff[c + 1] <= cell) ++c;
        const int lo = off[c], N = wall_curve_nodes(off, c, n_src);
        const int k0 = (cell - W.coff[c]) * kWallCell, len = min(kWallCell, N - k0);
        const double cx = x[lo + k0 + len / 2], cy = y[lo + k0 + len / 2];
        double r2 = 0.0;
        for (int j = k0; j < k0 + len; ++j) {
            const double ex = x[lo + j] - cx, ey = y[lo + j] - cy;
            r2 = fmax(r2, ex * ex + ey * ey);
        }
        W.cx[cell] = cx;
        W.cy[cell] = cy;
        W.rad[cell] = sqrt(r2) * (1.0 + 1e-12);
    }
    // mean weight per curve, in a fixed order (strided partial sums, then a tree)
    for (int c = 0; c < n_curves; ++c) {
        const int lo = off[c], N = wall_curve_nodes(off, c, n_src);
        double sacc = 0.0;
        for (int k = threadIdx.x; k < N; k += blockDim.x) sacc += w[lo + k];
        red[threadIdx.x] = sacc;
        __syncthreads();
        for (int st = blockDim.x / 2; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) W.h[c] = N > 0 ? red[0] / (double)N : 0.0;
        __syncthreads();
    }
}

// nearest unrolled node K = m N + k (m = -1, 0, 1) of curve c to (px, py):
// returns K and writes its squared distance to best
__device__ int wall_nearest(const WallCells &W, bool cells, int c, int lo, int N, double sg, double d, double px,
                            double py, const double *x, const double *y, double &best) {
    best = 1e300;
    int ks = 0;
    const auto scan = [&](int m, int k0, int k1) {
        const double sh = sg * d * (double)m;
        for (int k = k0; k < k1; ++k) {
            const double dx = px - (x[lo + k] + sh), dy = py - y[lo + k];
            const double d2 = dx * dx + dy * dy;
            if (d2 < best) { best = d2; ks = m * N + k; }
        }
    };
    if (!cells) {
        for (int m = -1; m <= 1; ++m) scan(m, 0, N);
        return ks;
    }
    const int cb = W.coff[c], ce = W.coff[c + 1];
    double ub = 1e300;
    for (int m = -1; m <= 1; ++m) {
        const double sh = sg * d * (double)m;
        for (int q = cb; q < ce; ++q) {
            const double dx = px - (W.cx[q] + sh), dy = py - W.cy[q];
            ub = fmin(ub, dx * dx + dy * dy);
        }
    }
    const double bound = sqrt(ub) * (1.0 + 1e-9);
    // passing cells, as 12-bit codes (m + 1) * kWallMaxCells + (q - cb)
    uint64_t wd[2] = {0, 0};
    int nl = 0;
    for (int m = -1; m <= 1; ++m) {
        const double sh = sg * d * (double)m;
        for (int q = cb; q < ce; ++q) {
            const double dx = px - (W.cx[q] + sh), dy = py - W.cy[q];
            const double lim = bound + W.rad[q];
            if (dx * dx + dy * dy <= lim * lim) {
                if (nl < kWallScan) {
                    const uint64_t code = (uint64_t)((m + 1) * kWallMaxCells + (q - cb));
                    if (nl < 5) wd[0] |= code << (12 * nl);
                    else wd[1] |= code << (12 * (nl - 5));
                }
                ++nl;
            }
        }
    }
    if (nl <= kWallScan) {
        for (int t = 0; t < nl; ++t) {
            const int code = (int)(((t < 5 ? wd[0] : wd[1]) >> (12 * (t < 5 ? t : t - 5))) & 0xfff);
            const int k0 = (code % kWallMaxCells) * kWallCell;
            scan(code / kWallMaxCells - 1, k0, min(N, k0 + kWallCell));
        }
    } else {
        for (int m = -1; m <= 1; ++m) {
            const double sh = sg * d * (double)m;
            for (int q = cb; q < ce; ++q) {
                const double dx = px - (W.cx[q] + sh), dy = py - W.cy[q];
                const double lim = bound + W.rad[q];
                if (dx * dx + dy * dy <= lim * lim) {
                    const int k0 = (q - cb) * kWallCell;
                    scan(m, k0, min(N, k0 + kWallCell));
                }
            }
        }
    }
    return ks;
}

// Features of targets near periodic walls (grid-stride over targets; the cell
// table is built once per block in LDS).
__global__ __launch_bounds__(256) void near_wall_features(int64_t n_trg, const double *__restrict__ tx,
                                                          const double *__restrict__ ty,
                                                          const int32_t *__restrict__ tc,
                                                          const int32_t *__restrict__ off, int32_t n_curves,
                                                          int64_t n_src, const double *__restrict__ x,
                                                          const double *__restrict__ y,
                                                          const double *__restrict__ nx,
                                                          const double *__restrict__ ny,
                                                          const double *__restrict__ kap,
                                                          const double *__restrict__ w,
                                                          const double *__restrict__ fx,
                                                          const double *__restrict__ fy, double d,
                                                          float *__restrict__ X, double *__restrict__ frame) {
    __shared__ WallCells W;
    wall_cells_build(W, off, n_curves, n_src, x, y, w);
    const bool cells = W.ok != 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_trg; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = tc[i];
        const int lo = (c >= 0 && c < n_curves) ? off[c] : 0;
        const int N = (c >= 0 && c < n_curves) ? off[c + 1] - lo : 0;
        float *xi = X + i * kNearFeat;
        double *fr = frame + i * 6;
        if (c < 0 || c >= n_curves || N < 8 || lo < 0 || (int64_t)lo + N > n_src) {
            for (int k = 0; k < kNearFeat; ++k) xi[k] = __builtin_nanf("");
            for (int k = 0; k < 6; ++k) fr[k] = __builtin_nan("");
            continue;
        }
        const double sg = x[lo + 1] > x[lo] ? 1.0 : -1.0;
        const double px = tx[i], py = ty[i];
        double best = 0.0, h = 0.0;
        if (cells) {
            h = W.h[c];
        } else {
            for (int k = 0; k < N; ++k) h += w[lo + k];
            h /= (double)N;
        }
        const int ks = wall_nearest(W, cells, c, lo, N, sg, d, px, py, x, y, best);
        const auto md = [N](int K) { return ((K % N) + N) % N; };
        const auto fl = [N](int K) { return K >= 0 ? K / N : -((-K + N - 1) / N); };
        const int ms = md(ks);
        const double xs = x[lo + ms] + sg * d * (double)fl(ks), ys = y[lo + ms];
        const double ts0 = -ny[lo + ms], ts1 = nx[lo + ms];
        const int k0 = ((px - xs) * ts0 + (py - ys) * ts1 >= 0.0) ? ks : ks - 1;
        const int m0 = md(k0);
        const double t0 = -ny[lo + m0], t1 = nx[lo + m0];
        const double n0 = nx[lo + m0], n1 = ny[lo + m0];
        const double ox = px - (x[lo + m0] + sg * d * (double)fl(k0)), oy = py - y[lo + m0];
        double ft[8], fn[8], F = 0.0;
        for (int j = 0; j < 8; ++j) {
            const int k = lo + md(k0 + j - 3);
            ft[j] = fx[k] * t0 + fy[k] * t1;
            fn[j] = fx[k] * n0 + fy[k] * n1;
            F = fmax(F, sqrt(ft[j] * ft[j] + fn[j] * fn[j]));
        }
        if (F == 0.0) F = 1.0;
        xi[0] = (float)((ox * t0 + oy * t1) / h);
        xi[1] = (float)((ox * n0 + oy * n1) / h);
        xi[2] = (float)log(sqrt(best) / h);
        xi[3] = (float)(kap[lo + m0] * h);
        for (int j = 0; j < 8; ++j) {
            xi[4 + j] = (float)(ft[j] / F);
            xi[12 + j] = (float)(fn[j] / F);
        }
        fr[0] = t0;
        fr[1] = t1;
        fr[2] = n0;
        fr[3] = n1;
        fr[4] = 1.0;
        fr[5] = F;
    }
}

// scaled labels in the local frame: (Delta . t0, Delta . n0) * 4 pi mu / (h F)
__global__ __launch_bounds__(256) void near_scale_labels_k(int64_t n, const double *__restrict__ du,
                                                           const double *__restrict__ dv,
                                                           const double *__restrict__ frame, double mu,
                                                           float *__restrict__ Y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *fr = frame + 6 * i;
    const double sc = 4.0 * M_PI * mu / (fr[4] * fr[5]);
    Y[2 * i] = (float)((du[i] * fr[0] + dv[i] * fr[1]) * sc);
    Y[2 * i + 1] = (float)((du[i] * fr[2] + dv[i] * fr[3]) * sc);
}

// ---------------------------------------------------------------------------
// MLP pieces
// ---------------------------------------------------------------------------
__device__ __forceinline__ float gelu_f(float z) {
    const float u = 0.7978845608028654f * (z + 0.044715f * z * z * z);
    // tanh(u) = 1 - 2 / (exp(2u) + 1); exp via the hardware exp2
    const float e = __builtin_amdgcn_exp2f(fminf(2.8853900817779268f * u, 126.f));
    const float th = 1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f);
    return 0.5f * z * (1.f + th);
}

__device__ __forceinline__ float gelu_grad_f(float z) {
    const float u = 0.7978845608028654f * (z + 0.044715f * z * z * z);
    const float e = __builtin_amdgcn_exp2f(fminf(2.8853900817779268f * u, 126.f));
    const float th = 1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f);
    const float du = 0.7978845608028654f * (1.f + 3.f * 0.044715f * z * z);
    return 0.5f * (1.f + th) + 0.5f * z * (1.f - th * th) * du;
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    // round to nearest even, as the hardware conversion does
    bf16x2_t v;
    v[0] = (__bf16)a;
    v[1] = (__bf16)b;
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ float dot2_bf16(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a), __builtin_bit_cast(bf16x2_t, b), c,
                                           false);
}

// MLP inference, with the fallback decision taken first (from the target's
// bin of |normal offset| / h and the calibrated bounds, scaled into velocity
// units by h F / (4 pi mu)): no correction, the network, or the upsampled
// quadrature (the target joins the fallback list).  nb: the packed BF16
// network.  The network runs on the matrix cores: a wave takes one group of
// 32 targets and evaluates each layer as out^T = W in^T with
// v_mfma_f32_32x32x8_bf16: A = 32 output features x 8 inputs of W (read from
// the blob's [out][in/2] pairs), B = 8 inputs x the 32 targets, C = 32
// features x 32 targets in FP32, started at the bias.  Lane l holds target
// l % 32; in C it holds features 8 (r / 4) + 4 (l / 32) + r % 4 of each
// 32-feature tile (r = 0..15), which are exactly the inputs 8 s + 4 (l / 32) +
// 0..3 of K-step s of the next layer's B: the activations stay in their
// lanes between layers.  GELU in FP32 and rounding to BF16 between layers; the
// last 64 -> 2 layer is a dot2 over the lane's 32 features plus the partner
// lane's half.
typedef short bf16x4v_t __attribute__((ext_vector_type(4)));
typedef float f32x16v_t __attribute__((ext_vector_type(16)));

// 4 bf16 of row `row` of a [out][in2] pair array, inputs k0..k0+3 (k0 % 4 == 0)
__device__ __forceinline__ bf16x4v_t mfma_wrow(const uint32_t *W, int in2, int row, int k0) {
    const uint32_t *q = W + row * in2 + k0 / 2;
    const uint32_t lo = q[0], hi = q[1];
    return __builtin_bit_cast(bf16x4v_t, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ bf16x4v_t mfma_pack4(float a, float b, float c, float d) {
    return __builtin_bit_cast(bf16x4v_t, ((uint64_t)pack_bf16(c, d) << 32) | pack_bf16(a, b));
}

template <int KSTEPS, int IN2>
__device__ __forceinline__ void mfma_layer(const uint32_t *W, const float *b, const bf16x4v_t (&in)[KSTEPS],
                                           int c, int h, f32x16v_t (&acc)[2]) {
#pragma unroll
    for (int T = 0; T < 2; ++T) {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[T][r] = b[32 * T + 8 * (r / 4) + 4 * h + (r % 4)];
#pragma unroll
        for (int s = 0; s < KSTEPS; ++s) {
            const int k0 = 8 * s + 4 * h;
            const bf16x4v_t a = (2 * IN2 > k0) ? mfma_wrow(W, IN2, 32 * T + c, k0) : bf16x4v_t{0, 0, 0, 0};
            acc[T] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, in[s], acc[T], 0, 0, 0);
        }
    }
}

// GELU of a layer's output, rounded to the next layer's B operands
__device__ __forceinline__ void mfma_act(const f32x16v_t (&acc)[2], bf16x4v_t (&out)[8]) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int T = s / 4, r = 4 * (s % 4);
        out[s] = mfma_pack4(gelu_f(acc[T][r]), gelu_f(acc[T][r + 1]), gelu_f(acc[T][r + 2]), gelu_f(acc[T][r + 3]));
    }
}

__global__ __launch_bounds__(256) void near_mlp_infer_mfma(int64_t n_trg, const float *__restrict__ X,
                                                           const double *__restrict__ frame,
                                                           const NearBlob *__restrict__ nb, double mu,
                                                           double threshold, int use_bound,
                                                           double *__restrict__ du, double *__restrict__ dv,
                                                           int32_t *__restrict__ flag) {
    static_assert(kNearFeat <= 24, "three K-steps of the first layer");
    const int lane = threadIdx.x & (kWave - 1), h = lane >> 5, c = lane & 31;
    const int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;   // this wave's group
    if (g * 32 < n_trg) {                                            // wave-uniform
        const int64_t i = g * 32 + c;
        const bool valid = i < n_trg;
        const float *xi = X + (valid ? i : 0) * kNearFeat;
        const double *fr = frame + 6 * (valid ? i : 0);
        int dec = 0;                                                 // 0 network, 1 quadrature, 2 none
        double sc = 0.0;
        if (valid) {
            sc = fr[4] * fr[5] / (4.0 * M_PI * mu);
            if (use_bound) {
                const float noff = fabsf(xi[1]);
                int bin = (int)floorf((log10f(fmaxf(noff, 1e-30f)) - nb->bin_lo) / nb->bin_w);
                bin = bin < 0 ? 0 : (bin >= nb->n_bins ? nb->n_bins - 1 : bin);
                const bool bad = !(noff == noff);
                if (!bad && (double)nb->bound_zero[bin] * sc <= threshold) dec = 2;
                else if (bad || (double)nb->bound[bin] * sc > threshold) dec = 1;
            }
        }
        // the network runs only if some target of the group needs it
        float y0 = 0.f, y1 = 0.f;
        if (__any(valid && dec == 0)) {                              // wave-uniform
            // first layer: the standardised features of the lane's target
            bf16x4v_t in1[3];
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = 8 * s + 4 * h + e;
                    v[e] = (valid && k < kNearFeat) ? (xi[k] - nb->mu_in[k]) * nb->isd_in[k] : 0.f;
                }
                in1[s] = mfma_pack4(v[0], v[1], v[2], v[3]);
            }
            f32x16v_t acc[2];
            bf16x4v_t hb[8];
            mfma_layer<3, kNearFeat / 2>(nb->W1, nb->b1, in1, c, h, acc);
            mfma_act(acc, hb);
            mfma_layer<8, 32>(nb->W2, nb->b2, hb, c, h, acc);
            mfma_act(acc, hb);
            mfma_layer<8, 32>(nb->W3, nb->b3, hb, c, h, acc);
#pragma unroll
            for (int T = 0; T < 2; ++T) {
#pragma unroll
                for (int r = 0; r < 16; r += 2) {
                    const int f = 32 * T + 8 * (r / 4) + 4 * h + (r % 4);
                    const uint32_t p = pack_bf16(gelu_f(acc[T][r]), gelu_f(acc[T][r + 1]));
                    y0 = dot2_bf16(nb->W4[f / 2], p, y0);
                    y1 = dot2_bf16(nb->W4[32 + f / 2], p, y1);
                }
            }
            y0 += __shfl_xor(y0, 32, kWave);
            y1 += __shfl_xor(y1, 32, kWave);
            y0 += nb->b4[0];
            y1 += nb->b4[1];
        }
        if (valid && h == 0) {
            if (dec == 2) {
                if (flag) flag[i] = 2;
                du[i] = 0.0;
                dv[i] = 0.0;
            } else if (dec == 1) {
                flag[i] = 1;               // the quadrature kernel writes du, dv
            } else {
                if (flag) flag[i] = 0;
                du[i] = sc * ((double)y0 * fr[0] + (double)y1 * fr[2]);
                dv[i] = sc * ((double)y0 * fr[1] + (double)y1 * fr[3]);
            }
        }
    }
}

// Pack FP32 master parameters into the BF16 inference blob.
__global__ __launch_bounds__(256) void near_pack(const float *__restrict__ prm, const float *__restrict__ bound,
                                                 const float *__restrict__ bound_zero, int32_t n_bins, float bin_lo,
                                                 float bin_w, NearBlob *__restrict__ nb) {
    const MlpOffsets O;
    constexpr int r0 = kNearFeat;                  // W1 pairs
    constexpr int r1 = r0 + 64 * kNearFeat / 2;    // W2
    constexpr int r2 = r1 + 64 * 32;               // W3
    constexpr int r3 = r2 + 64 * 32;               // W4
    constexpr int r4 = r3 + 2 * 32;                // biases, bounds
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < kNearBlobWork; q += gridDim.x * blockDim.x) {
        if (q < r0) {
            nb->mu_in[q] = prm[O.mu + q];
            nb->isd_in[q] = 1.f / prm[O.sd + q];
        } else if (q < r1) {
            const int r = q - r0, o = r / (kNearFeat / 2), k = r % (kNearFeat / 2);
            nb->W1[r] = pack_bf16(prm[O.W1 + (2 * k) * 64 + o], prm[O.W1 + (2 * k + 1) * 64 + o]);
        } else if (q < r2) {
            const int r = q - r1, o = r / 32, k = r % 32;
            nb->W2[r] = pack_bf16(prm[O.W2 + (2 * k) * 64 + o], prm[O.W2 + (2 * k + 1) * 64 + o]);
        } else if (q < r3) {
            const int r = q - r2, o = r / 32, k = r % 32;
            nb->W3[r] = pack_bf16(prm[O.W3 + (2 * k) * 64 + o], prm[O.W3 + (2 * k + 1) * 64 + o]);
        } else if (q < r4) {
            const int r = q - r3, o = r / 32, k = r % 32;
            nb->W4[r] = pack_bf16(prm[O.W4 + (2 * k) * 2 + o], prm[O.W4 + (2 * k + 1) * 2 + o]);
        } else {
            const int o = q - r4;                  // 0 .. 63
            nb->b1[o] = prm[O.b1 + o];
            nb->b2[o] = prm[O.b2 + o];
            nb->b3[o] = prm[O.b3 + o];
            if (o < 2) nb->b4[o] = prm[O.b4 + o];
            nb->bound[o] = o < n_bins ? bound[o] : 3e38f;
            nb->bound_zero[o] = (o < n_bins && bound_zero) ? bound_zero[o] : 3e38f;
            if (o == 0) {
                nb->n_bins = n_bins;
                nb->bin_lo = bin_lo;
                nb->bin_w = bin_w;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// a11: training (FP32)
// ---------------------------------------------------------------------------
// The training kernels give each sample a wave and each neuron a lane (the
// batch of a step is a few hundred samples: one thread per sample would leave
// most of the chip idle).  A neuron's sum runs over its inputs in the same
// order as a plain per-sample loop.  The wave passes a layer's activations to
// the next layer through its own row of LDS; the fences keep the compiler from
// moving the LDS accesses across the hand-over (LDS instructions of one wave
// complete in issue order).
__device__ __forceinline__ void mlp_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// one 64-neuron layer of sample's forward pass: lane o; in: the wave's LDS row
// (n_in values), written over by the layer's activations on return
__device__ __forceinline__ void mlp_fwd_layer(int n_in, const float *__restrict__ W, const float *__restrict__ b,
                                              float *row, int o, float *z, float *h) {
    float a = b[o];
    for (int k = 0; k < n_in; ++k) a = fmaf(row[k], W[k * 64 + o], a);
    const float hv = gelu_f(a);
    z[o] = a;
    h[o] = hv;
    mlp_wave_sync();                     // every lane has read the inputs
    row[o] = hv;
    mlp_wave_sync();
}

// per sample: forward, loss term, output delta dY = (Y - T) / B, and the
// pre-activations z1..z3 and activations h0..h3 kept for the backward pass
__global__ __launch_bounds__(256) void mlp_fwd(int32_t B, const int32_t *__restrict__ idx,
                                               const float *__restrict__ X, const float *__restrict__ T,
                                               const float *__restrict__ prm, float *__restrict__ act,
                                               float *__restrict__ dY, float *__restrict__ lossv) {
    __shared__ float rows[kBlock / kWave][64];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int s = blockIdx.x * (kBlock / kWave) + wv;
    if (s >= B) return;                  // wave-uniform; no block barrier below
    float *row = rows[wv];
    const MlpOffsets O;
    const int64_t i = idx ? idx[s] : s;
    float *A = act + (int64_t)s * kActStride;   // h0[20] z1[64] h1[64] z2[64] h2[64] z3[64] h3[64]
    float *h0 = A, *z1 = A + 20, *h1 = A + 84, *z2 = A + 148, *h2 = A + 212, *z3 = A + 276, *h3 = A + 340;
    if (lane < kNearFeat) {
        const float v = (X[i * kNearFeat + lane] - prm[O.mu + lane]) / prm[O.sd + lane];
        h0[lane] = v;
        row[lane] = v;
    }
    mlp_wave_sync();
    mlp_fwd_layer(kNearFeat, prm + O.W1, prm + O.b1, row, lane, z1, h1);
    mlp_fwd_layer(64, prm + O.W2, prm + O.b2, row, lane, z2, h2);
    mlp_fwd_layer(64, prm + O.W3, prm + O.b3, row, lane, z3, h3);
    float r = 0.f;
    if (lane < 2) {
        float a = prm[O.b4 + lane];
        for (int k = 0; k < 64; ++k) a = fmaf(row[k], prm[O.W4 + k * 2 + lane], a);
        r = a - T[i * 2 + lane];
        dY[s * 2 + lane] = r / (float)B;
    }
    const float r1 = __shfl(r, 1, kWave);
    if (lane == 0) lossv[s] = 0.5f * (r * r + r1 * r1) / (float)B;
}

// per sample: the deltas of the three hidden layers, written over z3, z2, z1
__global__ __launch_bounds__(256) void mlp_bwd(int32_t B, const float *__restrict__ prm, float *__restrict__ act,
                                               const float *__restrict__ dY) {
    __shared__ float rows[kBlock / kWave][64];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int s = blockIdx.x * (kBlock / kWave) + wv;
    if (s >= B) return;                  // wave-uniform
    float *row = rows[wv];
    const MlpOffsets O;
    float *A = act + (int64_t)s * kActStride;
    float *z1 = A + 20, *z2 = A + 148, *z3 = A + 276;
    const float g0 = dY[2 * s], g1 = dY[2 * s + 1];
    const float d3 = (prm[O.W4 + lane * 2] * g0 + prm[O.W4 + lane * 2 + 1] * g1) * gelu_grad_f(z3[lane]);
    z3[lane] = d3;
    row[lane] = d3;
    mlp_wave_sync();
    float a = 0.f;
    for (int o = 0; o < 64; ++o) a = fmaf(prm[O.W3 + lane * 64 + o], row[o], a);
    const float d2 = a * gelu_grad_f(z2[lane]);
    z2[lane] = d2;
    mlp_wave_sync();
    row[lane] = d2;
    mlp_wave_sync();
    a = 0.f;
    for (int o = 0; o < 64; ++o) a = fmaf(prm[O.W2 + lane * 64 + o], row[o], a);
    z1[lane] = a * gelu_grad_f(z1[lane]);
}

// gradient of every parameter: the sum over the batch of (input activation x
// delta), in kGradChunks contiguous runs of samples, each summed in sample
// order, then the runs added in order (fixed order: deterministic); a block
// holds 256 / kGradChunks parameters.  The loss is the sum of lossv.
constexpr int kGradChunks = 8;
__global__ __launch_bounds__(256) void mlp_grad(int32_t B, const float *__restrict__ act,
                                                const float *__restrict__ dY, const float *__restrict__ lossv,
                                                float *__restrict__ grad, float *__restrict__ loss) {
    constexpr int kPer = kBlock / kGradChunks;
    __shared__ float part[kGradChunks][kPer];
    const int pp = threadIdx.x % kPer, ch = threadIdx.x / kPer;
    const int p = blockIdx.x * kPer + pp;
    const MlpOffsets O;
    int hin = -1, dl = -1, dk = 0, width = 64;   // activation column, delta column
    if (p >= O.W1 && p < O.b1) { const int r = p - O.W1; hin = r / 64; dl = 20 + r % 64; }
    else if (p >= O.b1 && p < O.W2) { dl = 20 + (p - O.b1); }
    else if (p >= O.W2 && p < O.b2) { const int r = p - O.W2; hin = 84 + r / 64; dl = 148 + r % 64; }
    else if (p >= O.b2 && p < O.W3) { dl = 148 + (p - O.b2); }
    else if (p >= O.W3 && p < O.b3) { const int r = p - O.W3; hin = 212 + r / 64; dl = 276 + r % 64; }
    else if (p >= O.b3 && p < O.W4) { dl = 276 + (p - O.b3); }
    else if (p >= O.W4 && p < O.b4) { const int r = p - O.W4; hin = 340 + r / 2; dk = r % 2; width = 2; }
    else if (p >= O.b4 && p < O.total) { dk = p - O.b4; width = 2; }
    float g = 0.f;
    if (p >= O.W1 && p < O.total) {              // mu_in / sd_in are not trained
        const int s0 = (int)((int64_t)B * ch / kGradChunks), s1 = (int)((int64_t)B * (ch + 1) / kGradChunks);
        for (int s = s0; s < s1; ++s) {
            const float *A = act + (int64_t)s * kActStride;
            const float d = width == 2 ? dY[2 * s + dk] : A[dl];
            g = fmaf(hin >= 0 ? A[hin] : 1.f, d, g);
        }
    }
    part[ch][pp] = g;
    __syncthreads();
    if (ch == 0 && p < O.total) {
        float t = 0.f;
        for (int c = 0; c < kGradChunks; ++c) t += part[c][pp];
        grad[p] = t;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
        float l = 0.f;
        for (int s = 0; s < B; ++s) l += lossv[s];
        *loss = l;
    }
}

__global__ __launch_bounds__(256) void mlp_adam(float *__restrict__ prm, const float *__restrict__ grad,
                                                float *__restrict__ m, float *__restrict__ v, int32_t step, float lr,
                                                float b1, float b2, float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const MlpOffsets O;
    if (p >= O.total || p < O.W1) return;
    const float g = grad[p];
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.f - powf(b1, (float)step));
    const float vh = vv / (1.f - powf(b2, (float)step));
    prm[p] -= lr * mh / (sqrtf(vh) + eps);
}

// FP32 forward only (reference-precision inference, gradient checks)
__global__ __launch_bounds__(256) void mlp_fwd_only(int64_t n, const float *__restrict__ X,
                                                    const float *__restrict__ prm, float *__restrict__ Y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const MlpOffsets O;
    float h0[kNearFeat], h1[64], h2[64];
    for (int k = 0; k < kNearFeat; ++k) h0[k] = (X[i * kNearFeat + k] - prm[O.mu + k]) / prm[O.sd + k];
    for (int o = 0; o < 64; ++o) {
        float a = prm[O.b1 + o];
        for (int k = 0; k < kNearFeat; ++k) a = fmaf(h0[k], prm[O.W1 + k * 64 + o], a);
        h1[o] = gelu_f(a);
    }
    for (int o = 0; o < 64; ++o) {
        float a = prm[O.b2 + o];
        for (int k = 0; k < 64; ++k) a = fmaf(h1[k], prm[O.W2 + k * 64 + o], a);
        h2[o] = gelu_f(a);
    }
    for (int o = 0; o < 64; ++o) {
        float a = prm[O.b3 + o];
        for (int k = 0; k < 64; ++k) a = fmaf(h2[k], prm[O.W3 + k * 64 + o], a);
        h1[o] = gelu_f(a);
    }
    for (int o = 0; o < 2; ++o) {
        float a = prm[O.b4 + o];
        for (int k = 0; k < 64; ++k) a = fmaf(h1[k], prm[O.W4 + k * 2 + o], a);
        Y[i * 2 + o] = a;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static unsigned grid_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

hipError_t near_launch_upsample(const s2d_curves *c, int P, double *up, hipStream_t st) {
    if (c->n_curves <= 0) return hipSuccess;
    // LDS: 8 H node pairs and 12 (H + 1) coefficients at the largest N (21 KB)
    const size_t lds = (4 * (size_t)kUpMaxN + 12 * ((size_t)kUpMaxN / 2 + 1)) * sizeof(double);
    hipLaunchKernelGGL(near_upsample, dim3((unsigned)c->n_curves), dim3(kUpThreads), lds, st, c->curve_off, c->n_curves,
                       c->n_nodes, c->x, c->y, c->w, c->fx, c->fy, P, up);
    return hipGetLastError();
}

hipError_t near_launch_quad(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, const int32_t *list,
                            const int32_t *list_len, int P, const double *up, double mu, double *du, double *dv,
                            hipStream_t st, double *uf, double *vf, double *uc, double *vc) {
    if (t->n <= 0) return hipSuccess;
    const unsigned g = grid_for(t->n, kWave);
    hipLaunchKernelGGL(near_quad, dim3(g), dim3(kWave * kQuadParts), 0, st, t->n, list, list_len, t->x, t->y, tc,
                       c->curve_off,
                       c->n_curves, c->n_nodes, P, up, 1.0 / (4.0 * M_PI * mu), du,
                       dv, uf, vf, uc, vc);
    return hipGetLastError();
}

hipError_t near_launch_compact(int64_t n, const int32_t *flag, int32_t *cnt, int32_t *list, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kCompactBlock - 1) / kCompactBlock;
    hipLaunchKernelGGL(near_compact_count, dim3((unsigned)nb), dim3(kCompactBlock), 0, st, n, flag, cnt);
    hipLaunchKernelGGL(near_compact_scan, dim3(1), dim3(1024), 0, st, nb, cnt);
    hipLaunchKernelGGL(near_compact_scatter, dim3((unsigned)nb), dim3(kCompactBlock), 0, st, n, flag, cnt, list);
    return hipGetLastError();
}

hipError_t near_launch_features(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, float *X,
                                double *frame, hipStream_t st) {
    if (t->n <= 0) return hipSuccess;
    hipLaunchKernelGGL(near_features, dim3(grid_for(t->n)), dim3(256), 0, st, t->n, t->x, t->y, tc, c->curve_off,
                       c->n_curves, c->n_nodes, c->x, c->y, c->nx, c->ny, c->kappa, c->w, c->fx, c->fy, X, frame);
    return hipGetLastError();
}

hipError_t near_launch_wall_features(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, double d,
                                     float *X, double *frame, hipStream_t st) {
    if (t->n <= 0) return hipSuccess;
    // grid-stride: each block builds the cell table once for up to a few
    // thousand targets
    const int64_t blocks = std::min<int64_t>((t->n + 255) / 256, 1024);
    hipLaunchKernelGGL(near_wall_features, dim3((unsigned)blocks), dim3(256), 0, st, t->n, t->x, t->y,
                       tc, c->curve_off, c->n_curves, c->n_nodes, c->x, c->y, c->nx, c->ny, c->kappa, c->w, c->fx,
                       c->fy, d, X, frame);
    return hipGetLastError();
}

hipError_t near_launch_scale_labels(int64_t n, const double *du, const double *dv, const double *frame, double mu,
                                    float *Y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(near_scale_labels_k, dim3(grid_for(n)), dim3(256), 0, st, n, du, dv, frame, mu, Y);
    return hipGetLastError();
}

hipError_t near_launch_infer(int64_t n, const float *X, const double *frame, const NearBlob *nb, double mu,
                             double threshold, int use_bound, double *du, double *dv, int32_t *flag, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    // 32 targets per wave, 4 waves per block
    const int64_t groups = (n + 31) / 32;
    const int64_t blocks = (groups + 3) / 4;
    hipLaunchKernelGGL(near_mlp_infer_mfma, dim3((unsigned)blocks), dim3(256), 0, st, n, X, frame, nb, mu, threshold,
                       use_bound, du, dv, flag);
    return hipGetLastError();
}

hipError_t near_launch_pack(const float *prm, const float *bound, const float *bound_zero, int32_t n_bins,
                            float bin_lo, float bin_w, NearBlob *nb, hipStream_t st) {
    hipLaunchKernelGGL(near_pack, dim3(grid_for(kNearBlobWork)), dim3(256), 0, st, prm, bound, bound_zero, n_bins,
                       bin_lo, bin_w, nb);
    return hipGetLastError();
}

hipError_t near_launch_train_step(int32_t B, const int32_t *idx, const float *X, const float *T, float *prm,
                                  float *m, float *v, int32_t step, float lr, float *grad, float *act, float *dY,
                                  float *lossv, float *loss, int update, hipStream_t st) {
    const MlpOffsets O;
    const unsigned wave_blocks = (unsigned)((B + kBlock / kWave - 1) / (kBlock / kWave));   // a wave per sample
    hipLaunchKernelGGL(mlp_fwd, dim3(wave_blocks), dim3(kBlock), 0, st, B, idx, X, T, prm, act, dY, lossv);
    hipLaunchKernelGGL(mlp_bwd, dim3(wave_blocks), dim3(kBlock), 0, st, B, prm, act, dY);
    hipLaunchKernelGGL(mlp_grad, dim3((unsigned)((O.total + kBlock / kGradChunks - 1) / (kBlock / kGradChunks))),
                       dim3(kBlock), 0, st, B, act, dY, lossv, grad, loss);
    if (update)
        hipLaunchKernelGGL(mlp_adam, dim3(grid_for(O.total)), dim3(256), 0, st, prm, grad, m, v, step, lr, 0.9f,
                           0.999f, 1e-8f);
    return hipGetLastError();
}

hipError_t near_launch_fwd(int64_t n, const float *X, const float *prm, float *Y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_fwd_only, dim3(grid_for(n)), dim3(256), 0, st, n, X, prm, Y);
    return hipGetLastError();
}

}  // namespace s2d
