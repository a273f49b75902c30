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
//  * learned correction: the density's node derivatives d_p (p = 0..4) per
//    curve; per target its nearest node k*, the frame of k* (tangent along
//    the node order, normal towards the target), offsets (s, b) in units of
//    the local spacing and 14 geometry features; the correction is
//    Delta = scale sum_p (Cflat_p(s, b) + exp(-2 pi b) dC_p) d_p, with Cflat
//    the exact correction of a straight line with equispaced nodes (closed
//    form, by Poisson summation) and dC the output of a 14 -> 64 -> 64 -> 64
//    -> 20 tanh-form GELU network, weights and activations rounded to BF16,
//    products accumulated in FP32 on the matrix cores
//    (v_mfma_f32_32x32x8_bf16, 32 targets per wave).  A per-bin error bound
//    (bins in log10 b) calibrated on held-out data decides between no
//    correction, the network and the upsampled quadrature.
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
constexpr int kUpThreads = 192;   // the stages stride over their items (measured best of 128-320)

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

// The coarse node k and the fine node k P are the same point (the
// interpolant passes through the nodes): one squared distance, log and
// reciprocal serve both rules, with the fine record's weight (gfx, gfy) and
// the coarse one's (gcx, gcy); the node's FP64 coordinates are the coarse
// record's.
__device__ __forceinline__ void slp64_acc2(double px, double py, double sx, double sy, double gfx, double gfy,
                                           double gcx, double gcy, const double *ltab, double (&s)[8]) {
    const double rx = px - sx, ry = py - sy;
    const double q = __builtin_fma(rx, rx, ry * ry);
    const double lq = log64_tab(q, ltab);
    const double iq = rcp64(q);
    const double tf = __builtin_fma(rx, gfx, ry * gfy) * iq, tc = __builtin_fma(rx, gcx, ry * gcy) * iq;
    s[4] = __builtin_fma(gfx, lq, s[4]);
    s[5] = __builtin_fma(gfy, lq, s[5]);
    s[6] = __builtin_fma(rx, tf, s[6]);
    s[7] = __builtin_fma(ry, tf, s[7]);
    s[0] = __builtin_fma(gcx, lq, s[0]);
    s[1] = __builtin_fma(gcy, lq, s[1]);
    s[2] = __builtin_fma(rx, tc, s[2]);
    s[3] = __builtin_fma(ry, tc, s[3]);
}

// Part `part` of `parts` of the coarse (N nodes) and fine (P N nodes)
// single-layer sums of one curve, from the records {x, y, g_x, g_y} written
// by near_upsample: the coarse nodes k of the part (N part / parts <= k <
// N (part + 1) / parts) with the fine nodes k P .. k P + P - 1 that follow
// each; coarse sums go to s[0..3], fine ones to s[4..7].  PK: P known at
// compile time (its fine nodes unrolled), or 0.
template <bool UNIFORM, int PK>
__device__ __forceinline__ void near_sums(double px, double py, int lo, int N, int P, int64_t n_src, int part,
                                          int parts, const double *__restrict__ up, const double *ltab,
                                          double (&s)[8]) {
    if (UNIFORM) {
        lo = __builtin_amdgcn_readfirstlane(lo);
        N = __builtin_amdgcn_readfirstlane(N);
    }
    if (PK > 0) P = PK;
    const int ka = N * part / parts, kb = N * (part + 1) / parts;
    const double *cr = up + 4 * ((int64_t)n_src * P + lo);
    const double *fr = up + 4 * (int64_t)lo * P;
    // the fine nodes between coarse ones alternate between two accumulator
    // sets (t), added at the end: two independent chains
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = ka; k < kb; ++k) {
        const double *c = cr + 4 * k, *f = fr + 4 * (int64_t)k * P;
        slp64_acc2(px, py, c[0], c[1], f[2], f[3], c[2], c[3], ltab, s);
        if constexpr (PK > 0) {
#pragma unroll
            for (int j = 1; j < PK; ++j) {
                if (j & 1)
                    slp64_acc(px, py, f[4 * j], f[4 * j + 1], f[4 * j + 2], f[4 * j + 3], ltab, t[0], t[1], t[2],
                              t[3]);
                else
                    slp64_acc(px, py, f[4 * j], f[4 * j + 1], f[4 * j + 2], f[4 * j + 3], ltab, s[4], s[5], s[6],
                              s[7]);
            }
        } else {
            int j = 1;
            for (; j + 1 < P; j += 2) {
                slp64_acc(px, py, f[4 * j], f[4 * j + 1], f[4 * j + 2], f[4 * j + 3], ltab, t[0], t[1], t[2], t[3]);
                slp64_acc(px, py, f[4 * j + 4], f[4 * j + 5], f[4 * j + 6], f[4 * j + 7], ltab, s[4], s[5], s[6],
                          s[7]);
            }
            if (j < P)
                slp64_acc(px, py, f[4 * j], f[4 * j + 1], f[4 * j + 2], f[4 * j + 3], ltab, t[0], t[1], t[2], t[3]);
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) s[4 + e] += t[e];
}

// Delta for the 64 targets q = 64 blk + lane, or, with an index list, for
// targets list[q], q < *list_len (the list keeps the targets' order, so its
// waves stay on one curve).  The kQuadParts waves of the workgroup take the
// same targets and an equal share of the coarse nodes (with their fine
// nodes) each; wave 0 adds the others' partial sums in fixed order.  Short
// workgroups keep the launch balanced across curves of different sizes.  When every live target of the
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
    const double px = live ? tx[i] : tx[0], py = live ? ty[i] : ty[0];
    if (uniform) {
        // idle lanes follow the wave's curve (their results are dropped)
        const int cu = __builtin_amdgcn_readfirstlane(cmin);
        const int lou = off[cu], Nu = off[cu + 1] - lou;
        if (P == 8) near_sums<true, 8>(px, py, lou, Nu, P, n_src, part, kQuadParts, up, ltab, s);
        else near_sums<true, 0>(px, py, lou, Nu, P, n_src, part, kQuadParts, up, ltab, s);
    } else if (ok) {
        if (P == 8) near_sums<false, 8>(px, py, lo, N, P, n_src, part, kQuadParts, up, ltab, s);
        else near_sums<false, 0>(px, py, lo, N, P, n_src, part, kQuadParts, up, ltab, s);
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

// Order-keeping compaction of the targets with flag == value (AUTO's
// learned and fallback targets, one or both in the same pass): per-workgroup
// counts, one exclusive scan per value, then each workgroup writes its
// targets' indices at its offset in target order.
constexpr int kCompactBlock = 256;
constexpr int kScanThreads = 1024;

// one compaction: targets with flag == value into list, per-workgroup
// counts (then their exclusive scan and the total) in cnt; list == NULL
// switches it off
struct CompactOut {
    int value;
    int32_t *cnt, *list;
};

__device__ __forceinline__ int compact_flag(int64_t n, const int32_t *__restrict__ flag, int64_t i) {
    return i < n ? flag[i] : -1;
}

__global__ __launch_bounds__(kCompactBlock) void near_compact_count(int64_t n, const int32_t *__restrict__ flag,
                                                                    CompactOut a, CompactOut b) {
    __shared__ int wsum[2][kCompactBlock / kWave];
    const int64_t i = (int64_t)blockIdx.x * kCompactBlock + threadIdx.x;
    const int f = compact_flag(n, flag, i);
    const uint64_t ba = __ballot(f == a.value), bb = __ballot(f == b.value);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        wsum[0][threadIdx.x / kWave] = __popcll(ba);
        wsum[1][threadIdx.x / kWave] = __popcll(bb);
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const CompactOut &o = threadIdx.x == 0 ? a : b;
        int s = 0;
        for (int w = 0; w < kCompactBlock / kWave; ++w) s += wsum[threadIdx.x][w];
        if (o.list) o.cnt[blockIdx.x] = s;
    }
}

// exclusive scan of cnt[0 .. nb) in place, total in cnt[nb]: workgroup 0
// scans a's counts, workgroup 1 b's; each thread sums a contiguous segment,
// the segment sums are scanned by wave prefix sums and the waves' totals,
// then each thread writes its segment's prefixes
__global__ __launch_bounds__(kScanThreads) void near_compact_scan(int64_t nb, CompactOut a, CompactOut b) {
    __shared__ int wtot[kScanThreads / kWave];
    const CompactOut &o = blockIdx.x == 0 ? a : b;
    if (!o.list) return;                                   // workgroup-uniform
    int32_t *cnt = o.cnt;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int64_t seg = (nb + kScanThreads - 1) / kScanThreads;
    const int64_t b0 = min((int64_t)threadIdx.x * seg, nb), b1 = min(b0 + seg, nb);
    int s = 0;
    for (int64_t k = b0; k < b1; ++k) s += cnt[k];
    int x = s;                                             // inclusive prefix within the wave
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) wtot[wv] = x;
    __syncthreads();
    if (wv == 0) {
        int t = lane < kScanThreads / kWave ? wtot[lane] : 0;
#pragma unroll
        for (int d = 1; d < kScanThreads / kWave; d <<= 1) {
            const int y = __shfl_up(t, d, kWave);
            if (lane >= d) t += y;
        }
        if (lane < kScanThreads / kWave) wtot[lane] = t;   // inclusive totals
    }
    __syncthreads();
    int run = x - s + (wv > 0 ? wtot[wv - 1] : 0);
    for (int64_t k = b0; k < b1; ++k) {
        const int v = cnt[k];
        cnt[k] = run;
        run += v;
    }
    if (threadIdx.x == kScanThreads - 1) cnt[nb] = wtot[kScanThreads / kWave - 1];
}

__global__ __launch_bounds__(kCompactBlock) void near_compact_scatter(int64_t n, const int32_t *__restrict__ flag,
                                                                      CompactOut a, CompactOut b) {
    __shared__ int wsum[2][kCompactBlock / kWave];
    const int64_t i = (int64_t)blockIdx.x * kCompactBlock + threadIdx.x;
    const int f = compact_flag(n, flag, i);
    const uint64_t ba = __ballot(f == a.value), bb = __ballot(f == b.value);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) {
        wsum[0][w] = __popcll(ba);
        wsum[1][w] = __popcll(bb);
    }
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1;
    if (a.list && ((ba >> lane) & 1)) {
        int base = a.cnt[blockIdx.x];
        for (int k = 0; k < w; ++k) base += wsum[0][k];
        a.list[base + __popcll(ba & below)] = (int32_t)i;
    }
    if (b.list && ((bb >> lane) & 1)) {
        int base = b.cnt[blockIdx.x];
        for (int k = 0; k < w; ++k) base += wsum[1][k];
        b.list[base + __popcll(bb & below)] = (int32_t)i;
    }
}

// ---------------------------------------------------------------------------
// a9: the learned correction's inputs
// ---------------------------------------------------------------------------
// The correction Delta is linear in the density, and the trapezoid rules see
// the density only through its trigonometric interpolant.  Near the target's
// nearest node k* the interpolant is summarised by its derivatives there,
// d_p = (2 pi / N)^p d^p f / dt^p (p = 0..4, per-node units), and
//   Delta = scale * sum_p (Cflat_p(s, b) + exp(-2 pi b) dC_p) d_p
// in the frame (t, n) of k*: t along growing node index, n the normal turned
// towards the target, lengths in units of the local spacing hl = w_k*,
// (s, b) the target's offsets, scale = hl / 4 pi mu (single layer) or 1 / pi
// (double layer).  Cflat_p is the exact correction of a straight line with
// equispaced nodes (closed form, flat_* below), dC_p the network's output.

// Node derivatives of the density, one workgroup per curve (even N, 4 <= N <=
// kUpMaxN; larger even curves go to the kernels below): the interpolant's
// coefficients a_m, b_m (m = 0..N/2, the Nyquist mode's weight split evenly),
// then at each node sum_m (m h)^p times the p-th derivative of a_m cos(m t) +
// b_m sin(m t) at t_k (h = 2 pi / N; the Nyquist term keeps its even
// derivatives only: the odd ones vanish at the nodes).  Both stages use the
// reflection k -> N - k: the coefficients sum the even and odd parts
// f_k +- f_{N-k} over k < N/2, and a thread of the second stage evaluates the
// nodes k and N - k together (cos(m t) the same, sin(m t) of opposite sign).
// A thread takes one coefficient (mode, component) in the first stage and one
// node pair and component, all five p, in the second; each steps cos and sin
// of the multiple angles by rotation through its base angle (at most 128
// steps, rounding growing at most linearly), so no lane gathers from a
// table; the powers of m h come from a per-mode table in LDS (read as a
// broadcast).  Invalid curves get NaN.
__global__ __launch_bounds__(256) void near_derivs(const int32_t *__restrict__ off, int32_t n_curves, int64_t n_src,
                                                   const double *__restrict__ fx, const double *__restrict__ fy,
                                                   double *__restrict__ dtab, int32_t *__restrict__ big) {
    __shared__ double co[2][kUpMaxN / 2 + 1][2];
    __shared__ double eo[2][kUpMaxN / 2 + 1][2];      // {f_k + f_{N-k}, f_k - f_{N-k}}; k = 0, N/2: {f_k, 0}
    __shared__ double mp[kUpMaxN / 2 + 1][4];         // m h, -(m h)^2, -(m h)^3, (m h)^4
    const int c = blockIdx.x;
    if (c >= n_curves) return;
    const int lo = off[c], N = off[c + 1] - lo;
    if (lo < 0 || N <= 0 || (int64_t)lo + N > n_src) return;          // no rows of its own to fill
    if (N > kUpMaxN && !(N & 1)) {                                     // the large-curve kernels' work
        if (threadIdx.x == 0) big[0] = 1;
        return;
    }
    if (N < 4 || (N & 1)) {
        for (int q = threadIdx.x; q < N * 2 * kNearDeriv; q += blockDim.x)
            dtab[(int64_t)lo * 2 * kNearDeriv + q] = __builtin_nan("");
        return;
    }
    const int H = N / 2;
    const double h = 2.0 * M_PI / (double)N;
    for (int q = threadIdx.x; q < 2 * (H + 1); q += blockDim.x) {
        const int comp = q / (H + 1), k = q % (H + 1);
        const double *f = (comp ? fy : fx) + lo;
        const bool edge = k == 0 || k == H;
        const double p = f[k], r = edge ? 0.0 : f[N - k];
        eo[comp][k][0] = p + r;
        eo[comp][k][1] = p - r;
    }
    for (int m = threadIdx.x; m <= H; m += blockDim.x) {
        const double mh = (double)m * h, mh2 = mh * mh;
        mp[m][0] = mh;
        mp[m][1] = -mh2;
        mp[m][2] = -mh * mh2;
        mp[m][3] = mh2 * mh2;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * (H + 1); q += blockDim.x) {
        const int comp = q / (H + 1), m = q % (H + 1);
        double cb, sb;                                                 // cos, sin(2 pi m / N)
        sincospi(2.0 * (double)m / (double)N, &sb, &cb);
        double cm = cb, sm = sb;                                       // cos, sin(2 pi m k / N), k = 1
        // k = 0 and k = N/2 (cos = (-1)^m, sin = 0)
        double a = (m & 1) ? eo[comp][0][0] - eo[comp][H][0] : eo[comp][0][0] + eo[comp][H][0];
        double b = 0.0;
        for (int k = 1; k < H; ++k) {
            a = __builtin_fma(eo[comp][k][0], cm, a);
            b = __builtin_fma(eo[comp][k][1], sm, b);
            const double cn = __builtin_fma(cm, cb, -sm * sb);
            sm = __builtin_fma(sm, cb, cm * sb);
            cm = cn;
        }
        const double sc = (m == 0 || m == H) ? 1.0 / N : 2.0 / N;
        co[comp][m][0] = a * sc;
        co[comp][m][1] = (m == 0 || m == H) ? 0.0 : b * sc;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * (H + 1); q += blockDim.x) {
        const int comp = q / (H + 1), k = q % (H + 1);
        const bool pair = k != 0 && k != H;                            // node N - k is another node
        double cb, sb;                                                 // cos, sin(2 pi k / N)
        sincospi(2.0 * (double)k / (double)N, &sb, &cb);
        double cm = 1.0, sm = 0.0;                                     // cos, sin(2 pi m k / N)
        double acc[kNearDeriv], acr[kNearDeriv];                       // node k, node N - k
        acc[0] = acr[0] = co[comp][0][0];
#pragma unroll
        for (int p = 1; p < kNearDeriv; ++p) acc[p] = acr[p] = 0.0;
        for (int m = 1; m <= H; ++m) {
            const double cn = __builtin_fma(cm, cb, -sm * sb);
            sm = __builtin_fma(sm, cb, cm * sb);
            cm = cn;
            const double a = co[comp][m][0], b = co[comp][m][1];
            // (m h)^p times the p-th derivative of a cos + b sin: the
            // derivatives cycle through g0, g1, -g0, -g1; at N - k the sine
            // changes sign
            const double bs = b * sm, ac = a * cm;
            const double g0 = ac + bs, r0 = ac - bs;
            const double bc = b * cm;
            const double g1 = __builtin_fma(-a, sm, bc), r1 = __builtin_fma(a, sm, bc);
            const double p1 = mp[m][0], p2 = mp[m][1], p3 = mp[m][2], p4 = mp[m][3];
            acc[0] += g0;
            acr[0] += r0;
            if (m < H) {
                acc[1] = __builtin_fma(p1, g1, acc[1]);
                acr[1] = __builtin_fma(p1, r1, acr[1]);
                acc[3] = __builtin_fma(p3, g1, acc[3]);
                acr[3] = __builtin_fma(p3, r1, acr[3]);
            }
            acc[2] = __builtin_fma(p2, g0, acc[2]);
            acr[2] = __builtin_fma(p2, r0, acr[2]);
            acc[4] = __builtin_fma(p4, g0, acc[4]);
            acr[4] = __builtin_fma(p4, r0, acr[4]);
        }
        double *row = dtab + ((int64_t)lo + k) * 2 * kNearDeriv + comp;
#pragma unroll
        for (int p = 0; p < kNearDeriv; ++p) row[2 * p] = acc[p];
        if (pair) {
            double *rr = dtab + ((int64_t)lo + N - k) * 2 * kNearDeriv + comp;
#pragma unroll
            for (int p = 0; p < kNearDeriv; ++p) rr[2 * p] = acr[p];
        }
    }
}

// The same derivatives for curves of more than kUpMaxN nodes (walls of
// thousands of nodes), spread over the chip: the table of cos, sin(2 pi j /
// N) (row lo + j), then one wave per coefficient m (row lo + m, m <= N/2 <
// N) summing over the nodes in lane-strided order, then one wave per node
// summing over the modes.  Wave partial sums are added by a fixed butterfly.
// The kernels stride over the rows with a fixed grid and return at once
// unless near_derivs flagged a large curve (big[0] != 0).
__device__ __forceinline__ int curve_of(const int32_t *__restrict__ off, int n_curves, int64_t q) {
    int lo = 0, hi = n_curves - 1;                       // last c with off[c] <= q
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)off[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// the curve of row q and its range, if it is a valid curve of more than
// kUpMaxN (even) nodes
__device__ __forceinline__ bool big_curve(const int32_t *__restrict__ off, int32_t n_curves, int64_t n_src, int64_t q,
                                          int &lo, int &N) {
    if (n_curves <= 0 || q >= n_src) return false;
    const int c = curve_of(off, n_curves, q);
    lo = off[c];
    N = off[c + 1] - lo;
    return lo >= 0 && (int64_t)lo + N <= n_src && q >= lo && q < (int64_t)lo + N && N > kUpMaxN && !(N & 1);
}

constexpr int kBigBlocks = 1024;
constexpr int kInferCUs = 256;

__global__ __launch_bounds__(256) void near_derivs_table(const int32_t *__restrict__ off, int32_t n_curves,
                                                         int64_t n_src, const int32_t *__restrict__ big,
                                                         double *__restrict__ tab) {
    if (big[0] == 0) return;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_src; q += (int64_t)gridDim.x * blockDim.x) {
        int lo, N;
        if (!big_curve(off, n_curves, n_src, q, lo, N)) continue;
        double sv, cv;
        sincospi(2.0 * (double)(q - lo) / (double)N, &sv, &cv);
        tab[2 * q] = cv;
        tab[2 * q + 1] = sv;
    }
}

// coefficients {a_x, b_x, a_y, b_y} of mode m at coef[4 (lo + m)]
__global__ __launch_bounds__(256) void near_derivs_coef(const int32_t *__restrict__ off, int32_t n_curves,
                                                        int64_t n_src, const int32_t *__restrict__ big,
                                                        const double *__restrict__ fx, const double *__restrict__ fy,
                                                        const double *__restrict__ tab, double *__restrict__ coef) {
    if (big[0] == 0) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; q < n_src; q += waves) {
        int lo, N;
        if (!big_curve(off, n_curves, n_src, q, lo, N)) continue;       // wave-uniform
        const int H = N / 2, m = (int)(q - lo);
        if (m > H) continue;
        double ax = 0.0, bx = 0.0, ay = 0.0, by = 0.0;
        int j = (int)(((int64_t)m * lane) % N);                         // (m k) mod N, stepped by 64 m
        const int step = (int)(((int64_t)m * kWave) % N);
        for (int k = lane; k < N; k += kWave) {
            const double c = tab[2 * ((int64_t)lo + j)], sn = tab[2 * ((int64_t)lo + j) + 1];
            ax = __builtin_fma(fx[lo + k], c, ax);
            bx = __builtin_fma(fx[lo + k], sn, bx);
            ay = __builtin_fma(fy[lo + k], c, ay);
            by = __builtin_fma(fy[lo + k], sn, by);
            j += step;
            j = j >= N ? j - N : j;
        }
        ax = wave_sum_d(ax);
        bx = wave_sum_d(bx);
        ay = wave_sum_d(ay);
        by = wave_sum_d(by);
        if (lane == 0) {
            const bool edge = m == 0 || m == H;
            const double sc = edge ? 1.0 / N : 2.0 / N;
            coef[4 * q] = ax * sc;
            coef[4 * q + 1] = edge ? 0.0 : bx * sc;
            coef[4 * q + 2] = ay * sc;
            coef[4 * q + 3] = edge ? 0.0 : by * sc;
        }
    }
}

__global__ __launch_bounds__(256) void near_derivs_nodes(const int32_t *__restrict__ off, int32_t n_curves,
                                                         int64_t n_src, const int32_t *__restrict__ big,
                                                         const double *__restrict__ tab,
                                                         const double *__restrict__ coef, double *__restrict__ dtab) {
    if (big[0] == 0) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; q < n_src; q += waves) {
        int lo, N;
        if (!big_curve(off, n_curves, n_src, q, lo, N)) continue;       // wave-uniform
        const int H = N / 2, k = (int)(q - lo);
        const double h = 2.0 * M_PI / (double)N;
        double acc[2 * kNearDeriv];
#pragma unroll
        for (int r = 0; r < 2 * kNearDeriv; ++r) acc[r] = 0.0;
        int j = (int)(((int64_t)(1 + lane) * k) % N);                   // (m k) mod N, stepped by 64 k
        const int step = (int)(((int64_t)kWave * k) % N);
        for (int m = 1 + lane; m <= H; m += kWave) {
            const double c = tab[2 * ((int64_t)lo + j)], sn = tab[2 * ((int64_t)lo + j) + 1];
            j += step;
            j = j >= N ? j - N : j;
            const double *co = coef + 4 * ((int64_t)lo + m);
            // (m h)^p times the p-th derivative of a cos + b sin: the derivatives
            // cycle through g0, g1, -g0, -g1
            const double gx0 = __builtin_fma(co[0], c, co[1] * sn), gx1 = __builtin_fma(-co[0], sn, co[1] * c);
            const double gy0 = __builtin_fma(co[2], c, co[3] * sn), gy1 = __builtin_fma(-co[2], sn, co[3] * c);
            const double mh = (double)m * h;
            double mp = 1.0;
#pragma unroll
            for (int p = 0; p < kNearDeriv; ++p) {
                if (!(m == H && (p & 1))) {
                    const double sg = (p & 2) ? -1.0 : 1.0;
                    acc[2 * p] = __builtin_fma(mp, sg * ((p & 1) ? gx1 : gx0), acc[2 * p]);
                    acc[2 * p + 1] = __builtin_fma(mp, sg * ((p & 1) ? gy1 : gy0), acc[2 * p + 1]);
                }
                mp *= mh;
            }
        }
#pragma unroll
        for (int r = 0; r < 2 * kNearDeriv; ++r) acc[r] = wave_sum_d(acc[r]);
        if (lane == 0) {
            acc[0] += coef[4 * (int64_t)lo];
            acc[1] += coef[4 * (int64_t)lo + 2];
#pragma unroll
            for (int r = 0; r < 2 * kNearDeriv; ++r) dtab[q * 2 * kNearDeriv + r] = acc[r];
        }
    }
}

// The frame in registers: the kNearFrame words of the frame record, then
// exp(-2 pi b), cos(-2 pi s) and sin(-2 pi s) (Q of the plain rule, kept for
// the straight-line part; not part of the stored record).
constexpr int kNearRec = kNearFrame + 3;

// exp(-2 pi b) and (cos, sin)(-2 pi s) (the one expression every caller uses)
__device__ __forceinline__ void flat_q(double s, double b, double &aq, double &cq, double &sq) {
    sincospi(-2.0 * s, &sq, &cq);
    aq = exp(-2.0 * M_PI * b);
}

// Geometry features and frame of a target p whose nearest node is at (X, Y)
// with unit normal (NX, NY), curvature kap and spacing hl, nb[j] the nodes
// k* - 2, k* - 1, k* + 1, k* + 2: xi = [s, b, ln(|p - x_k*| / hl), sg kap hl,
// the four nodes in the frame (units hl), Re Q, Im Q], Q = exp(-2 pi (b + i s));
// fr[0..8] = s, b, t, n_f, hl, (F later), sg; fr[19] = sg kap hl; fr[20..22]
// = exp(-2 pi b), cos(-2 pi s), sin(-2 pi s).
__device__ __forceinline__ void near_frame_features(double px, double py, double X, double Y, double NX,
                                                    double NY, double kap, double hl, const double (&nb)[4][2],
                                                    float *__restrict__ xi, double *__restrict__ fr) {
    const double st = ((nb[2][0] - nb[1][0]) * -NY + (nb[2][1] - nb[1][1]) * NX) >= 0.0 ? 1.0 : -1.0;
    const double tx = -st * NY, ty = st * NX;
    const double ox = px - X, oy = py - Y;
    const double ih = 1.0 / hl;
    const double sv = (ox * tx + oy * ty) * ih;
    const double nv = (ox * NX + oy * NY) * ih;
    const double sg = nv >= 0.0 ? 1.0 : -1.0;
    const double nfx = sg * NX, nfy = sg * NY;
    const double b = sg * nv;
    xi[0] = (float)sv;
    xi[1] = (float)b;
    xi[2] = (float)log(sqrt(ox * ox + oy * oy) * ih);
    xi[3] = (float)(sg * kap * hl);
    for (int j = 0; j < 4; ++j) {
        const double gx = nb[j][0] - X, gy = nb[j][1] - Y;
        xi[4 + 2 * j] = (float)((gx * tx + gy * ty) * ih);
        xi[5 + 2 * j] = (float)((gx * nfx + gy * nfy) * ih);
    }
    double aq, cq, sq;
    flat_q(sv, b, aq, cq, sq);
    xi[12] = (float)(aq * cq);
    xi[13] = (float)(aq * sq);
    fr[kNearFrame] = aq;
    fr[kNearFrame + 1] = cq;
    fr[kNearFrame + 2] = sq;
    fr[0] = sv;
    fr[1] = b;
    fr[2] = tx;
    fr[3] = ty;
    fr[4] = nfx;
    fr[5] = nfy;
    fr[6] = hl;
    fr[8] = sg;
    fr[kNearFrame - 1] = sg * kap * hl;
}

// the density's derivatives at the node (row of the derivative table) in
// the frame, and F = sum |d| over p and both components (1 if zero): the
// unit of AUTO's calibrated bounds
__device__ __forceinline__ void near_frame_head(const double *__restrict__ drow, double *__restrict__ fr) {
    double F = 0.0;
#pragma unroll
    for (int p = 0; p < kNearDeriv; ++p) {
        const double dx = drow[2 * p], dy = drow[2 * p + 1];
        const double dt = dx * fr[2] + dy * fr[3], dn = dx * fr[4] + dy * fr[5];
        fr[9 + 2 * p] = dt;
        fr[10 + 2 * p] = dn;
        F += fabs(dt) + fabs(dn);
    }
    fr[7] = F > 0.0 ? F : 1.0;
}

__device__ __forceinline__ void near_invalid(float *__restrict__ xi, double *__restrict__ fr) {
    for (int k = 0; k < kNearFeat; ++k) xi[k] = __builtin_nanf("");
    for (int k = 0; k < kNearRec; ++k) fr[k] = __builtin_nan("");
}

// nearest node k* (smallest index on ties) of the curve at [lo, lo + N);
// UNIFORM: lo and N are the same in every lane (loads take the scalar path)
template <bool UNIFORM>
__device__ __forceinline__ int near_scan(double px, double py, int lo, int N, const double *__restrict__ x,
                                         const double *__restrict__ y, double &best) {
    if (UNIFORM) {
        lo = __builtin_amdgcn_readfirstlane(lo);
        N = __builtin_amdgcn_readfirstlane(N);
    }
    best = 1e300;
    int ks = 0;
#pragma unroll 4
    for (int k = 0; k < N; ++k) {
        const double dx = px - x[lo + k], dy = py - y[lo + k];
        const double d2 = dx * dx + dy * dy;
        if (d2 < best) { best = d2; ks = k; }
    }
    return ks;
}

template <int OP>
__device__ __forceinline__ int near_decide_one(int64_t i, const double *fr, const DecideArgs &a, int c);
template <int OP>
__device__ void near_learned_head(int64_t i, const double *rec, const DecideArgs &a, float *__restrict__ nrec);

// What a launch of near_features computes:
// - kFeatFrame: the features X and the frame records (training, calibration);
// - kFeatScan: the features X and the nearest node k* (kstar, -1 for an
//   invalid target), without the density: it can run beside near_derivs;
// - kFeatHead: from kstar and the derivative table, the frame in registers,
//   AUTO's decision (near_decide_one) and, for a learned target, its
//   straight-line part and network record (near_learned_head);
// - kFeatFused: kFeatScan and kFeatHead in one launch (the frame stays in
//   registers; no kstar).
// The frames of kFeatHead and kFeatFused are the one kFeatFrame writes, bit
// for bit (the same code from the same nearest node).
constexpr int kFeatFrame = 0, kFeatScan = 1, kFeatHead = 2, kFeatFused = 3;

template <int MODE>
__global__ __launch_bounds__(256) void near_features(int64_t n_trg, const double *__restrict__ tx,
                                                     const double *__restrict__ ty, const int32_t *__restrict__ tc,
                                                     const int32_t *__restrict__ off, int32_t n_curves, int64_t n_src,
                                                     const double *__restrict__ x, const double *__restrict__ y,
                                                     const double *__restrict__ nx, const double *__restrict__ ny,
                                                     const double *__restrict__ kap, const double *__restrict__ w,
                                                     const double *__restrict__ dtab, float *__restrict__ X,
                                                     double *__restrict__ frame, int32_t *__restrict__ kstar,
                                                     float *__restrict__ nrec, DecideArgs da) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = q < n_trg;
    const int64_t i = live ? q : 0;
    const int c = live ? tc[i] : -1;
    const int lo = (c >= 0 && c < n_curves) ? off[c] : 0;
    const int N = (c >= 0 && c < n_curves) ? off[c + 1] - lo : 0;
    bool ok = c >= 0 && c < n_curves && N >= 8 && lo >= 0 && (int64_t)lo + N <= n_src;
    const double px = live ? tx[i] : 0.0, py = live ? ty[i] : 0.0;
    int ks = 0;
    if constexpr (MODE == kFeatHead) {
        if (!live) return;
        ks = kstar[i];
        ok = ok && ks >= 0 && ks < N;
    } else {
        // a wave is uniform when all its live lanes share one valid curve
        // (every lane of the wave reaches this vote)
        const int cl = ok ? c : INT_MAX;
        const int cmin = wave_min(cl);
        const bool uniform = cmin != INT_MAX && __all(!live || (ok && c == cmin));
        double best = 0.0;
        if (uniform) {
            const int cu = __builtin_amdgcn_readfirstlane(cmin);
            const int lou = off[cu];
            ks = near_scan<true>(px, py, lou, off[cu + 1] - lou, x, y, best);
        } else if (ok) {
            ks = near_scan<false>(px, py, lo, N, x, y, best);
        }
        if (!live) return;
        if constexpr (MODE == kFeatScan) kstar[i] = ok ? ks : -1;
    }
    float xl[kNearFeat];
    float *xi = MODE == kFeatHead ? xl : X + i * kNearFeat;
    double rec[kNearRec];
    if (!ok) {
        near_invalid(xi, rec);
    } else {
        double nb[4][2];
        const int js[4] = {-2, -1, 1, 2};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = lo + (ks + js[j] + N) % N;
            nb[j][0] = x[k];
            nb[j][1] = y[k];
        }
        const int k = lo + ks;
        near_frame_features(px, py, x[k], y[k], nx[k], ny[k], kap[k], w[k], nb, xi, rec);
        if constexpr (MODE != kFeatScan) near_frame_head(dtab + (int64_t)k * 2 * kNearDeriv, rec);
    }
    if constexpr (MODE == kFeatHead || MODE == kFeatFused) {
        if (near_decide_one<S2D_OP_SLP>(i, rec, da, c) == 0) near_learned_head<S2D_OP_SLP>(i, rec, da, nrec);
    } else if constexpr (MODE == kFeatFrame) {
        double *fr = frame + i * kNearFrame;
#pragma unroll
        for (int r = 0; r < kNearFrame; ++r) fr[r] = rec[r];
    }
}

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
// table is built once per block in LDS): one period of wall curve tc[i] (N >=
// 8 nodes advancing by sgd d in x), unrolled over three periods (node K in
// [-N, 2N) at (x_{K mod N} + sgd d floor(K / N), y_{K mod N})); the nearest
// unrolled node k* (smallest K on ties) and its unrolled neighbours give the
// features as for closed curves.
// FUSE as for near_features (the double layer's straight-line part)
template <bool FUSE>
__global__ __launch_bounds__(256) void near_wall_features(int64_t n_trg, const double *__restrict__ tx,
                                                          const double *__restrict__ ty,
                                                          const int32_t *__restrict__ tc,
                                                          const int32_t *__restrict__ off, int32_t n_curves,
                                                          int64_t n_src, const double *__restrict__ x,
                                                          const double *__restrict__ y,
                                                          const double *__restrict__ nx,
                                                          const double *__restrict__ ny,
                                                          const double *__restrict__ kap,
                                                          const double *__restrict__ w, double d,
                                                          const double *__restrict__ dtab, float *__restrict__ X,
                                                          double *__restrict__ frame, float *__restrict__ nrec,
                                                          DecideArgs da) {
    __shared__ WallCells W;
    wall_cells_build(W, off, n_curves, n_src, x, y, w);
    const bool cells = W.ok != 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_trg; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = tc[i];
        const int lo = (c >= 0 && c < n_curves) ? off[c] : 0;
        const int N = (c >= 0 && c < n_curves) ? off[c + 1] - lo : 0;
        float *xi = X + i * kNearFeat;
        double rec[kNearRec];
        // the frame record's destination: the frame array, or the fused
        // decision and learned head
        const auto emit = [&]() {
            if constexpr (FUSE) {
                if (near_decide_one<S2D_OP_DLP>(i, rec, da, c) == 0) near_learned_head<S2D_OP_DLP>(i, rec, da, nrec);
            } else {
                double *fr = frame + i * kNearFrame;
#pragma unroll
                for (int r = 0; r < kNearFrame; ++r) fr[r] = rec[r];
            }
        };
        if (c < 0 || c >= n_curves || N < 8 || lo < 0 || (int64_t)lo + N > n_src) {
            near_invalid(xi, rec);
            emit();
            continue;
        }
        const double sgd = x[lo + 1] > x[lo] ? 1.0 : -1.0;
        const double px = tx[i], py = ty[i];
        double best = 0.0;
        const int ks = wall_nearest(W, cells, c, lo, N, sgd, d, px, py, x, y, best);
        const auto md = [N](int K) { return ((K % N) + N) % N; };
        const auto fl = [N](int K) { return K >= 0 ? K / N : -((-K + N - 1) / N); };
        double nb[4][2];
        const int js[4] = {-2, -1, 1, 2};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int K = ks + js[j];
            nb[j][0] = x[lo + md(K)] + sgd * d * (double)fl(K);
            nb[j][1] = y[lo + md(K)];
        }
        const int m = lo + md(ks);
        near_frame_features(px, py, x[m] + sgd * d * (double)fl(ks), y[m], nx[m], ny[m], kap[m], w[m], nb, xi,
                            rec);
        near_frame_head(dtab + (int64_t)m * 2 * kNearDeriv, rec);
        emit();
    }
}

// ---------------------------------------------------------------------------
// the straight-line coefficients (closed form)
// ---------------------------------------------------------------------------
// On the line y = 0 with nodes at the integers (weight 1), density tau^p / p!,
// target (s, b), b > 0, the error of the trapezoid rule of spacing D is, by
// Poisson summation, sum_{l != 0} g^(2 pi l / D).  For the single-layer
// kernel (-1/2 log q + a^2/q, a b/q, -1/2 log q + b^2/q with a = s - tau,
// q = a^2 + b^2) the transforms are e^{-i w s - b |w|} times pi/|w| - pi b,
// i pi b sgn(w), pi/|w| + pi b; multiplying by tau^p is (i d/dw)^p, pairs
// l, -l are complex conjugates, and the sums over l are polylogarithms of
// Q = exp(-c z), c = 2 pi / D, z = b + i s:
//   S1_p = pi sum_j C(p, j) (-z)^(p-j) (-1)^j j! c^-(j+1) Li_{j+1}(Q),
//   S0_p = (-z)^p Li_0(Q),
//   E_TT = (2/p!) Re[i^p (S1_p - pi b S0_p)], E_NN = (2/p!) Re[i^p (S1_p + pi b S0_p)],
//   E_TN = (2/p!) Re[i^(p+1) pi b S0_p].
// Li_0 = Q / (1 - Q) and Li_1 = -log(1 - Q) are closed; Li_2..Li_5 are their
// series, truncated after L terms (|Q| = exp(-2 pi b / D)).  The double
// layer's kernel b r r^T / q^2 has the transforms (pi/2)(1 - b|w|),
// i (pi/2) b w, (pi/2)(1 + b|w|) times the same phase, polynomial in w: its
// sums need only Li_0 and Li_-1 = Q / (1 - Q)^2.  Each rule's coefficients
// are returned contracted with the density derivatives d[p][in] (frame).
struct Cx {
    double re, im;
};
__device__ __forceinline__ Cx cx_mul(Cx a, Cx b) {
    return {__builtin_fma(a.re, b.re, -a.im * b.im), __builtin_fma(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ Cx cx_add(Cx a, Cx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Cx cx_scale(Cx a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ Cx cx_div(Cx a, Cx b) {
    const double d = __builtin_fma(b.re, b.re, b.im * b.im);
    return {__builtin_fma(a.re, b.re, a.im * b.im) / d, __builtin_fma(a.im, b.re, -a.re * b.im) / d};
}
// i^p c for p = 0..3 (mod 4)
__device__ __forceinline__ Cx cx_ipow(int p, Cx c) {
    switch (p & 3) {
    case 0: return c;
    case 1: return {-c.im, c.re};
    case 2: return {-c.re, -c.im};
    default: return {c.im, -c.re};
    }
}

// 1 / l^k for l = 1..64, k = 2..5 (the polylogarithm series)
struct InvPowTab {
    double v[65][4];
    constexpr InvPowTab() : v() {
        for (int l = 1; l <= 64; ++l) {
            const double r = 1.0 / (double)l;
            double q = r * r;
            for (int k = 0; k < 4; ++k) {
                v[l][k] = q;
                q *= r;
            }
        }
    }
};
__constant__ InvPowTab kInvPow = InvPowTab();
constexpr int kPolyCoarse = 64, kPolyFine = 16;

// C(p, j) (-1)^j j! and 2 / p! (the coefficients of S1_p and of E_p)
struct FlatCoef {
    double bj[kNearDeriv][kNearDeriv];
    double f[kNearDeriv];
    constexpr FlatCoef() : bj(), f() {
        double fact = 1.0;
        for (int p = 0; p < kNearDeriv; ++p) {
            if (p > 0) fact *= (double)p;
            f[p] = 2.0 / fact;
            double binom = 1.0, jf = 1.0;
            for (int j = 0; j <= p; ++j) {
                if (j > 0) {
                    binom = binom * (double)(p - j + 1) / (double)j;
                    jf *= (double)j;
                }
                bj[p][j] = binom * ((j & 1) ? -jf : jf);
            }
        }
    }
};
__constant__ FlatCoef kFlat = FlatCoef();

// sum_p E_p(rule of spacing D = 1 / inv_d) d_p for the single (OP =
// S2D_OP_SLP) or double layer; out = (t, n) components
// Q = exp(-2 pi inv_d (b + i s)) is passed in (flat_pair)
template <int OP>
__device__ void flat_rule(double s, double b, double inv_d, Cx Q, int L, const double *__restrict__ dfr,
                          double (&out)[2]) {
    const double c = 2.0 * M_PI * inv_d;
    const Cx om = {1.0 - Q.re, -Q.im};                       // 1 - Q
    const Cx L0 = cx_div(Q, om);
    Cx zp[kNearDeriv];                                       // (-z)^k
    zp[0] = {1.0, 0.0};
    for (int k = 1; k < kNearDeriv; ++k) zp[k] = cx_mul(zp[k - 1], {-b, -s});
    out[0] = out[1] = 0.0;
    if constexpr (OP == S2D_OP_SLP) {
        Cx Li[kNearDeriv + 1];
        Li[0] = L0;
        Li[1] = {-0.5 * log(om.re * om.re + om.im * om.im), -atan2(om.im, om.re)};   // -log(1 - Q)
        Cx acc[kNearDeriv - 1] = {};
        Cx ql = {1.0, 0.0};
        for (int l = 1; l <= L; ++l) {
            ql = cx_mul(ql, Q);
#pragma unroll
            for (int k = 0; k < kNearDeriv - 1; ++k) acc[k] = cx_add(acc[k], cx_scale(ql, kInvPow.v[l][k]));
        }
        for (int k = 2; k <= kNearDeriv; ++k) Li[k] = acc[k - 2];
        const double ic = (0.5 / M_PI) / inv_d;              // 1 / c
#pragma unroll
        for (int p = 0; p < kNearDeriv; ++p) {
            Cx S1 = {0.0, 0.0};
            double icj = ic;                                 // c^-(j+1)
#pragma unroll
            for (int j = 0; j <= p; ++j) {
                if (j > 0) icj *= ic;
                S1 = cx_add(S1, cx_scale(cx_mul(zp[p - j], Li[j + 1]), kFlat.bj[p][j] * icj));
            }
            S1 = cx_scale(S1, M_PI);
            const Cx S0 = cx_mul(zp[p], L0);
            const double f = kFlat.f[p];
            const double ett = f * cx_ipow(p, {S1.re - M_PI * b * S0.re, S1.im - M_PI * b * S0.im}).re;
            const double enn = f * cx_ipow(p, {S1.re + M_PI * b * S0.re, S1.im + M_PI * b * S0.im}).re;
            const double etn = f * cx_ipow(p + 1, cx_scale(S0, M_PI * b)).re;
            const double dt = dfr[2 * p], dn = dfr[2 * p + 1];
            out[0] = __builtin_fma(ett, dt, __builtin_fma(etn, dn, out[0]));
            out[1] = __builtin_fma(etn, dt, __builtin_fma(enn, dn, out[1]));
        }
    } else {
        const Cx Lm1 = cx_div(L0, om);                       // Q / (1 - Q)^2
#pragma unroll
        for (int p = 0; p < kNearDeriv; ++p) {
            // sum_l d^p/dw^p [e^{-wz} (alpha + beta w)] = alpha (-z)^p L0 + beta ((-z)^p c Lm1 + p (-z)^(p-1) L0)
            const Cx base = cx_mul(zp[p], L0);
            Cx lin = cx_scale(cx_mul(zp[p], Lm1), c);
            if (p > 0) lin = cx_add(lin, cx_scale(cx_mul(zp[p - 1], L0), (double)p));
            const double f = kFlat.f[p];
            const double h = 0.5 * M_PI;
            const double ett = f * cx_ipow(p, {h * (base.re - b * lin.re), h * (base.im - b * lin.im)}).re;
            const double enn = f * cx_ipow(p, {h * (base.re + b * lin.re), h * (base.im + b * lin.im)}).re;
            const double etn = f * cx_ipow(p + 1, cx_scale(lin, h * b)).re;
            const double dt = dfr[2 * p], dn = dfr[2 * p + 1];
            out[0] = __builtin_fma(ett, dt, __builtin_fma(etn, dn, out[0]));
            out[1] = __builtin_fma(etn, dt, __builtin_fma(enn, dn, out[1]));
        }
    }
}

// The straight-line parts of the refined rule (spacing 1 / P: Q^P, by
// repeated squaring) and of the plain one (Q = aq (cq + i sq)), the refined
// with L = kPolyFine polylogarithm terms and the plain with kPolyCoarse.
template <int OP>
__device__ __forceinline__ void flat_pair(double s, double b, int P, double aq, double cq, double sq,
                                          const double *__restrict__ dfr, double (&ff)[2], double (&fc)[2]) {
    const Cx Q = {aq * cq, aq * sq};
    Cx QP = {1.0, 0.0}, base = Q;
    for (int e = P; e > 0; e >>= 1) {
        if (e & 1) QP = cx_mul(QP, base);
        if (e > 1) base = cx_mul(base, base);
    }
    flat_rule<OP>(s, b, (double)P, QP, kPolyFine, dfr, ff);
    flat_rule<OP>(s, b, 1.0, Q, kPolyCoarse, dfr, fc);
}

// ---------------------------------------------------------------------------
// MLP pieces
// ---------------------------------------------------------------------------
// tanh-form GELU, 0.5 z (1 + tanh u) with u = sqrt(2/pi) (z + 0.044715 z^3),
// taken as z / (1 + exp(-2u)) (the same function: 1 + tanh u = 2 / (1 +
// exp(-2u))): one exponential, one reciprocal and six other instructions
// per neuron; exp via the hardware exp2, its argument clamped so that the
// sum stays finite
constexpr float kGeluK = -2.0f * 0.7978845608028654f * 1.4426950408889634f;   // -2 sqrt(2/pi) log2(e)

__device__ __forceinline__ float gelu_sig(float z) {
    // 1 / (1 + exp(-2u)) = (1 + tanh u) / 2
    const float t = z * __builtin_fmaf(0.044715f * kGeluK, z * z, kGeluK);
    return __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(fminf(t, 126.f)) + 1.f);
}

__device__ __forceinline__ float gelu_f(float z) { return z * gelu_sig(z); }

// d/dz: s + 2 z s (1 - s) du/dz with s = (1 + tanh u) / 2 (the tanh form's
// derivative 0.5 (1 + tanh u) + 0.5 z (1 - tanh^2 u) du/dz, rewritten)
__device__ __forceinline__ float gelu_grad_f(float z) {
    const float sg = gelu_sig(z);
    const float du = 0.7978845608028654f * (1.f + 3.f * 0.044715f * z * z);
    return __builtin_fmaf(2.f * z * sg * (1.f - sg), du, sg);
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    // round to nearest even, as the hardware conversion does
    bf16x2_t v;
    v[0] = (__bf16)a;
    v[1] = (__bf16)b;
    return __builtin_bit_cast(uint32_t, v);
}

// MLP inference on the matrix cores: a pass of a wave takes 32 targets and
// evaluates each layer as out^T = W in^T with v_mfma_f32_32x32x8_bf16: A = 32
// output features x 8 inputs of W (read from the blob's [out][in/2] pairs),
// B = 8 inputs x the 32 targets, C = 32 features x 32 targets in FP32,
// started at the bias.  Lane l holds target l % 32; in C it holds features
// 8 (r / 4) + 4 (l / 32) + r % 4 of each 32-feature tile (r = 0..15), which
// are exactly the inputs 8 s + 4 (l / 32) + 0..3 of K-step s of the next
// layer's B: the activations stay in their lanes between layers.  GELU in
// FP32 and rounding to BF16 between layers.
typedef short bf16x4v_t __attribute__((ext_vector_type(4)));
typedef float f32x16v_t __attribute__((ext_vector_type(16)));

// 4 bf16 of row `row` of a pair array with rows of `stride` words, inputs
// k0..k0+3 (k0 % 4 == 0)
__device__ __forceinline__ bf16x4v_t mfma_wrow(const uint32_t *W, int stride, int row, int k0) {
    const uint32_t *q = W + row * stride + k0 / 2;
    const uint32_t lo = q[0], hi = q[1];
    return __builtin_bit_cast(bf16x4v_t, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ bf16x4v_t mfma_pack4(float a, float b, float c, float d) {
    return __builtin_bit_cast(bf16x4v_t, ((uint64_t)pack_bf16(c, d) << 32) | pack_bf16(a, b));
}

// TILES 32-feature output tiles of a layer with KSTEPS K-steps (weight rows
// of IN2 words)
template <int TILES, int KSTEPS, int IN2>
__device__ __forceinline__ void mfma_layer(const uint32_t *W, const float *b, const bf16x4v_t (&in)[KSTEPS],
                                           int c, int h, f32x16v_t (&acc)[TILES]) {
#pragma unroll
    for (int T = 0; T < TILES; ++T) {
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[T][r] = b[32 * T + 8 * (r / 4) + 4 * h + (r % 4)];
#pragma unroll
        for (int s = 0; s < KSTEPS; ++s)
            acc[T] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(mfma_wrow(W, IN2, 32 * T + c, 8 * s + 4 * h), in[s],
                                                             acc[T], 0, 0, 0);
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

// AUTO's bins: the FP32 position of log10 b among bins of width bin_w from
// bin_lo (NaN for NaN b); within a b bin, the cell of |s| (width 1/8, the
// last one open) and of log10 |kappa h| (width 3/16 from -2, both ends
// open; NaN goes to the last cells)
__device__ __forceinline__ float near_bpos(float bf, float bin_lo, float bin_w) {
    return floorf((log10f(bf) - bin_lo) / bin_w);
}
__device__ __forceinline__ int near_cell(float sf, float khf) {
    const float a = fabsf(sf) * 8.f;
    const int j = a < (float)(kNearSBins - 1) ? (int)a : kNearSBins - 1;
    const float k = (log10f(fabsf(khf)) + 2.f) * (16.f / 3.f);
    const int m = k < 1.f ? 0 : (k < (float)(kNearKBins - 1) ? (int)k : kNearKBins - 1);
    return j * kNearKBins + m;
}

// MLP and AUTO inference.  Per target, the decision first (AUTO): bins of
// log10(b) and |s| in FP32 (the calibration bins them the same way); b below
// the blob's b_min, NaN, a target on the unexpected side of the curve (inside
// a vesicle, whose normals point outwards; beyond a wall, whose normals point
// out of the fluid) or a b bin below the first go to the quadrature (flag 1);
// past the last b bin only "no correction" (if the last b bin's largest
// correction is within the target's tolerance) or the quadrature; inside, no
// correction, the network or the quadrature by the bin's calibrated bounds
// (scaled by scale * F into velocity units) against the tolerance (the
// target's curve's entry of curve_tol, else threshold); the bins of |s| >=
// 1/2 hold no network bound (near_calib_finish).  For a learned target the
// feature kernel's head writes the straight-line part of both rules (FP64,
// contracted with the density derivatives) to du, dv and the network's
// record; near_net then adds the network's part, so that
//   Delta = scale [t n_f] (sum_p Cflat_p d_p + exp(-2 pi b) sum_p dC_p d_p)
// in FP64 (the double layer's flat part times sg).
// The network's weights and biases staged in LDS once per workgroup.  Rows
// are padded by two words (strides 10 and 34) so that the 32 rows a wave's
// lanes read for one MFMA fall in distinct LDS banks.
constexpr int kS1 = 10, kS2 = 34;
struct NetLds {
    uint32_t W1[64 * kS1], W2[64 * kS2], W3[64 * kS2], W4[32 * kS2];
    float b1[64], b2[64], b3[64], b4[32];
};

__device__ void net_stage(const NearBlob *__restrict__ nb, NetLds &L) {
    for (int q = threadIdx.x; q < 64 * 32; q += blockDim.x) {
        const int r = q / 32, k = q % 32;
        if (k < 8) L.W1[r * kS1 + k] = nb->W1[r * 8 + k];
        L.W2[r * kS2 + k] = nb->W2[q];
        L.W3[r * kS2 + k] = nb->W3[q];
        if (r < 32) L.W4[r * kS2 + k] = nb->W4[q];
    }
    for (int q = threadIdx.x; q < 64; q += blockDim.x) {
        L.b1[q] = nb->b1[q];
        L.b2[q] = nb->b2[q];
        L.b3[q] = nb->b3[q];
        if (q < 32) L.b4[q] = nb->b4[q];
    }
}

// AUTO's decision for one target from its frame record fr (flag value: 0
// learned, 1 quadrature, 2 no correction; 0 when use_bound == 0), and the
// zero correction of dec 2 written to du, dv.
template <int OP>
__device__ __forceinline__ int near_decide_one(int64_t i, const double *fr, const DecideArgs &a, int c) {
    int dec = 0;
    if (a.use_bound) {
        const NearBlob *nb = a.nb;
        const double b = fr[1], sg = fr[8], F = fr[7];
        const double scale = OP == S2D_OP_SLP ? fr[6] / (4.0 * M_PI * a.mu) : 1.0 / M_PI;
        const float bf = (float)b;
        const bool side = OP == S2D_OP_SLP ? sg > 0.0 : sg < 0.0;
        const double sF = scale * F;
        const int nbins = nb->n_bins;
        const float pos = near_bpos(bf, nb->bin_lo, nb->bin_w);
        double tol = a.threshold;
        if (a.curve_tol) tol = (c >= 0 && c < a.n_curves) ? a.curve_tol[c] : -1.0;
        if (!(bf >= nb->b_min) || !side || !(sF == sF) || !(pos >= 0.f) || nbins <= 0) {
            dec = 1;
        } else {
            const bool past = !(pos < (float)nbins);
            const int bin = (past ? nbins - 1 : (int)pos) * kNearCell + near_cell((float)fr[0], (float)fr[19]);
            if ((double)nb->bound_zero[bin] * sF <= tol) dec = 2;
            else if (past) dec = 1;
            else dec = (double)nb->bound[bin] * sF <= tol ? 0 : 1;
        }
    }
    a.flag[i] = dec;
    if (dec == 2) {
        a.du[i] = 0.0;
        a.dv[i] = 0.0;
    }
    return dec;
}

// The learned route's part that needs the frame, for one target: the
// straight-line part (the refined rule of spacing 1 / P minus the plain one,
// FP64) written to du, dv, and the network's record nrec[kNetRec]: the
// derivatives d_p in the frame, t, n_f, and scale exp(-2 pi b) (FP32).
template <int OP>
__device__ void near_learned_head(int64_t i, const double *rec, const DecideArgs &a, float *__restrict__ nrec) {
    const double b = rec[1];
    const double scale = OP == S2D_OP_SLP ? rec[6] / (4.0 * M_PI * a.mu) : 1.0 / M_PI;
    double yt = 0.0, yn = 0.0;
    if (b > 0.0) {
        double ff[2], fc[2];
        flat_pair<OP>(rec[0], b, a.nb->P, rec[kNearFrame], rec[kNearFrame + 1], rec[kNearFrame + 2], rec + 9, ff,
                      fc);
        yt = ff[0] - fc[0];
        yn = ff[1] - fc[1];
        if (OP != S2D_OP_SLP) {
            yt *= rec[8];
            yn *= rec[8];
        }
    }
    a.du[i] = scale * (yt * rec[2] + yn * rec[4]);               // NaN for an invalid frame
    a.dv[i] = scale * (yt * rec[3] + yn * rec[5]);
    float *r = nrec + i * kNetRec;
#pragma unroll
    for (int k = 0; k < 2 * kNearDeriv; ++k) r[k] = (float)rec[9 + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) r[2 * kNearDeriv + k] = (float)rec[2 + k];
    r[2 * kNearDeriv + 4] = (float)(scale * rec[kNearFrame]);           // scale exp(-2 pi b)
    r[2 * kNearDeriv + 5] = 0.f;
}

// The network's part of the learned route, added to du, dv of the listed
// targets (list[q], q < *list_len, or all when list is NULL) from their
// features X and records nrec (near_learned_head): a wave takes
// 64 of them in two MFMA passes of 32; pass h2 feeds target 32 h2 + c from
// lanes c and c + 32, and after the exchange lane 32 h2 + c holds it.
// Persistent workgroups stage the network in LDS once; 4 waves per SIMD (128
// registers) keep the LDS and MFMA latencies covered.
template <int OP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void near_net(
    int64_t n_trg, const int32_t *__restrict__ list, const int32_t *__restrict__ list_len,
    const float *__restrict__ X, const float *__restrict__ nrec, const NearBlob *__restrict__ nb,
    double *__restrict__ du, double *__restrict__ dv) {
    static_assert(kNearFeat <= 16, "two K-steps of the first layer");
    __shared__ NetLds L;
    net_stage(nb, L);
    __syncthreads();
    const int64_t n = list ? (int64_t)*list_len : n_trg;
    const int lane = threadIdx.x & (kWave - 1), h = lane >> 5, c = lane & 31;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t g = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; g * kWave < n; g += waves) {
        const int64_t q0 = g * kWave + lane;
        const bool mine = q0 < n;
        const int64_t i = mine ? (list ? (int64_t)list[q0] : q0) : 0;
        double net[2] = {0.0, 0.0};
#pragma unroll 1
        for (int h2 = 0; h2 < 2; ++h2) {
            const int64_t qt = g * kWave + 32 * h2 + c;
            if (g * kWave + 32 * h2 >= n) break;                 // wave-uniform
            const bool vt = qt < n;
            const int64_t it = vt ? (list ? (int64_t)list[qt] : qt) : 0;
            const float *xi = X + it * kNearFeat;
            const float *ft = nrec + kNetRec * it;
            bf16x4v_t in1[2];
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = 8 * s2 + 4 * h + e;
                    v[e] = (vt && k < kNearFeat) ? (xi[k] - nb->mu_in[k]) * nb->isd_in[k] : 0.f;
                }
                in1[s2] = mfma_pack4(v[0], v[1], v[2], v[3]);
            }
            f32x16v_t acc[2];
            bf16x4v_t hb[8];
            mfma_layer<2, 2, kS1>(L.W1, L.b1, in1, c, h, acc);
            mfma_act(acc, hb);
            mfma_layer<2, 8, kS2>(L.W2, L.b2, hb, c, h, acc);
            mfma_act(acc, hb);
            mfma_layer<2, 8, kS2>(L.W3, L.b3, hb, c, h, acc);
            mfma_act(acc, hb);
            f32x16v_t y[1];
            mfma_layer<1, 8, kS2>(L.W4, L.b4, hb, c, h, y);
            // the lane's outputs o = 8 (r / 4) + 4 h + r % 4 < 20: dC[p][out][in] with
            // p = o / 4, out = (o % 4) / 2, in = o % 2, contracted with d[p][in]
            double nt[2] = {0.0, 0.0};
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int o = 8 * (r / 4) + 4 * h + (r % 4);
                if (o < kNearOut) {
                    const int p = o / 4, out = (o % 4) / 2, in = o % 2;
                    nt[out] = __builtin_fma((double)y[0][r], (double)ft[2 * p + in], nt[out]);
                }
            }
            nt[0] += __shfl_xor(nt[0], 32, kWave);
            nt[1] += __shfl_xor(nt[1], 32, kWave);
            if (h == h2) {
                net[0] = nt[0];
                net[1] = nt[1];
            }
        }
        if (!mine) continue;
        const float *fr = nrec + kNetRec * i + 2 * kNearDeriv;      // t, n_f, scale exp(-2 pi b)
        const double se = fr[4];
        du[i] = __builtin_fma(se, net[0] * (double)fr[0] + net[1] * (double)fr[2], du[i]);
        dv[i] = __builtin_fma(se, net[0] * (double)fr[1] + net[1] * (double)fr[3], dv[i]);
    }
}

// Pack FP32 master parameters into the BF16 inference blob (first layer rows
// padded to 8 input pairs, the last layer to 32 output rows, with zeros).
__global__ __launch_bounds__(256) void near_pack(const float *__restrict__ prm, const float *__restrict__ bound,
                                                 const float *__restrict__ bound_zero, int32_t n_bins, float bin_lo,
                                                 float bin_w, float b_min, int32_t P, NearBlob *__restrict__ nb) {
    using O = MlpOffsets;
    constexpr int r0 = kNearFeat;                  // W1 pairs
    constexpr int r1 = r0 + 64 * 8;                // W2
    constexpr int r2 = r1 + 64 * 32;               // W3
    constexpr int r3 = r2 + 64 * 32;               // W4
    constexpr int r4 = r3 + 32 * 32;               // biases, bounds
    constexpr int total = r4 + kNearTable;
    static_assert(kNearTable >= 64, "the bias pass rides on the bound pass");
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
        if (q < r0) {
            nb->mu_in[q] = prm[O::mu + q];
            nb->isd_in[q] = 1.f / prm[O::sd + q];
        } else if (q < r1) {
            const int r = q - r0, o = r / 8, k = r % 8;
            const float a = 2 * k < kNearFeat ? prm[O::W1 + (2 * k) * 64 + o] : 0.f;
            const float bq = 2 * k + 1 < kNearFeat ? prm[O::W1 + (2 * k + 1) * 64 + o] : 0.f;
            nb->W1[r] = pack_bf16(a, bq);
        } else if (q < r2) {
            const int r = q - r1, o = r / 32, k = r % 32;
            nb->W2[r] = pack_bf16(prm[O::W2 + (2 * k) * 64 + o], prm[O::W2 + (2 * k + 1) * 64 + o]);
        } else if (q < r3) {
            const int r = q - r2, o = r / 32, k = r % 32;
            nb->W3[r] = pack_bf16(prm[O::W3 + (2 * k) * 64 + o], prm[O::W3 + (2 * k + 1) * 64 + o]);
        } else if (q < r4) {
            const int r = q - r3, o = r / 32, k = r % 32;
            nb->W4[r] = o < kNearOut ? pack_bf16(prm[O::W4 + (2 * k) * kNearOut + o],
                                                 prm[O::W4 + (2 * k + 1) * kNearOut + o])
                                     : 0u;
        } else {
            const int o = q - r4;                  // 0 .. kNearTable - 1
            if (o < 64) {
                nb->b1[o] = prm[O::b1 + o];
                nb->b2[o] = prm[O::b2 + o];
                nb->b3[o] = prm[O::b3 + o];
            }
            if (o < 32) nb->b4[o] = o < kNearOut ? prm[O::b4 + o] : 0.f;
            nb->bound[o] = o < n_bins * kNearCell ? bound[o] : 3e38f;
            nb->bound_zero[o] = (o < n_bins * kNearCell && bound_zero) ? bound_zero[o] : 3e38f;
            if (o == 0) {
                nb->n_bins = n_bins;
                nb->bin_lo = bin_lo;
                nb->bin_w = bin_w;
                nb->b_min = b_min;
                nb->P = P;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// training data: the flat prediction's residual and the per-sample weight
// ---------------------------------------------------------------------------
// largest |(ur, vr)| of each curve's targets (non-negative floats order like
// their bit patterns, so an atomic max on the bits is exact and order-free)
__global__ __launch_bounds__(256) void near_curve_scale(int64_t n, const int32_t *__restrict__ tc, int32_t n_curves,
                                                        const double *__restrict__ ur, const double *__restrict__ vr,
                                                        uint32_t *__restrict__ cscale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = tc[i];
    if (c < 0 || c >= n_curves) return;
    const float v = (float)sqrt(ur[i] * ur[i] + vr[i] * vr[i]);
    if (v == v) atomicMax(cscale + c, __builtin_bit_cast(uint32_t, v));
}

// per sample: T = [d (10, frame), R (2) = label / scale - flat prediction
// (frame), weight = gain scale / curve scale, exp(-2 pi b)]; the labels are the
// quadrature's corrections (du, dv), the curve scale is its curve's largest
// |(ur, vr)| (the error measure's normalisation)
template <int OP>
__global__ __launch_bounds__(256) void near_train_targets_k(int64_t n, const double *__restrict__ frame,
                                                            const double *__restrict__ du,
                                                            const double *__restrict__ dv,
                                                            const int32_t *__restrict__ tc, int32_t n_curves,
                                                            double mu, int32_t P, float gain,
                                                            const uint32_t *__restrict__ cscale,
                                                            float *__restrict__ T) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *fr = frame + kNearFrame * i;
    const double b = fr[1];
    const double scale = OP == S2D_OP_SLP ? fr[6] / (4.0 * M_PI * mu) : 1.0 / M_PI;
    double y0 = (du[i] * fr[2] + dv[i] * fr[3]) / scale, y1 = (du[i] * fr[4] + dv[i] * fr[5]) / scale;
    double fc[2] = {0.0, 0.0}, ff[2] = {0.0, 0.0};
    double aq, cq, sq;
    flat_q(fr[0], b, aq, cq, sq);
    if (b > 0.0) flat_pair<OP>(fr[0], b, P, aq, cq, sq, fr + 9, ff, fc);
    const double sgn = OP == S2D_OP_SLP ? 1.0 : fr[8];
    y0 -= sgn * (ff[0] - fc[0]);
    y1 -= sgn * (ff[1] - fc[1]);
    const int c = tc[i];
    const float cs = (c >= 0 && c < n_curves) ? __builtin_bit_cast(float, cscale[c]) : 0.f;
    float *t = T + kNearTStride * i;
    for (int k = 0; k < 2 * kNearDeriv; ++k) t[k] = (float)fr[9 + k];
    t[10] = (float)y0;
    t[11] = (float)y1;
    t[12] = cs > 0.f ? (float)((double)gain * scale / (double)cs) : 0.f;
    t[13] = (float)aq;
}

// per-feature mean and standard deviation (population) over n samples into
// the parameter vector's standardisation slots: one workgroup per feature,
// strided FP64 partial sums added in a fixed tree order (deterministic)
__global__ __launch_bounds__(256) void near_feature_stats_k(int64_t n, const float *__restrict__ X,
                                                            float *__restrict__ prm) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += (double)X[i * kNearFeat + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    const double mean = red[0] / (double)(n > 0 ? n : 1);
    __syncthreads();
    s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double e = (double)X[i * kNearFeat + k] - mean;
        s = __builtin_fma(e, e, s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double sd = sqrt(red[0] / (double)(n > 0 ? n : 1));
        prm[MlpOffsets::mu + k] = (float)mean;
        prm[MlpOffsets::sd + k] = sd > 1e-30 ? (float)sd : 1.f;
    }
}

// Calibration of AUTO's rule: per bin of log10(b) and |s| (FP32, as the
// inference bins them), the largest network error |pred - label| and the largest
// correction |label|, both over scale * F; targets that AUTO would not trust
// the network with (b < b_min, the wrong side, NaN) are skipped.  bound and
// bound_zero hold float bits (atomic max); empty bins become 3e38 and the
// others are multiplied by margin (1 + count_margin / sqrt(count)) in the
// finishing pass (a wider margin where a bin has few samples).
template <int OP>
__global__ __launch_bounds__(256) void near_calib_acc(int64_t n, const double *__restrict__ frame,
                                                      const double *__restrict__ dup, const double *__restrict__ dvp,
                                                      const double *__restrict__ du, const double *__restrict__ dv,
                                                      double mu, int32_t n_bins, float bin_lo, float bin_w,
                                                      float b_min, uint32_t *__restrict__ bound,
                                                      uint32_t *__restrict__ bound_zero, int32_t *__restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *fr = frame + kNearFrame * i;
    const float bf = (float)fr[1];
    const bool side = OP == S2D_OP_SLP ? fr[8] > 0.0 : fr[8] < 0.0;
    if (!(bf >= b_min) || !side) return;
    const float pos = near_bpos(bf, bin_lo, bin_w);
    if (!(pos >= 0.f && pos < (float)n_bins)) return;
    const int bin = (int)pos * kNearCell + near_cell((float)fr[0], (float)fr[19]);
    const double scale = OP == S2D_OP_SLP ? fr[6] / (4.0 * M_PI * mu) : 1.0 / M_PI;
    const double sF = scale * fr[7];
    const float e = (float)(sqrt((dup[i] - du[i]) * (dup[i] - du[i]) + (dvp[i] - dv[i]) * (dvp[i] - dv[i])) / sF);
    const float z = (float)(sqrt(du[i] * du[i] + dv[i] * dv[i]) / sF);
    if (!(e == e) || !(z == z)) return;
    atomicMax(bound + bin, __builtin_bit_cast(uint32_t, e));
    atomicMax(bound_zero + bin, __builtin_bit_cast(uint32_t, z));
    atomicAdd(count + bin, 1);
}

__global__ __launch_bounds__(256) void near_calib_init(int32_t n_bins, uint32_t *bound, uint32_t *bound_zero,
                                                       int32_t *count) {
    for (int b = threadIdx.x; b < n_bins * kNearCell; b += blockDim.x) {
        bound[b] = 0u;
        bound_zero[b] = 0u;
        count[b] = 0;
    }
}

// Targets past the midpoint between two nodes (|s| >= 1/2, where the
// nearest node by distance is not the nearest by arc) never take the learned
// route: the network's held-out errors there underestimate its errors on new
// targets by up to three times (heavy tails), so their cells keep the
// no-correction bound only.
__global__ __launch_bounds__(256) void near_calib_finish(int32_t n_bins, float margin, float count_margin,
                                                         uint32_t *bound, uint32_t *bound_zero, const int32_t *count) {
    for (int b = threadIdx.x; b < n_bins * kNearCell; b += blockDim.x) {
        const int n = count[b];
        const bool past_mid = (b % kNearCell) / kNearKBins == kNearSBins - 1;
        const float m = n > 0 ? margin * (1.f + count_margin / sqrtf((float)n)) : 0.f;
        const float e = n > 0 && !past_mid ? __builtin_bit_cast(float, bound[b]) * m : 3e38f;
        const float z = n > 0 ? __builtin_bit_cast(float, bound_zero[b]) * m : 3e38f;
        bound[b] = __builtin_bit_cast(uint32_t, e);
        bound_zero[b] = __builtin_bit_cast(uint32_t, z);
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

// activation columns of a training sample's record
constexpr int kA_h0 = 0, kA_z1 = kNearFeat, kA_h1 = kA_z1 + 64, kA_z2 = kA_h1 + 64, kA_h2 = kA_z2 + 64,
              kA_z3 = kA_h2 + 64, kA_h3 = kA_z3 + 64;

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

// per sample: forward, the head (the 20 outputs dC contracted with the
// sample's d, times exp(-2 pi b)), the weighted residual e = wt (head - R),
// its loss term |e|^2 / 2B, the output deltas dY[o] = wt e_out(o) env d[p][in] / B,
// and the pre-activations z1..z3 and activations h0..h3 for the backward pass
__global__ __launch_bounds__(256) void mlp_fwd(int32_t B, const int32_t *__restrict__ idx,
                                               const float *__restrict__ X, const float *__restrict__ T,
                                               const float *__restrict__ prm, float *__restrict__ act,
                                               float *__restrict__ dY, float *__restrict__ lossv) {
    __shared__ float rows[kBlock / kWave][64];
    using O = MlpOffsets;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int s = blockIdx.x * (kBlock / kWave) + wv;
    if (s >= B) return;                  // wave-uniform; no block barrier below
    float *row = rows[wv];
    const int64_t i = idx ? idx[s] : s;
    float *A = act + (int64_t)s * kActStride;
    if (lane < kNearFeat) {
        const float v = (X[i * kNearFeat + lane] - prm[O::mu + lane]) / prm[O::sd + lane];
        A[kA_h0 + lane] = v;
        row[lane] = v;
    }
    mlp_wave_sync();
    mlp_fwd_layer(kNearFeat, prm + O::W1, prm + O::b1, row, lane, A + kA_z1, A + kA_h1);
    mlp_fwd_layer(64, prm + O::W2, prm + O::b2, row, lane, A + kA_z2, A + kA_h2);
    mlp_fwd_layer(64, prm + O::W3, prm + O::b3, row, lane, A + kA_z3, A + kA_h3);
    float yo = 0.f;
    if (lane < kNearOut) {
        float a = prm[O::b4 + lane];
        for (int k = 0; k < 64; ++k) a = fmaf(row[k], prm[O::W4 + k * kNearOut + lane], a);
        yo = a;
    }
    mlp_wave_sync();
    if (lane < kNearOut) row[lane] = yo;
    mlp_wave_sync();
    // every lane contracts the 20 outputs in the same order
    const float *t = T + (int64_t)kNearTStride * i;
    float hd[2] = {0.f, 0.f};
    for (int o = 0; o < kNearOut; ++o) {
        const int p = o / 4, out = (o % 4) / 2, in = o % 2;
        hd[out] = fmaf(row[o], t[2 * p + in], hd[out]);
    }
    const float wt = t[12], env = t[13];
    const float e0 = wt * (env * hd[0] - t[10]), e1 = wt * (env * hd[1] - t[11]);
    if (lane < kNearOut) {
        const int p = lane / 4, out = (lane % 4) / 2, in = lane % 2;
        dY[(int64_t)s * kNearOut + lane] = wt * (out ? e1 : e0) * env * t[2 * p + in] / (float)B;
    }
    if (lane == 0) lossv[s] = 0.5f * (e0 * e0 + e1 * e1) / (float)B;
}

// per sample: the deltas of the three hidden layers, written over z3, z2, z1
__global__ __launch_bounds__(256) void mlp_bwd(int32_t B, const float *__restrict__ prm, float *__restrict__ act,
                                               const float *__restrict__ dY) {
    __shared__ float rows[kBlock / kWave][64];
    using O = MlpOffsets;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int s = blockIdx.x * (kBlock / kWave) + wv;
    if (s >= B) return;                  // wave-uniform
    float *row = rows[wv];
    float *A = act + (int64_t)s * kActStride;
    const float *g = dY + (int64_t)s * kNearOut;
    float a = 0.f;
    for (int o = 0; o < kNearOut; ++o) a = fmaf(prm[O::W4 + lane * kNearOut + o], g[o], a);
    const float d3 = a * gelu_grad_f(A[kA_z3 + lane]);
    A[kA_z3 + lane] = d3;
    row[lane] = d3;
    mlp_wave_sync();
    a = 0.f;
    for (int o = 0; o < 64; ++o) a = fmaf(prm[O::W3 + lane * 64 + o], row[o], a);
    const float d2 = a * gelu_grad_f(A[kA_z2 + lane]);
    A[kA_z2 + lane] = d2;
    mlp_wave_sync();
    row[lane] = d2;
    mlp_wave_sync();
    a = 0.f;
    for (int o = 0; o < 64; ++o) a = fmaf(prm[O::W2 + lane * 64 + o], row[o], a);
    A[kA_z1 + lane] = a * gelu_grad_f(A[kA_z1 + lane]);
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
    using O = MlpOffsets;
    const int pp = threadIdx.x % kPer, ch = threadIdx.x / kPer;
    const int p = blockIdx.x * kPer + pp;
    int hin = -1, dl = -1, dk = 0;               // activation column, delta column (act) or output (dY)
    bool outd = false;
    if (p >= O::W1 && p < O::b1) { const int r = p - O::W1; hin = kA_h0 + r / 64; dl = kA_z1 + r % 64; }
    else if (p >= O::b1 && p < O::W2) { dl = kA_z1 + (p - O::b1); }
    else if (p >= O::W2 && p < O::b2) { const int r = p - O::W2; hin = kA_h1 + r / 64; dl = kA_z2 + r % 64; }
    else if (p >= O::b2 && p < O::W3) { dl = kA_z2 + (p - O::b2); }
    else if (p >= O::W3 && p < O::b3) { const int r = p - O::W3; hin = kA_h2 + r / 64; dl = kA_z3 + r % 64; }
    else if (p >= O::b3 && p < O::W4) { dl = kA_z3 + (p - O::b3); }
    else if (p >= O::W4 && p < O::b4) { const int r = p - O::W4; hin = kA_h3 + r / kNearOut; dk = r % kNearOut; outd = true; }
    else if (p >= O::b4 && p < O::total) { dk = p - O::b4; outd = true; }
    float g = 0.f;
    if (p >= O::W1 && p < O::total) {            // mu_in / sd_in are not trained
        const int s0 = (int)((int64_t)B * ch / kGradChunks), s1 = (int)((int64_t)B * (ch + 1) / kGradChunks);
        // the loads of 8 samples are issued before their (ordered) FMAs
        const float *dsrc = outd ? dY + dk : act + dl;
        const int64_t dstr = outd ? kNearOut : kActStride;
        int s = s0;
        for (; s + 8 <= s1; s += 8) {
            float dv[8], hv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                dv[u] = dsrc[(int64_t)(s + u) * dstr];
                hv[u] = hin >= 0 ? act[(int64_t)(s + u) * kActStride + hin] : 1.f;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) g = fmaf(hv[u], dv[u], g);
        }
        for (; s < s1; ++s) g = fmaf(hin >= 0 ? act[(int64_t)s * kActStride + hin] : 1.f, dsrc[(int64_t)s * dstr], g);
    }
    part[ch][pp] = g;
    __syncthreads();
    if (ch == 0 && p < O::total) {
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
    using O = MlpOffsets;
    if (p >= O::total || p < O::W1) return;
    const float g = grad[p];
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.f - powf(b1, (float)step));
    const float vh = vv / (1.f - powf(b2, (float)step));
    prm[p] -= lr * mh / (sqrtf(vh) + eps);
}

// FP32 forward only: the 20 raw outputs dC (reference-precision inference,
// gradient checks)
__global__ __launch_bounds__(256) void mlp_fwd_only(int64_t n, const float *__restrict__ X,
                                                    const float *__restrict__ prm, float *__restrict__ Y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    using O = MlpOffsets;
    float h0[kNearFeat], h1[64], h2[64];
    for (int k = 0; k < kNearFeat; ++k) h0[k] = (X[i * kNearFeat + k] - prm[O::mu + k]) / prm[O::sd + k];
    for (int o = 0; o < 64; ++o) {
        float a = prm[O::b1 + o];
        for (int k = 0; k < kNearFeat; ++k) a = fmaf(h0[k], prm[O::W1 + k * 64 + o], a);
        h1[o] = gelu_f(a);
    }
    for (int o = 0; o < 64; ++o) {
        float a = prm[O::b2 + o];
        for (int k = 0; k < 64; ++k) a = fmaf(h1[k], prm[O::W2 + k * 64 + o], a);
        h2[o] = gelu_f(a);
    }
    for (int o = 0; o < 64; ++o) {
        float a = prm[O::b3 + o];
        for (int k = 0; k < 64; ++k) a = fmaf(h2[k], prm[O::W3 + k * 64 + o], a);
        h1[o] = gelu_f(a);
    }
    for (int o = 0; o < kNearOut; ++o) {
        float a = prm[O::b4 + o];
        for (int k = 0; k < 64; ++k) a = fmaf(h1[k], prm[O::W4 + k * kNearOut + o], a);
        Y[i * kNearOut + o] = a;
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

hipError_t near_launch_compact(int64_t n, const int32_t *flag, int value, int32_t *cnt, int32_t *list,
                               hipStream_t st, int value2, int32_t *cnt2, int32_t *list2) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + kCompactBlock - 1) / kCompactBlock;
    const CompactOut a{value, cnt, list}, b{list2 ? value2 : -2, list2 ? cnt2 : nullptr, list2};
    hipLaunchKernelGGL(near_compact_count, dim3((unsigned)nb), dim3(kCompactBlock), 0, st, n, flag, a, b);
    hipLaunchKernelGGL(near_compact_scan, dim3(list2 ? 2 : 1), dim3(kScanThreads), 0, st, nb, a, b);
    hipLaunchKernelGGL(near_compact_scatter, dim3((unsigned)nb), dim3(kCompactBlock), 0, st, n, flag, a, b);
    return hipGetLastError();
}


size_t near_derivs_scratch(const s2d_curves *c) {
    // a flag (256 bytes), then for curves above kUpMaxN nodes the cos / sin
    // table and the mode coefficients
    return 256 + (c->n_nodes > kUpMaxN ? (size_t)c->n_nodes * 6 * sizeof(double) : 0);
}

hipError_t near_launch_derivs(const s2d_curves *c, double *dtab, void *scratch, hipStream_t st) {
    if (c->n_curves <= 0 || c->n_nodes <= 0) return hipSuccess;
    int32_t *big = (int32_t *)scratch;
    hipError_t e = zero_int_launch(big, 1, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(near_derivs, dim3((unsigned)c->n_curves), dim3(256), 0, st, c->curve_off, c->n_curves,
                       c->n_nodes, c->fx, c->fy, dtab, big);
    if (c->n_nodes > kUpMaxN) {
        // some curve may exceed kUpMaxN nodes: the kernels return at once
        // unless near_derivs found one
        double *tab = (double *)((char *)scratch + 256), *coef = tab + 2 * c->n_nodes;
        const unsigned g = (unsigned)std::min<int64_t>(kBigBlocks, (c->n_nodes + 255) / 256 * 4);
        hipLaunchKernelGGL(near_derivs_table, dim3(g), dim3(256), 0, st, c->curve_off, c->n_curves, c->n_nodes, big,
                           tab);
        hipLaunchKernelGGL(near_derivs_coef, dim3(g), dim3(256), 0, st, c->curve_off, c->n_curves, c->n_nodes, big,
                           c->fx, c->fy, tab, coef);
        hipLaunchKernelGGL(near_derivs_nodes, dim3(g), dim3(256), 0, st, c->curve_off, c->n_curves, c->n_nodes, big,
                           tab, coef, dtab);
    }
    return hipGetLastError();
}

hipError_t near_launch_features(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, const double *dtab,
                                float *X, double *frame, hipStream_t st) {
    if (t->n <= 0) return hipSuccess;
    hipLaunchKernelGGL(near_features<kFeatFrame>, dim3(grid_for(t->n)), dim3(256), 0, st, t->n, t->x, t->y, tc,
                       c->curve_off, c->n_curves, c->n_nodes, c->x, c->y, c->nx, c->ny, c->kappa, c->w, dtab, X,
                       frame, nullptr, nullptr, DecideArgs{});
    return hipGetLastError();
}

hipError_t near_launch_scan(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, float *X, int32_t *kstar,
                            hipStream_t st) {
    if (t->n <= 0) return hipSuccess;
    hipLaunchKernelGGL(near_features<kFeatScan>, dim3(grid_for(t->n)), dim3(256), 0, st, t->n, t->x, t->y, tc,
                       c->curve_off, c->n_curves, c->n_nodes, c->x, c->y, c->nx, c->ny, c->kappa, c->w, nullptr, X,
                       nullptr, kstar, nullptr, DecideArgs{});
    return hipGetLastError();
}

hipError_t near_launch_head(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, const double *dtab,
                            const int32_t *kstar, const DecideArgs &da, float *nrec, hipStream_t st, float *X) {
    if (t->n <= 0) return hipSuccess;
    if (kstar)
        hipLaunchKernelGGL(near_features<kFeatHead>, dim3(grid_for(t->n)), dim3(256), 0, st, t->n, t->x, t->y, tc,
                           c->curve_off, c->n_curves, c->n_nodes, c->x, c->y, c->nx, c->ny, c->kappa, c->w, dtab,
                           nullptr, nullptr, (int32_t *)kstar, nrec, da);
    else
        hipLaunchKernelGGL(near_features<kFeatFused>, dim3(grid_for(t->n)), dim3(256), 0, st, t->n, t->x, t->y, tc,
                           c->curve_off, c->n_curves, c->n_nodes, c->x, c->y, c->nx, c->ny, c->kappa, c->w, dtab, X,
                           nullptr, nullptr, nrec, da);
    return hipGetLastError();
}

hipError_t near_launch_wall_features(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, double d,
                                     const double *dtab, float *X, double *frame, hipStream_t st,
                                     const DecideArgs *fused, float *nrec) {
    if (t->n <= 0) return hipSuccess;
    // grid-stride: each block builds the cell table once for up to a few
    // thousand targets
    const int64_t blocks = std::min<int64_t>((t->n + 255) / 256, 1024);
    const DecideArgs da = fused ? *fused : DecideArgs{};
    if (fused)
        hipLaunchKernelGGL(near_wall_features<true>, dim3((unsigned)blocks), dim3(256), 0, st, t->n, t->x, t->y, tc,
                           c->curve_off, c->n_curves, c->n_nodes, c->x, c->y, c->nx, c->ny, c->kappa, c->w, d, dtab,
                           X, nullptr, nrec, da);
    else
        hipLaunchKernelGGL(near_wall_features<false>, dim3((unsigned)blocks), dim3(256), 0, st, t->n, t->x, t->y, tc,
                           c->curve_off, c->n_curves, c->n_nodes, c->x, c->y, c->nx, c->ny, c->kappa, c->w, d, dtab,
                           X, frame, nullptr, da);
    return hipGetLastError();
}

hipError_t near_launch_infer(int op, int64_t n, const float *X, const float *nrec, const NearBlob *nb,
                             const int32_t *list, const int32_t *list_len, double *du, double *dv, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    // the network 64 targets per wave (4 waves per block, persistent blocks
    // that stage the network in LDS once, four per compute unit at most)
    const int64_t groups = (n + kWave - 1) / kWave;
    const unsigned nbk = (unsigned)std::min<int64_t>((groups + 3) / 4, 4 * kInferCUs);
    if (op == S2D_OP_SLP)
        hipLaunchKernelGGL(near_net<S2D_OP_SLP>, dim3(nbk), dim3(256), 0, st, n, list, list_len, X, nrec, nb, du, dv);
    else
        hipLaunchKernelGGL(near_net<S2D_OP_DLP>, dim3(nbk), dim3(256), 0, st, n, list, list_len, X, nrec, nb, du, dv);
    return hipGetLastError();
}

hipError_t near_launch_pack(const float *prm, const float *bound, const float *bound_zero, int32_t n_bins,
                            float bin_lo, float bin_w, float b_min, int32_t P, NearBlob *nb, hipStream_t st) {
    hipLaunchKernelGGL(near_pack, dim3(32), dim3(256), 0, st, prm, bound, bound_zero, n_bins, bin_lo, bin_w, b_min, P,
                       nb);
    return hipGetLastError();
}

hipError_t near_launch_train_targets(int op, int64_t n, const double *frame, const double *du, const double *dv,
                                     const int32_t *tc, int32_t n_curves, const double *ur, const double *vr,
                                     double mu, int32_t P, float gain, uint32_t *cscale, float *T,
                                     hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (n_curves > 0) {
        hipError_t e = zero_int_launch((int32_t *)cscale, n_curves, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(near_curve_scale, dim3(grid_for(n)), dim3(256), 0, st, n, tc, n_curves, ur, vr, cscale);
    }
    if (op == S2D_OP_SLP)
        hipLaunchKernelGGL(near_train_targets_k<S2D_OP_SLP>, dim3(grid_for(n)), dim3(256), 0, st, n, frame, du, dv, tc,
                           n_curves, mu, P, gain, cscale, T);
    else
        hipLaunchKernelGGL(near_train_targets_k<S2D_OP_DLP>, dim3(grid_for(n)), dim3(256), 0, st, n, frame, du, dv, tc,
                           n_curves, mu, P, gain, cscale, T);
    return hipGetLastError();
}

hipError_t near_launch_train_step(int32_t B, const int32_t *idx, const float *X, const float *T, float *prm,
                                  float *m, float *v, int32_t step, float lr, float *grad, float *act, float *dY,
                                  float *lossv, float *loss, int update, hipStream_t st) {
    using O = MlpOffsets;
    const unsigned wave_blocks = (unsigned)((B + kBlock / kWave - 1) / (kBlock / kWave));   // a wave per sample
    hipLaunchKernelGGL(mlp_fwd, dim3(wave_blocks), dim3(kBlock), 0, st, B, idx, X, T, prm, act, dY, lossv);
    hipLaunchKernelGGL(mlp_bwd, dim3(wave_blocks), dim3(kBlock), 0, st, B, prm, act, dY);
    hipLaunchKernelGGL(mlp_grad, dim3((unsigned)((O::total + kBlock / kGradChunks - 1) / (kBlock / kGradChunks))),
                       dim3(kBlock), 0, st, B, act, dY, lossv, grad, loss);
    if (update)
        hipLaunchKernelGGL(mlp_adam, dim3(grid_for(O::total)), dim3(256), 0, st, prm, grad, m, v, step, lr, 0.9f,
                           0.999f, 1e-8f);
    return hipGetLastError();
}

hipError_t near_launch_fwd(int64_t n, const float *X, const float *prm, float *Y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_fwd_only, dim3(grid_for(n)), dim3(256), 0, st, n, X, prm, Y);
    return hipGetLastError();
}

hipError_t near_launch_feature_stats(int64_t n, const float *X, float *prm, hipStream_t st) {
    hipLaunchKernelGGL(near_feature_stats_k, dim3(kNearFeat), dim3(256), 0, st, n, X, prm);
    return hipGetLastError();
}

hipError_t near_launch_calibrate(int op, int64_t n, const double *frame, const double *dup, const double *dvp,
                                 const double *du, const double *dv, double mu, int32_t n_bins, float bin_lo,
                                 float bin_w, float b_min, float margin, float count_margin, uint32_t *bound,
                                 uint32_t *bound_zero, int32_t *count, hipStream_t st) {
    hipLaunchKernelGGL(near_calib_init, dim3(1), dim3(256), 0, st, n_bins, bound, bound_zero, count);
    if (n > 0) {
        if (op == S2D_OP_SLP)
            hipLaunchKernelGGL(near_calib_acc<S2D_OP_SLP>, dim3(grid_for(n)), dim3(256), 0, st, n, frame, dup, dvp, du,
                               dv, mu, n_bins, bin_lo, bin_w, b_min, bound, bound_zero, count);
        else
            hipLaunchKernelGGL(near_calib_acc<S2D_OP_DLP>, dim3(grid_for(n)), dim3(256), 0, st, n, frame, dup, dvp, du,
                               dv, mu, n_bins, bin_lo, bin_w, b_min, bound, bound_zero, count);
    }
    hipLaunchKernelGGL(near_calib_finish, dim3(1), dim3(256), 0, st, n_bins, margin, count_margin, bound,
                       bound_zero, count);
    return hipGetLastError();
}

}  // namespace s2d
