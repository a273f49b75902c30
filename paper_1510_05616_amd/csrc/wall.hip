// Spectral upsampling of periodic channel walls, the first step of the walls'
// close evaluation (the paper leaves close evaluation of the wall double
// layer to future work: Section 5 footnote; Section 6).
//
// Each wall curve is one period of a d-periodic wall with N (even, >= 4)
// nodes equispaced in its parameter t in [0, 2 pi), advancing by s d in x
// (s = +-1, from the first two nodes).  Its periodic parts x - s d t / 2 pi
// and y and the density are expanded in their discrete Fourier coefficients
// V_k = sum_j v_j e^{-2 pi i j k / N}, k = 0 .. N/2 (stage 1, a direct sum per
// coefficient), and evaluated at the P N parameter values 2 pi m / (P N)
// (stage 2, the trigonometric interpolant with the Nyquist mode split evenly
// between +-N/2), with spectral derivatives for the speed |x'(t)|, the
// weights (2 pi / P N) |x'| and the unit normals, oriented like the given
// normal of the coarse node at or before the fine one.
//
// Coefficients are stored interleaved, 8 doubles per (curve, k): re and im of
// the four series.  Both sums are split into chunks (over the nodes in stage
// 1, over the modes in stage 2) along the grid's y dimension so that the
// launch fills the device, and the chunks' partial sums are added in chunk
// order by a second kernel (deterministic results).  A wave whose lanes all
// lie in one curve reads the coefficients (and in stage 1 the nodes) through
// the scalar data path; twiddle factors follow a rotation recurrence
// re-anchored with sincospi every 32 steps.
#include "s2d_near.h"

#include <algorithm>

namespace s2d {

namespace {

constexpr int kAnchor = 32;

struct alignas(16) Coef8 { double v[8]; };        // (re, im) of x~, y, fx, fy

// element i of a device array, read through the constant address space (the
// scalar path when the address is wave-uniform), one dword at a time
template <class T>
__device__ __forceinline__ T load_ro(const void *base, int64_t i) {
    constexpr int n = (int)(sizeof(T) / 4);
    using CP = const __attribute__((address_space(4))) uint32_t *;
    const CP p = (CP)((const char *)base + i * (int64_t)sizeof(T));
    struct Words { uint32_t w[n]; } t;
#pragma unroll
    for (int k = 0; k < n; ++k) t.w[k] = p[k];
    return __builtin_bit_cast(T, t);
}

template <bool UNI, class T>
__device__ __forceinline__ T ld(const T *p, int64_t i) {
    if constexpr (UNI) return load_ro<T>(p, i);
    else return p[i];
}

// the curve c with off[c] * scale <= g < off[c + 1] * scale (off ascending)
__device__ __forceinline__ int find_curve(const int32_t *__restrict__ off, int n, int64_t g, int64_t scale) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)off[mid] * scale <= g) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool curve_ok(int64_t lo, int64_t hi, int64_t n_nodes) {
    return lo >= 0 && hi <= n_nodes && hi - lo >= 4 && ((hi - lo) & 1) == 0;
}

// stage 1 sums for coefficient k of the curve at lo with N nodes, over its
// nodes jb .. je-1
template <bool UNI>
__device__ __forceinline__ void dft_sums(const WallArgs &a, int64_t lo, int64_t N, int64_t k, int64_t jb,
                                         int64_t je, double s, double re[4], double im[4]) {
    double wr, wi;
    sincospi(2.0 * (double)k / (double)N, &wi, &wr);
    wi = -wi;                                           // e^{-2 pi i k / N}
    const double sd = s * a.d / (double)N;
    for (int64_t j0 = jb; j0 < je; j0 += kAnchor) {
        double zr, zi;
        sincospi(2.0 * (double)((j0 * k) % N) / (double)N, &zi, &zr);
        zi = -zi;
        const int64_t j1 = min(j0 + (int64_t)kAnchor, je);
        for (int64_t j = j0; j < j1; ++j) {
            const double v[4] = {ld<UNI>(a.x, lo + j) - sd * (double)j, ld<UNI>(a.y, lo + j), ld<UNI>(a.fx, lo + j),
                                 ld<UNI>(a.fy, lo + j)};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                re[q] = __builtin_fma(v[q], zr, re[q]);
                im[q] = __builtin_fma(v[q], zi, im[q]);
            }
            const double tr = zr * wr - zi * wi;
            zi = zr * wi + zi * wr;
            zr = tr;
        }
    }
}

// stage 1, split over the nodes: work-item g, chunk blockIdx.y ->
// coefficient k = g - off[c] of curve c (k <= N/2) over the chunk's nodes
__global__ __launch_bounds__(256) void wall_dft_part(WallArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n_nodes) return;
    const int c = find_curve(a.off, a.n_curves, g, 1);
    const int64_t lo = a.off[c], hi = a.off[c + 1], N = hi - lo, k = g - lo;
    if (!curve_ok(lo, hi, a.n_nodes) || k < 0 || k > N / 2) return;
    const int64_t S = a.s1, sc = blockIdx.y, len = (N + S - 1) / S;
    const int64_t jb = min(sc * len, N), je = min(jb + len, N);
    const double s = a.x[lo + 1] > a.x[lo] ? 1.0 : -1.0;
    double re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
    const int lo_u = __builtin_amdgcn_readfirstlane((int)lo);
    if (__all(lo == (int64_t)lo_u)) {
        // one curve: N and the chunk bounds are wave-uniform (scalar loop,
        // scalar loads of the nodes)
        const int N_u = __builtin_amdgcn_readfirstlane((int)N);
        const int jb_u = __builtin_amdgcn_readfirstlane((int)jb), je_u = __builtin_amdgcn_readfirstlane((int)je);
        dft_sums<true>(a, lo_u, N_u, k, jb_u, je_u, s, re, im);
    } else {
        dft_sums<false>(a, lo, N, k, jb, je, s, re, im);
    }
    Coef8 o;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        o.v[2 * q] = re[q];
        o.v[2 * q + 1] = im[q];
    }
    ((Coef8 *)a.part1)[sc * a.n_nodes + lo + k] = o;
}

// the chunks' partial coefficients summed in chunk order
__global__ __launch_bounds__(256) void wall_dft_sum(WallArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.n_nodes) return;
    const int c = find_curve(a.off, a.n_curves, g, 1);
    const int64_t lo = a.off[c], hi = a.off[c + 1], N = hi - lo, k = g - lo;
    if (!curve_ok(lo, hi, a.n_nodes) || k < 0 || k > N / 2) return;
    const Coef8 *p = (const Coef8 *)a.part1;
    Coef8 o = p[g];
    for (int sc = 1; sc < a.s1; ++sc) {
        const Coef8 t = p[(int64_t)sc * a.n_nodes + g];
#pragma unroll
        for (int q = 0; q < 8; ++q) o.v[q] += t.v[q];
    }
    ((Coef8 *)a.coef)[g] = o;
}

// stage 2 sums over modes k = kb .. ke-1 at the fine angle th = 2 pi j / M,
// kept apart by the parity of k - kb (A: even, B: odd) and split into
// C = sum Re V_k cos k th, S = sum Im V_k sin k th (four series) and
// DS = sum k Re V_k sin k th, DC = sum k Im V_k cos k th (x~ and y only).
// Then Re sum V_k e^{ik th} = C - S and Re sum i k V_k e^{ik th} = -(DS + DC);
// at -th the sine parts change sign, and at th + pi the odd-k parts do.
struct SynthAcc { double C[4], S[4], DS[2], DC[2]; };

template <bool UNI>
__device__ __forceinline__ void synth_step(const Coef8 *coef, int64_t lo, int64_t k, double zr, double zi,
                                           SynthAcc &X) {
    const Coef8 V = ld<UNI>(coef, lo + k);
    const double kd = (double)k;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        X.C[q] = __builtin_fma(V.v[2 * q], zr, X.C[q]);
        X.S[q] = __builtin_fma(V.v[2 * q + 1], zi, X.S[q]);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        X.DS[q] = __builtin_fma(kd * V.v[2 * q], zi, X.DS[q]);
        X.DC[q] = __builtin_fma(kd * V.v[2 * q + 1], zr, X.DC[q]);
    }
}

template <bool UNI>
__device__ __forceinline__ void synth_sums(const Coef8 *coef, int64_t lo, int64_t kb, int64_t ke, int64_t j,
                                           int64_t M, SynthAcc &A, SynthAcc &B) {
    double wr, wi;
    sincospi(2.0 * (double)j / (double)M, &wi, &wr);   // e^{i th}
    for (int64_t k0 = kb; k0 < ke; k0 += kAnchor) {      // kAnchor is even: k0 - kb stays even
        double zr, zi;
        sincospi(2.0 * (double)((k0 * j) % M) / (double)M, &zi, &zr);
        const int64_t k1 = min(k0 + (int64_t)kAnchor, ke);
        int64_t k = k0;
        for (; k + 1 < k1; k += 2) {
            synth_step<UNI>(coef, lo, k, zr, zi, A);
            double tr = zr * wr - zi * wi;
            zi = zr * wi + zi * wr;
            zr = tr;
            synth_step<UNI>(coef, lo, k + 1, zr, zi, B);
            tr = zr * wr - zi * wi;
            zi = zr * wi + zi * wr;
            zr = tr;
        }
        if (k < k1) synth_step<UNI>(coef, lo, k, zr, zi, A);
    }
}

// stage 2, split over the modes 1 .. h-1: work-item g, chunk blockIdx.y.
// Curve c owns the P N / 2 work-items from ceil(P off[c] / 2); item j <= M / 4
// of the curve serves the fine points j, M - j, M/2 + j and M/2 - j (the
// rest return at once).  Six partial sums per fine point and chunk.
__global__ __launch_bounds__(256) void wall_synth_part(WallArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t P = a.P, nf = P * a.n_nodes;
    if (2 * g >= nf) return;
    const int c = find_curve(a.off, a.n_curves, 2 * g, P);
    const int64_t lo = a.off[c], hi = a.off[c + 1], N = hi - lo, M = P * N, h = N / 2;
    const int64_t j = g - (P * lo + 1) / 2;
    if (!curve_ok(lo, hi, a.n_nodes) || j < 0 || j > M / 4) return;
    const int64_t S = a.s2, sc = blockIdx.y, len = (h - 1 + S - 1) / S;
    const int64_t kb = min(1 + sc * len, h), ke = min(kb + len, h);
    const Coef8 *coef = (const Coef8 *)a.coef;
    SynthAcc A = {}, B = {};
    const int lo_u = __builtin_amdgcn_readfirstlane((int)lo);
    if (__all(lo == (int64_t)lo_u)) {
        // one curve: the mode range is wave-uniform (scalar loop, scalar
        // loads of the coefficients)
        const int kb_u = __builtin_amdgcn_readfirstlane((int)kb), ke_u = __builtin_amdgcn_readfirstlane((int)ke);
        synth_sums<true>(coef, lo_u, kb_u, ke_u, j, M, A, B);
    } else {
        synth_sums<false>(coef, lo, kb, ke, j, M, A, B);
    }
    const bool odd = kb & 1;                            // A holds the odd k when kb is odd
    SynthAcc E, O;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        E.C[q] = odd ? B.C[q] : A.C[q];
        O.C[q] = odd ? A.C[q] : B.C[q];
        E.S[q] = odd ? B.S[q] : A.S[q];
        O.S[q] = odd ? A.S[q] : B.S[q];
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        E.DS[q] = odd ? B.DS[q] : A.DS[q];
        O.DS[q] = odd ? A.DS[q] : B.DS[q];
        E.DC[q] = odd ? B.DC[q] : A.DC[q];
        O.DC[q] = odd ? A.DC[q] : B.DC[q];
    }
    const int64_t pts[4] = {j, j ? M - j : 0, M / 2 + j, M / 2 - j};
    double *base = a.part2 + sc * 6 * nf + P * lo;
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        const double ho = (o & 2) ? -1.0 : 1.0, rs = (o & 1) ? -1.0 : 1.0;
        double *p = base + pts[o];
#pragma unroll
        for (int q = 0; q < 4; ++q) p[q * nf] = (E.C[q] + ho * O.C[q]) - rs * (E.S[q] + ho * O.S[q]);
#pragma unroll
        for (int q = 0; q < 2; ++q) p[(4 + q) * nf] = -rs * (E.DS[q] + ho * O.DS[q]) - (E.DC[q] + ho * O.DC[q]);
    }
}

// stage 2 finish: the chunks' sums in chunk order, the mean and Nyquist
// terms, then nodes, normals, weights and density of fine point g
__global__ __launch_bounds__(256) void wall_synth_fin(WallArgs a) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t P = a.P, nf = P * a.n_nodes;
    if (g >= nf) return;
    const int c = find_curve(a.off, a.n_curves, g, P);
    const int64_t lo = a.off[c], hi = a.off[c + 1], N = hi - lo, M = P * N, m = g - P * lo, h = N / 2;
    if (!curve_ok(lo, hi, a.n_nodes) || m < 0 || m >= M) {
        const double nan = __builtin_nan("");
        a.ox[g] = a.oy[g] = a.onx[g] = a.ony[g] = a.ow[g] = a.ofx[g] = a.ofy[g] = nan;
        return;
    }
    double acc[4] = {0, 0, 0, 0}, dac[2] = {0, 0};
    for (int sc = 0; sc < a.s2; ++sc) {
        const double *p = a.part2 + (int64_t)sc * 6 * nf + g;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += p[q * nf];
        dac[0] += p[4 * nf];
        dac[1] += p[5 * nf];
    }
    const double s = a.x[lo + 1] > a.x[lo] ? 1.0 : -1.0;
    const Coef8 *coef = (const Coef8 *)a.coef;
    const Coef8 V0 = coef[lo], Vh = coef[lo + h];
    double sh, ch;
    sincospi(2.0 * (double)((h * m) % M) / (double)M, &sh, &ch);
    const double invN = 1.0 / (double)N;
    double val[4], der[2];
#pragma unroll
    for (int q = 0; q < 4; ++q) val[q] = (V0.v[2 * q] + 2.0 * acc[q] + Vh.v[2 * q] * ch) * invN;
#pragma unroll
    for (int q = 0; q < 2; ++q) der[q] = (2.0 * dac[q] - (double)h * Vh.v[2 * q] * sh) * invN;
    const double dX = der[0] + s * a.d / (2.0 * M_PI), dY = der[1];
    const double sp = sqrt(dX * dX + dY * dY);
    const int64_t j = lo + m / P;
    const double o = (-dY * a.nx[j] + dX * a.ny[j]) > 0.0 ? 1.0 : -1.0;
    a.ox[g] = val[0] + s * a.d * ((double)m / (double)M);
    a.oy[g] = val[1];
    a.onx[g] = -o * dY / sp;
    a.ony[g] = o * dX / sp;
    a.ow[g] = (2.0 * M_PI / (double)M) * sp;
    a.ofx[g] = val[2];
    a.ofy[g] = val[3];
}

__global__ void wall_fine_offsets(const int32_t *__restrict__ off, int n_curves, int P, int32_t *__restrict__ foff) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n_curves) foff[i] = off[i] * P;
}

// u (+)= uf - uc, v (+)= vf - vc: the difference is rounded first, so an
// accumulated result equals the written one added to the prior contents
__global__ __launch_bounds__(256) void delta_combine(int64_t n, int acc, double *__restrict__ u,
                                                     double *__restrict__ v, const double *__restrict__ t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double du = t[i] - t[2 * n + i], dv = t[n + i] - t[3 * n + i];
    u[i] = acc ? u[i] + du : du;
    v[i] = acc ? v[i] + dv : dv;
}

__global__ __launch_bounds__(256) void add_or_write(int64_t n, int acc, double *__restrict__ u,
                                                    double *__restrict__ v, const double *__restrict__ tu,
                                                    const double *__restrict__ tv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    u[i] = acc ? u[i] + tu[i] : tu[i];
    v[i] = acc ? v[i] + tv[i] : tv[i];
}

// one vector atomic per fallback target
__global__ __launch_bounds__(256) void fallback_compact(int64_t n, const int32_t *__restrict__ flag,
                                                        const double *__restrict__ tx, const double *__restrict__ ty,
                                                        int32_t *__restrict__ list, int32_t *__restrict__ count,
                                                        double *__restrict__ cx, double *__restrict__ cy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || flag[i] != 1) return;
    const int32_t j = atomicAdd(count, 1);
    list[j] = (int32_t)i;
    cx[j] = tx[i];
    cy[j] = ty[i];
}

__global__ __launch_bounds__(256) void fallback_scatter(int64_t m, const int32_t *__restrict__ list,
                                                        const double *__restrict__ t4, double *__restrict__ tu,
                                                        double *__restrict__ tv) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int32_t i = list[j];
    tu[i] = t4[j] - t4[2 * m + j];
    tv[i] = t4[m + j] - t4[3 * m + j];
}

__global__ void zero_int(int32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

unsigned grid(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void wall_splits(int64_t n_nodes, int P, int *s1, int *s2) {
    // chunks enough for about 8 (stage 1) and 16 (stage 2) waves per SIMD
    // of a 256-CU device; more work per chunk than that gains nothing
    constexpr int64_t kItems1 = 256LL * 4 * 8 * 64, kItems2 = 2 * kItems1;
    const int64_t n1 = std::max<int64_t>(n_nodes, 1), n2 = std::max<int64_t>((int64_t)P * n_nodes, 1);
    *s1 = (int)std::min<int64_t>(std::max<int64_t>((kItems1 + n1 - 1) / n1, 1), 32);
    *s2 = (int)std::min<int64_t>(std::max<int64_t>((kItems2 + n2 - 1) / n2, 1), 16);
}

WallScratch wall_scratch(int64_t n_nodes, int P) {
    WallScratch w{};
    wall_splits(n_nodes, P, &w.s1, &w.s2);
    const auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    w.coef = 0;
    w.part1 = al((size_t)n_nodes * sizeof(Coef8));
    w.part2 = w.part1 + al((size_t)w.s1 * n_nodes * sizeof(Coef8));
    w.total = w.part2 + al((size_t)w.s2 * 6 * P * n_nodes * sizeof(double));
    return w;
}

hipError_t wall_upsample_launch(const WallArgs &a, hipStream_t st) {
    if (a.n_curves > 0 && a.off && a.ooff) {
        hipLaunchKernelGGL(wall_fine_offsets, dim3((unsigned)((a.n_curves + 1 + 255) / 256)), dim3(256), 0, st,
                           a.off, a.n_curves, a.P, a.ooff);
    }
    if (a.n_nodes > 0) {
        const unsigned g1 = grid(a.n_nodes), g2 = grid(((int64_t)a.P * a.n_nodes + 1) / 2);
        hipLaunchKernelGGL(wall_dft_part, dim3(g1, (unsigned)a.s1), dim3(256), 0, st, a);
        hipLaunchKernelGGL(wall_dft_sum, dim3(g1), dim3(256), 0, st, a);
        hipLaunchKernelGGL(wall_synth_part, dim3(g2, (unsigned)a.s2), dim3(256), 0, st, a);
        hipLaunchKernelGGL(wall_synth_fin, dim3(grid((int64_t)a.P * a.n_nodes)), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t add_or_write_launch(int64_t n, int accumulate, double *u, double *v, const double *tu, const double *tv,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(add_or_write, dim3(grid(n)), dim3(256), 0, st, n, accumulate ? 1 : 0, u, v, tu, tv);
    return hipGetLastError();
}

hipError_t fallback_compact_launch(int64_t n, const int32_t *flag, const double *tx, const double *ty, int32_t *list,
                                   int32_t *count, double *cx, double *cy, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fallback_compact, dim3(grid(n)), dim3(256), 0, st, n, flag, tx, ty, list, count, cx, cy);
    return hipGetLastError();
}

hipError_t fallback_scatter_launch(int64_t m, const int32_t *list, const double *t4, double *tu, double *tv,
                                   hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(fallback_scatter, dim3(grid(m)), dim3(256), 0, st, m, list, t4, tu, tv);
    return hipGetLastError();
}

hipError_t zero_int_launch(int32_t *p, int n, hipStream_t st) {
    hipLaunchKernelGGL(zero_int, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t delta_combine_launch(int64_t n, int accumulate, double *u, double *v, const double *t, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(delta_combine, dim3(grid(n)), dim3(256), 0, st, n, accumulate ? 1 : 0, u, v, t);
    return hipGetLastError();
}

}  // namespace s2d
