// Periodization system of one channel cell on the GPU (Section 2.2,
// Eqs. (urep)-(bsys); Nystrom discretisation, Section 2.3; block solve,
// Section 4.1).
//
// Unknowns: the double-layer density tau at the N wall nodes (interleaved
// (x, y) per node) and the coefficients c of M proxy Stokeslets on a circle
// around the cell.  Rows: the wall velocity data at the N wall nodes
// (-1/2 tau + the double layer over the images |n| <= 1, the n = 0 self term
// by the diagonal limit), then at K side heights the velocity difference
// R - L and the traction difference R - L (side normal (1, 0)), where only
// the far wall copies (R against the walls shifted by -d, L against +d) and
// the proxies remain after the near interactions cancel (Eqs. (BIEgu),
// (BIEgT)).
//
// The four blocks are filled by one kernel each (one thread per 2 x 2 node
// block, column-major for the solver).  Factor: blocked LU of A with partial
// pivoting (rocSOLVER panels, rocBLAS TRSM / GEMM updates, row interchanges
// by a kernel of its own; the call schedule in lu_plan.h keeps every library
// operand within 2^30 elements), X = A^-1 B by the triangular sweeps,
// S = Q - C X (GEMM), SVD of the small S and its truncated pseudo-inverse.
// Solve: y = A^-1 v (row permutation, forward and backward sweeps),
// c = S^+ (g - C y), tau = y - X c.
#include "lu_plan.h"
#include "s2d_cell.h"
#include "s2d_internal.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

namespace s2d {

namespace {

constexpr double kPi = 3.14159265358979323846;

// 2 x 2 kernel blocks, o[2 a + b] = K_ab, r = target - source

__device__ __forceinline__ void stresslet_blk(double rx, double ry, double nx, double ny, double (&o)[4]) {
    const double q = rx * rx + ry * ry;
    const double f = (rx * nx + ry * ny) / (q * q * kPi);
    o[0] = rx * rx * f;
    o[1] = rx * ry * f;
    o[2] = o[1];
    o[3] = ry * ry * f;
}

__device__ __forceinline__ void stokeslet_blk(double rx, double ry, double mu, double (&o)[4]) {
    const double q = rx * rx + ry * ry;
    const double s = 1.0 / (4.0 * kPi * mu);
    const double l = -0.5 * log(q);
    o[0] = s * (l + rx * rx / q);
    o[1] = s * (rx * ry / q);
    o[2] = o[1];
    o[3] = s * (l + ry * ry / q);
}

// traction of the Stokeslet at a target with normal m (Eq. (K))
__device__ __forceinline__ void stokeslet_traction_blk(double rx, double ry, double mx, double my, double (&o)[4]) {
    const double q = rx * rx + ry * ry;
    const double f = -(rx * mx + ry * my) / (q * q * kPi);
    o[0] = rx * rx * f;
    o[1] = rx * ry * f;
    o[2] = o[1];
    o[3] = ry * ry * f;
}

// traction of the double-layer velocity and pressure pair (Eqs. (D), (P)) of
// a source with normal n at a target with normal m (Eq. (T), its dipole
// functions paired as the stress of the pair: a = r.n/r^2 goes with the
// target-normal term, b = r.m/r^2 with the source-normal term)
__device__ __forceinline__ void stresslet_traction_blk(double rx, double ry, double mx, double my, double nx,
                                                       double ny, double mu, double (&o)[4]) {
    const double q = rx * rx + ry * ry;
    const double a = (rx * nx + ry * ny) / q;
    const double b = (rx * mx + ry * my) / q;
    const double c1 = ((nx * mx + ny * my) / q - 8.0 * a * b) / q;
    const double r[2] = {rx, ry}, m[2] = {mx, my}, n[2] = {nx, ny};
    const double s = mu / kPi;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int k = 0; k < 2; ++k)
            o[2 * i + k] = s * (c1 * r[i] * r[k] + (i == k ? a * b : 0.0) + m[i] * n[k] / q + b * n[i] * r[k] / q +
                                a * r[i] * m[k] / q);
}

__device__ __forceinline__ void proxy_point(const CellArgs &g, int m, double &px, double &py) {
    const double th = 2.0 * kPi * (double)m / (double)g.M;
    px = g.cx + g.R * cos(th);
    py = g.cy + g.R * sin(th);
}

__device__ __forceinline__ void put(double *A, int64_t ld, int64_t row0, int64_t col0, const double (&o)[4]) {
    A[row0 + col0 * ld] = o[0];
    A[row0 + 1 + col0 * ld] = o[2];
    A[row0 + (col0 + 1) * ld] = o[1];
    A[row0 + 1 + (col0 + 1) * ld] = o[3];
}

// A: -1/2 I + sum_{|n| <= 1} D(x_i, y_j + n d) w_j, diagonal limit at n = 0
__global__ __launch_bounds__(256) void cell_fill_A(CellArgs g, double *A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = g.n_wall;
    if (t >= N * N) return;
    const int64_t i = t % N, j = t / N;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const double nx = g.nx[j], ny = g.ny[j], w = g.w[j];
    for (int n = -1; n <= 1; ++n) {
        double o[4];
        if (n == 0 && i == j) {
            // -(kappa / 2 pi) t t^T, t t^T = I - n n^T
            const double k = -g.kap[j] / (2.0 * kPi);
            o[0] = k * (1.0 - nx * nx);
            o[1] = k * (-nx * ny);
            o[2] = o[1];
            o[3] = k * (1.0 - ny * ny);
        } else {
            stresslet_blk(g.x[i] - g.x[j] - n * g.d, g.y[i] - g.y[j], nx, ny, o);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] += o[e] * w;
    }
    if (i == j) {
        acc[0] -= 0.5;
        acc[3] -= 0.5;
    }
    put(A, 2 * N, 2 * i, 2 * j, acc);
}

// B: the proxy Stokeslets at the wall nodes
__global__ __launch_bounds__(256) void cell_fill_B(CellArgs g, double *B) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = g.n_wall;
    if (t >= N * g.M) return;
    const int64_t i = t % N;
    const int m = (int)(t / N);
    double px, py, o[4];
    proxy_point(g, m, px, py);
    stokeslet_blk(g.x[i] - px, g.y[i] - py, g.mu, o);
    put(B, 2 * N, 2 * i, 2 * m, o);
}

// C: velocity (rows 2k + a) and traction (rows 2K + 2k + a) differences of
// the far wall copies, R against the walls shifted by -d, L by +d
__global__ __launch_bounds__(256) void cell_fill_C(CellArgs g, double *C) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t K = g.K;
    if (t >= K * g.n_wall) return;
    const int64_t k = t % K, j = t / K;
    const double yk = g.side_y[k], w = g.w[j], nx = g.nx[j], ny = g.ny[j];
    const double rxR = g.xl + g.d - (g.x[j] - g.d), rxL = g.xl - (g.x[j] + g.d), ry = yk - g.y[j];
    double a[4], b[4], o[4];
    stresslet_blk(rxR, ry, nx, ny, a);
    stresslet_blk(rxL, ry, nx, ny, b);
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = (a[e] - b[e]) * w;
    put(C, 4 * K, 2 * k, 2 * j, o);
    stresslet_traction_blk(rxR, ry, 1.0, 0.0, nx, ny, g.mu, a);
    stresslet_traction_blk(rxL, ry, 1.0, 0.0, nx, ny, g.mu, b);
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = (a[e] - b[e]) * w;
    put(C, 4 * K, 2 * K + 2 * k, 2 * j, o);
}

// Q: the same differences of the proxy Stokeslets
__global__ __launch_bounds__(256) void cell_fill_Q(CellArgs g, double *Q) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t K = g.K;
    if (t >= K * g.M) return;
    const int64_t k = t % K;
    const int m = (int)(t / K);
    double px, py, a[4], b[4], o[4];
    proxy_point(g, m, px, py);
    const double yk = g.side_y[k];
    stokeslet_blk(g.xl + g.d - px, yk - py, g.mu, a);
    stokeslet_blk(g.xl - px, yk - py, g.mu, b);
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = a[e] - b[e];
    put(Q, 4 * K, 2 * k, 2 * m, o);
    stokeslet_traction_blk(g.xl + g.d - px, yk - py, 1.0, 0.0, a);
    stokeslet_traction_blk(g.xl - px, yk - py, 1.0, 0.0, b);
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = a[e] - b[e];
    put(Q, 4 * K, 2 * K + 2 * k, 2 * m, o);
}

// P (n x m) = V diag(1/s) U^T over the singular values above rcond * s_0,
// from U (m x r, ld m) and V^T (r x n, ld r), r = min(m, n)
__global__ __launch_bounds__(256) void cell_pinv(int m, int n, int r, const double *sv, const double *U,
                                                 const double *Vt, double rcond, double *P) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)m * n) return;
    const int j = (int)(t % n), i = (int)(t / n);
    const double cut = rcond * sv[0];
    double acc = 0.0;
    for (int l = 0; l < r; ++l)
        if (sv[l] > cut) acc += Vt[l + (int64_t)j * r] * U[i + (int64_t)l * m] / sv[l];
    P[j + (int64_t)i * n] = acc;
}

// the row interchanges of one LU panel on columns of T (column c at
// T + c ld): for i < k in order, rows i and ipiv[i] - 1 (1-based, relative to
// T's first row), skipping pivots outside the m rows; one thread per column,
// the pivots staged through LDS
__global__ __launch_bounds__(64) void lu_laswp(double *T, int64_t ld, int64_t cols, int64_t m, const int32_t *ipiv,
                                               int64_t k) {
    __shared__ int32_t sp[1024];
    const int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x;
    double *col = T + (c < cols ? c : 0) * ld;
    for (int64_t i0 = 0; i0 < k; i0 += 1024) {
        const int cnt = (int)(k - i0 < 1024 ? k - i0 : 1024);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += 64) sp[t] = ipiv[i0 + t] - 1;
        __syncthreads();
        if (c >= cols) continue;
        for (int t = 0; t < cnt; ++t) {
            const int64_t i = i0 + t, r = sp[t];
            if (r == i || r < 0 || r >= m) continue;
            const double a = col[i];
            col[i] = col[r];
            col[r] = a;
        }
    }
}

// out[i + j ldo] = in[perm[i] + j ldi], i < n, j < nrhs (NaN for an index
// outside 0..n-1, as in a workspace that was never factored)
__global__ __launch_bounds__(256) void lu_gather(int64_t n, int64_t nrhs, const double *in, int64_t ldi,
                                                 const int32_t *perm, double *out, int64_t ldo) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nrhs) return;
    const int64_t i = t % n, j = t / n, p = perm[i];
    out[i + j * ldo] = p >= 0 && p < n ? in[p + j * ldi] : __builtin_nan("");
}

// Rows per block of the one-right-hand-side sweeps.  Each sweep keeps, per
// block t, a row-major tile of 2 kTb doubles per row (n rows in all, block t
// at rows t kTb..): [D_t | -G_t], D_t the inverse of the diagonal block of L
// (forward) or U (backward), G_t = D_t F[t rows, s columns] with s the block
// the sweep finishes t from (forward s = t - 1, backward s = t + 1); zeros
// past the blocks' sizes.
constexpr int kTb = 256;
constexpr int kTileW = 2 * kTb;

// identity in the D_t part of every tile, zeros elsewhere
__global__ __launch_bounds__(256) void tri_tile_init(int64_t n, double *T) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * kTileW) return;
    const int64_t r = t / kTileW, e = t % kTileW;
    T[t] = e == r % kTb ? 1.0 : 0.0;
}

// sum_j col[j n] v[j], j < jn <= NJ, in order; all NJ loads in flight at once
// when the block is whole
template <int NJ>
__device__ __forceinline__ double dot_cols(const double *col, int64_t n, const double *v, int jn) {
    double acc = 0.0;
    if (jn == NJ) {
        double a[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) a[j] = col[j * n];
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc += a[j] * v[j];
    } else {
        for (int j = 0; j < jn; ++j) acc += col[j * n] * v[j];
    }
    return acc;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// One step of a triangular sweep of one right-hand side: y is the working
// vector (the right-hand side less the finished blocks' contributions), x
// receives the finished blocks.  Block s is finished (x_s final) when the
// step runs; the step finishes block t and updates the rows [r0, r1):
//   x_t = [D_t | -G_t] [y_t; x_s]  (y_t alone when s0 < 0: the first block),
//   y_r -= F[r, s columns] x_s     for r in [r0, r1), outside blocks s and t.
// y_t is complete, since every block before s updated it in an earlier
// step.  Forward (unit lower L): t = s + 1, r0 = the row after t; backward
// (U): t = s - 1, [r0, r1) = the rows above t.
// Workgroups of 8 waves: the first ceil(bt / 32) finish block t, 4 rows per
// wave, each row's tile read contiguously across the lanes and summed over
// the wave; the others update 64 rows each, every wave an eighth of the kTb
// columns of F.
constexpr int kTriThreads = 512;
__global__ __launch_bounds__(kTriThreads) void tri_step(const double *__restrict__ F, const double *__restrict__ T,
                                                        int64_t n, double *__restrict__ y, double *__restrict__ x,
                                                        int64_t s0, int bs, int64_t t0, int bt, int64_t r0,
                                                        int64_t r1) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nfin = (bt + 31) / 32;
    if ((int)blockIdx.x < nfin) {
        constexpr int KE = kTileW / 64;
        double in[KE];
#pragma unroll
        for (int k = 0; k < KE; ++k) {
            const int e = lane + 64 * k;
            in[k] = e < kTb ? (e < bt ? y[t0 + e] : 0.0) : (e - kTb < bs ? x[s0 + e - kTb] : 0.0);
        }
        const int i0 = (int)blockIdx.x * 32 + w * 4;
        double acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc[q] = 0.0;
            if (i0 + q < bt) {
                const double *row = T + (t0 + i0 + q) * kTileW + lane;
                double a[KE];
#pragma unroll
                for (int k = 0; k < KE; ++k) a[k] = row[64 * k];
#pragma unroll
                for (int k = 0; k < KE; ++k) acc[q] += a[k] * in[k];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double v = wave_sum(acc[q]);
            if (lane == 0 && i0 + q < bt) x[t0 + i0 + q] = v;
        }
        return;
    }
    __shared__ double red[kTriThreads];
    constexpr int NJ = kTb / 8;
    const int64_t r = r0 + (int64_t)((int)blockIdx.x - nfin) * 64 + lane;
    const bool live = r < r1;
    double acc = 0.0;
    if (live) acc = dot_cols<NJ>(F + r + (s0 + w * NJ) * n, n, x + s0 + w * NJ, min(NJ, bs - w * NJ));
    red[threadIdx.x] = acc;
    __syncthreads();
    if (w == 0 && live) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) t += red[k * 64 + lane];
        y[r] -= t;
    }
}

unsigned grid(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int64_t cell_panels(const CellArgs &g) { return g.panel < 1 ? 0 : (2 * g.n_wall + g.panel - 1) / g.panel; }

CellLayout cell_layout(const CellArgs &g) {
    CellLayout L{};
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const int64_t n = 2 * g.n_wall, nc = 2 * (int64_t)g.M, mr = 4 * (int64_t)g.K;
    const int64_t r = std::min(mr, nc);
    size_t off = 0;
    L.A = off;    off = al(off + (size_t)n * n * 8);
    L.B = off;    off = al(off + (size_t)n * nc * 8);
    L.X = off;    off = al(off + (size_t)n * nc * 8);
    L.C = off;    off = al(off + (size_t)mr * n * 8);
    L.S = off;    off = al(off + (size_t)mr * nc * 8);
    L.U = off;    off = al(off + (size_t)mr * r * 8);
    L.Vt = off;   off = al(off + (size_t)r * nc * 8);
    L.sv = off;   off = al(off + (size_t)r * 8);
    L.E = off;    off = al(off + (size_t)r * 8);
    L.P = off;    off = al(off + (size_t)nc * mr * 8);
    L.y = off;    off = al(off + (size_t)n * 8);
    L.rr = off;   off = al(off + (size_t)mr * 8);
    L.ipiv = off; off = al(off + (size_t)n * 4);
    L.perm = off; off = al(off + (size_t)n * 4);
    L.Tf = off;   off = al(off + (size_t)n * kTileW * 8);
    L.Tb = off;   off = al(off + (size_t)n * kTileW * 8);
    L.w = off;    off = al(off + (size_t)n * 8);
    L.info = off; off = al(off + (size_t)(cell_panels(g) + 1) * 4);
    L.total = off;
    return L;
}

hipError_t cell_fill(const CellArgs &g, double *A, double *B, double *C, double *Q, hipStream_t st) {
    const int64_t N = g.n_wall;
    if (A && N > 0) hipLaunchKernelGGL(cell_fill_A, dim3(grid(N * N)), dim3(256), 0, st, g, A);
    if (B && N > 0 && g.M > 0) hipLaunchKernelGGL(cell_fill_B, dim3(grid(N * g.M)), dim3(256), 0, st, g, B);
    if (C && N > 0 && g.K > 0) hipLaunchKernelGGL(cell_fill_C, dim3(grid(g.K * N)), dim3(256), 0, st, g, C);
    if (Q && g.K > 0 && g.M > 0) hipLaunchKernelGGL(cell_fill_Q, dim3(grid((int64_t)g.K * g.M)), dim3(256), 0, st, g, Q);
    return hipGetLastError();
}

hipError_t cell_pinv_launch(int m, int n, const double *sv, const double *U, const double *Vt, double rcond, double *P,
                            hipStream_t st) {
    const int r = std::min(m, n);
    hipLaunchKernelGGL(cell_pinv, dim3(grid((int64_t)m * n)), dim3(256), 0, st, m, n, r, sv, U, Vt, rcond, P);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// data of the channel's response to vesicles (Algorithm 1, steps 3-5)
// ---------------------------------------------------------------------------
namespace {

// side-wall targets: L = (xl, side_y), R = (xl + d, side_y), normal (1, 0)
__global__ __launch_bounds__(256) void resp_side(int K, const double *side_y, double xl, double d, double *sxl,
                                                 double *sxr, double *mx, double *my) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    sxl[k] = xl;
    sxr[k] = xl + d;
    mx[k] = 1.0;
    my[k] = 0.0;
}

// v = -(S^near f on the walls), interleaved per node
__global__ __launch_bounds__(256) void resp_pack_v(int64_t nw, const double *vwx, const double *vwy, double *v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw) return;
    v[2 * i] = -vwx[i];
    v[2 * i + 1] = -vwy[i];
}

// g = [L - R velocity ; L - R traction + p_drive (1, 0)], interleaved per height;
// s = [rx | ry | lx | ly | trx | try | tlx | tly], K each
__global__ __launch_bounds__(256) void resp_pack_g(int K, const double *s, double p_drive, double *g) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    g[2 * k] = s[2 * K + k] - s[k];
    g[2 * k + 1] = s[3 * K + k] - s[K + k];
    g[2 * K + 2 * k] = s[6 * K + k] - s[4 * K + k] + p_drive;
    g[2 * K + 2 * k + 1] = s[7 * K + k] - s[5 * K + k];
}

// tau, c de-interleaved; proxy points on their circle, unit weights
__global__ __launch_bounds__(256) void resp_unpack(int64_t nw, const double *tau, double *tx, double *ty, int M,
                                                   const double *c, double pcx, double pcy, double R, double *cx,
                                                   double *cy, double *px, double *py, double *pw, int32_t *poff) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nw) {
        tx[i] = tau[2 * i];
        ty[i] = tau[2 * i + 1];
    }
    if (i < M) {
        cx[i] = c[2 * i];
        cy[i] = c[2 * i + 1];
        double sn, cs;
        sincospi(2.0 * (double)i / (double)M, &sn, &cs);
        px[i] = pcx + R * cs;
        py[i] = pcy + R * sn;
        pw[i] = 1.0;
    }
    if (i == 0) {
        poff[0] = 0;
        poff[1] = M;
    }
}

}  // namespace

hipError_t resp_side_launch(int K, const double *side_y, double xl, double d, double *sxl, double *sxr, double *mx,
                            double *my, hipStream_t st) {
    hipLaunchKernelGGL(resp_side, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, K, side_y, xl, d, sxl, sxr,
                       mx, my);
    return hipGetLastError();
}

hipError_t resp_pack_launch(int64_t nw, const double *vwx, const double *vwy, int K, const double *s, double p_drive,
                            double *v, double *g, hipStream_t st) {
    if (nw > 0) hipLaunchKernelGGL(resp_pack_v, dim3(grid(nw)), dim3(256), 0, st, nw, vwx, vwy, v);
    hipLaunchKernelGGL(resp_pack_g, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, K, s, p_drive, g);
    return hipGetLastError();
}

hipError_t resp_unpack_launch(int64_t nw, const double *tau, double *tx, double *ty, int M, const double *c,
                              double pcx, double pcy, double R, double *cx, double *cy, double *px, double *py,
                              double *pw, int32_t *poff, hipStream_t st) {
    const int64_t n = std::max<int64_t>(std::max<int64_t>(nw, M), 1);
    hipLaunchKernelGGL(resp_unpack, dim3(grid(n)), dim3(256), 0, st, nw, tau, tx, ty, M, c, pcx, pcy, R, cx, cy, px,
                       py, pw, poff);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// factor and solve (rocSOLVER / rocBLAS on the caller's stream)
// ---------------------------------------------------------------------------
namespace {

std::mutex g_hmu;
rocblas_handle g_handle[64] = {};

std::string rb_err(const char *what, rocblas_status s) {
    return std::string(what) + ": " + rocblas_status_to_string(s);
}

// one handle per device, created on first use; the caller holds g_hmu
rocblas_handle handle_for(hipStream_t st, std::string &err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        err = "no current HIP device";
        return nullptr;
    }
    if (!g_handle[dev]) {
        const rocblas_status s = rocblas_create_handle(&g_handle[dev]);
        if (s != rocblas_status_success) {
            err = rb_err("rocblas_create_handle", s);
            g_handle[dev] = nullptr;
            return nullptr;
        }
    }
    const rocblas_status s = rocblas_set_stream(g_handle[dev], st);
    if (s != rocblas_status_success) {
        err = rb_err("rocblas_set_stream", s);
        return nullptr;
    }
    return g_handle[dev];
}

}  // namespace

std::mutex &blas_mutex() { return g_hmu; }

void *blas_handle(hipStream_t st, std::string &err) { return (void *)handle_for(st, err); }

namespace {

// the calls of an LU schedule (lu_plan.h): F is the n x n factored matrix
// (ld n), T the target (F itself when factoring), ldt its leading dimension
std::string lu_run(rocblas_handle h, const std::vector<lu::Call> &plan, double *F, int64_t n, double *T,
                   int64_t ldt, int32_t *ipiv, int32_t *info, hipStream_t st) {
    const double one = 1.0, minus_one = -1.0;
    const rocblas_int ld = (rocblas_int)n, lt = (rocblas_int)ldt;
    for (const lu::Call &c : plan) {
        rocblas_status s = rocblas_status_success;
        const rocblas_int m = (rocblas_int)c.m, nn = (rocblas_int)c.n, k = (rocblas_int)c.k;
        switch (c.op) {
            case lu::kGetrf:
                s = rocsolver_dgetrf(h, m, nn, F + c.a, ld, ipiv + c.piv, info + c.slot);
                if (s != rocblas_status_success) return rb_err("rocsolver_dgetrf", s);
                break;
            case lu::kLaswp: {
                hipLaunchKernelGGL(lu_laswp, dim3((unsigned)((c.n + 63) / 64)), dim3(64), 0, st, T + c.b, ldt, c.n,
                                   c.m, ipiv + c.piv, c.k);
                const hipError_t e = hipGetLastError();
                if (e != hipSuccess) return std::string("lu_laswp: ") + hipGetErrorString(e);
                break;
            }
            case lu::kTrsm: {
                const rocblas_fill fill = c.upper ? rocblas_fill_upper : rocblas_fill_lower;
                const rocblas_diagonal diag = c.upper ? rocblas_diagonal_non_unit : rocblas_diagonal_unit;
                s = rocblas_dtrsm(h, rocblas_side_left, fill, rocblas_operation_none, diag, m, nn, &one, F + c.a, ld,
                                  T + c.b, lt);
                if (s != rocblas_status_success) return rb_err("rocblas_dtrsm", s);
                break;
            }
            case lu::kGemm:
                s = rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, m, nn, k, &minus_one, F + c.a,
                                  ld, T + c.b, lt, &one, T + c.c, lt);
                if (s != rocblas_status_success) return rb_err("rocblas_dgemm", s);
                break;
            default:
                return "unknown LU call";
        }
    }
    return "";
}

hipError_t gather_launch(int64_t n, int64_t nrhs, const double *in, int64_t ldi, const int32_t *perm, double *out,
                         int64_t ldo, hipStream_t st) {
    hipLaunchKernelGGL(lu_gather, dim3(grid(n * nrhs)), dim3(256), 0, st, n, nrhs, in, ldi, perm, out, ldo);
    return hipGetLastError();
}

// the sweeps' tiles.  Viewed column-major with leading dimension kTileW,
// block t's tile holds D_t^T in rows 0..bt-1 and -G_t^T in rows kTb..:
// D^T = L^-T (U^-T) by TRSM from the right with the transposed triangle on
// an identity, -G^T = -F[t rows, s columns]^T D^T by GEMM.
std::string tri_prepare(rocblas_handle h, const double *F, int64_t n, double *Tf, double *Tb, hipStream_t st) {
    hipLaunchKernelGGL(tri_tile_init, dim3(grid(n * kTileW)), dim3(256), 0, st, n, Tf);
    hipLaunchKernelGGL(tri_tile_init, dim3(grid(n * kTileW)), dim3(256), 0, st, n, Tb);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return std::string("tri_tile_init: ") + hipGetErrorString(e);
    const double one = 1.0, minus_one = -1.0, zero = 0.0;
    const rocblas_int ld = (rocblas_int)n, lt = kTileW;
    auto bsz = [&](int64_t q) { return (rocblas_int)std::min<int64_t>(kTb, n - q); };
    for (int64_t q = 0; q < n; q += kTb) {
        const rocblas_int b = bsz(q);
        const double *Fq = F + q + q * n;
        double *tf = Tf + q * kTileW, *tb = Tb + q * kTileW;
        rocblas_status s = rocblas_dtrsm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                                         rocblas_diagonal_unit, b, b, &one, Fq, ld, tf, lt);
        if (s == rocblas_status_success)
            s = rocblas_dtrsm(h, rocblas_side_right, rocblas_fill_upper, rocblas_operation_transpose,
                              rocblas_diagonal_non_unit, b, b, &one, Fq, ld, tb, lt);
        if (s != rocblas_status_success) return rb_err("rocblas_dtrsm", s);
        if (q > 0) {                                  // forward: block q from q - kTb
            const int64_t p = q - kTb;
            s = rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, bsz(p), b, b, &minus_one,
                              F + q + p * n, ld, tf, lt, &zero, tf + kTb, lt);
        }
        if (s == rocblas_status_success && q + kTb < n) {   // backward: block q from q + kTb
            const int64_t p = q + kTb;
            s = rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, bsz(p), b, b, &minus_one,
                              F + q + p * n, ld, tb, lt, &zero, tb + kTb, lt);
        }
        if (s != rocblas_status_success) return rb_err("rocblas_dgemm", s);
    }
    return "";
}

// x = U^-1 L^-1 y, y and w scratch (both overwritten): the forward sweep
// from y into w, then the backward sweep from w into x; one launch per block
hipError_t tri_solve(const double *F, const double *Tf, const double *Tb, int64_t n, double *y, double *w, double *x,
                     hipStream_t st) {
    const int64_t nq = (n + kTb - 1) / kTb;
    auto bsz = [&](int64_t q) { return (int)std::min<int64_t>(kTb, n - q * kTb); };
    auto step = [&](const double *T, double *yy, double *xx, int64_t s, int64_t t, int64_t r0, int64_t r1) {
        const unsigned g = (unsigned)((bsz(t) + 31) / 32 + (r1 - r0 + 63) / 64);
        hipLaunchKernelGGL(tri_step, dim3(g), dim3(kTriThreads), 0, st, F, T, n, yy, xx, s < 0 ? -1 : s * kTb,
                           s < 0 ? 0 : bsz(s), t * kTb, bsz(t), r0, r1);
    };
    step(Tf, y, w, -1, 0, 0, 0);
    for (int64_t q = 0; q + 1 < nq; ++q) step(Tf, y, w, q, q + 1, std::min(n, (q + 2) * kTb), n);
    step(Tb, w, x, -1, nq - 1, 0, 0);
    for (int64_t q = nq - 1; q >= 1; --q) step(Tb, w, x, q, q - 1, 0, (q - 1) * kTb);
    return hipGetLastError();
}

}  // namespace

std::string cell_factor(const CellArgs &g, double rcond, void *ws, hipStream_t st) {
    const CellLayout L = cell_layout(g);
    char *b = (char *)ws;
    double *A = (double *)(b + L.A), *B = (double *)(b + L.B), *X = (double *)(b + L.X), *C = (double *)(b + L.C);
    double *S = (double *)(b + L.S);
    double *U = (double *)(b + L.U), *Vt = (double *)(b + L.Vt), *sv = (double *)(b + L.sv), *E = (double *)(b + L.E);
    double *P = (double *)(b + L.P);
    int32_t *ipiv = (int32_t *)(b + L.ipiv), *perm = (int32_t *)(b + L.perm), *info = (int32_t *)(b + L.info);
    const int64_t n = 2 * g.n_wall, np = cell_panels(g);
    const rocblas_int nc = 2 * g.M, mr = 4 * g.K, r = std::min(mr, nc);
    if (g.panel < 1 || lu::panel_width(n, lu::kMaxSpan, g.panel) != g.panel) return "cell: bad LU panel width";
    hipError_t e = cell_fill(g, A, B, C, S, st);    // Q into S
    if (e != hipSuccess) return std::string("cell fill: ") + hipGetErrorString(e);
    std::lock_guard<std::mutex> lk(g_hmu);
    std::string err;
    rocblas_handle h = handle_for(st, err);
    if (!h) return err;
    err = lu_run(h, lu::factor_plan(n, g.panel, lu::kMaxSpan), A, n, A, n, ipiv, info, st);
    if (err.empty())
        err = tri_prepare(h, A, n, (double *)(b + L.Tf), (double *)(b + L.Tb), st);
    if (!err.empty()) return err;
    // the solves' row permutation: the panels' interchanges in order
    std::vector<int32_t> hp((size_t)n), hinfo((size_t)np + 1, 0);
    e = hipMemcpyAsync(hp.data(), ipiv, (size_t)n * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(hinfo.data(), info, (size_t)np * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return std::string("cell factor: ") + hipGetErrorString(e);
    for (int64_t p = 0; p < np; ++p)
        if (hinfo[(size_t)p] != 0)
            return "the wall block A is singular (LU pivot " + std::to_string(p * g.panel + hinfo[(size_t)p]) +
                   " is zero)";
    std::vector<int32_t> pm((size_t)n);
    for (int64_t i = 0; i < n; ++i) pm[(size_t)i] = (int32_t)i;
    for (int64_t k = 0; k < n; k += g.panel)
        for (int64_t i = k; i < std::min(n, k + g.panel); ++i) {
            const int64_t q = k + hp[(size_t)i] - 1;
            if (q < k || q >= n) return "cell factor: pivot out of range";
            std::swap(pm[(size_t)i], pm[(size_t)q]);
        }
    e = hipMemcpyAsync(perm, pm.data(), (size_t)n * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = gather_launch(n, nc, B, n, perm, X, n, st);            // P B
    if (e != hipSuccess) return std::string("cell factor: ") + hipGetErrorString(e);
    err = lu_run(h, lu::solve_plan(n, nc, n, g.panel, lu::kMaxSpan), A, n, X, n, ipiv, info, st);  // X = A^-1 B
    if (!err.empty()) return err;
    const double one = 1.0, minus_one = -1.0;
    rocblas_status s = rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, mr, nc, (rocblas_int)n,
                                     &minus_one, C, mr, X, (rocblas_int)n, &one, S, mr);    // S = Q - C X
    if (s != rocblas_status_success) return rb_err("rocblas_dgemm", s);
    s = rocsolver_dgesvd(h, rocblas_svect_singular, rocblas_svect_singular, mr, nc, S, mr, sv, U, mr, Vt, r, E,
                         rocblas_outofplace, info + np);
    if (s != rocblas_status_success) return rb_err("rocsolver_dgesvd", s);
    e = cell_pinv_launch(mr, nc, sv, U, Vt, rcond, P, st);
    if (e != hipSuccess) return std::string("cell pinv: ") + hipGetErrorString(e);
    int32_t svd_info = 0;
    e = hipMemcpyAsync(&svd_info, info + np, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return std::string("cell factor: ") + hipGetErrorString(e);
    if (svd_info != 0) return "the SVD of the Schur complement did not converge";
    return "";
}

std::string cell_solve(const CellArgs &g, const double *v, const double *gv, double *tau, double *c, void *ws,
                       hipStream_t st) {
    const CellLayout L = cell_layout(g);
    char *b = (char *)ws;
    double *A = (double *)(b + L.A), *X = (double *)(b + L.X), *C = (double *)(b + L.C), *P = (double *)(b + L.P);
    double *y = (double *)(b + L.y), *rr = (double *)(b + L.rr);
    const int32_t *perm = (const int32_t *)(b + L.perm);
    const int64_t n = 2 * g.n_wall;
    const rocblas_int nc = 2 * g.M, mr = 4 * g.K;
    hipError_t e = hipMemcpyAsync(rr, gv, (size_t)mr * 8, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = gather_launch(n, 1, v, n, perm, y, n, st);                 // P v
    if (e == hipSuccess)                                                                 // y = A^-1 v
        e = tri_solve(A, (const double *)(b + L.Tf), (const double *)(b + L.Tb), n, y, (double *)(b + L.w), y, st);
    if (e != hipSuccess) return std::string("cell solve: ") + hipGetErrorString(e);
    std::lock_guard<std::mutex> lk(g_hmu);
    std::string err;
    rocblas_handle h = handle_for(st, err);
    if (!h) return err;
    const double one = 1.0, minus_one = -1.0, zero = 0.0;
    rocblas_status s = rocblas_dgemv(h, rocblas_operation_none, mr, (rocblas_int)n, &minus_one, C, mr, y, 1, &one,
                                     rr, 1);                                             // g - C y
    if (s != rocblas_status_success) return rb_err("rocblas_dgemv", s);
    s = rocblas_dgemv(h, rocblas_operation_none, nc, mr, &one, P, nc, rr, 1, &zero, c, 1);         // c = S^+ (.)
    if (s != rocblas_status_success) return rb_err("rocblas_dgemv", s);
    e = hipMemcpyAsync(tau, y, (size_t)n * 8, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return std::string("cell solve: ") + hipGetErrorString(e);
    s = rocblas_dgemv(h, rocblas_operation_none, (rocblas_int)n, nc, &minus_one, X, (rocblas_int)n, c, 1, &one, tau,
                      1);                                                                // y - X c
    if (s != rocblas_status_success) return rb_err("rocblas_dgemv", s);
    return "";
}

}  // namespace s2d
