// Call schedule of the blocked dense LU (partial pivoting) and of its
// triangular solves for the periodization cell's wall block (block solve,
// Section 4.1).  Plain C++ with no device code, so that the index arithmetic
// can be checked on the host.
//
// The n x n matrix F is column-major with leading dimension n.  It is cut
// into column panels of width W; panel p starts at column k = p W:
//   getrf   the (n - k) x W panel below the diagonal, pivots into ipiv[k..]
//           (1-based, relative to row k), its status into info[p];
//   laswp   the panel's row interchanges on every column left and right of it;
//   trsm    U_12 = L_11^-1 A_12 (unit lower triangle of the panel);
//   gemm    A_22 -= L_21 U_12.
// A solve with right-hand sides T (ld >= n, rows already permuted) runs the
// forward sweep over the panels of L and the backward sweep over those of U,
// each a triangular solve on the diagonal block and a product that updates
// the rows below (above).
//
// Every library call addresses at most `lim` elements from its operand's
// base pointer (rows - 1 + (cols - 1) ld < lim): the panel width follows
// from lim, and wide operands are cut into column chunks.  The dense
// libraries' 32-bit interfaces then never form an element offset of lim or
// more, whatever the matrix size.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace s2d {
namespace lu {

// 2^30 elements: the size the 32-bit library interfaces have been run at
// (a 32,256 x 32,256 matrix is 1.04e9 elements)
constexpr int64_t kMaxSpan = int64_t(1) << 30;

enum : int { kGetrf = 0, kLaswp = 1, kTrsm = 2, kGemm = 3 };

// One call.  Offsets are in elements: a into F, b and c into the target T
// (T is F itself for the factorisation).
//   kGetrf  F[a] m x n panel, pivots ipiv[piv .. piv + n), status info[slot]
//   kLaswp  pivots ipiv[piv .. piv + k) applied to the n columns of T[b]
//           (b at the panel's first row; pivots relative to that row)
//   kTrsm   T[b] (m x n) = tri(F[a])^-1 T[b]; F[a] is m x m, unit lower
//           (upper == 0) or non-unit upper (upper == 1)
//   kGemm   T[c] (m x n) -= F[a] (m x k) T[b] (k x n)
struct Call {
    int op, upper;
    int64_t m, n, k;
    int64_t a, b, c;
    int64_t piv, slot;
};

// element span of an r x c operand with leading dimension ld
inline int64_t span(int64_t r, int64_t c, int64_t ld) { return r <= 0 || c <= 0 ? 0 : (r - 1) + (c - 1) * ld + 1; }

// the widest number of columns of an r-row operand (leading dimension ld)
// within lim elements; 0 if not even one column fits
inline int64_t col_chunk(int64_t r, int64_t ld, int64_t lim) {
    if (r < 1 || ld < r || lim < r) return 0;
    return (lim - r) / ld + 1;
}

// panel width: req when 1 <= req <= the widest allowed, the widest allowed
// (rounded down to a multiple of 256 above 512) when req == 0, else 0
inline int64_t panel_width(int64_t n, int64_t lim, int64_t req) {
    if (n < 1) return 0;
    int64_t w = col_chunk(n, n, lim);
    if (w < 1) return 0;
    if (w >= n) w = n;
    else if (w > 512) w &= ~int64_t(255);
    if (req == 0) return w;
    return req >= 1 && req <= w ? req : 0;
}

// columns [c0, c1) of T cut into chunks of at most W columns that keep an
// r-row block at leading dimension ld within lim; fn(c, cols) per chunk
template <class Fn>
inline void chunks(int64_t c0, int64_t c1, int64_t r, int64_t ld, int64_t W, int64_t lim, Fn fn) {
    int64_t cc = std::min(W, col_chunk(r, ld, lim));
    if (cc < 1) cc = 1;
    for (int64_t c = c0; c < c1; c += cc) fn(c, std::min(cc, c1 - c));
}

inline std::vector<Call> factor_plan(int64_t n, int64_t W, int64_t lim) {
    std::vector<Call> out;
    if (n < 1 || W < 1) return out;
    const int64_t ld = n;
    int64_t slot = 0;
    for (int64_t k = 0; k < n; k += W, ++slot) {
        const int64_t kb = std::min(W, n - k), r = n - k, k2 = k + kb;
        out.push_back({kGetrf, 0, r, kb, 0, k + k * ld, 0, 0, k, slot});
        // interchanges on the columns left and right of the panel (the
        // swap kernel indexes in 64 bits; chunked like the rest all the same)
        chunks(0, k, r, ld, W, lim, [&](int64_t c, int64_t w) {
            out.push_back({kLaswp, 0, r, w, kb, 0, k + c * ld, 0, k, 0});
        });
        chunks(k2, n, r, ld, W, lim, [&](int64_t c, int64_t w) {
            out.push_back({kLaswp, 0, r, w, kb, 0, k + c * ld, 0, k, 0});
        });
        if (k2 >= n) break;
        chunks(k2, n, kb, ld, W, lim, [&](int64_t c, int64_t w) {
            out.push_back({kTrsm, 0, kb, w, 0, k + k * ld, k + c * ld, 0, 0, 0});
        });
        chunks(k2, n, std::max(n - k2, kb), ld, W, lim, [&](int64_t c, int64_t w) {
            out.push_back({kGemm, 0, n - k2, w, kb, k2 + k * ld, k + c * ld, k2 + c * ld, 0, 0});
        });
    }
    return out;
}

// solve of F x = T (rows of T already permuted) in place, nrhs columns of T
// at leading dimension ldt; the sweeps use blocks of S rows (at most the
// widest panel for lim)
inline std::vector<Call> solve_plan(int64_t n, int64_t nrhs, int64_t ldt, int64_t S, int64_t lim) {
    std::vector<Call> out;
    S = std::min(S, panel_width(n, lim, 0));
    if (n < 1 || nrhs < 1 || ldt < n || S < 1) return out;
    const int64_t ld = n;
    for (int64_t k = 0; k < n; k += S) {              // L y = T
        const int64_t kb = std::min(S, n - k), k2 = k + kb;
        chunks(0, nrhs, kb, ldt, nrhs, lim, [&](int64_t c, int64_t w) {
            out.push_back({kTrsm, 0, kb, w, 0, k + k * ld, k + c * ldt, 0, 0, 0});
        });
        if (k2 < n)
            chunks(0, nrhs, std::max(n - k2, kb), ldt, nrhs, lim, [&](int64_t c, int64_t w) {
                out.push_back({kGemm, 0, n - k2, w, kb, k2 + k * ld, k + c * ldt, k2 + c * ldt, 0, 0});
            });
    }
    const int64_t last = ((n - 1) / S) * S;
    for (int64_t k = last; k >= 0; k -= S) {          // U x = y
        const int64_t kb = std::min(S, n - k);
        chunks(0, nrhs, kb, ldt, nrhs, lim, [&](int64_t c, int64_t w) {
            out.push_back({kTrsm, 1, kb, w, 0, k + k * ld, k + c * ldt, 0, 0, 0});
        });
        if (k > 0)
            chunks(0, nrhs, std::max(k, kb), ldt, nrhs, lim, [&](int64_t c, int64_t w) {
                out.push_back({kGemm, 0, k, w, kb, k * ld, k + c * ldt, c * ldt, 0, 0});
            });
    }
    return out;
}

}  // namespace lu
}  // namespace s2d
