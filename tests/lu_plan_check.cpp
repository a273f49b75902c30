// Host check of the blocked LU call schedule (paper_1510_05616_amd/csrc/lu_plan.h).
//
// check <n> <lim> <W> <S>: every call's operands stay within lim elements
//   of their base pointers and inside their buffers (index arithmetic only,
//   for sizes up to the largest cells).
// run <n> <lim> <W> <S> <nrhs> <seed>: executes the schedule with plain
//   loops for getrf / laswp / trsm / gemm on a random matrix and compares
//   the solution of A x = b with that of unblocked Gaussian elimination with
//   partial pivoting on the same matrix.
// Prints "OK ..." on success, "FAIL ..." and exits 1 otherwise.
#include "../paper_1510_05616_amd/csrc/lu_plan.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

using namespace s2d::lu;

static int fail(const std::string &m) {
    std::printf("FAIL %s\n", m.c_str());
    return 1;
}

// operand r x c at offset off, leading dimension ld, in a buffer of len
// elements: within lim from its base and inside the buffer
static bool operand_ok(int64_t off, int64_t r, int64_t c, int64_t ld, int64_t len, int64_t lim, std::string &why,
                       const char *what) {
    if (r < 1 || c < 1) return true;
    const int64_t sp = span(r, c, ld);
    if (off < 0 || ld < r || sp > lim || off + sp > len) {
        why = std::string(what) + " off " + std::to_string(off) + " r " + std::to_string(r) + " c " +
              std::to_string(c) + " ld " + std::to_string(ld) + " span " + std::to_string(sp);
        return false;
    }
    return true;
}

static bool check_plan(const std::vector<Call> &plan, int64_t n, int64_t ldt, int64_t nrhs, int64_t lim,
                       bool factor, std::string &why) {
    const int64_t lenF = n * n, lenT = factor ? lenF : ldt * nrhs, ld = n;
    const int64_t tld = factor ? ld : ldt;
    for (const Call &c : plan) {
        switch (c.op) {
            case kGetrf:
                if (!factor) return why = "getrf in a solve", false;
                if (!operand_ok(c.a, c.m, c.n, ld, lenF, lim, why, "getrf")) return false;
                if (c.piv < 0 || c.piv + c.n > n || c.a != c.piv + c.piv * ld) return why = "getrf pivots", false;
                break;
            case kLaswp:
                if (!operand_ok(c.b, c.m, c.n, tld, lenT, lim, why, "laswp")) return false;
                if (c.piv < 0 || c.piv + c.k > n || c.k > c.m) return why = "laswp pivots", false;
                break;
            case kTrsm:
                if (!operand_ok(c.a, c.m, c.m, ld, lenF, lim, why, "trsm triangle")) return false;
                if (!operand_ok(c.b, c.m, c.n, tld, lenT, lim, why, "trsm block")) return false;
                break;
            case kGemm:
                if (!operand_ok(c.a, c.m, c.k, ld, lenF, lim, why, "gemm left")) return false;
                if (!operand_ok(c.b, c.k, c.n, tld, lenT, lim, why, "gemm right")) return false;
                if (!operand_ok(c.c, c.m, c.n, tld, lenT, lim, why, "gemm out")) return false;
                break;
            default:
                return why = "unknown op", false;
        }
        // the 32-bit library interfaces take every size as a 32-bit int
        if (c.m > INT32_MAX || c.n > INT32_MAX || c.k > INT32_MAX) return why = "size above 2^31", false;
    }
    return true;
}

// --- plain loops -----------------------------------------------------------
static int64_t getrf(double *A, int64_t m, int64_t n, int64_t ld, int32_t *ipiv) {
    int64_t info = 0;
    for (int64_t j = 0; j < std::min(m, n); ++j) {
        int64_t p = j;
        for (int64_t i = j + 1; i < m; ++i)
            if (std::fabs(A[i + j * ld]) > std::fabs(A[p + j * ld])) p = i;
        ipiv[j] = (int32_t)(p + 1);
        if (A[p + j * ld] == 0.0) {
            if (!info) info = j + 1;
            continue;
        }
        if (p != j)
            for (int64_t c = 0; c < n; ++c) std::swap(A[j + c * ld], A[p + c * ld]);
        for (int64_t i = j + 1; i < m; ++i) A[i + j * ld] /= A[j + j * ld];
        for (int64_t c = j + 1; c < n; ++c)
            for (int64_t i = j + 1; i < m; ++i) A[i + c * ld] -= A[i + j * ld] * A[j + c * ld];
    }
    return info;
}

static void laswp(double *T, int64_t cols, int64_t ld, const int32_t *ipiv, int64_t k) {
    for (int64_t c = 0; c < cols; ++c)
        for (int64_t i = 0; i < k; ++i) {
            const int64_t r = ipiv[i] - 1;
            if (r != i) std::swap(T[i + c * ld], T[r + c * ld]);
        }
}

static void trsm(const double *F, int64_t m, int64_t ld, bool upper, double *T, int64_t n, int64_t ldt) {
    for (int64_t c = 0; c < n; ++c) {
        double *x = T + c * ldt;
        if (!upper) {
            for (int64_t j = 0; j < m; ++j)
                for (int64_t i = j + 1; i < m; ++i) x[i] -= F[i + j * ld] * x[j];
        } else {
            for (int64_t j = m - 1; j >= 0; --j) {
                x[j] /= F[j + j * ld];
                for (int64_t i = 0; i < j; ++i) x[i] -= F[i + j * ld] * x[j];
            }
        }
    }
}

// T[c] -= F (m x k) T[b] (k x n)
static void gemm(const double *F, int64_t ld, double *T, int64_t ldt, int64_t m, int64_t n, int64_t k, int64_t b,
                 int64_t c) {
    for (int64_t jc = 0; jc < n; ++jc)
        for (int64_t l = 0; l < k; ++l) {
            const double x = T[b + l + jc * ldt];
            for (int64_t i = 0; i < m; ++i) T[c + i + jc * ldt] -= F[i + l * ld] * x;
        }
}

// the schedule on A in place; returns the status, fills ipiv
static int64_t run_factor(const std::vector<Call> &plan, double *A, int64_t n, int32_t *ipiv) {
    int64_t info = 0;
    for (const Call &c : plan) {
        if (c.op == kGetrf) {
            const int64_t s = getrf(A + c.a, c.m, c.n, n, ipiv + c.piv);
            if (s && !info) info = c.piv + s;
        } else if (c.op == kLaswp) {
            laswp(A + c.b, c.n, n, ipiv + c.piv, c.k);
        } else if (c.op == kTrsm) {
            trsm(A + c.a, c.m, n, c.upper != 0, A + c.b, c.n, n);
        } else if (c.op == kGemm) {
            gemm(A + c.a, n, A, n, c.m, c.n, c.k, c.b, c.c);
        }
    }
    return info;
}

static void run_solve(const std::vector<Call> &plan, const double *F, int64_t n, double *T, int64_t ldt) {
    for (const Call &c : plan) {
        if (c.op == kTrsm) trsm(F + c.a, c.m, n, c.upper != 0, T + c.b, c.n, ldt);
        else if (c.op == kGemm) gemm(F + c.a, n, T, ldt, c.m, c.n, c.k, c.b, c.c);
    }
}

static uint64_t rng_state;
static double urand() {
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

int main(int argc, char **argv) {
    if (argc < 6) return fail("usage");
    const std::string mode = argv[1];
    const int64_t n = std::atoll(argv[2]), lim = std::atoll(argv[3]), Wreq = std::atoll(argv[4]),
                  S = std::atoll(argv[5]);
    const int64_t W = panel_width(n, lim, Wreq);
    if (W < 1) return fail("no panel width for n " + std::to_string(n));
    const std::vector<Call> fp = factor_plan(n, W, lim);
    std::string why;
    if (!check_plan(fp, n, n, n, lim, true, why)) return fail("factor: " + why);
    // every column is factored exactly once
    int64_t cols = 0;
    for (const Call &c : fp)
        if (c.op == kGetrf) cols += c.n;
    if (cols != n) return fail("panels cover " + std::to_string(cols) + " columns");
    if (mode == "check") {
        const int64_t nrhs = argc > 6 ? std::atoll(argv[6]) : 1;
        const std::vector<Call> sp = solve_plan(n, nrhs, n, S, lim);
        if (sp.empty()) return fail("empty solve plan");
        if (!check_plan(sp, n, n, nrhs, lim, false, why)) return fail("solve: " + why);
        int64_t maxspan = 0;
        for (const Call &c : fp) maxspan = std::max(maxspan, span(c.m, c.op == kTrsm ? c.m : c.n, n));
        std::printf("OK check n %lld W %lld calls %zu + %zu max span %lld\n", (long long)n, (long long)W, fp.size(),
                    sp.size(), (long long)maxspan);
        return 0;
    }
    if (mode != "run" || argc < 8) return fail("usage");
    const int64_t nrhs = std::atoll(argv[6]);
    rng_state = (uint64_t)std::atoll(argv[7]) * 2654435761ull + 1;
    std::vector<double> A(n * n), B(n * nrhs);
    for (auto &v : A) v = urand() - 0.5;
    for (int64_t i = 0; i < n; ++i) A[i + i * n] += 0.1 * (urand() - 0.5);   // pivoting matters
    for (auto &v : B) v = urand() - 0.5;
    // reference: unblocked elimination on a copy
    std::vector<double> R = A, X = B;
    std::vector<int32_t> rp(n), ip(n);
    if (getrf(R.data(), n, n, n, rp.data())) return fail("reference singular");
    laswp(X.data(), nrhs, n, rp.data(), n);
    trsm(R.data(), n, n, false, X.data(), nrhs, n);
    trsm(R.data(), n, n, true, X.data(), nrhs, n);
    // the schedule
    std::vector<double> F = A;
    if (run_factor(fp, F.data(), n, ip.data())) return fail("blocked factor singular");
    // the solves' row permutation from the panels' pivots
    std::vector<int64_t> perm(n);
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    for (int64_t k = 0; k < n; k += W)
        for (int64_t i = 0; i < std::min(W, n - k); ++i) std::swap(perm[k + i], perm[k + ip[k + i] - 1]);
    const int64_t ldt = n + 3;
    std::vector<double> T(ldt * nrhs, 0.0);
    for (int64_t c = 0; c < nrhs; ++c)
        for (int64_t i = 0; i < n; ++i) T[i + c * ldt] = B[perm[i] + c * n];
    const std::vector<Call> sp = solve_plan(n, nrhs, ldt, S, lim);
    if (!check_plan(sp, n, ldt, nrhs, lim, false, why)) return fail("solve: " + why);
    run_solve(sp, F.data(), n, T.data(), ldt);
    double err = 0.0, scale = 0.0;
    for (int64_t c = 0; c < nrhs; ++c)
        for (int64_t i = 0; i < n; ++i) {
            err = std::max(err, std::fabs(T[i + c * ldt] - X[i + c * n]));
            scale = std::max(scale, std::fabs(X[i + c * n]));
        }
    // the same pivot rows as the unblocked elimination
    for (int64_t i = 0; i < n; ++i)
        if (ip[i] + (i / W) * W != rp[i]) return fail("pivot " + std::to_string(i) + " differs");
    if (!(err <= 1e-9 * scale)) return fail("solution differs: " + std::to_string(err / scale));
    std::printf("OK run n %lld W %lld calls %zu + %zu rel err %.3e\n", (long long)n, (long long)W, fp.size(),
                sp.size(), err / scale);
    return 0;
}
