// Internal declarations of the periodization cell and the channel's
// response (cell.hip), apart from the pair kernels' shared header.
#pragma once
#include "s2d_internal.h"

namespace s2d {

// Periodization system of one channel cell (device-passable by value).
struct CellArgs {
    int64_t n_wall;                                   // wall nodes N (both walls)
    const double *x, *y, *nx, *ny, *w, *kap;
    int32_t K;                                        // side collocation heights
    const double *side_y;
    double xl;                                        // x of the left side wall
    int32_t M;                                        // proxy Stokeslets
    double cx, cy, R;                                 // proxy circle
    double d, mu;
    int64_t panel;                                    // LU panel width (columns)
};
// workspace of a factored cell (byte offsets): A holds the LU factors, ipiv
// the panels' pivots, perm the row permutation of the solves, Tf / Tb the
// forward and backward sweeps' block tiles, w sweep scratch, info the panels'
// LU status then the SVD's
struct CellLayout {
    size_t A, B, X, C, S, U, Vt, sv, E, P, y, rr, ipiv, perm, Tf, Tb, w, info, total;
};
CellLayout cell_layout(const CellArgs &g);
int64_t cell_panels(const CellArgs &g);
hipError_t cell_fill(const CellArgs &g, double *A, double *B, double *C, double *Q, hipStream_t st);
hipError_t cell_pinv_launch(int m, int n, const double *sv, const double *U, const double *Vt, double rcond,
                            double *P, hipStream_t st);
// data of the channel's response to vesicles (cell.hip)
hipError_t resp_side_launch(int K, const double *side_y, double xl, double d, double *sxl, double *sxr, double *mx,
                            double *my, hipStream_t st);
hipError_t resp_pack_launch(int64_t nw, const double *vwx, const double *vwy, int K, const double *s, double p_drive,
                            double *v, double *g, hipStream_t st);
hipError_t resp_unpack_launch(int64_t nw, const double *tau, double *tx, double *ty, int M, const double *c,
                              double pcx, double pcy, double R, double *cx, double *cy, double *px, double *py,
                              double *pw, int32_t *poff, hipStream_t st);
// "" on success, else a message; factor waits for the stream
std::string cell_factor(const CellArgs &g, double rcond, void *ws, hipStream_t st);
std::string cell_solve(const CellArgs &g, const double *v, const double *gv, double *tau, double *c, void *ws,
                       hipStream_t st);

}  // namespace s2d
