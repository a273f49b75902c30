/*
 * stokes2d_vesicle.h -- C ABI of libstokes2d.so for the vesicle time step
 * (Marple, Barnett, Gillman, Veerapaneni, arXiv 1510.05616, Section 3.2 and
 * Algorithm 1, steps 2 and 6-9; Appendices A-C).
 *
 * A vesicle set is n_curves closed curves, curve c owning the global nodes
 * [curve_off[c], curve_off[c+1]).  Each curve is counter-clockwise with N
 * nodes (even, 4 <= N <= 512) equispaced in a parameter alpha_j = 2 pi j / N.
 * Discrete operators:
 *   - D_alpha: the spectral derivative of the trigonometric interpolant (the
 *     Nyquist mode has zero derivative at the nodes), i.e. the circulant
 *     (D_alpha v)_m = sum_{j != m} 1/2 (-1)^(m-j) cot(pi (m-j) / N) v_j;
 *   - D_s = D_alpha / |x_alpha| (arc-length derivative); x_ssss = D_s^4 x;
 *   - trapezoid weights w_j = (2 pi / N) |x_alpha|_j, outward normal
 *     (y_alpha, -x_alpha) / |x_alpha|.
 * A curve that is odd, shorter than 4 or longer than 512 nodes, or
 * inconsistent with curve_off gets NaN outputs.
 *
 * Memory: every array is a DEVICE pointer, FP64 (int32 offsets), caller
 * owned; workspaces are 256-byte aligned and sized by the *_workspace_size
 * calls.  Calls are asynchronous on `stream` except ves_step_solve and
 * ves_time_step, whose GMRES reads dot products back to the host each
 * iteration (they return when the solve has finished; the update,
 * corrections and outputs are enqueued on `stream`).  Errors as in
 * stokes2d.h (s2d_status, stokes2d_last_error()); stokes2d_init() must have
 * been called for the current device.
 */
#ifndef STOKES2D_VESICLE_H
#define STOKES2D_VESICLE_H

#include "stokes2d.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Per node: speed |x_alpha|, weight w, unit outward normal (nx, ny) and
 * unit tangent (tx, ty) = x_alpha / |x_alpha| = x_s.  Any output may be NULL. */
S2D_API int ves_geometry(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off,
                         const double *x, const double *y, double *speed, double *w,
                         double *nx, double *ny, double *tx, double *ty, void *stream);

/* Membrane forces of Algorithm 1, step 2 (Section 3.1): bending
 * f_b = -kappa_B x_ssss and tension f_sigma = (sigma x_s)_s.  sigma may be
 * NULL (zero tension); an output pair may be NULL (not computed). */
S2D_API int ves_forces(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off,
                       const double *x, const double *y, const double *sigma, double kappa_b,
                       double *fbx, double *fby, double *fsx, double *fsy, void *stream);

/* The total membrane force f = f_b + f_sigma (Algorithm 1, step 2) into
 * fx, fy; sigma may be NULL (bending only). */
S2D_API int ves_total_force(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off,
                            const double *x, const double *y, const double *sigma, double kappa_b,
                            double *fx, double *fy, void *stream);

/* Perimeter (sum of weights) and enclosed area (integral of x y_alpha
 * d alpha, Appendix B) of every curve: [n_curves] each; either may be NULL. */
S2D_API int ves_measure(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off,
                        const double *x, const double *y, double *length, double *area,
                        void *stream);

/* Parameters of the semi-implicit step, Eq. (tsteplinsys):
 *     [ I + dt kappa_B S D_s^4      -S D_s(x_s .) ] [ u     ]   [ -kappa_B S x_ssss + u_resp ]
 *     [ x_s . D_s                    0            ] [ sigma ] = [ (L0 - L) / (dt L)          ]
 * S = S^near_{gamma,gamma}: the single layer (Section 2.1 Eq. (S), viscosity
 * mu) of all vesicles at all vesicle nodes, images img_lo..img_hi of period d,
 * Kress's product quadrature on each node's own curve at image 0.  The last
 * row is Eq. (ALC) with L0 [n_curves] the reference perimeters; L0 = NULL
 * gives x_s . u_s = 0.  u_resp_x, u_resp_y: the channel's response velocity
 * at the nodes ([n_nodes] each) or NULL (none, e.g. free space).  mode: the
 * s2d_mode of the single-layer sums in ves_step_apply.  The solves
 * (ves_step_solve, ves_time_step) with S2D_FP32C refine iteratively: the
 * right-hand side and every residual b - A z in FP64, each correction
 * A dz = r by GMRES with FP32C sums to a relative 1e-4 (FP32C sums alone
 * stall GMRES near 1e-5: D_s^4 amplifies their rounding); they reach the
 * same tolerance as S2D_FP64. */
typedef struct ves_step_params {
    int32_t mode;
    double dt, kappa_b, mu;
    double d;
    int32_t img_lo, img_hi;
    const double *L0;
    const double *u_resp_x, *u_resp_y;
    double tol;            /* GMRES: stop at ||b - A z|| <= tol ||b|| */
    int32_t restart;       /* Krylov vectors per cycle (1..128) */
    int32_t max_iter;      /* total iterations */
    int32_t precond;       /* 1: right preconditioning by the block-diagonal self
                              interactions (each curve's block of the matrix above
                              with S restricted to the curve itself, image 0),
                              rebuilt every solve; 0: none */
    int32_t nmax;          /* largest node count of any curve (>= the actual one;
                              sizes the preconditioner's workspace) */
    int32_t near;          /* close evaluation between vesicles (Section 3.2): 0 none, the
                              trapezoid rule for every pair of distinct vesicles; 1 upsampled:
                              a node closer than near_band h_c to another vesicle c, or to an
                              image of one (h_c the largest trapezoid weight of c, the
                              distance to c's nearest node), gets the difference between
                              c's single layer by the near_P-times upsampled quadrature and
                              by the trapezoid rule (near_correct_eval's
                              S2D_NEAR_UPSAMPLE), in S and in b.  The pairs are found once
                              per call (one read-back: ves_step_apply then waits for the
                              stream too).  Needs nmax in 4..256. */
    int32_t near_P;        /* upsampling factor: near_P >= 2, near_P nmax <= 2048 */
    double near_band;      /* > 0, in units of h_c */
    int32_t near_max;      /* capacity for the (node, vesicle, image) pairs (>= 1; sizes the
                              workspace); a call that finds more returns S2D_EINVAL */
    int32_t warm;          /* 0: GMRES starts from z = 0; 1: from a given z (ves_step_solve:
                              the z passed in; ves_time_step: (u, v, sigma), u and v holding
                              the previous step's velocity), GMRES then solves for the
                              correction of the FP64 residual b - A z; the same tolerance
                              relative to ||b|| */
} ves_step_params;

/* Workspace bytes for ves_step_apply / ves_step_solve / ves_time_step. */
S2D_API size_t ves_step_workspace_size(int64_t n_nodes, int32_t n_curves, const ves_step_params *p);

/* out = A z for the step matrix above (z, out: [3 n_nodes] = [u_x; u_y;
 * sigma]), and b, its right-hand side ([3 n_nodes], may be NULL). */
S2D_API int ves_step_apply(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off,
                           const double *x, const double *y, const ves_step_params *p,
                           const double *z, double *out, double *b,
                           void *ws, size_t ws_bytes, void *stream);

/* Solves the step system by restarted GMRES from z = 0, or from the z
 * passed in when p->warm (classical Gram-Schmidt applied twice, fixed-order
 * reductions: bitwise reproducible).  z: [3 n_nodes] solution.  iters, rel_res: host pointers
 * (may be NULL) for the iteration count and the final ||b - A z|| / ||b||.
 * Returns S2D_OK also when max_iter is reached; check rel_res.  iters
 * counts the GMRES iterations of all corrections in S2D_FP32C mode. */
S2D_API int ves_step_solve(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off,
                           const double *x, const double *y, const ves_step_params *p,
                           double *z, int32_t *iters, double *rel_res,
                           void *ws, size_t ws_bytes, void *stream);

/* Appendix B: x <- x + c (y_alpha, -x_alpha) per curve, c the root nearest
 * zero of the quadratic that makes the area A0[c]; in place. */
S2D_API int ves_area_correct(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off,
                             double *x, double *y, const double *A0, void *stream);

/* Appendix C, Algorithm 2: the arc length s(alpha) from the Fourier series of
 * |x_alpha| integrated term by term, parameters alpha*_k with s = k L / N by
 * linear interpolation in the table s(2 pi j / N), then x, y (and sigma, if
 * not NULL) replaced by their trigonometric interpolants at alpha*; in place. */
S2D_API int ves_reparameterize(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off,
                               double *x, double *y, double *sigma, void *stream);

/* One time step (Algorithm 1, steps 6-9): solve the step system, then
 * x <- x + dt u, area correction to A0 (if not NULL), reparameterization of
 * x, y and sigma (if reparam != 0).  sigma: [n_nodes] in/out, receives
 * sigma^{k+1}.  u, v: [n_nodes] outputs (may be NULL unless p->warm; with
 * p->warm they are also inputs: the starting guess of the velocity, such as
 * the last step's output). */
S2D_API int ves_time_step(int64_t n_nodes, int32_t n_curves, const int32_t *curve_off,
                          double *x, double *y, double *sigma, const ves_step_params *p,
                          const double *A0, int reparam, double *u, double *v,
                          int32_t *iters, double *rel_res,
                          void *ws, size_t ws_bytes, void *stream);

/* The channel's response to the vesicles, Algorithm 1 steps 3-5 (Section
 * 3.1), for the force density (fx, fy) on the vesicles (e.g. f_b + f_sigma
 * from ves_forces) and a cell factored by stokes2d_cell_factor (cell_ws):
 *   v_U, v_D = -S^near f on the walls (Eq. (vesU)),
 *   g_u = -S_{gamma-d} f|_R + S_{gamma+d} f|_L,
 *   g_T = -T(S_{gamma-d} f, Q_{gamma-d} f)|_R + T(S_{gamma+d} f, Q_{gamma+d} f)|_L
 *         + p_drive (1, 0)                   (Eq. (vesgT); p_drive is the
 *                                           pressure drop p(L) - p(R) per period),
 * the cell system for tau and c, and u_resp = D^near tau + sum_m c_m phi_m
 * (Eq. (urep)) at the vesicle nodes: u_resp_x, u_resp_y [n_nodes] (written),
 * the input u_resp of ves_step_params.  mode: the s2d_mode of the layer
 * sums; the wall double layer at the vesicles uses the plain trapezoid rule
 * (close evaluation: near_wall_correct_eval).  cell_ws also serves as the
 * solve's scratch: calls sharing it must be ordered on one stream. */
S2D_API size_t ves_response_workspace_size(const s2d_cell *cell, int64_t n_nodes, int32_t n_curves,
                                           int mode);
S2D_API int ves_channel_response(const s2d_cell *cell, void *cell_ws, size_t cell_ws_bytes,
                                 int64_t n_nodes, int32_t n_curves, const int32_t *curve_off,
                                 const double *x, const double *y, const double *fx,
                                 const double *fy, double p_drive, int mode, double *u_resp_x,
                                 double *u_resp_y, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* STOKES2D_VESICLE_H */
