/*
 * stokes2d.h -- C ABI of libstokes2d.so: free-space 2D Stokes layer
 * potentials with periodic near images on MI355X (gfx950).
 *
 * What is computed (Marple, Barnett, Gillman, Veerapaneni, "A fast algorithm
 * for simulating multiphase flows through periodic geometries of arbitrary
 * shape", arXiv 1510.05616):
 *
 *   single layer, Section 2.1 Eq. (S) summed as the imposed flow of
 *   Section 3.1 Eq. (utotrep):
 *     u(x) = 1/(4 pi mu) sum_{n=img_lo}^{img_hi} sum_j
 *            [ -1/2 log|r|^2 I + r r^T / |r|^2 ] w_j f_j,  r = x - y_j - n d e1
 *
 *   double layer, Section 2.1 Eq. (D) summed as Eq. (Dnr):
 *     u(x) = 1/pi sum_{n=img_lo}^{img_hi} sum_j r (r . n_j)(r . tau_j) w_j / |r|^4
 *
 * The source nodes carry periodic-trapezoid weights w_j (Section 2.3).  A
 * target that is node i of source curve c (declared through on_curve and
 * on_node) is treated as the paper's Nystrom discretisation does:
 *   - single layer: the n = 0 interaction with its own curve c is replaced by
 *     Kress's product quadrature for the logarithmic singularity (Section 3.2,
 *     spectrally accurate Nystrom method with periodic Kress corrections);
 *     curve c must have an even node count N = 2m with nodes equispaced in a
 *     smooth parameter, w_k = (2 pi / N) |x'(t_k)|;
 *   - double layer: the n = 0 term of node i itself is replaced by the
 *     diagonal limit -(kappa_i / 2 pi) t_i t_i^T tau_i w_i (Section 2.3); the
 *     result is the principal-value operator D_{Gamma,Gamma}; the caller adds
 *     the -1/2 tau jump of Eq. (JR) if it wants the interior limit.
 * With img_lo = -1, img_hi = 1 this is the |n| <= 1 near-image sum of the
 * paper; img_lo = img_hi = +-1 gives the single far images of the
 * periodicity blocks (Section 2.2, Eqs. (BIEgu) and (vesU)-(vesgT)).
 *
 * Conventions (the paper shows them only in a figure):
 *   - signed curvature kappa = -(x'' . n) / |x'|^2 (positive on a convex curve
 *     with outward normal);  normals are taken as given.
 *
 * Memory and ownership.  Every array argument is a DEVICE pointer to
 * caller-owned memory, structure-of-arrays, FP64 (int32 for indices), in
 * every mode; the mode selects only the internal arithmetic.  The library
 * never allocates, frees or keeps user memory: scratch comes from the
 * caller's workspace (size from stokes2d_workspace_size(), 256-byte aligned).
 * Calls are asynchronous on `stream` (a hipStream_t, or NULL for the null
 * stream); the caller synchronises.  Two calls that share a workspace must be
 * ordered on one stream.
 *
 * Errors.  Every entry point returns an s2d_status.  Argument checks run on
 * the host before any launch: a call that fails them launches nothing and
 * leaves the outputs untouched.  Index contents of device arrays (curve_off,
 * on_curve, on_node) are not read on the host; a target whose on_curve /
 * on_node entry is out of range, or that sits on an odd-sized curve in a
 * single-layer call, gets NaN outputs.  stokes2d_last_error() returns a
 * message for the calling thread's last failure.
 */
#ifndef STOKES2D_H
#define STOKES2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define S2D_API __attribute__((visibility("default")))

typedef enum {
    S2D_OK = 0,
    S2D_EINVAL = -1,      /* bad argument (NULL pointer, size, image range, mu <= 0, ...) */
    S2D_EHIP = -2,        /* a HIP runtime call failed */
    S2D_ENOTSUP = -3,     /* unsupported mode / device */
    S2D_EWORKSPACE = -4,  /* workspace NULL, too small or misaligned */
    S2D_ENOINIT = -5      /* stokes2d_init() was not called for the current device */
} s2d_status;

typedef enum {
    S2D_FP64 = 0,         /* every pair term in FP64 */
    S2D_FP32C = 1         /* pair terms in FP32, exact FP64 coordinate differences,
                             FP32 sub-blocks merged into FP64 accumulators; the own-curve
                             Kress quadrature and the diagonal limit stay FP64 */
} s2d_mode;

typedef enum {
    S2D_OP_SLP = 0,               /* single-layer velocity */
    S2D_OP_DLP = 1,               /* double-layer velocity */
    S2D_OP_SLP_PRESSURE = 2,      /* single-layer pressure (free targets) */
    S2D_OP_DLP_PRESSURE = 3,      /* double-layer pressure (free targets) */
    S2D_OP_SLP_TRACTION = 4       /* single-layer traction (free targets with normals) */
} s2d_op;

/* A set of source curves (device pointers).  Curve c owns global nodes
 * [curve_off[c], curve_off[c+1]). */
typedef struct s2d_curves {
    int64_t n_nodes;
    int32_t n_curves;
    const int32_t *curve_off;   /* [n_curves + 1], curve_off[0] = 0, curve_off[n_curves] = n_nodes */
    const double *x, *y;        /* node coordinates */
    const double *nx, *ny;      /* unit normals: DLP always; SLP only when targets sit on curves */
    const double *w;            /* trapezoid weights */
    const double *kappa;        /* signed curvature: DLP with on-curve targets only, else may be NULL */
    const double *fx, *fy;      /* density: force f (SLP) or double-layer density tau (DLP) */
} s2d_curves;

/* Target points (device pointers).  on_curve / on_node are both NULL (no
 * target sits on a source node) or both [n]: on_curve[i] = c >= 0 says target
 * i IS global source node on_node[i] of curve c (its coordinates must equal
 * that node's); -1 means a free target. */
typedef struct s2d_targets {
    int64_t n;
    const double *x, *y;
    const int32_t *on_curve, *on_node;
} s2d_targets;

/* Selects the device for the calling thread's later calls and sets up the
 * library's per-device state (device properties, launch tuning table, the
 * no-allocation entry point's scratch address, and the second stream and
 * events near_correct_eval's AUTO method uses).  Not capturable; call once
 * per device before any evaluation. */
S2D_API int stokes2d_init(int device);

/* Bytes of workspace an evaluation with these arguments needs (0 on bad
 * arguments).  op is an s2d_op; mode an s2d_mode. */
S2D_API size_t stokes2d_workspace_size(int op, int mode, const s2d_curves *src,
                                       const s2d_targets *trg);

/* Single-layer potential (Stokeslet) of density src->fx, fy at the targets,
 * summed over source images n = img_lo..img_hi shifted by n * d along x.
 * Writes u, v ([trg->n] device FP64), or adds to them when accumulate != 0.
 * Requires mu > 0, img_lo <= img_hi, |img| <= 64, d > 0 if any image is
 * nonzero.  Pointers in src may be NULL only when their count is 0. */
S2D_API int stokes2d_slp_eval(int mode, const s2d_curves *src, const s2d_targets *trg,
                              double d, int32_t img_lo, int32_t img_hi, double mu,
                              double *u, double *v, int accumulate,
                              void *ws, size_t ws_bytes, void *stream);

/* The same evaluation for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no workspace argument; the scratch lives in a device array
 * inside the library, S2D_NOALLOC_SCRATCH_BYTES (32 MiB) per device, set up
 * by stokes2d_init and held until the process ends.  The call allocates
 * nothing and returns S2D_EWORKSPACE, launching nothing, when the problem
 * needs more scratch than that, i.e. when stokes2d_workspace_size(S2D_OP_SLP,
 * ...) exceeds S2D_NOALLOC_SCRATCH_BYTES (about 34 bytes per source node,
 * 8 more with on-curve targets, plus 16 per on-curve target: the 128k-node
 * channel needs about 6 MB; a million source nodes do not fit).
 * The result equals stokes2d_slp_eval's bit for bit.  Every call on one device
 * shares that device's scratch: calls that overlap on one device (several
 * streams, several host threads) race and must be serialised by the caller.
 * Nothing in the scratch needs to start at zero; each call overwrites what
 * it reads. */
#define S2D_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
S2D_API int stokes2d_slp_eval_noalloc(int mode, const s2d_curves *src, const s2d_targets *trg,
                                      double d, int32_t img_lo, int32_t img_hi, double mu,
                                      double *u, double *v, int accumulate, void *stream);

/* Double-layer potential (stresslet, principal value on source curves) of
 * density src->fx, fy (the paper's tau).  The double-layer velocity kernel has
 * no viscosity factor (Section 2.1, Eq. (D)). */
S2D_API int stokes2d_dlp_eval(int mode, const s2d_curves *src, const s2d_targets *trg,
                              double d, int32_t img_lo, int32_t img_hi,
                              double *u, double *v, int accumulate,
                              void *ws, size_t ws_bytes, void *stream);

/* Pressure and traction of the layer potentials at free targets (the
 * pressure representation and the traction data of the periodicity
 * conditions).  The kernels are singular where a target meets a source node,
 * so trg->on_curve / on_node must be NULL (S2D_EINVAL otherwise); targets are
 * assumed off the source curves.  Sums over source images n = img_lo..img_hi
 * as for the velocities; the same modes (FP64, FP32C with FP32 pair terms from
 * exact FP64 coordinate differences).  Output arrays are [trg->n] device FP64,
 * written, or added to when accumulate != 0.
 *
 * Single-layer pressure (Section 2.1, Eq. (Q)) of force density src->fx, fy:
 *   p(x) = 1/(2 pi) sum_n sum_j (r . w_j f_j) / |r|^2,  r = x - y_j - n d e1
 * (no viscosity factor). */
S2D_API int stokes2d_slp_pressure_eval(int mode, const s2d_curves *src, const s2d_targets *trg,
                                       double d, int32_t img_lo, int32_t img_hi,
                                       double *p, int accumulate,
                                       void *ws, size_t ws_bytes, void *stream);

/* Double-layer pressure (Section 2.1, Eq. (P)) of density src->fx, fy (tau),
 * source normals src->nx, ny:
 *   p(x) = mu/pi sum_n sum_j [ -(nu_j . tau_j) / |r|^2
 *                              + 2 (r . nu_j)(r . tau_j) / |r|^4 ],  nu_j = w_j n_j.
 * Requires mu > 0. */
S2D_API int stokes2d_dlp_pressure_eval(int mode, const s2d_curves *src, const s2d_targets *trg,
                                       double d, int32_t img_lo, int32_t img_hi, double mu,
                                       double *p, int accumulate,
                                       void *ws, size_t ws_bytes, void *stream);

/* Single-layer traction (Section 2.1, Eq. (K)) at targets with unit normals
 * (trg_nx[i], trg_ny[i]) (device FP64 [trg->n]):
 *   t(x) = -1/pi sum_n sum_j r (r . w_j f_j)(r . m) / |r|^4,  m the target normal
 * (no viscosity factor).  With single images n = -1 and n = +1 at the side
 * walls this gives the traction discrepancy data of the periodicity
 * conditions (Section 3.1, Eq. (vesgT)). */
S2D_API int stokes2d_slp_traction_eval(int mode, const s2d_curves *src, const s2d_targets *trg,
                                       const double *trg_nx, const double *trg_ny,
                                       double d, int32_t img_lo, int32_t img_hi,
                                       double *tx, double *ty, int accumulate,
                                       void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Periodization system of one channel cell (Section 2.2, Eqs. (urep)-(bsys);
 * Nystrom discretisation, Section 2.3; block solve, Section 4.1).
 *
 * The velocity in the cell is the wall double layer of density tau summed
 * over the images |n| <= 1 plus M Stokeslets c_m at proxy points on a circle
 * around the cell; the pressure correspondingly.  Rows: the velocity data v
 * at the N wall nodes (the n = 0 term with the -1/2 jump and the diagonal
 * limit), then at the K side heights the velocity difference u(R) - u(L) and
 * the traction difference T(R) - T(L) for the side normal (1, 0), R = L + d:
 *     [A B; C Q] [tau; c] = [v; g],
 * solved as S = Q - C A^-1 B, c = S^+ (g - C A^-1 v), tau = A^-1 (v - B c),
 * S^+ the pseudo-inverse over the singular values above rcond * s_max.
 * Every 2-vector is interleaved (x, y) per node: v, tau [2N], g [4K] (the K
 * velocity differences, then the K traction differences), c [2M].  Matrices
 * are column-major with leading dimension = rows: A 2N x 2N, B 2N x 2M,
 * C 4K x 2N, Q 4K x 2M.  The pair kernels of Eqs. (D), (S), (K) and the
 * double-layer traction of Eq. (T) fill them on the GPU.  A is factored by a
 * blocked LU with partial pivoting: column panels of lu_panel columns
 * (rocSOLVER getrf), their row interchanges on the other columns, and
 * rocBLAS TRSM / GEMM updates of the columns to their right; each solve
 * permutes its right-hand side and runs the forward and backward triangular
 * sweeps.  No library call is given an operand that spans more than 2^30
 * elements, which bounds the panel width: at most 16,640 columns at
 * N = 32,128, 8,192 at N = 65,536.  The libraries may allocate their own
 * device scratch.
 * ------------------------------------------------------------------------- */
typedef struct s2d_cell {
    s2d_curves walls;             /* the wall nodes of one period (x, y, nx, ny, w, kappa; the
                                     densities are not used); normals point out of the fluid;
                                     1 <= N <= 65,536 */
    int32_t n_side;               /* K >= 1 collocation heights on each side wall */
    const double *side_y;         /* [K] device */
    double x_left;                /* L at x = x_left, R at x = x_left + d */
    int32_t n_proxy;              /* M >= 1 proxy Stokeslets, equispaced from angle 0 */
    double proxy_cx, proxy_cy, proxy_r;
    double d, mu;                 /* period > 0, viscosity > 0 */
    int32_t lu_panel;             /* LU panel width in columns: 0 for the widest within the
                                     2^30-element bound (a single panel when (2N)^2 fits it),
                                     else 1 .. that width */
} s2d_cell;

/* Limits: N <= 65,536 wall nodes, and 4K * 2N and 2M * 2N at most 2^30
 * (S2D_EINVAL beyond).
 *
 * Workspace bytes of a factored cell (0 on bad arguments): the LU factors of
 * A (2N)^2 * 8 bytes, B, A^-1 B, C, the pseudo-inverse of S, the pivots, the
 * solves' row permutation and scratch. */
S2D_API size_t stokes2d_cell_workspace_size(const s2d_cell *cell);

/* Fills the four blocks into caller buffers (any may be NULL to skip). */
S2D_API int stokes2d_cell_assemble(const s2d_cell *cell, double *A, double *B, double *C, double *Q,
                                   void *stream);

/* Assembles and factors the system into ws; waits for `stream` (it reads
 * the LU and SVD status).  Not capturable.  rcond: relative cut-off of S^+
 * (the paper gives none; 1e-8 is about the square root of the noise level
 * of S).  S2D_EHIP with a message if A is singular or the SVD fails. */
S2D_API int stokes2d_cell_factor(const s2d_cell *cell, double rcond, void *ws, size_t ws_bytes,
                                 void *stream);

/* Solves for one right-hand side with a workspace factored by
 * stokes2d_cell_factor (same cell): v [2N], g [4K] in; tau [2N], c [2M]
 * out (device FP64).  Asynchronous on `stream`. */
S2D_API int stokes2d_cell_solve(const s2d_cell *cell, const double *v, const double *g, double *tau,
                                double *c, void *ws, size_t ws_bytes, void *stream);

/* One independent channel instance of a batched evaluation: the single
 * layer of the vesicles plus the double layer of the walls, images -1..1,
 * at the same n target points (trg_ves and trg_wall describe the same points;
 * their on_curve / on_node refer to ves and wall respectively). */
typedef struct s2d_instance {
    s2d_curves ves;
    s2d_curves wall;
    s2d_targets trg_ves;
    s2d_targets trg_wall;
    double d, mu;
    double *u, *v;               /* [n] outputs (written, not accumulated) */
} s2d_instance;

/* Workspace bytes for stokes2d_batch_eval over the host array inst[n_inst]
 * (0 on bad arguments).  The size covers every tile shape the tuner tries. */
S2D_API size_t stokes2d_batch_workspace_size(int mode, int32_t n_inst, const s2d_instance *inst);

/* Evaluates u = S(ves) f + D(wall) tau for every instance.  The work of all
 * instances is cut into (instance, operator, target tile, source split)
 * items, sorted longest first per operator, and run by one persistent launch
 * per operator; the whole evaluation is recorded in a HIP graph.  The first call for a given argument
 * set (mode, every pointer and size in inst[], d, mu, ws, ws_bytes) waits for
 * `stream`, picks the tile shape (timing a few candidates on the real inputs
 * unless a tuned choice for this size is cached; environment S2D_TUNE=0 keeps
 * the default, S2D_TUNE_CACHE names the JSON cache file), records the graph
 * and launches it; it is not capturable and may allocate (pinned table
 * image, graph).  Later calls with the same argument set are one graph launch
 * on `stream`: device data behind the pointers may change between calls, the
 * pointers and sizes may not.  `inst` is read only during the call.  The
 * workspace holds the call's tables and partial sums until the launched work
 * completes. */
S2D_API int stokes2d_batch_eval(int mode, int32_t n_inst, const s2d_instance *inst,
                                void *ws, size_t ws_bytes, void *stream);

/* Frees every cached batch plan and graph (waits for the device). */
S2D_API int stokes2d_batch_release(void);

/* The tile shape stokes2d_batch_eval uses for this instance set's size
 * bucket: targets per lane (*tpt: 1, 2 or 4), 256-source superblocks per
 * source split (*sbps) and resident waves per compute unit of the persistent
 * grid (*wpc).  Returns 1 when the shape comes from the tuner (this process
 * or the cache file), 0 when it is the built-in default, or a negative
 * s2d_status.  Host only; launches nothing. */
S2D_API int stokes2d_batch_tuned(int mode, int32_t n_inst, const s2d_instance *inst, int32_t *tpt,
                                 int32_t *sbps, int32_t *wpc);

/* ---------------------------------------------------------------------------
 * Near-field correction of the single layer (learned, with FFT-upsampled
 * quadrature as reference and fallback).
 *
 * For a target x near closed source curve c (given by trg_curve[i]), the
 * plain N-node trapezoid single layer of curve c loses accuracy (the paper
 * notes the trapezoid rule's near-curve error band: Section 5 footnote,
 * Section 5.1 error figure).  The
 * correction is Delta(x) = u_P(x) - u_1(x): the single layer of curve c
 * evaluated on P*N nodes obtained by FFT upsampling of the curve and its
 * density (the paper represents curves in a Fourier basis), minus the N-node
 * trapezoid value; images and other curves are not involved.  Curves must
 * have an even node count N with 8 <= N <= 256 and P*N <= 2048.
 *
 * The learned route writes Delta in the frame of the target's nearest node
 * k* (tangent t along growing node index, normal n_f turned towards the
 * target, lengths in units of the local spacing h = w_k*, offsets (s, b)):
 *   Delta = scale sum_{p=0..4} (Cflat_p(s, b) + exp(-2 pi b) dC_p) d_p,
 * d_p = (2 pi / N)^p d^p f / dt^p at k* (the density's node derivatives in
 * the frame), Cflat_p the exact correction of a straight line with
 * equispaced nodes (closed form by Poisson summation), dC_p (2 x 2 each) the
 * output of a 14-64-64-64-20 network (BF16 weights, MFMA inference), scale =
 * h / (4 pi mu) for the single layer and 1 / pi for the double layer.
 * ------------------------------------------------------------------------- */
#define S2D_NEAR_NFEAT 14            /* geometry features per target */
#define S2D_NEAR_NFRAME 20           /* FP64 frame words per target */
#define S2D_NEAR_NDERIV 10           /* FP64 derivative-table words per node */
#define S2D_NEAR_TSTRIDE 14          /* FP32 training-record words per sample */
#define S2D_NEAR_NOUT 20             /* network outputs dC[p][out][in] */
#define S2D_NEAR_NBINS 64            /* AUTO's largest number of bins of log10 b */
#define S2D_NEAR_SBINS 5             /* AUTO's bins of |s| per b bin: width 1/8, the last (|s| >= 1/2) open */
#define S2D_NEAR_KBINS 8             /* AUTO's bins of log10 |kappa h|: width 3/16 from -2, ends open */
#define S2D_NEAR_CELL (S2D_NEAR_SBINS * S2D_NEAR_KBINS)   /* table entries per b bin */
#define S2D_MLP_NPARAM 10608         /* FP32 master parameters of the 14-64-64-64-20 network */

typedef enum {
    S2D_NEAR_UPSAMPLE = 0,           /* FP64 upsampled quadrature for every target */
    S2D_NEAR_MLP = 1,                /* straight-line part plus BF16 network for every target, no fallback */
    S2D_NEAR_AUTO = 2                /* per target: none, learned or upsampled by calibrated bounds */
} s2d_near_method;

/* Workspace bytes for near_correct_eval. */
S2D_API size_t near_workspace_size(int method, const s2d_curves *ves, const s2d_targets *trg, int32_t upsample);

/* Delta at every target (du, dv: [n] device FP64, written).  trg->on_curve /
 * on_node are ignored; trg_curve[i] names the curve of `ves` the correction
 * is for.  upsample = P (1..32) of the quadrature (UPSAMPLE, and AUTO's
 * fallback); the learned route's straight-line part uses the P stored in
 * the blob (the one the network was trained for), so AUTO callers pass the
 * same P.  mlp: device blob from near_mlp_pack (MLP, AUTO).
 * AUTO decides per target against its tolerance: curve_tol[trg_curve[i]]
 * when curve_tol ([n_curves] device FP64, absolute velocity tolerances per
 * curve) is not NULL, else threshold.  Its bin is (log10 b, |s|,
 * log10 |kappa h|) in FP32 (near_calibrate):
 * b < the blob's b_min, a target inside its vesicle (against the outward
 * normal), NaN or a b bin below the first go to the quadrature; otherwise
 * Delta = 0 where the bin's largest correction times scale F (F = sum_p
 * |d_p|, both components) is within the tolerance, the learned value where
 * the bin's network bound times scale F is, the quadrature otherwise (past
 * the last b bin: 0 or the quadrature).  used_fallback: [n] device int32 or
 * NULL, set (MLP, AUTO) to 0 learned, 1 upsampled quadrature, 2 no
 * correction.  Targets of invalid curves get NaN.
 * Streams: every kernel is ordered after the caller's earlier work on
 * `stream`, and the call's last kernel runs on `stream`.  Outside stream
 * capture AUTO runs its derivatives and upsampling on a second stream of
 * the device (created by stokes2d_init, default priority), forked from and
 * joined back into `stream` by events; AUTO calls on one device take a
 * library lock while they enqueue.  Under capture everything stays on
 * `stream`; the results are the same either way. */
S2D_API int near_correct_eval(int method, const s2d_curves *ves, const s2d_targets *trg,
                              const int32_t *trg_curve, int32_t upsample, const void *mlp,
                              double threshold, const double *curve_tol, double mu, double *du,
                              double *dv, int32_t *used_fallback, void *ws, size_t ws_bytes,
                              void *stream);

/* The single layer of each target's own curve by the P-times upsampled
 * trapezoid rule (u_up, v_up) and by the plain N-node rule (u_trap, v_trap),
 * FP64 (their difference is Delta).  For normalising near-field errors. */
S2D_API size_t near_upsampled_slp_workspace_size(const s2d_curves *ves, const s2d_targets *trg, int32_t upsample);
S2D_API int near_upsampled_slp(const s2d_curves *ves, const s2d_targets *trg, const int32_t *trg_curve,
                               int32_t upsample, double mu, double *u_up, double *v_up, double *u_trap,
                               double *v_trap, void *ws, size_t ws_bytes, void *stream);

/* The density's node derivatives d_p = (2 pi / N)^p d^p f / dt^p, p = 0..4,
 * of every curve's trigonometric interpolant (N even and >= 4; other curves
 * get NaN), the Nyquist mode split evenly (its odd derivatives vanish at the
 * nodes): dtab [n_nodes][10] device FP64, d_p of fx at 2p and of fy at
 * 2p + 1.  Direct sums in FP64: one workgroup per curve up to 256 nodes,
 * a wave per coefficient and per node above (O(N^2) work per curve).  Serves
 * closed curves and wall periods alike (curves needs fx, fy and curve_off).
 * ws: near_derivs_workspace_size(curves) bytes of device scratch, 256-byte
 * aligned (256 bytes when n_nodes <= 256). */
S2D_API size_t near_derivs_workspace_size(const s2d_curves *curves);
S2D_API int near_derivs_eval(const s2d_curves *curves, double *dtab, void *ws, size_t ws_bytes, void *stream);

/* Per target, relative to curve trg_curve[i] of `ves`: the nearest node k*
 * (smallest index on ties), the geometry features X [n][14] FP32 =
 * (s, b, log(|x - x_k*| / h), sg kappa h, the nodes k*-2, k*-1, k*+1, k*+2
 * in the frame (units h), Re Q, Im Q with Q = exp(-2 pi (b + i s))) and the
 * frame [n][20] FP64 = (s, b, t_x, t_y, n_x, n_y, h, F, sg, d_0t, d_0n, ...,
 * d_4t, d_4n, sg kappa h): sg the sign of the offset along the node normal,
 * d_p from dtab (near_derivs_eval) in the frame, F = sum_p (|d_pt| + |d_pn|)
 * (1 if all vanish). */
S2D_API int near_features_eval(const s2d_curves *ves, const s2d_targets *trg, const int32_t *trg_curve,
                               const double *dtab, float *X, double *frame, void *stream);

/* Training records T [n][14] FP32 from labels (du, dv: the upsampled
 * quadrature's Delta) and frames: (d_0t, d_0n, ..., d_4t, d_4n, R_t, R_n,
 * wt, exp(-2 pi b)), R the label over scale minus the straight-line part
 * (op S2D_OP_SLP: single layer, scale h / 4 pi mu; S2D_OP_DLP: double
 * layer, scale 1 / pi, straight-line part times sg), wt = weight_gain
 * scale / (the largest |(u_ref, v_ref)| over the targets of the same
 * curve), so that the loss weighs errors as the normalised error measure
 * does (weight_gain > 0, a constant factor that keeps the gradients well
 * above Adam's eps).  curve_scale: [n_curves] device float, written with
 * those largest norms; targets of other curves get wt = 0.  upsample: the
 * P of the labels. */
S2D_API int near_train_targets(int op, int64_t n, const double *frame, const double *du, const double *dv,
                               const int32_t *trg_curve, int32_t n_curves, const double *u_ref,
                               const double *v_ref, double mu, int32_t upsample, float weight_gain,
                               float *curve_scale, float *T, void *stream);

/* Workspace bytes for a training step with `batch` samples. */
S2D_API size_t near_mlp_train_workspace_size(int32_t batch);

/* One minibatch step of weighted least squares on the learned part:
 * L = 1/(2B) sum_i |wt_i (exp(-2 pi b_i) sum_p dC_p(X_i) d_p,i - R_i)|^2 over
 * the records T (near_train_targets): forward, backward and per-parameter
 * gradient sums over the batch in fixed sample order, then an Adam update
 * (beta 0.9, 0.999, eps 1e-8) at step >= 1; step == 0 computes grad and
 * loss only.  params, adam_m, adam_v, grad: [S2D_MLP_NPARAM] device FP32
 * (the first 28 entries are the input standardisation mean and scale, not
 * trained).  loss: device float or NULL.  idx: [batch] sample indices into
 * X / T, or NULL for 0..batch-1. */
S2D_API int near_mlp_train_step(int32_t batch, const int32_t *idx, const float *X, const float *T,
                                float *params, float *adam_m, float *adam_v, int32_t step, float lr,
                                float *grad, float *loss, void *ws, size_t ws_bytes, void *stream);

/* FP32 forward pass of the master parameters: Y [n][20] = dC[p][out][in]
 * at 4p + 2 out + in. */
S2D_API int near_mlp_forward(int64_t n, const float *X, const float *params, float *Y, void *stream);

/* The input standardisation: mean and population standard deviation (1
 * where it vanishes) of each feature over X [n][14], written into params'
 * first 28 entries (FP64 sums in a fixed order). */
S2D_API int near_feature_stats(int64_t n, const float *X, float *params, void *stream);

/* Calibration of AUTO's rule on held-out targets: per bin (k, j, m), all
 * in FP32: k the bin of log10 b ([bin_lo + k bin_w, bin_lo + (k + 1)
 * bin_w), k < n_bins <= 64), j = min(floor(8 |s|), 4) the bin of |s| and m
 * = clamp(floor((log10 |kappa h| + 2) 16 / 3), 0, 7) the bin of the
 * curvature over the spacing (kappa h = frame[19]), over targets with b >=
 * b_min on the expected side (sg > 0 for the single layer, sg < 0 for the
 * double layer), the largest |(du_pred, dv_pred) - (du, dv)| and the largest
 * |(du, dv)|, both over scale F, times margin (1 + count_margin / sqrt(c))
 * for a bin of c targets (margin >= 1, count_margin >= 0: a wider margin
 * where the maximum rests on few samples): bound, bound_zero [n_bins *
 * S2D_NEAR_CELL] device float at S2D_NEAR_CELL k + 8 j + m; empty bins get
 * 3e38, and so does bound in the bins of j = 4 (|s| >= 1/2: past the
 * midpoint between two nodes the network's held-out errors underestimate
 * its errors on new targets, so the learned route is never admitted there).
 * count: [n_bins * S2D_NEAR_CELL] device int32, the targets per bin. */
S2D_API int near_calibrate(int op, int64_t n, const double *frame, const double *du_pred, const double *dv_pred,
                           const double *du, const double *dv, double mu, int32_t n_bins, float bin_lo,
                           float bin_w, float b_min, float margin, float count_margin, float *bound,
                           float *bound_zero, int32_t *count, void *stream);

/* Bytes of the BF16 inference blob; near_mlp_pack fills it (device, 256-byte
 * aligned) from FP32 master parameters, the calibrated bounds ([n_bins *
 * S2D_NEAR_CELL] as near_calibrate writes them; bound: NULL only with n_bins == 0;
 * bound_zero NULL: never skip), the bins, b_min and the upsampling factor P
 * the network was trained for. */
S2D_API size_t near_mlp_blob_size(void);
S2D_API int near_mlp_pack(const float *params, const float *bound, const float *bound_zero, int32_t n_bins,
                          float bin_lo, float bin_w, float b_min, int32_t upsample, void *blob, void *stream);

/* ---- walls: spectral upsampling and the near-wall correction ------------
 *
 * The paper evaluates the wall double layer at vesicles near a wall by the
 * plain trapezoid rule and leaves its close evaluation to future work
 * (Section 5 footnote; Section 6).  These entry points supply the
 * upsampled-quadrature correction for it, in the form the vesicles' near
 * field uses: Delta = D_P - D_1, the double layer of the P-times refined
 * wall minus that of the given one.
 *
 * Wall curves: each curve of `walls` is one period of a d-periodic wall, N
 * nodes (even, >= 4) equispaced in a parameter t in [0, 2 pi), advancing by
 * +d or -d in x per period (the sign from its first two nodes), normals nx,
 * ny, density fx, fy (w and kappa are not read).  A curve that is odd, has
 * fewer than 4 nodes or is inconsistent with curve_off gets NaN outputs. */

/* Workspace bytes for stokes2d_wall_upsample (0 on bad arguments). */
S2D_API size_t stokes2d_wall_upsample_workspace_size(const s2d_curves *walls, int32_t upsample);

/* The P N-node refinement of every wall curve (upsample = P in 1..32) by
 * trigonometric interpolation of x - s d t / (2 pi), y, fx and fy (the
 * Nyquist mode split evenly), with the speed |x'(t)| from spectral
 * derivatives: outputs [P * walls->n_nodes] device FP64 nodes x, y, unit
 * normals nx, ny (oriented like the given normal of the coarse node at or
 * before each fine one), trapezoid weights w = (2 pi / (P N)) |x'|, density
 * fx, fy; curve_off [n_curves + 1] device int32 = P * walls->curve_off.
 * FP64, direct DFT per curve (O(P N^2) work). */
S2D_API int stokes2d_wall_upsample(const s2d_curves *walls, double d, int32_t upsample,
                                   double *x, double *y, double *nx, double *ny, double *w,
                                   double *fx, double *fy, int32_t *curve_off,
                                   void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes for near_wall_correct_eval with `method` (0 on bad
 * arguments). */
S2D_API size_t near_wall_workspace_size(int method, const s2d_curves *walls, const s2d_targets *trg,
                                        int32_t upsample);

/* The learned route for the walls: features and frames as for
 * near_features_eval, of target i relative to wall curve trg_curve[i], the
 * wall unrolled over three periods so that the nearest node and its
 * neighbours may lie across the period boundary (h = w_k*).  dtab: the
 * walls' node derivatives (near_derivs_eval).  Needs the walls' w and kappa;
 * curves with fewer than 8 nodes give NaN. */
S2D_API int near_wall_features_eval(const s2d_curves *walls, const s2d_targets *trg,
                                    const int32_t *trg_curve, double d, const double *dtab, float *X,
                                    double *frame, void *stream);

/* Delta = D_P - D_1 of the wall double layer (Section 2.1 Eq. (D)) summed over
 * images img_lo..img_hi, at free targets (trg->on_curve must be NULL), FP64:
 * du, dv ([trg->n] device) are written, or Delta is added to them when
 * accumulate != 0 (so a caller adds it to the plain double layer it holds).
 * method (s2d_near_method as for near_correct_eval):
 *   UPSAMPLE: the refined-wall quadrature at every target;
 *   MLP:      the straight-line part and the network (mlp: a blob from
 *             near_mlp_pack trained on wall labels with S2D_OP_DLP) at
 *             every target, relative to wall trg_curve[i];
 *   AUTO:     per target as near_correct_eval decides (no correction, the
 *             learned route, or the refined quadrature, against
 *             curve_tol[trg_curve[i]] or threshold), the quadrature only at
 *             the fallback targets.  AUTO reads the fallback count back to
 *             the host (it waits for `stream`).
 * used_fallback: [n] device int32 or NULL, set (MLP, AUTO) to 0 network,
 * 1 quadrature, 2 no correction.  Same image and period rules as
 * stokes2d_dlp_eval. */
S2D_API int near_wall_correct_eval(int method, const s2d_curves *walls, const s2d_targets *trg,
                                   const int32_t *trg_curve, double d, int32_t img_lo,
                                   int32_t img_hi, int32_t upsample, const void *mlp,
                                   double threshold, const double *curve_tol, double *du,
                                   double *dv, int32_t *used_fallback, int accumulate, void *ws,
                                   size_t ws_bytes, void *stream);

/* Benchmarking aid: the VALU instruction issue rate reachable on this chip.
 * Launches blocks x 256 threads on `stream`, each running 8 independent
 * fused multiply-add chains of `iters` steps and writing their sum to
 * sink[thread] ([blocks * 256] device floats): form 0 FP32 with every
 * operand in a VGPR, form 1 FP32 with the multiplier a wave-uniform SGPR
 * value, form 2 FP64.  The caller times the launch (8 FMA per thread and
 * step). */
S2D_API int stokes2d_valu_probe(int form, int32_t blocks, int32_t iters, float *sink, void *stream);

/* Benchmarking aid (not capturable, not for production loops): while
 * enabled, each evaluation records a HIP event pair around its pair-sum
 * kernel launch on the caller's stream.  stokes2d_profile_read() waits for
 * the recorded events of operation `op` (an s2d_op), returns their summed
 * elapsed milliseconds and launch count, and releases them. */
S2D_API int stokes2d_profile_enable(int on);
S2D_API int stokes2d_profile_read(int op, double *total_ms, int64_t *launches);

/* Message describing the calling thread's last non-OK return. */
S2D_API const char *stokes2d_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
S2D_API int stokes2d_version(void);

#ifdef __cplusplus
}
#endif
#endif /* STOKES2D_H */
