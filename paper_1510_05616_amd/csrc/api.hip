// C ABI of libstokes2d: argument checks, launch planning, workspace carve-up
// and the launch sequence for each evaluation.  No allocation happens here:
// all scratch lives in the caller's workspace.
#include "lu_plan.h"
#include "s2d_cell.h"
#include "s2d_internal.h"
#include "s2d_near.h"
#include "../../include/stokes2d_vesicle.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

// Scratch memory of stokes2d_slp_eval_noalloc: the records, Kress tables and
// partial sums that stokes2d_slp_eval keeps in the caller's workspace.  Each
// device the library runs on holds its own copy until the process ends.  In
// host code `scratch` names a host-side stand-in, not device memory: kernels
// and copies use the address hipGetSymbolAddress returns for it on each
// device (DevState::scratch, set by stokes2d_init).
constexpr size_t kScratchBytes = S2D_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

struct DevState {
    bool init = false;
    int cus = 256;
    void *scratch = nullptr;     // this device's copy of `scratch`
    // AUTO's second stream (default priority) and its events: the
    // derivatives run beside the nearest-node search and the upsampling
    // beside the head kernel; side_mu orders the calls that use them
    hipStream_t side = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    std::mutex side_mu;
};
constexpr int kMaxDev = 64;
DevState g_dev[kMaxDev];
std::mutex g_mu;

// Optional timing of the pair kernels (benchmarking aid, not capturable):
// while enabled, each evaluation records a start/stop event pair around its
// pair-kernel launch on the caller's stream.
struct ProfEvent {
    int op;
    hipEvent_t a, b;
};
bool g_prof_on = false;
std::vector<ProfEvent> g_prof;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

using s2d::rec_bytes;

// Checks that do not depend on the device; returns S2D_OK or an error code
// with g_err set.
int check_args(int op, int mode, const s2d_curves *s, const s2d_targets *t, double d, int img_lo,
               int img_hi, double mu) {
    if (mode != S2D_FP64 && mode != S2D_FP32C) return fail(S2D_EINVAL, "mode must be S2D_FP64 or S2D_FP32C");
    if (op < S2D_OP_SLP || op > S2D_OP_SLP_TRACTION) return fail(S2D_EINVAL, "op must be an s2d_op");
    if (!s || !t) return fail(S2D_EINVAL, "src and trg must not be NULL");
    if (s->n_nodes < 0 || s->n_nodes > INT32_MAX - 2 * s2d::kSuperBlock)
        return fail(S2D_EINVAL, "src->n_nodes out of range [0, 2^31 - 513]");
    if (s->n_curves < 0) return fail(S2D_EINVAL, "src->n_curves < 0");
    if (t->n < 0) return fail(S2D_EINVAL, "trg->n < 0");
    if (s->n_nodes > 0) {
        if (!s->x || !s->y || !s->w || !s->fx || !s->fy)
            return fail(S2D_EINVAL, "src x, y, w, fx, fy must not be NULL when n_nodes > 0");
        if (!s2d::slp_sources(op) && (!s->nx || !s->ny)) return fail(S2D_EINVAL, "double layer needs src nx, ny");
    }
    if (t->n > 0 && (!t->x || !t->y)) return fail(S2D_EINVAL, "trg x, y must not be NULL when n > 0");
    if ((t->on_curve == nullptr) != (t->on_node == nullptr))
        return fail(S2D_EINVAL, "trg on_curve and on_node must both be NULL or both be set");
    if (op > S2D_OP_DLP && t->on_curve)
        return fail(S2D_EINVAL, "pressure and traction are evaluated at free targets: trg on_curve must be NULL");
    if (t->on_curve && t->n > 0) {
        if (!s->curve_off) return fail(S2D_EINVAL, "on-curve targets need src->curve_off");
        if (op == S2D_OP_SLP && s->n_nodes > 0 && (!s->nx || !s->ny))
            return fail(S2D_EINVAL, "single layer with on-curve targets needs src nx, ny");
        if (op == S2D_OP_DLP && s->n_nodes > 0 && !s->kappa)
            return fail(S2D_EINVAL, "double layer with on-curve targets needs src kappa");
    }
    if (img_lo > img_hi) return fail(S2D_EINVAL, "img_lo > img_hi");
    if (img_lo < -s2d::kMaxImages || img_hi > s2d::kMaxImages) return fail(S2D_EINVAL, "|image| > 64");
    if ((img_lo != 0 || img_hi != 0) && !(std::isfinite(d) && d > 0.0))
        return fail(S2D_EINVAL, "period d must be finite and > 0 when images are used");
    if ((op == S2D_OP_SLP || op == S2D_OP_DLP_PRESSURE) && !(std::isfinite(mu) && mu > 0.0))
        return fail(S2D_EINVAL, "mu must be finite and > 0");
    return S2D_OK;
}

int check_batch_inst(int mode, const s2d_instance &I, int32_t k) {
    const std::string where = "instance " + std::to_string(k) + ": ";
    int rc = check_args(S2D_OP_SLP, mode, &I.ves, &I.trg_ves, I.d, -1, 1, I.mu);
    if (rc != S2D_OK) return fail(rc, where + g_err);
    rc = check_args(S2D_OP_DLP, mode, &I.wall, &I.trg_wall, I.d, -1, 1, 1.0);
    if (rc != S2D_OK) return fail(rc, where + g_err);
    if (I.trg_ves.n != I.trg_wall.n) return fail(S2D_EINVAL, where + "trg_ves.n != trg_wall.n");
    if (I.trg_ves.n > 0 && (!I.u || !I.v)) return fail(S2D_EINVAL, where + "outputs u, v must not be NULL");
    if (I.ves.n_nodes > INT32_MAX / 4 || I.wall.n_nodes > INT32_MAX / 4 || I.trg_ves.n > INT32_MAX / 4)
        return fail(S2D_EINVAL, where + "instance too large for the batched path");
    return S2D_OK;
}

int current_device(int *dev) {
    if (hipGetDevice(dev) != hipSuccess) return fail(S2D_EHIP, "hipGetDevice failed");
    if (*dev < 0 || *dev >= kMaxDev || !g_dev[*dev].init)
        return fail(S2D_ENOINIT, "stokes2d_init() was not called for the current device");
    return S2D_OK;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(S2D_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int eval(int op, int mode, const s2d_curves *src, const s2d_targets *trg, double d, int32_t img_lo,
         int32_t img_hi, double mu, double *u, double *v, int accumulate, void *ws, size_t ws_bytes,
         void *stream, const double *tnx = nullptr, const double *tny = nullptr, bool may_profile = true) {
    using namespace s2d;
    int rc = check_args(op, mode, src, trg, d, img_lo, img_hi, mu);
    if (rc != S2D_OK) return rc;
    const int ncomp = (op == S2D_OP_SLP_PRESSURE || op == S2D_OP_DLP_PRESSURE) ? 1 : 2;
    if (trg->n > 0) {
        if (!u || (ncomp == 2 && !v)) return fail(S2D_EINVAL, "output arrays must not be NULL");
        if (op == S2D_OP_SLP_TRACTION && (!tnx || !tny)) return fail(S2D_EINVAL, "traction needs target normals");
    }
    int dev = 0;
    rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    if (trg->n == 0) return S2D_OK;
    Plan p = s2d::make_plan(op, mode, src, trg, g_dev[dev].cus);
    if (p.n_blocks > (int64_t)INT32_MAX)
        return fail(S2D_EINVAL, "too many target tiles x source splits for one launch (" +
                                    std::to_string(p.n_blocks) + " workgroups)");
    const bool img0 = img_lo <= 0 && img_hi >= 0;
    p.self = op == S2D_OP_SLP && trg->on_curve != nullptr && img0;
    if (p.total > 0) {
        if (!ws) return fail(S2D_EWORKSPACE, "workspace is NULL");
        if (ws_bytes < p.total)
            return fail(S2D_EWORKSPACE, "workspace too small: need " + std::to_string(p.total) + " bytes");
        if (((uintptr_t)ws & 255) != 0) return fail(S2D_EWORKSPACE, "workspace must be 256-byte aligned");
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (p.n_sb > 0) {
        e = launch_prep(p, src, ws, st);
        if (e != hipSuccess) return hip_fail(e, "prep launch");
    }
    if (p.self) {
        e = launch_kress(p, src, trg, ws, st);
        if (e != hipSuccess) return hip_fail(e, "kress launch");
    }
    PairArgs a{};
    a.rec = (char *)ws + p.off_rec;
    a.sbsum = (const double *)((char *)ws + p.off_sbsum);
    a.sub = (const SubInfo *)((char *)ws + p.off_sub);
    a.n_src = p.n_src;
    a.tx = trg->x;
    a.ty = trg->y;
    a.on_curve = img0 ? trg->on_curve : nullptr;
    a.on_node = img0 ? trg->on_node : nullptr;
    a.curve_off = src->curve_off;
    a.n_curves = src->n_curves;
    a.n_trg = p.n_trg;
    a.n_tiles = p.n_tiles;
    a.n_splits = p.n_splits;
    a.n_groups = p.n_groups;
    a.sb_per_split = p.sb_per_split;
    a.n_sb = p.n_sb;
    a.d = d;
    a.img_lo = img_lo;
    a.img_hi = img_hi;
    a.part = (double *)((char *)ws + p.off_part);
    a.tnx = tnx;
    a.tny = tny;
    a.rec64 = (char *)ws + p.off_rec64;
    FinalArgs f{};
    f.part = a.part;
    f.self = p.self ? (const double *)((char *)ws + p.off_self) : nullptr;
    f.n_parts = p.n_blocks > 0 ? p.n_groups : 0;
    f.n_trg = p.n_trg;
    f.n_src = p.n_src;
    switch (op) {
    case S2D_OP_SLP: f.pref = 1.0 / (4.0 * M_PI * mu); break;             // Eq. (S)
    case S2D_OP_DLP: f.pref = 1.0 / M_PI; break;                          // Eq. (D)
    case S2D_OP_SLP_PRESSURE: f.pref = 1.0 / (2.0 * M_PI); break;         // Eq. (Q)
    case S2D_OP_DLP_PRESSURE: f.pref = mu / M_PI; break;                  // Eq. (P)
    default: f.pref = -1.0 / M_PI; break;                                 // Eq. (K)
    }
    f.accumulate = accumulate ? 1 : 0;
    f.ncomp = ncomp;
    f.u = u;
    f.v = v;
    // on-curve targets with an empty or inconsistent curve come out NaN
    f.dlp_diag = op == S2D_OP_DLP && trg->on_curve != nullptr && img0;
    f.on_curve = trg->on_curve;
    f.on_node = trg->on_node;
    f.curve_off = src->curve_off;
    f.n_curves = src->n_curves;
    f.nx = src->nx;
    f.ny = src->ny;
    f.w = src->w;
    f.kappa = src->kappa;
    f.fx = src->fx;
    f.fy = src->fy;
    if (p.n_blocks > 0) {
        ProfEvent pe{op, nullptr, nullptr};
        if (g_prof_on && may_profile) {
            std::lock_guard<std::mutex> lk(g_mu);
            if (hipEventCreate(&pe.a) == hipSuccess && hipEventCreate(&pe.b) == hipSuccess) {
                hipEventRecord(pe.a, st);
            } else {
                pe.a = pe.b = nullptr;
            }
        }
        e = launch_pair(p, a, f, st);
        if (e != hipSuccess) return hip_fail(e, "pair launch");
        if (pe.a) {
            hipEventRecord(pe.b, st);
            std::lock_guard<std::mutex> lk(g_mu);
            g_prof.push_back(pe);
        }
    }
    // the pair kernel finishes the targets itself when it has one split group
    if (p.n_blocks > 0 && p.n_groups == 1) return S2D_OK;
    e = launch_final(p, f, st);
    if (e != hipSuccess) return hip_fail(e, "finalize launch");
    return S2D_OK;
}

}  // namespace

namespace s2d {
int set_error(int code, const std::string &msg) { return fail(code, msg); }
int device_ready(int *dev) { return current_device(dev); }
}  // namespace s2d

extern "C" {

S2D_API int stokes2d_init(int device) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(S2D_EHIP, "no HIP device");
    if (device < 0 || device >= n || device >= kMaxDev) return fail(S2D_EINVAL, "device index out of range");
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(S2D_ENOTSUP, std::string("libstokes2d is built for gfx950, device is ") + prop.gcnArchName);
    std::lock_guard<std::mutex> lk(g_mu);
    g_dev[device].cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (!g_dev[device].scratch) {
        // this device's address of the no-allocation entry point's scratch
        void *sp = nullptr;
        e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !sp) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_dev[device].scratch = sp;
    }
    if (!g_dev[device].side) {
        e = hipStreamCreateWithFlags(&g_dev[device].side, hipStreamNonBlocking);
        for (int k = 0; k < 3 && e == hipSuccess; ++k)
            e = hipEventCreateWithFlags(&g_dev[device].ev[k], hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "AUTO side stream");
    }
    g_dev[device].init = true;
    return S2D_OK;
}

S2D_API size_t stokes2d_workspace_size(int op, int mode, const s2d_curves *src, const s2d_targets *trg) {
    if (check_args(op, mode, src, trg, 1.0, 0, 0, 1.0) != S2D_OK) return 0;
    int dev = 0;
    int cus = 256;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDev && g_dev[dev].init) cus = g_dev[dev].cus;
    s2d::Plan p = s2d::make_plan(op, mode, src, trg, cus);
    return p.total > 0 ? p.total : 256;
}

S2D_API int stokes2d_slp_eval(int mode, const s2d_curves *src, const s2d_targets *trg, double d, int32_t img_lo,
                              int32_t img_hi, double mu, double *u, double *v, int accumulate, void *ws,
                              size_t ws_bytes, void *stream) {
    return eval(S2D_OP_SLP, mode, src, trg, d, img_lo, img_hi, mu, u, v, accumulate, ws, ws_bytes, stream);
}

S2D_API int stokes2d_slp_eval_noalloc(int mode, const s2d_curves *src, const s2d_targets *trg, double d,
                                      int32_t img_lo, int32_t img_hi, double mu, double *u, double *v,
                                      int accumulate, void *stream) {
    int rc = check_args(S2D_OP_SLP, mode, src, trg, d, img_lo, img_hi, mu);
    if (rc != S2D_OK) return rc;
    int dev = 0;
    rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    void *sp = g_dev[dev].scratch;
    if (!sp) return fail(S2D_ENOINIT, "stokes2d_init() did not set up the scratch memory of this device");
    const s2d::Plan p = s2d::make_plan(S2D_OP_SLP, mode, src, trg, g_dev[dev].cus);
    if (p.total > kScratchBytes)
        return fail(S2D_EWORKSPACE, "problem needs " + std::to_string(p.total) +
                                        " bytes of scratch; stokes2d_slp_eval_noalloc holds " +
                                        std::to_string(kScratchBytes) + " (use stokes2d_slp_eval with a workspace)");
    return eval(S2D_OP_SLP, mode, src, trg, d, img_lo, img_hi, mu, u, v, accumulate, sp, kScratchBytes, stream,
                nullptr, nullptr, false);
}

S2D_API int stokes2d_dlp_eval(int mode, const s2d_curves *src, const s2d_targets *trg, double d, int32_t img_lo,
                              int32_t img_hi, double *u, double *v, int accumulate, void *ws, size_t ws_bytes,
                              void *stream) {
    return eval(S2D_OP_DLP, mode, src, trg, d, img_lo, img_hi, 1.0, u, v, accumulate, ws, ws_bytes, stream);
}

S2D_API int stokes2d_slp_pressure_eval(int mode, const s2d_curves *src, const s2d_targets *trg, double d,
                                       int32_t img_lo, int32_t img_hi, double *p, int accumulate, void *ws,
                                       size_t ws_bytes, void *stream) {
    return eval(S2D_OP_SLP_PRESSURE, mode, src, trg, d, img_lo, img_hi, 1.0, p, nullptr, accumulate, ws, ws_bytes,
                stream);
}

S2D_API int stokes2d_dlp_pressure_eval(int mode, const s2d_curves *src, const s2d_targets *trg, double d,
                                       int32_t img_lo, int32_t img_hi, double mu, double *p, int accumulate,
                                       void *ws, size_t ws_bytes, void *stream) {
    return eval(S2D_OP_DLP_PRESSURE, mode, src, trg, d, img_lo, img_hi, mu, p, nullptr, accumulate, ws, ws_bytes,
                stream);
}

S2D_API int stokes2d_slp_traction_eval(int mode, const s2d_curves *src, const s2d_targets *trg,
                                       const double *trg_nx, const double *trg_ny, double d, int32_t img_lo,
                                       int32_t img_hi, double *tx, double *ty, int accumulate, void *ws,
                                       size_t ws_bytes, void *stream) {
    return eval(S2D_OP_SLP_TRACTION, mode, src, trg, d, img_lo, img_hi, 1.0, tx, ty, accumulate, ws, ws_bytes,
                stream, trg_nx, trg_ny);
}

// ---------------------------------------------------------------------------
// periodization system of one channel cell
// ---------------------------------------------------------------------------
namespace {

int check_cell(const s2d_cell *c, s2d::CellArgs *g) {
    if (!c) return fail(S2D_EINVAL, "cell must not be NULL");
    const s2d_curves &w = c->walls;
    if (w.n_nodes < 1 || w.n_nodes > 65536) return fail(S2D_EINVAL, "cell walls: n_nodes must be in 1..65536");
    if (!w.x || !w.y || !w.nx || !w.ny || !w.w || !w.kappa)
        return fail(S2D_EINVAL, "cell walls need x, y, nx, ny, w and kappa");
    if (c->n_side < 1 || c->n_side > 4096 || !c->side_y) return fail(S2D_EINVAL, "cell: n_side in 1..4096 and side_y set");
    if (c->n_proxy < 1 || c->n_proxy > 8192) return fail(S2D_EINVAL, "cell: n_proxy in 1..8192");
    if (!(std::isfinite(c->d) && c->d > 0.0)) return fail(S2D_EINVAL, "cell: d must be finite and > 0");
    if (!(std::isfinite(c->mu) && c->mu > 0.0)) return fail(S2D_EINVAL, "cell: mu must be finite and > 0");
    if (!(std::isfinite(c->proxy_r) && c->proxy_r > 0.0) || !std::isfinite(c->proxy_cx) ||
        !std::isfinite(c->proxy_cy) || !std::isfinite(c->x_left))
        return fail(S2D_EINVAL, "cell: proxy circle and x_left must be finite, proxy_r > 0");
    g->n_wall = w.n_nodes;
    g->x = w.x;
    g->y = w.y;
    g->nx = w.nx;
    g->ny = w.ny;
    g->w = w.w;
    g->kap = w.kappa;
    g->K = c->n_side;
    g->side_y = c->side_y;
    g->xl = c->x_left;
    g->M = c->n_proxy;
    g->cx = c->proxy_cx;
    g->cy = c->proxy_cy;
    g->R = c->proxy_r;
    g->d = c->d;
    g->mu = c->mu;
    // the blocked LU keeps every library operand within lu::kMaxSpan
    // elements; the blocks C (4K x 2N) and X (2N x 2M) go to the libraries
    // whole and must fit it too
    const int64_t n = 2 * w.n_nodes;
    if (4 * (int64_t)c->n_side * n > s2d::lu::kMaxSpan || 2 * (int64_t)c->n_proxy * n > s2d::lu::kMaxSpan)
        return fail(S2D_EINVAL, "cell: 4 n_side * 2 n_nodes and 2 n_proxy * 2 n_nodes must be at most 2^30");
    g->panel = s2d::lu::panel_width(n, s2d::lu::kMaxSpan, c->lu_panel);
    if (g->panel < 1)
        return fail(S2D_EINVAL, "cell: lu_panel must be 0 or in 1.." +
                                    std::to_string(s2d::lu::panel_width(n, s2d::lu::kMaxSpan, 0)));
    return S2D_OK;
}

int check_cell_ws(const s2d::CellArgs &g, void *ws, size_t ws_bytes) {
    const size_t need = s2d::cell_layout(g).total;
    if (!ws) return fail(S2D_EWORKSPACE, "workspace is NULL");
    if (ws_bytes < need) return fail(S2D_EWORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    if (((uintptr_t)ws & 255) != 0) return fail(S2D_EWORKSPACE, "workspace must be 256-byte aligned");
    return S2D_OK;
}

}  // namespace

S2D_API size_t stokes2d_cell_workspace_size(const s2d_cell *cell) {
    s2d::CellArgs g{};
    if (check_cell(cell, &g) != S2D_OK) return 0;
    return s2d::cell_layout(g).total;
}

S2D_API int stokes2d_cell_assemble(const s2d_cell *cell, double *A, double *B, double *C, double *Q, void *stream) {
    s2d::CellArgs g{};
    int rc = check_cell(cell, &g);
    if (rc != S2D_OK) return rc;
    int dev = 0;
    rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    const hipError_t e = s2d::cell_fill(g, A, B, C, Q, (hipStream_t)stream);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "cell assemble");
}

S2D_API int stokes2d_cell_factor(const s2d_cell *cell, double rcond, void *ws, size_t ws_bytes, void *stream) {
    s2d::CellArgs g{};
    int rc = check_cell(cell, &g);
    if (rc != S2D_OK) return rc;
    if (!(std::isfinite(rcond) && rcond >= 0.0 && rcond < 1.0)) return fail(S2D_EINVAL, "rcond must be in [0, 1)");
    rc = check_cell_ws(g, ws, ws_bytes);
    if (rc != S2D_OK) return rc;
    int dev = 0;
    rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    const std::string err = s2d::cell_factor(g, rcond, ws, (hipStream_t)stream);
    return err.empty() ? S2D_OK : fail(S2D_EHIP, err);
}

S2D_API int stokes2d_cell_solve(const s2d_cell *cell, const double *v, const double *gv, double *tau, double *c,
                                void *ws, size_t ws_bytes, void *stream) {
    s2d::CellArgs g{};
    int rc = check_cell(cell, &g);
    if (rc != S2D_OK) return rc;
    if (!v || !gv || !tau || !c) return fail(S2D_EINVAL, "v, g, tau and c must not be NULL");
    rc = check_cell_ws(g, ws, ws_bytes);
    if (rc != S2D_OK) return rc;
    int dev = 0;
    rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    const std::string err = s2d::cell_solve(g, v, gv, tau, c, ws, (hipStream_t)stream);
    return err.empty() ? S2D_OK : fail(S2D_EHIP, err);
}

// ---------------------------------------------------------------------------
// the channel's response to vesicles (Algorithm 1, steps 3-5)
// ---------------------------------------------------------------------------
namespace {

struct RespLayout {
    size_t v, g, tau, c, vw, side, s, tauxy, cxy, prox, poff, geo, eval, eval_bytes, total;
};

RespLayout resp_layout(const s2d_cell *cell, int64_t n, int32_t nc, int mode) {
    const size_t d = sizeof(double);
    const int64_t nw = cell->walls.n_nodes;
    const size_t K = (size_t)cell->n_side, M = (size_t)cell->n_proxy;
    RespLayout L{};
    size_t o = 0;
    L.v = o;
    o += align256(2 * nw * d);
    L.g = o;
    o += align256(4 * K * d);
    L.tau = o;
    o += align256(2 * nw * d);
    L.c = o;
    o += align256(2 * M * d);
    L.vw = o;
    o += align256(2 * nw * d);
    L.side = o;
    o += align256(4 * K * d);
    L.s = o;
    o += align256(8 * K * d);
    L.tauxy = o;
    o += align256(2 * nw * d);
    L.cxy = o;
    o += align256(2 * M * d);
    L.prox = o;
    o += align256(3 * M * d);
    L.poff = o;
    o += align256(2 * sizeof(int32_t));
    L.geo = o;
    o += align256(3 * (size_t)n * d);
    // the evaluations run in turn on one stream and share one workspace;
    // the shapes below carry placeholders for the arrays (only sizes are read)
    const double *a = (const double *)1;
    const int32_t *ia = (const int32_t *)1;
    const s2d_curves ves{n, nc, ia, a, a, a, a, a, nullptr, a, a};
    const s2d_curves wal{nw, cell->walls.n_curves, ia, a, a, a, a, a, nullptr, a, a};
    const s2d_curves prx{(int64_t)M, 1, ia, a, a, a, a, a, nullptr, a, a};
    const s2d_targets tw{nw, a, a, nullptr, nullptr}, ts{(int64_t)K, a, a, nullptr, nullptr},
        tv{n, a, a, nullptr, nullptr};
    size_t e = 256;
    e = std::max(e, stokes2d_workspace_size(S2D_OP_SLP, mode, &ves, &tw));
    e = std::max(e, stokes2d_workspace_size(S2D_OP_SLP, mode, &ves, &ts));
    e = std::max(e, stokes2d_workspace_size(S2D_OP_SLP_TRACTION, mode, &ves, &ts));
    e = std::max(e, stokes2d_workspace_size(S2D_OP_DLP, mode, &wal, &tv));
    e = std::max(e, stokes2d_workspace_size(S2D_OP_SLP, mode, &prx, &tv));
    L.eval = o;
    L.eval_bytes = e;
    o += align256(e);
    L.total = o;
    return L;
}

}  // namespace

S2D_API size_t ves_response_workspace_size(const s2d_cell *cell, int64_t n_nodes, int32_t n_curves, int mode) {
    s2d::CellArgs g{};
    if (check_cell(cell, &g) != S2D_OK || n_nodes < 0 || n_curves < 0 || (mode != S2D_FP64 && mode != S2D_FP32C))
        return 0;
    return resp_layout(cell, n_nodes, n_curves, mode).total;
}

S2D_API int ves_channel_response(const s2d_cell *cell, void *cell_ws, size_t cell_ws_bytes, int64_t n_nodes,
                                 int32_t n_curves, const int32_t *curve_off, const double *x, const double *y,
                                 const double *fx, const double *fy, double p_drive, int mode, double *u_resp_x,
                                 double *u_resp_y, void *ws, size_t ws_bytes, void *stream) {
    using namespace s2d;
    CellArgs g{};
    int rc = check_cell(cell, &g);
    if (rc != S2D_OK) return rc;
    rc = check_cell_ws(g, cell_ws, cell_ws_bytes);
    if (rc != S2D_OK) return rc;
    if (mode != S2D_FP64 && mode != S2D_FP32C) return fail(S2D_EINVAL, "mode must be an s2d_mode");
    if (n_nodes < 0 || n_curves < 0) return fail(S2D_EINVAL, "vesicle sizes out of range");
    if (n_nodes > 0 && (n_curves < 1 || !curve_off || !x || !y || !fx || !fy || !u_resp_x || !u_resp_y))
        return fail(S2D_EINVAL, "curve_off, x, y, fx, fy and the outputs must not be NULL");
    if (!std::isfinite(p_drive)) return fail(S2D_EINVAL, "p_drive must be finite");
    int dev = 0;
    rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    const RespLayout L = resp_layout(cell, n_nodes, n_curves, mode);
    if (!ws || ws_bytes < L.total)
        return fail(S2D_EWORKSPACE, "response workspace too small: need " + std::to_string(L.total) + " bytes");
    if (((uintptr_t)ws & 255) != 0) return fail(S2D_EWORKSPACE, "workspace must be 256-byte aligned");
    if (n_nodes == 0) return S2D_OK;
    char *b = (char *)ws;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = n_nodes, nw = cell->walls.n_nodes;
    const int K = cell->n_side, M = cell->n_proxy;
    const double d = cell->d, mu = cell->mu;
    void *ew = b + L.eval;
    const size_t eb = L.eval_bytes;
    // the vesicles as single-layer sources of f
    double *geo = (double *)(b + L.geo);
    rc = ves_geometry(n, n_curves, curve_off, x, y, nullptr, geo, geo + n, geo + 2 * n, nullptr, nullptr, stream);
    if (rc != S2D_OK) return rc;
    const s2d_curves ves{n, n_curves, curve_off, x, y, geo + n, geo + 2 * n, geo, nullptr, fx, fy};
    // step 3: -S^near f on the walls; S and T of the single far images at R and L
    double *vw = (double *)(b + L.vw);
    const s2d_targets tw{nw, cell->walls.x, cell->walls.y, nullptr, nullptr};
    rc = eval(S2D_OP_SLP, mode, &ves, &tw, d, -1, 1, mu, vw, vw + nw, 0, ew, eb, stream);
    if (rc != S2D_OK) return rc;
    double *side = (double *)(b + L.side), *sxl = side, *sxr = side + K, *mx = side + 2 * K, *my = side + 3 * K;
    hipError_t e = resp_side_launch(K, cell->side_y, cell->x_left, d, sxl, sxr, mx, my, st);
    if (e != hipSuccess) return hip_fail(e, "response side targets");
    double *s = (double *)(b + L.s);
    const s2d_targets tR{K, sxr, cell->side_y, nullptr, nullptr}, tL{K, sxl, cell->side_y, nullptr, nullptr};
    if ((rc = eval(S2D_OP_SLP, mode, &ves, &tR, d, -1, -1, mu, s, s + K, 0, ew, eb, stream)) != S2D_OK) return rc;
    if ((rc = eval(S2D_OP_SLP, mode, &ves, &tL, d, 1, 1, mu, s + 2 * K, s + 3 * K, 0, ew, eb, stream)) != S2D_OK)
        return rc;
    if ((rc = eval(S2D_OP_SLP_TRACTION, mode, &ves, &tR, d, -1, -1, mu, s + 4 * K, s + 5 * K, 0, ew, eb, stream,
                   mx, my)) != S2D_OK)
        return rc;
    if ((rc = eval(S2D_OP_SLP_TRACTION, mode, &ves, &tL, d, 1, 1, mu, s + 6 * K, s + 7 * K, 0, ew, eb, stream, mx,
                   my)) != S2D_OK)
        return rc;
    double *v = (double *)(b + L.v), *gv = (double *)(b + L.g);
    e = resp_pack_launch(nw, vw, vw + nw, K, s, p_drive, v, gv, st);
    if (e != hipSuccess) return hip_fail(e, "response data");
    // step 4: the cell system
    double *tau = (double *)(b + L.tau), *c = (double *)(b + L.c);
    const std::string err = cell_solve(g, v, gv, tau, c, cell_ws, st);
    if (!err.empty()) return fail(S2D_EHIP, err);
    // step 5: D^near tau + sum c_m phi_m at the vesicle nodes
    double *tx = (double *)(b + L.tauxy), *ty = tx + nw, *cx = (double *)(b + L.cxy), *cy = cx + M;
    double *px = (double *)(b + L.prox), *py = px + M, *pw = px + 2 * M;
    int32_t *poff = (int32_t *)(b + L.poff);
    e = resp_unpack_launch(nw, tau, tx, ty, M, c, cell->proxy_cx, cell->proxy_cy, cell->proxy_r, cx, cy, px, py, pw,
                           poff, st);
    if (e != hipSuccess) return hip_fail(e, "response densities");
    s2d_curves wal = cell->walls;
    wal.fx = tx;
    wal.fy = ty;
    const s2d_targets tv{n, x, y, nullptr, nullptr};
    if ((rc = eval(S2D_OP_DLP, mode, &wal, &tv, d, -1, 1, 1.0, u_resp_x, u_resp_y, 0, ew, eb, stream)) != S2D_OK)
        return rc;
    const s2d_curves prx{(int64_t)M, 1, poff, px, py, nullptr, nullptr, pw, nullptr, cx, cy};
    return eval(S2D_OP_SLP, mode, &prx, &tv, d, 0, 0, mu, u_resp_x, u_resp_y, 1, ew, eb, stream);
}

S2D_API int stokes2d_valu_probe(int form, int32_t blocks, int32_t iters, float *sink, void *stream) {
    if (form < 0 || form > 2) return fail(S2D_EINVAL, "form must be 0, 1 or 2");
    if (blocks < 1 || blocks > (1 << 20) || iters < 1) return fail(S2D_EINVAL, "blocks in 1..2^20, iters >= 1");
    if (!sink) return fail(S2D_EINVAL, "sink must not be NULL");
    int dev = 0;
    int rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    const hipError_t e = s2d::valu_probe_launch(form, blocks, iters, sink, (hipStream_t)stream);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "VALU probe launch");
}

S2D_API int stokes2d_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof_on = on != 0;
    return S2D_OK;
}

S2D_API int stokes2d_profile_read(int op, double *total_ms, int64_t *launches) {
    if (!total_ms || !launches) return fail(S2D_EINVAL, "total_ms and launches must not be NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    double tot = 0.0;
    int64_t n = 0;
    std::vector<ProfEvent> keep;
    for (auto &pe : g_prof) {
        if (pe.op != op) {
            keep.push_back(pe);
            continue;
        }
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(pe.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, pe.a, pe.b);
        if (e != hipSuccess) return hip_fail(e, "profile event");
        tot += ms;
        ++n;
        hipEventDestroy(pe.a);
        hipEventDestroy(pe.b);
    }
    g_prof.swap(keep);
    *total_ms = tot;
    *launches = n;
    return S2D_OK;
}

S2D_API size_t stokes2d_batch_workspace_size(int mode, int32_t n_inst, const s2d_instance *inst) {
    if (n_inst < 0 || (n_inst > 0 && !inst)) return 0;
    for (int32_t k = 0; k < n_inst; ++k)
        if (check_batch_inst(mode, inst[k], k) != S2D_OK) return 0;
    return std::max<size_t>(s2d::batch_workspace_size(mode, n_inst, inst), 256);
}

S2D_API int stokes2d_batch_eval(int mode, int32_t n_inst, const s2d_instance *inst, void *ws, size_t ws_bytes,
                                void *stream) {
    if (n_inst < 0) return fail(S2D_EINVAL, "n_inst < 0");
    if (n_inst > 0 && !inst) return fail(S2D_EINVAL, "inst must not be NULL");
    for (int32_t k = 0; k < n_inst; ++k) {
        const int rc = check_batch_inst(mode, inst[k], k);
        if (rc != S2D_OK) return rc;
    }
    int dev = 0;
    int rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    if (n_inst == 0) return S2D_OK;
    if (!ws) return fail(S2D_EWORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(S2D_EWORKSPACE, "workspace must be 256-byte aligned");
    std::string err;
    rc = s2d::batch_eval(dev, g_dev[dev].cus, mode, n_inst, inst, ws, ws_bytes, (hipStream_t)stream, err);
    if (rc != S2D_OK) return fail(rc, err);
    return S2D_OK;
}

S2D_API int stokes2d_batch_release(void) { return s2d::batch_release(); }

S2D_API int stokes2d_batch_tuned(int mode, int32_t n_inst, const s2d_instance *inst, int32_t *tpt, int32_t *sbps,
                                 int32_t *wpc) {
    if (!tpt || !sbps || !wpc) return fail(S2D_EINVAL, "tpt, sbps and wpc must not be NULL");
    if (mode != S2D_FP64 && mode != S2D_FP32C) return fail(S2D_EINVAL, "mode must be S2D_FP64 or S2D_FP32C");
    if (n_inst < 0) return fail(S2D_EINVAL, "n_inst < 0");
    if (n_inst > 0 && !inst) return fail(S2D_EINVAL, "inst must not be NULL");
    for (int32_t k = 0; k < n_inst; ++k) {
        const int rc = check_batch_inst(mode, inst[k], k);
        if (rc != S2D_OK) return rc;
    }
    int a = 0, b = 0, c = 0;
    const int tuned = s2d::batch_tuned(mode, n_inst, inst, &a, &b, &c);
    *tpt = a;
    *sbps = b;
    *wpc = c;
    return tuned;
}

// ---------------------------------------------------------------------------
// near-field correction
// ---------------------------------------------------------------------------
namespace {

static_assert(S2D_NEAR_NBINS == s2d::kNearMaxBins && S2D_NEAR_SBINS == s2d::kNearSBins &&
                  S2D_NEAR_KBINS == s2d::kNearKBins && S2D_NEAR_CELL == s2d::kNearCell,
              "the public bin counts match the kernels'");
static_assert(S2D_NEAR_NFEAT == s2d::kNearFeat && S2D_NEAR_NFRAME == s2d::kNearFrame &&
                  S2D_NEAR_NDERIV == 2 * s2d::kNearDeriv && S2D_NEAR_TSTRIDE == s2d::kNearTStride &&
                  S2D_NEAR_NOUT == s2d::kNearOut && S2D_MLP_NPARAM == s2d::MlpOffsets::total,
              "the public near-field sizes match the kernels'");

struct NearLayout {
    size_t up, dtab, dscr, X, nrec, flag, list, count, llist, lcount, total;
};

NearLayout near_layout(int method, const s2d_curves *c, const s2d_targets *t, int P) {
    NearLayout L{};
    size_t off = 0;
    L.up = off;
    if (method != S2D_NEAR_MLP) off = align256(off + 4 * ((size_t)P + 1) * (size_t)c->n_nodes * sizeof(double));
    L.dtab = L.dscr = L.X = off;
    if (method != S2D_NEAR_UPSAMPLE) {
        off = align256(off + (size_t)c->n_nodes * 2 * s2d::kNearDeriv * sizeof(double));
        L.dscr = off;
        off = align256(off + s2d::near_derivs_scratch(c));
        L.X = off;
        off = align256(off + (size_t)t->n * s2d::kNearFeat * sizeof(float));
        L.nrec = off;
        off = align256(off + (size_t)t->n * s2d::kNetRec * sizeof(float));
        // AUTO: per-target decisions, the fallback targets' list and the
        // compaction's per-workgroup counts
        L.flag = off;
        off = align256(off + (size_t)t->n * sizeof(int32_t));
        L.list = off;
        off = align256(off + (size_t)t->n * sizeof(int32_t));
        L.count = off;
        off = align256(off + ((size_t)(t->n + 255) / 256 + 1) * sizeof(int32_t));
        // the learned targets' list and its compaction counts
        L.llist = off;
        off = align256(off + (size_t)t->n * sizeof(int32_t));
        L.lcount = off;
        off = align256(off + ((size_t)(t->n + 255) / 256 + 1) * sizeof(int32_t));
    } else {
        L.nrec = L.flag = L.list = L.count = L.llist = L.lcount = off;
    }
    L.total = std::max<size_t>(off, 256);
    return L;
}

int check_near(int method, const s2d_curves *c, const s2d_targets *t, const int32_t *tc, int P, double mu) {
    if (method < S2D_NEAR_UPSAMPLE || method > S2D_NEAR_AUTO) return fail(S2D_EINVAL, "unknown near method");
    if (!c || !t) return fail(S2D_EINVAL, "ves and trg must not be NULL");
    if (c->n_nodes < 0 || c->n_nodes > INT32_MAX / 32 || c->n_curves < 0 || t->n < 0 || t->n > INT32_MAX)
        return fail(S2D_EINVAL, "sizes out of range");
    if (c->n_nodes > 0 && (!c->x || !c->y || !c->nx || !c->ny || !c->w || !c->kappa || !c->fx || !c->fy ||
                           !c->curve_off))
        return fail(S2D_EINVAL, "ves arrays (x, y, nx, ny, w, kappa, fx, fy, curve_off) must not be NULL");
    if (t->n > 0 && (!t->x || !t->y || !tc)) return fail(S2D_EINVAL, "trg x, y and trg_curve must not be NULL");
    if (P < 1 || P > 32) return fail(S2D_EINVAL, "upsample factor must be in 1..32");
    if (!(std::isfinite(mu) && mu > 0.0)) return fail(S2D_EINVAL, "mu must be finite and > 0");
    return S2D_OK;
}

int check_curves_derivs(const s2d_curves *c) {
    if (!c || c->n_nodes < 0 || c->n_curves < 0 || c->n_nodes > INT32_MAX / 16) return fail(S2D_EINVAL, "bad curves");
    if (c->n_nodes > 0 && (!c->fx || !c->fy || !c->curve_off))
        return fail(S2D_EINVAL, "curves fx, fy and curve_off must not be NULL");
    return S2D_OK;
}

bool valid_op(int op) { return op == S2D_OP_SLP || op == S2D_OP_DLP; }

}  // namespace

S2D_API size_t near_workspace_size(int method, const s2d_curves *ves, const s2d_targets *trg, int32_t upsample) {
    if (!ves || !trg || upsample < 1 || upsample > 32 || method < 0 || method > 2) return 0;
    return near_layout(method, ves, trg, upsample).total;
}

S2D_API int near_correct_eval(int method, const s2d_curves *ves, const s2d_targets *trg, const int32_t *trg_curve,
                              int32_t upsample, const void *mlp, double threshold, const double *curve_tol,
                              double mu, double *du, double *dv, int32_t *used_fallback, void *ws, size_t ws_bytes,
                              void *stream) {
    int rc = check_near(method, ves, trg, trg_curve, upsample, mu);
    if (rc != S2D_OK) return rc;
    if (method != S2D_NEAR_UPSAMPLE && !mlp) return fail(S2D_EINVAL, "MLP methods need the packed network");
    if (method == S2D_NEAR_AUTO && !curve_tol && !(threshold >= 0.0))
        return fail(S2D_EINVAL, "threshold must be >= 0");
    int dev = 0;
    rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    if (trg->n == 0) return S2D_OK;
    if (!du || !dv) return fail(S2D_EINVAL, "outputs du, dv must not be NULL");
    const NearLayout L = near_layout(method, ves, trg, upsample);
    if (!ws || ws_bytes < L.total)
        return fail(S2D_EWORKSPACE, "near workspace too small: need " + std::to_string(L.total) + " bytes");
    if (((uintptr_t)ws & 255) != 0) return fail(S2D_EWORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    double *up = (double *)(w + L.up);
    hipError_t e = hipSuccess;
    if (method == S2D_NEAR_UPSAMPLE) {
        e = s2d::near_launch_upsample(ves, upsample, up, st);
        if (e != hipSuccess) return hip_fail(e, "near upsample launch");
        e = s2d::near_launch_quad(ves, trg, trg_curve, nullptr, nullptr, upsample, up, mu, du, dv, st);
        if (e != hipSuccess) return hip_fail(e, "near quadrature launch");
        return S2D_OK;
    }
    double *dtab = (double *)(w + L.dtab);
    float *X = (float *)(w + L.X), *nrec = (float *)(w + L.nrec);
    const bool autom = method == S2D_NEAR_AUTO;
    // the per-target decisions: the caller's array or the workspace
    int32_t *flag = used_fallback ? used_fallback : (int32_t *)(w + L.flag);
    const s2d::DecideArgs da{(const s2d::NearBlob *)mlp, mu, threshold, curve_tol, ves->n_curves, autom ? 1 : 0,
                             du, dv, flag};
    const int64_t nb = (trg->n + 255) / 256;
    int32_t *lcnt = (int32_t *)(w + L.lcount), *llist = (int32_t *)(w + L.llist);
    int32_t *fcnt = (int32_t *)(w + L.count), *flist = (int32_t *)(w + L.list);
    // the nearest nodes, from the search to the head kernel, in the fallback
    // list's area (the compaction writes it only after the head kernel)
    int32_t *kstar = flist;
    if (!autom) {
        // the learned route: derivatives, then the search, features and head
        // in one launch, then the network
        e = s2d::near_launch_derivs(ves, dtab, w + L.dscr, st);
        if (e != hipSuccess) return hip_fail(e, "near derivative launch");
        e = s2d::near_launch_head(ves, trg, trg_curve, dtab, nullptr, da, nrec, st, X);
        if (e != hipSuccess) return hip_fail(e, "near features launch");
        e = s2d::near_launch_infer(S2D_OP_SLP, trg->n, X, nrec, (const s2d::NearBlob *)mlp, nullptr, nullptr, du,
                                   dv, st);
        return e == hipSuccess ? S2D_OK : hip_fail(e, "near MLP launch");
    }
    // AUTO outside stream capture: the derivatives and the upsampling on the
    // device's second stream, beside the nearest-node search and the head
    // kernel (fork / join by events); under capture every kernel stays on
    // the caller's stream in the same order, with the same results
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    e = hipStreamIsCapturing(st, &cap);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    DevState &D = g_dev[dev];
    const bool two = cap == hipStreamCaptureStatusNone && D.side;
    std::unique_lock<std::mutex> lk(D.side_mu, std::defer_lock);
    hipStream_t sd = st;
    if (two) {
        lk.lock();
        sd = D.side;
        e = hipEventRecord(D.ev[0], st);
        if (e == hipSuccess) e = hipStreamWaitEvent(sd, D.ev[0], 0);
        if (e != hipSuccess) return hip_fail(e, "near fork");
    }
    // the derivatives (the longer of the two chains) first, then the search
    e = s2d::near_launch_derivs(ves, dtab, w + L.dscr, sd);
    if (e != hipSuccess) return hip_fail(e, "near derivative launch");
    if (two && (e = hipEventRecord(D.ev[1], sd)) != hipSuccess) return hip_fail(e, "near derivative event");
    e = s2d::near_launch_scan(ves, trg, trg_curve, X, kstar, st);
    if (e != hipSuccess) return hip_fail(e, "near nearest-node launch");
    e = s2d::near_launch_upsample(ves, upsample, up, sd);
    if (e != hipSuccess) return hip_fail(e, "near upsample launch");
    if (two && (e = hipEventRecord(D.ev[2], sd)) != hipSuccess) return hip_fail(e, "near upsample event");
    if (two && (e = hipStreamWaitEvent(st, D.ev[1], 0)) != hipSuccess) return hip_fail(e, "near derivative wait");
    e = s2d::near_launch_head(ves, trg, trg_curve, dtab, kstar, da, nrec, st);
    if (e != hipSuccess) return hip_fail(e, "near head launch");
    // the learned and the fallback targets, each compacted in order (the
    // quadrature's cost follows the fallback targets' number rather than the
    // waves that hold one); the network, then the quadrature once the
    // upsampling is done (the network's persistent workgroups hold every
    // SIMD's registers, so the two would not overlap anyway)
    e = s2d::near_launch_compact(trg->n, flag, 0, lcnt, llist, st, 1, fcnt, flist);
    if (e != hipSuccess) return hip_fail(e, "near compaction launch");
    e = s2d::near_launch_infer(S2D_OP_SLP, trg->n, X, nrec, (const s2d::NearBlob *)mlp, llist, lcnt + nb, du, dv,
                               st);
    if (e != hipSuccess) return hip_fail(e, "near MLP launch");
    if (two && (e = hipStreamWaitEvent(st, D.ev[2], 0)) != hipSuccess) return hip_fail(e, "near upsample wait");
    e = s2d::near_launch_quad(ves, trg, trg_curve, flist, fcnt + nb, upsample, up, mu, du, dv, st);
    if (e != hipSuccess) return hip_fail(e, "near fallback launch");
    return S2D_OK;
}

S2D_API int near_upsampled_slp(const s2d_curves *ves, const s2d_targets *trg, const int32_t *trg_curve,
                               int32_t upsample, double mu, double *u_up, double *v_up, double *u_trap,
                               double *v_trap, void *ws, size_t ws_bytes, void *stream) {
    int rc = check_near(S2D_NEAR_UPSAMPLE, ves, trg, trg_curve, upsample, mu);
    if (rc != S2D_OK) return rc;
    int dev = 0;
    rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    if (trg->n == 0) return S2D_OK;
    if (!u_up || !v_up || !u_trap || !v_trap) return fail(S2D_EINVAL, "outputs must not be NULL");
    const NearLayout L = near_layout(S2D_NEAR_UPSAMPLE, ves, trg, upsample);
    const size_t need = L.total + align256(2 * (size_t)trg->n * sizeof(double));
    if (!ws || ws_bytes < need)
        return fail(S2D_EWORKSPACE, "near workspace too small: need " + std::to_string(need) + " bytes");
    if (((uintptr_t)ws & 255) != 0) return fail(S2D_EWORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    double *up = (double *)((char *)ws + L.up);
    double *d = (double *)((char *)ws + L.total);
    hipError_t e = s2d::near_launch_upsample(ves, upsample, up, st);
    if (e != hipSuccess) return hip_fail(e, "near upsample launch");
    e = s2d::near_launch_quad(ves, trg, trg_curve, nullptr, nullptr, upsample, up, mu, d, d + trg->n, st, u_up, v_up,
                              u_trap, v_trap);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "near quadrature launch");
}

S2D_API size_t near_upsampled_slp_workspace_size(const s2d_curves *ves, const s2d_targets *trg, int32_t upsample) {
    if (!ves || !trg || upsample < 1 || upsample > 32) return 0;
    return near_layout(S2D_NEAR_UPSAMPLE, ves, trg, upsample).total + align256(2 * (size_t)trg->n * sizeof(double));
}

S2D_API size_t near_derivs_workspace_size(const s2d_curves *curves) {
    if (!curves || curves->n_nodes < 0 || curves->n_nodes > INT32_MAX / 16) return 0;
    return std::max<size_t>(align256(s2d::near_derivs_scratch(curves)), 256);
}

S2D_API int near_derivs_eval(const s2d_curves *curves, double *dtab, void *ws, size_t ws_bytes, void *stream) {
    int rc = check_curves_derivs(curves);
    if (rc != S2D_OK) return rc;
    if (curves->n_nodes > 0 && !dtab) return fail(S2D_EINVAL, "dtab must not be NULL");
    const size_t need = s2d::near_derivs_scratch(curves);
    if (!ws || ws_bytes < need)
        return fail(S2D_EWORKSPACE, "derivative workspace too small: need " + std::to_string(need) + " bytes");
    if (((uintptr_t)ws & 255) != 0) return fail(S2D_EWORKSPACE, "workspace must be 256-byte aligned");
    int dev = 0;
    rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    const hipError_t e = s2d::near_launch_derivs(curves, dtab, ws, (hipStream_t)stream);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "near derivative launch");
}

S2D_API int near_features_eval(const s2d_curves *ves, const s2d_targets *trg, const int32_t *trg_curve,
                               const double *dtab, float *X, double *frame, void *stream) {
    int rc = check_near(S2D_NEAR_MLP, ves, trg, trg_curve, 1, 1.0);
    if (rc != S2D_OK) return rc;
    int dev = 0;
    rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    if (trg->n == 0) return S2D_OK;
    if (!X || !frame || (ves->n_nodes > 0 && !dtab)) return fail(S2D_EINVAL, "dtab, X and frame must not be NULL");
    hipError_t e = s2d::near_launch_features(ves, trg, trg_curve, dtab, X, frame, (hipStream_t)stream);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "near features launch");
}

S2D_API int near_train_targets(int op, int64_t n, const double *frame, const double *du, const double *dv,
                               const int32_t *trg_curve, int32_t n_curves, const double *u_ref,
                               const double *v_ref, double mu, int32_t upsample, float weight_gain,
                               float *curve_scale, float *T, void *stream) {
    if (!valid_op(op)) return fail(S2D_EINVAL, "op must be S2D_OP_SLP or S2D_OP_DLP");
    if (n < 0 || n > INT32_MAX || n_curves < 0) return fail(S2D_EINVAL, "sizes out of range");
    if (n > 0 && (!frame || !du || !dv || !trg_curve || !u_ref || !v_ref || !T))
        return fail(S2D_EINVAL, "arrays must not be NULL");
    if (n_curves > 0 && !curve_scale) return fail(S2D_EINVAL, "curve_scale must not be NULL");
    if (!(std::isfinite(mu) && mu > 0.0)) return fail(S2D_EINVAL, "mu must be finite and > 0");
    if (upsample < 1 || upsample > 32) return fail(S2D_EINVAL, "upsample factor must be in 1..32");
    if (!(weight_gain > 0.f) || !std::isfinite(weight_gain)) return fail(S2D_EINVAL, "weight_gain must be > 0");
    int dev = 0;
    int rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    const hipError_t e =
        s2d::near_launch_train_targets(op, n, frame, du, dv, trg_curve, n_curves, u_ref, v_ref, mu, upsample,
                                       weight_gain, (uint32_t *)curve_scale, T, (hipStream_t)stream);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "training targets launch");
}

S2D_API size_t near_mlp_train_workspace_size(int32_t batch) {
    if (batch <= 0) return 0;
    return align256((size_t)batch * s2d::kActStride * sizeof(float)) +
           align256((size_t)batch * s2d::kNearOut * sizeof(float)) + align256((size_t)batch * sizeof(float));
}

S2D_API int near_mlp_train_step(int32_t batch, const int32_t *idx, const float *X, const float *T, float *params,
                                float *adam_m, float *adam_v, int32_t step, float lr, float *grad, float *loss,
                                void *ws, size_t ws_bytes, void *stream) {
    if (batch <= 0 || batch > (1 << 22)) return fail(S2D_EINVAL, "batch must be in 1..4194304");
    if (!X || !T || !params || !grad) return fail(S2D_EINVAL, "X, T, params, grad must not be NULL");
    if (step > 0 && (!adam_m || !adam_v)) return fail(S2D_EINVAL, "Adam state must not be NULL when step > 0");
    if (step < 0) return fail(S2D_EINVAL, "step < 0");
    if (!(std::isfinite(lr) && lr >= 0.f)) return fail(S2D_EINVAL, "lr must be finite and >= 0");
    int dev = 0;
    int rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    const size_t need = near_mlp_train_workspace_size(batch);
    if (!ws || ws_bytes < need) return fail(S2D_EWORKSPACE, "train workspace too small: need " + std::to_string(need));
    if (((uintptr_t)ws & 255) != 0) return fail(S2D_EWORKSPACE, "workspace must be 256-byte aligned");
    char *w = (char *)ws;
    float *act = (float *)w;
    float *dY = (float *)(w + align256((size_t)batch * s2d::kActStride * sizeof(float)));
    float *lossv = (float *)((char *)dY + align256((size_t)batch * s2d::kNearOut * sizeof(float)));
    hipError_t e = s2d::near_launch_train_step(batch, idx, X, T, params, adam_m, adam_v, step, lr, grad, act, dY,
                                               lossv, loss, step > 0 ? 1 : 0, (hipStream_t)stream);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "train step launch");
}

S2D_API int near_mlp_forward(int64_t n, const float *X, const float *params, float *Y, void *stream) {
    if (n < 0) return fail(S2D_EINVAL, "n < 0");
    if (n > 0 && (!X || !params || !Y)) return fail(S2D_EINVAL, "arrays must not be NULL");
    int dev = 0;
    int rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    hipError_t e = s2d::near_launch_fwd(n, X, params, Y, (hipStream_t)stream);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "MLP forward launch");
}

S2D_API int near_feature_stats(int64_t n, const float *X, float *params, void *stream) {
    if (n < 0) return fail(S2D_EINVAL, "n < 0");
    if (!params || (n > 0 && !X)) return fail(S2D_EINVAL, "X and params must not be NULL");
    int dev = 0;
    int rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    hipError_t e = s2d::near_launch_feature_stats(n, X, params, (hipStream_t)stream);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "feature statistics launch");
}

S2D_API int near_calibrate(int op, int64_t n, const double *frame, const double *du_pred, const double *dv_pred,
                           const double *du, const double *dv, double mu, int32_t n_bins, float bin_lo, float bin_w,
                           float b_min, float margin, float count_margin, float *bound, float *bound_zero,
                           int32_t *count, void *stream) {
    if (!valid_op(op)) return fail(S2D_EINVAL, "op must be S2D_OP_SLP or S2D_OP_DLP");
    if (n < 0 || n > INT32_MAX) return fail(S2D_EINVAL, "n out of range");
    if (n > 0 && (!frame || !du_pred || !dv_pred || !du || !dv)) return fail(S2D_EINVAL, "arrays must not be NULL");
    if (n_bins < 1 || n_bins > s2d::kNearMaxBins) return fail(S2D_EINVAL, "n_bins must be in 1..64");
    if (!bound || !bound_zero || !count) return fail(S2D_EINVAL, "bound, bound_zero and count must not be NULL");
    if (!(bin_w > 0.f) || !std::isfinite(bin_lo) || !std::isfinite(bin_w))
        return fail(S2D_EINVAL, "bins: bin_w must be finite and > 0, bin_lo finite");
    if (!(b_min >= 0.f) || !(margin >= 1.f) || !std::isfinite(margin) || !(count_margin >= 0.f) ||
        !std::isfinite(count_margin))
        return fail(S2D_EINVAL, "b_min must be >= 0, margin finite and >= 1, count_margin finite and >= 0");
    if (!(std::isfinite(mu) && mu > 0.0)) return fail(S2D_EINVAL, "mu must be finite and > 0");
    int dev = 0;
    int rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    hipError_t e = s2d::near_launch_calibrate(op, n, frame, du_pred, dv_pred, du, dv, mu, n_bins, bin_lo, bin_w, b_min,
                                              margin, count_margin, (uint32_t *)bound, (uint32_t *)bound_zero, count,
                                              (hipStream_t)stream);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "calibration launch");
}

S2D_API size_t near_mlp_blob_size(void) { return align256(sizeof(s2d::NearBlob)); }

S2D_API int near_mlp_pack(const float *params, const float *bound, const float *bound_zero, int32_t n_bins,
                          float bin_lo, float bin_w, float b_min, int32_t upsample, void *blob, void *stream) {
    if (!params || !blob) return fail(S2D_EINVAL, "params and blob must not be NULL");
    if (n_bins < 0 || n_bins > s2d::kNearMaxBins) return fail(S2D_EINVAL, "n_bins must be in 0..64");
    if (n_bins > 0 && !bound) return fail(S2D_EINVAL, "bound must not be NULL when n_bins > 0");
    if (!(bin_w > 0.f) || !std::isfinite(bin_lo) || !std::isfinite(bin_w))
        return fail(S2D_EINVAL, "bins: bin_w must be finite and > 0, bin_lo finite");
    if (!(b_min >= 0.f)) return fail(S2D_EINVAL, "b_min must be >= 0");
    if (upsample < 1 || upsample > 32) return fail(S2D_EINVAL, "upsample factor must be in 1..32");
    if (((uintptr_t)blob & 255) != 0) return fail(S2D_EINVAL, "blob must be 256-byte aligned");
    int dev = 0;
    int rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    hipError_t e = s2d::near_launch_pack(params, bound, bound_zero, n_bins, bin_lo, bin_w, b_min, upsample,
                                         (s2d::NearBlob *)blob, (hipStream_t)stream);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "MLP pack launch");
}

// ---------------------------------------------------------------------------
// walls: spectral upsampling and the near-wall double-layer correction
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kWallMaxNodes = (INT32_MAX - 4 * s2d::kSuperBlock) / 32;

int check_walls(const s2d_curves *w, double d, int P) {
    if (!w) return fail(S2D_EINVAL, "walls must not be NULL");
    if (w->n_nodes < 0 || w->n_nodes > kWallMaxNodes || w->n_curves < 0)
        return fail(S2D_EINVAL, "walls sizes out of range");
    if (w->n_nodes > 0 && w->n_curves < 1) return fail(S2D_EINVAL, "walls with nodes need n_curves >= 1");
    if (w->n_nodes > 0 && (!w->x || !w->y || !w->nx || !w->ny || !w->fx || !w->fy || !w->curve_off))
        return fail(S2D_EINVAL, "walls x, y, nx, ny, fx, fy, curve_off must not be NULL");
    if (P < 1 || P > 32) return fail(S2D_EINVAL, "upsample factor must be in 1..32");
    if (!(std::isfinite(d) && d > 0.0)) return fail(S2D_EINVAL, "period d must be finite and > 0");
    return S2D_OK;
}

// fine curves, then the coefficients, in one workspace
struct WallLayout {
    size_t fine, foff, coef, total;
};

WallLayout wall_layout(const s2d_curves *w, int P) {
    WallLayout L{};
    const size_t nf = (size_t)P * (size_t)w->n_nodes;
    L.fine = 0;
    L.foff = align256(7 * nf * sizeof(double));
    L.coef = L.foff + align256(((size_t)w->n_curves + 1) * sizeof(int32_t));
    L.total = L.coef + align256(s2d::wall_scratch(w->n_nodes, P).total);
    return L;
}

s2d::WallArgs wall_args(const s2d_curves *w, double d, int P, void *scratch, double *const out[7], int32_t *ooff) {
    s2d::WallArgs a{};
    const s2d::WallScratch sc = s2d::wall_scratch(w->n_nodes, P);
    a.s1 = sc.s1;
    a.s2 = sc.s2;
    a.coef = (double *)((char *)scratch + sc.coef);
    a.part1 = (double *)((char *)scratch + sc.part1);
    a.part2 = (double *)((char *)scratch + sc.part2);
    a.n_nodes = w->n_nodes;
    a.n_curves = w->n_curves;
    a.P = P;
    a.off = w->curve_off;
    a.x = w->x;
    a.y = w->y;
    a.nx = w->nx;
    a.ny = w->ny;
    a.fx = w->fx;
    a.fy = w->fy;
    a.d = d;
    a.ox = out[0];
    a.oy = out[1];
    a.onx = out[2];
    a.ony = out[3];
    a.ow = out[4];
    a.ofx = out[5];
    a.ofy = out[6];
    a.ooff = ooff;
    return a;
}

// workspace of near_wall_correct_eval: upsampling, outputs, features and
// the fallback list (MLP, AUTO), pair sums
struct NearWallLayout {
    WallLayout up;
    size_t t4, dtab, dscr, X, nrec, flag, list, count, llist, lcount, cxy, pair, pair_bytes, total;
};

NearWallLayout near_wall_layout(int method, const s2d_curves *w, const s2d_targets *t, int P,
                                s2d_curves *fine_shape) {
    NearWallLayout L{};
    size_t o = 0;
    if (method != S2D_NEAR_MLP) {
        L.up = wall_layout(w, P);
        o = L.up.total;
    }
    const size_t n = (size_t)t->n;
    L.t4 = o;
    o += align256(4 * n * sizeof(double));
    if (method != S2D_NEAR_UPSAMPLE) {
        L.dtab = o;
        o += align256((size_t)w->n_nodes * 2 * s2d::kNearDeriv * sizeof(double));
        L.dscr = o;
        o += align256(s2d::near_derivs_scratch(w));
        L.X = o;
        o += align256(n * s2d::kNearFeat * sizeof(float));
        L.nrec = o;
        o += align256(n * s2d::kNetRec * sizeof(float));
        L.flag = o;
        o += align256(n * sizeof(int32_t));
        L.list = o;
        o += align256(n * sizeof(int32_t));
        L.count = o;
        o += 256;
        L.llist = o;
        o += align256(n * sizeof(int32_t));
        L.lcount = o;
        o += align256((n + 255) / 256 * sizeof(int32_t) + sizeof(int32_t));
        L.cxy = o;
        o += align256(2 * n * sizeof(double));
    }
    s2d_curves f = *w;
    f.n_nodes = (int64_t)P * w->n_nodes;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDev && g_dev[dev].init) cus = g_dev[dev].cus;
    size_t pb = 256;
    if (method == S2D_NEAR_UPSAMPLE) {
        pb = std::max(pb, s2d::make_plan(S2D_OP_DLP, S2D_FP64, &f, t, cus).total);
        pb = std::max(pb, s2d::make_plan(S2D_OP_DLP, S2D_FP64, w, t, cus).total);
    } else if (method == S2D_NEAR_AUTO) {
        // the fallback targets are known only at run time: the largest plan
        // over every tile count up to all targets (the plan depends on the
        // target count through its tiles)
        s2d_targets tm = *t;
        const int64_t tiles = ((int64_t)n + s2d::kWave - 1) / s2d::kWave;
        for (int64_t k = 1; k <= tiles; ++k) {
            tm.n = std::min<int64_t>(k * s2d::kWave, (int64_t)n);
            pb = std::max(pb, s2d::make_plan(S2D_OP_DLP, S2D_FP64, &f, &tm, cus).total);
            pb = std::max(pb, s2d::make_plan(S2D_OP_DLP, S2D_FP64, w, &tm, cus).total);
        }
    }
    L.pair = o;
    L.pair_bytes = pb;
    L.total = o + align256(pb);
    if (fine_shape) *fine_shape = f;
    return L;
}

}  // namespace

S2D_API size_t stokes2d_wall_upsample_workspace_size(const s2d_curves *walls, int32_t upsample) {
    if (!walls || walls->n_nodes < 0 || walls->n_nodes > kWallMaxNodes || upsample < 1 || upsample > 32) return 0;
    return std::max<size_t>(s2d::wall_scratch(walls->n_nodes, upsample).total, 256);
}

S2D_API int stokes2d_wall_upsample(const s2d_curves *walls, double d, int32_t upsample, double *x, double *y,
                                   double *nx, double *ny, double *w, double *fx, double *fy, int32_t *curve_off,
                                   void *ws, size_t ws_bytes, void *stream) {
    int rc = check_walls(walls, d, upsample);
    if (rc != S2D_OK) return rc;
    if (walls->n_nodes > 0 && (!x || !y || !nx || !ny || !w || !fx || !fy))
        return fail(S2D_EINVAL, "outputs x, y, nx, ny, w, fx, fy must not be NULL");
    if (walls->n_curves > 0 && !curve_off) return fail(S2D_EINVAL, "output curve_off must not be NULL");
    int dev = 0;
    rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    const size_t need = stokes2d_wall_upsample_workspace_size(walls, upsample);
    if (!ws || ws_bytes < need)
        return fail(S2D_EWORKSPACE, "wall workspace too small: need " + std::to_string(need) + " bytes");
    if (((uintptr_t)ws & 255) != 0) return fail(S2D_EWORKSPACE, "workspace must be 256-byte aligned");
    double *const out[7] = {x, y, nx, ny, w, fx, fy};
    const s2d::WallArgs a = wall_args(walls, d, upsample, ws, out, walls->n_curves > 0 ? curve_off : nullptr);
    if (walls->n_curves == 0) return S2D_OK;
    const hipError_t e = s2d::wall_upsample_launch(a, (hipStream_t)stream);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "wall upsample launch");
}

S2D_API size_t near_wall_workspace_size(int method, const s2d_curves *walls, const s2d_targets *trg,
                                        int32_t upsample) {
    if (!walls || !trg || trg->n < 0 || walls->n_nodes < 0 || walls->n_nodes > kWallMaxNodes ||
        walls->n_curves < 0 || upsample < 1 || upsample > 32 || method < S2D_NEAR_UPSAMPLE || method > S2D_NEAR_AUTO)
        return 0;
    return near_wall_layout(method, walls, trg, upsample, nullptr).total;
}

S2D_API int near_wall_features_eval(const s2d_curves *walls, const s2d_targets *trg, const int32_t *trg_curve,
                                    double d, const double *dtab, float *X, double *frame, void *stream) {
    int rc = check_walls(walls, d, 1);
    if (rc != S2D_OK) return rc;
    if (!trg || trg->n < 0 || trg->n > INT32_MAX || (trg->n > 0 && (!trg->x || !trg->y || !trg_curve)))
        return fail(S2D_EINVAL, "trg x, y and trg_curve must not be NULL");
    if (walls->n_nodes > 0 && (!walls->w || !walls->kappa || !dtab))
        return fail(S2D_EINVAL, "the features need the walls' w, kappa and derivative table");
    if (trg->n > 0 && (!X || !frame)) return fail(S2D_EINVAL, "X and frame must not be NULL");
    int dev = 0;
    rc = current_device(&dev);
    if (rc != S2D_OK || trg->n == 0) return rc;
    const hipError_t e =
        s2d::near_launch_wall_features(walls, trg, trg_curve, d, dtab, X, frame, (hipStream_t)stream);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "near-wall features launch");
}

S2D_API int near_wall_correct_eval(int method, const s2d_curves *walls, const s2d_targets *trg,
                                   const int32_t *trg_curve, double d, int32_t img_lo, int32_t img_hi,
                                   int32_t upsample, const void *mlp, double threshold, const double *curve_tol,
                                   double *du, double *dv, int32_t *used_fallback, int accumulate, void *ws,
                                   size_t ws_bytes, void *stream) {
    if (method < S2D_NEAR_UPSAMPLE || method > S2D_NEAR_AUTO) return fail(S2D_EINVAL, "unknown near method");
    int rc = check_walls(walls, d, upsample);
    if (rc != S2D_OK) return rc;
    rc = check_args(S2D_OP_DLP, S2D_FP64, walls, trg, d, img_lo, img_hi, 1.0);
    if (rc != S2D_OK) return rc;
    if (trg->on_curve) return fail(S2D_EINVAL, "the near-wall correction is for free targets: on_curve must be NULL");
    if (trg->n > 0 && (!du || !dv)) return fail(S2D_EINVAL, "outputs du, dv must not be NULL");
    if (method != S2D_NEAR_UPSAMPLE) {
        if (!mlp) return fail(S2D_EINVAL, "MLP methods need the packed network");
        if (trg->n > 0 && !trg_curve) return fail(S2D_EINVAL, "MLP methods need trg_curve");
        if (walls->n_nodes > 0 && (!walls->w || !walls->kappa))
            return fail(S2D_EINVAL, "MLP methods need the walls' w and kappa");
    }
    if (method == S2D_NEAR_AUTO && !curve_tol && !(threshold >= 0.0))
        return fail(S2D_EINVAL, "threshold must be >= 0");
    int dev = 0;
    rc = current_device(&dev);
    if (rc != S2D_OK) return rc;
    if (trg->n == 0) return S2D_OK;
    s2d_curves fine{};
    const NearWallLayout L = near_wall_layout(method, walls, trg, upsample, &fine);
    if (!ws || ws_bytes < L.total)
        return fail(S2D_EWORKSPACE, "near-wall workspace too small: need " + std::to_string(L.total) + " bytes");
    if (((uintptr_t)ws & 255) != 0) return fail(S2D_EWORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    const int64_t n = trg->n;
    double *t4 = (double *)(base + L.t4);     // D_P (u, v), then D_1 (u, v); or the result (u, v)
    hipError_t e = hipSuccess;
    if (walls->n_nodes == 0) {
        // no wall: the correction is zero
        return eval(S2D_OP_DLP, S2D_FP64, walls, trg, d, img_lo, img_hi, 1.0, du, dv, accumulate,
                    base + L.pair, L.pair_bytes, stream);
    }
    // the refined walls (UPSAMPLE; AUTO when some target falls back)
    const auto refine = [&]() -> int {
        const size_t nf = (size_t)fine.n_nodes;
        double *fp = (double *)(base + L.up.fine);
        double *const out[7] = {fp, fp + nf, fp + 2 * nf, fp + 3 * nf, fp + 4 * nf, fp + 5 * nf, fp + 6 * nf};
        int32_t *foff = (int32_t *)(base + L.up.foff);
        const s2d::WallArgs a = wall_args(walls, d, upsample, base + L.up.coef, out, foff);
        const hipError_t ee = s2d::wall_upsample_launch(a, st);
        if (ee != hipSuccess) return hip_fail(ee, "wall upsample launch");
        fine.curve_off = foff;
        fine.x = out[0];
        fine.y = out[1];
        fine.nx = out[2];
        fine.ny = out[3];
        fine.w = out[4];
        fine.kappa = nullptr;
        fine.fx = out[5];
        fine.fy = out[6];
        return S2D_OK;
    };
    if (method == S2D_NEAR_UPSAMPLE) {
        if ((rc = refine()) != S2D_OK) return rc;
        rc = eval(S2D_OP_DLP, S2D_FP64, &fine, trg, d, img_lo, img_hi, 1.0, t4, t4 + n, 0, base + L.pair,
                  L.pair_bytes, stream);
        if (rc != S2D_OK) return rc;
        rc = eval(S2D_OP_DLP, S2D_FP64, walls, trg, d, img_lo, img_hi, 1.0, t4 + 2 * n, t4 + 3 * n, 0,
                  base + L.pair, L.pair_bytes, stream);
        if (rc != S2D_OK) return rc;
        e = s2d::delta_combine_launch(n, accumulate, du, dv, t4, st);
        return e == hipSuccess ? S2D_OK : hip_fail(e, "near-wall combine launch");
    }
    // MLP, AUTO: density derivatives, features, then the straight-line
    // coefficients and the network (AUTO: with the per-bin decision)
    double *dtab = (double *)(base + L.dtab);
    float *X = (float *)(base + L.X), *nrec = (float *)(base + L.nrec);
    e = s2d::near_launch_derivs(walls, dtab, base + L.dscr, st);
    if (e != hipSuccess) return hip_fail(e, "near-wall derivative launch");
    const bool autom = method == S2D_NEAR_AUTO;
    int32_t *flag = used_fallback ? used_fallback : (int32_t *)(base + L.flag);
    double *tu = t4, *tv = t4 + n;
    const s2d::DecideArgs da{(const s2d::NearBlob *)mlp, 1.0, threshold, curve_tol, walls->n_curves, autom ? 1 : 0,
                             tu, tv, flag};
    e = s2d::near_launch_wall_features(walls, trg, trg_curve, d, dtab, X, nullptr, st, &da, nrec);
    if (e != hipSuccess) return hip_fail(e, "near-wall features launch");
    const int32_t *llist = nullptr, *llen = nullptr;
    if (autom) {
        int32_t *lcnt = (int32_t *)(base + L.lcount);
        e = s2d::near_launch_compact(n, flag, 0, lcnt, (int32_t *)(base + L.llist), st);
        if (e != hipSuccess) return hip_fail(e, "near-wall compaction launch");
        llist = (const int32_t *)(base + L.llist);
        llen = lcnt + (n + 255) / 256;
    }
    e = s2d::near_launch_infer(S2D_OP_DLP, n, X, nrec, (const s2d::NearBlob *)mlp, llist, llen, tu, tv, st);
    if (e != hipSuccess) return hip_fail(e, "near-wall MLP launch");
    if (autom) {
        // the fallback targets: the refined quadrature at a compacted list
        int32_t *list = (int32_t *)(base + L.list), *count = (int32_t *)(base + L.count);
        double *cx = (double *)(base + L.cxy), *cy = cx + n;
        e = s2d::zero_int_launch(count, 1, st);
        if (e == hipSuccess) e = s2d::fallback_compact_launch(n, flag, trg->x, trg->y, list, count, cx, cy, st);
        int32_t m = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&m, count, sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "near-wall fallback list");
        if (m > 0) {
            if ((rc = refine()) != S2D_OK) return rc;
            // fine and coarse sums of the m targets into the feature area
            // (the features are no longer needed)
            static_assert(s2d::kNetRec * sizeof(float) >= 4 * sizeof(double), "four doubles per target fit");
            double *f4 = (double *)(base + L.nrec);
            const s2d_targets tl{m, cx, cy, nullptr, nullptr};
            rc = eval(S2D_OP_DLP, S2D_FP64, &fine, &tl, d, img_lo, img_hi, 1.0, f4, f4 + m, 0, base + L.pair,
                      L.pair_bytes, stream);
            if (rc != S2D_OK) return rc;
            rc = eval(S2D_OP_DLP, S2D_FP64, walls, &tl, d, img_lo, img_hi, 1.0, f4 + 2 * m, f4 + 3 * m, 0,
                      base + L.pair, L.pair_bytes, stream);
            if (rc != S2D_OK) return rc;
            e = s2d::fallback_scatter_launch(m, list, f4, tu, tv, st);
            if (e != hipSuccess) return hip_fail(e, "near-wall fallback scatter");
        }
    }
    e = s2d::add_or_write_launch(n, accumulate, du, dv, tu, tv, st);
    return e == hipSuccess ? S2D_OK : hip_fail(e, "near-wall output launch");
}

S2D_API const char *stokes2d_last_error(void) { return g_err.c_str(); }

S2D_API int stokes2d_version(void) { return 100; }

}  // extern "C"
