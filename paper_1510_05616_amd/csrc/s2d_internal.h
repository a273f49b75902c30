// Internal declarations shared by the HIP translation units of libstokes2d.
// Nothing here is part of the public ABI (include/stokes2d.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <mutex>
#include <string>

#include "../../include/stokes2d.h"

namespace s2d {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kWavesPerBlock = 4;    // batched pair kernel: 4 independent waves per workgroup
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kMaxPairWaves = 16;    // single-call pair kernel: up to 16 waves (splits) per target tile
constexpr int kSuperBlock = 256;     // sources per superblock (split granularity, FP32 log reference)
constexpr int kSubBlock = 16;        // FP32 sub-block: local origin, merged into the FP64 accumulators
constexpr double kFarRadii = 4.0;    // a sub-block is far from a target beyond this many radii
constexpr int kMaxImages = 64;

// Source records written by the preparation kernels: one wave-uniform record
// per source, read through the scalar data path by the pair kernels.
struct alignas(32) RecSlp64 { double x, y, gx, gy; };                 // g = w f
// FP32C records carry the FP64 node (exact path) and its offset from the
// sub-block origin in FP32 (far path).
struct alignas(16) RecSlp32 { double x, y; float xl, yl, gx, gy; };
struct alignas(16) RecDlp64 { double x, y, nx, ny, tx, ty; };         // nu = w n, tau
struct alignas(16) RecDlp32 { double x, y; float xl, yl, nx, ny, tx, ty; };
// per FP32C sub-block: origin and (kFarRadii * radius)^2
struct SubInfo { double ox, oy, r2; };

// One launch's decomposition of (targets x sources).
struct Plan {
    int op, mode, tpt;
    int64_t n_src, n_trg;
    int64_t n_sb;            // superblocks (sources padded to kSuperBlock)
    int64_t n_tiles;         // target tiles of kWave targets
    int waves;               // waves (splits) per workgroup, <= kMaxPairWaves
    int n_groups;            // split groups: workgroups per tile, partial planes when > 1
    int n_splits;            // source splits = waves * n_groups (each a whole number of superblocks or empty)
    int64_t sb_per_split;
    int64_t n_blocks;        // workgroups of the pair kernel
    bool self;               // targets carry on_curve/on_node and image 0 is in range
    // workspace carve-out (byte offsets)
    size_t off_rec, off_rec64, off_sub, off_sbsum, off_part, off_self, off_kress, total;
};

struct PairArgs {
    const void *rec;
    const double *sbsum;      // FP32 SLP: per-superblock sum of g (2 doubles each)
    const SubInfo *sub;       // FP32C: per sub-block origin and far radius
    int64_t n_src;
    const double *tx, *ty;
    const int32_t *on_curve, *on_node, *curve_off;
    int32_t n_curves;
    int64_t n_trg;
    int64_t n_tiles;
    int32_t n_splits;
    int32_t n_groups;         // single-call kernel: split groups (partial planes when > 1)
    int64_t sb_per_split;
    int64_t n_sb;
    double d;
    int32_t img_lo, img_hi;
    double *part;             // single call: [n_groups][2][n_trg]; batched: [n_splits][2][n_trg]
    const double *tnx, *tny;  // target unit normals (single-layer traction) or NULL
    const void *rec64;        // FP32C pressures and traction: FP64 records for near sub-blocks
};

// FP32C pressures and traction evaluate near sub-blocks from FP64 records.
constexpr bool near_fp64(int op) { return op > S2D_OP_DLP; }

// bytes of one source record of (op, mode), and the launch plan of an
// evaluation with `cus` compute units (plan.hip)
size_t rec_bytes(int op, int mode);
Plan make_plan(int op, int mode, const s2d_curves *s, const s2d_targets *t, int cus);

// VALU issue-rate probe (probe.hip): blocks x 256 threads, each 8 FMA chains
// of `iters` steps; sink: [blocks * 256] floats
hipError_t valu_probe_launch(int form, int32_t blocks, int32_t iters, float *sink, hipStream_t st);

// Operators whose sources are force densities g = w f (single-layer records)
// rather than double-layer densities (nu = w n, tau).
constexpr bool slp_sources(int op) {
    return op == S2D_OP_SLP || op == S2D_OP_SLP_PRESSURE || op == S2D_OP_SLP_TRACTION;
}

struct FinalArgs {
    const double *part;
    const double *self;       // SLP own-curve Kress sums [2][n_trg] or NULL
    int32_t n_parts;          // partial planes of part
    int64_t n_trg;
    int64_t n_src;
    double pref;
    int accumulate;
    int ncomp;                // 2: (u, v); 1: a scalar (pressure) written to u only
    double *u, *v;
    // DLP diagonal limit
    int dlp_diag;
    const int32_t *on_curve, *on_node, *curve_off;
    int32_t n_curves;
    const double *nx, *ny, *w, *kappa, *fx, *fy;
};

// launchers (return hipError_t of the launch)
hipError_t launch_prep(const Plan &p, const s2d_curves *src, void *ws, hipStream_t st);
hipError_t launch_pair(const Plan &p, const PairArgs &a, const FinalArgs &f, hipStream_t st);
hipError_t launch_kress(const Plan &p, const s2d_curves *src, const s2d_targets *trg,
                        void *ws, hipStream_t st);
hipError_t launch_final(const Plan &p, const FinalArgs &a, hipStream_t st);

// the rocBLAS handle of the current device bound to stream st (a
// rocblas_handle; cell.hip), created on first use; hold blas_mutex() while
// using it
std::mutex &blas_mutex();
void *blas_handle(hipStream_t st, std::string &err);

// error state and device checks shared by the entry points (api.hip):
// set_error records the calling thread's message and returns code;
// device_ready fails unless stokes2d_init ran for the current device
int set_error(int code, const std::string &msg);
int device_ready(int *dev);

// batched evaluation (batch.hip)
size_t batch_workspace_size(int mode, int32_t n_inst, const s2d_instance *inst);
int batch_eval(int dev, int cus, int mode, int32_t n_inst, const s2d_instance *inst, void *ws, size_t ws_bytes,
               hipStream_t stream, std::string &err);
int batch_release();
int batch_tuned(int mode, int32_t n_inst, const s2d_instance *inst, int *tpt, int *sbps, int *wpc);

}  // namespace s2d
