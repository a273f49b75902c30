// Single-call pair-sum kernel: a grid of independent waves, one (target
// tile, source split) each; the per-wave work is pair_tile() in pair_impl.h.
#include "pair_impl.h"

namespace s2d {

template <int OP, int PREC, int TPT>
__global__ __launch_bounds__(kBlock) void pair_kernel(PairArgs a) {
    __shared__ __attribute__((aligned(16))) double ltab[kLogTabWords];
    if (PREC == S2D_FP64 && OP == S2D_OP_SLP) fill_log_table(ltab);   // before any wave returns
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int64_t blk = blockIdx.x;
    const int split = (int)(blk % a.n_splits);
    const int64_t tile = (blk / a.n_splits) * kWavesPerBlock + wid;
    if (tile >= a.n_tiles) return;                  // wave-uniform
    pair_tile<OP, PREC, TPT>(a, tile, split, lane, ltab);
}

template <int OP, int PREC, int TPT>
static hipError_t launch_t(const Plan &p, const PairArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((pair_kernel<OP, PREC, TPT>), dim3((unsigned)p.n_blocks), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_pair(const Plan &p, const PairArgs &a, hipStream_t st) {
    if (p.n_blocks <= 0) return hipSuccess;
    const bool f64 = p.mode == S2D_FP64;
    // pressures and traction: one target per lane
    switch (p.op) {
    case S2D_OP_SLP_PRESSURE:
        return f64 ? launch_t<S2D_OP_SLP_PRESSURE, S2D_FP64, 1>(p, a, st)
                   : launch_t<S2D_OP_SLP_PRESSURE, S2D_FP32C, 1>(p, a, st);
    case S2D_OP_DLP_PRESSURE:
        return f64 ? launch_t<S2D_OP_DLP_PRESSURE, S2D_FP64, 1>(p, a, st)
                   : launch_t<S2D_OP_DLP_PRESSURE, S2D_FP32C, 1>(p, a, st);
    case S2D_OP_SLP_TRACTION:
        return f64 ? launch_t<S2D_OP_SLP_TRACTION, S2D_FP64, 1>(p, a, st)
                   : launch_t<S2D_OP_SLP_TRACTION, S2D_FP32C, 1>(p, a, st);
    default:
        break;
    }
    const bool slp = p.op == S2D_OP_SLP;
    switch (p.tpt) {
    case 1:
        if (slp) return f64 ? launch_t<S2D_OP_SLP, S2D_FP64, 1>(p, a, st) : launch_t<S2D_OP_SLP, S2D_FP32C, 1>(p, a, st);
        return f64 ? launch_t<S2D_OP_DLP, S2D_FP64, 1>(p, a, st) : launch_t<S2D_OP_DLP, S2D_FP32C, 1>(p, a, st);
    case 2:
        if (slp) return f64 ? launch_t<S2D_OP_SLP, S2D_FP64, 2>(p, a, st) : launch_t<S2D_OP_SLP, S2D_FP32C, 2>(p, a, st);
        return f64 ? launch_t<S2D_OP_DLP, S2D_FP64, 2>(p, a, st) : launch_t<S2D_OP_DLP, S2D_FP32C, 2>(p, a, st);
    case 4:
        if (slp) return f64 ? launch_t<S2D_OP_SLP, S2D_FP64, 4>(p, a, st) : launch_t<S2D_OP_SLP, S2D_FP32C, 4>(p, a, st);
        return f64 ? launch_t<S2D_OP_DLP, S2D_FP64, 4>(p, a, st) : launch_t<S2D_OP_DLP, S2D_FP32C, 4>(p, a, st);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace s2d

