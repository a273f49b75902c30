// Single-call pair-sum kernel.  A workgroup of W waves owns one target tile
// (kWave targets) and W consecutive source splits of one split group; its
// waves evaluate pair_sum() (pair_impl.h) on their splits, and wave 0 adds the
// W results in wave order through LDS.  With one split group (every source
// in the workgroup) wave 0 then finishes the targets itself: the own-curve
// Kress sums, the double layer's diagonal limit, the prefactor and the
// accumulate flag, exactly as finalize() does.  With G > 1 groups it writes
// the group's FP64 partial, and finalize() adds the G partials in order.
//
// blockIdx -> (tile, group): group = blockIdx % G, tile = blockIdx / G.  The
// dispatcher assigns workgroups to the 8 XCDs round-robin, so with G a
// multiple of 8 each XCD sees only its own groups and streams only their
// sources through its L2; with G = 1 every XCD streams all sources, which
// the planner allows only when the source records fit in one XCD's L2.
#include "pair_impl.h"
#include "self_impl.h"

namespace s2d {

template <int OP, int PREC, int NI>
// register allocation held to 8 waves per SIMD (64 VGPRs): every pair kernel
// fits without spills, and two 16-wave workgroups then share a CU
__global__ __launch_bounds__(kMaxPairWaves * kWave) __attribute__((amdgpu_waves_per_eu(8, 8)))
void pair_kernel(PairArgs a, FinalArgs f) {
    __shared__ __attribute__((aligned(16))) double ltab[kLogTabWords];
    __shared__ double red[2][kMaxPairWaves - 1][kWave];
    if (PREC == S2D_FP64 && OP == S2D_OP_SLP) fill_log_table(ltab);
    const int lane = threadIdx.x & (kWave - 1);
    // wave index made wave-uniform for the compiler: the split, and with it
    // every source record address, must be uniform so records take the scalar path
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int W = blockDim.x / kWave;
    const int64_t blk = blockIdx.x;
    const int group = (int)(blk % a.n_groups);
    const int64_t tile = blk / a.n_groups;
    double ox[1], oy[1];
    pair_sum<OP, PREC, 1, NI>(a, tile, group * W + wid, lane, ltab, ox, oy);
    if (wid > 0) {
        red[0][wid - 1][lane] = ox[0];
        red[1][wid - 1][lane] = oy[0];
    }
    __syncthreads();
    if (wid != 0) return;
    double sx = ox[0], sy = oy[0];
    for (int w = 1; w < W; ++w) {
        sx += red[0][w - 1][lane];
        sy += red[1][w - 1][lane];
    }
    const int64_t i = tile * kWave + lane;
    if (i >= a.n_trg) return;
    if (a.n_groups > 1) {
        a.part[(int64_t)(2 * group) * a.n_trg + i] = sx;
        a.part[(int64_t)(2 * group + 1) * a.n_trg + i] = sy;
        return;
    }
    final_one(f, i, sx, sy);
}

template <int OP, int PREC, int NI>
static hipError_t launch_t(const Plan &p, const PairArgs &a, const FinalArgs &f, hipStream_t st) {
    hipLaunchKernelGGL((pair_kernel<OP, PREC, NI>), dim3((unsigned)p.n_blocks), dim3(p.waves * kWave), 0, st, a, f);
    return hipGetLastError();
}

template <int NI>
static hipError_t launch_ni(const Plan &p, const PairArgs &a, const FinalArgs &f, hipStream_t st) {
    const bool f64 = p.mode == S2D_FP64;
    switch (p.op) {
    case S2D_OP_SLP:
        return f64 ? launch_t<S2D_OP_SLP, S2D_FP64, NI>(p, a, f, st) : launch_t<S2D_OP_SLP, S2D_FP32C, NI>(p, a, f, st);
    case S2D_OP_DLP:
        return f64 ? launch_t<S2D_OP_DLP, S2D_FP64, NI>(p, a, f, st) : launch_t<S2D_OP_DLP, S2D_FP32C, NI>(p, a, f, st);
    case S2D_OP_SLP_PRESSURE:
        return f64 ? launch_t<S2D_OP_SLP_PRESSURE, S2D_FP64, NI>(p, a, f, st)
                   : launch_t<S2D_OP_SLP_PRESSURE, S2D_FP32C, NI>(p, a, f, st);
    case S2D_OP_DLP_PRESSURE:
        return f64 ? launch_t<S2D_OP_DLP_PRESSURE, S2D_FP64, NI>(p, a, f, st)
                   : launch_t<S2D_OP_DLP_PRESSURE, S2D_FP32C, NI>(p, a, f, st);
    case S2D_OP_SLP_TRACTION:
        return f64 ? launch_t<S2D_OP_SLP_TRACTION, S2D_FP64, NI>(p, a, f, st)
                   : launch_t<S2D_OP_SLP_TRACTION, S2D_FP32C, NI>(p, a, f, st);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_pair(const Plan &p, const PairArgs &a, const FinalArgs &f, hipStream_t st) {
    if (p.n_blocks <= 0) return hipSuccess;
    if (p.waves < 1 || p.waves > kMaxPairWaves || a.n_groups < 1) return hipErrorInvalidValue;
    // images three at a time when the count allows it
    const int n_img = a.img_hi - a.img_lo + 1;
    if (n_img % 3 == 0) return launch_ni<3>(p, a, f, st);
    return launch_ni<1>(p, a, f, st);
}

}  // namespace s2d
