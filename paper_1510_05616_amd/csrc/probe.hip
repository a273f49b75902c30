// VALU issue-rate probes (a benchmarking aid): the instruction issue rate a
// wave can reach on this chip when nothing but independent FMA chains is in
// flight, the ceiling against which the pair kernels' measured VALU rate is
// judged.  Each thread runs kChains independent chains for `iters`
// iterations, one fused multiply-add per chain and iteration:
//   form 0: FP32, every operand in a VGPR (two instructions may issue in one
//           cycle);
//   form 1: FP32, the multiplier a wave-uniform kernel argument held in an
//           SGPR (the operand pattern of the pair kernels' source records);
//   form 2: FP64, every operand in a VGPR.
// The chains' final values are summed into sink[thread] so that none is
// removed.  Packed FP32 instructions are disabled for the library build, so
// the FP32 forms issue plain v_fma_f32.
#include "s2d_internal.h"

namespace s2d {

constexpr int kChains = 8;

template <int FORM>
__global__ __launch_bounds__(256) void valu_probe(int32_t iters, float s_mul, float *__restrict__ sink) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float lane = (float)(threadIdx.x & (kWave - 1));
    if constexpr (FORM == 2) {
        double a[kChains];
        const double m = 1.0 + 1e-12 * lane, c = 1e-7 * lane;
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = 1e-3 * (double)(k + 1) + 1e-9 * lane;
#pragma unroll 4
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) a[k] = __builtin_fma(a[k], m, c);
        }
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kChains; ++k) s += a[k];
        sink[t] = (float)s;
    } else {
        float a[kChains];
        const float m = FORM == 1 ? s_mul : 1.f + 1e-7f * lane, c = 1e-7f * lane;
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = 1e-3f * (float)(k + 1) + 1e-6f * lane;
#pragma unroll 4
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) a[k] = __builtin_fmaf(a[k], m, c);
        }
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < kChains; ++k) s += a[k];
        sink[t] = s;
    }
}

hipError_t valu_probe_launch(int form, int32_t blocks, int32_t iters, float *sink, hipStream_t st) {
    if (form == 0)
        hipLaunchKernelGGL(valu_probe<0>, dim3((unsigned)blocks), dim3(256), 0, st, iters, 1.f, sink);
    else if (form == 1)
        hipLaunchKernelGGL(valu_probe<1>, dim3((unsigned)blocks), dim3(256), 0, st, iters, 1.0000001f, sink);
    else
        hipLaunchKernelGGL(valu_probe<2>, dim3((unsigned)blocks), dim3(256), 0, st, iters, 1.f, sink);
    return hipGetLastError();
}

}  // namespace s2d
