// Source preparation kernels of a single evaluation (device code in
// prep_impl.h).
#include "prep_impl.h"

namespace s2d {

template <int OP, int PREC>
__global__ __launch_bounds__(256) void prep_records(int64_t n_src, int64_t n_pad,
                                                    const double *__restrict__ x, const double *__restrict__ y,
                                                    const double *__restrict__ nx, const double *__restrict__ ny,
                                                    const double *__restrict__ w,
                                                    const double *__restrict__ fx, const double *__restrict__ fy,
                                                    void *rec_out, SubInfo *sub) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (PREC == S2D_FP64) {
        if (j >= n_pad) return;
        prep_one64<OP>(j, n_src, x, y, nx, ny, w, fx, fy, rec_out);
    } else {
        if (j >= n_pad / kSubBlock) return;           // one thread per sub-block
        prep_sub32<OP>(j, n_src, x, y, nx, ny, w, fx, fy, rec_out, sub);
    }
}

__global__ __launch_bounds__(256) void prep_sbsum(int64_t n_src, int64_t n_sb,
                                                  const double *__restrict__ w,
                                                  const double *__restrict__ fx, const double *__restrict__ fy,
                                                  double *sbsum) {
    const int64_t sb = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;   // a wave per superblock
    if (sb >= n_sb) return;                                                           // wave-uniform
    sbsum_wave(sb, n_src, w, fx, fy, sbsum, threadIdx.x & (kWave - 1));
}

template <int OP, int PREC>
static hipError_t prep_t(const Plan &p, const s2d_curves *s, void *ws, hipStream_t st) {
    const int64_t n_pad = p.n_sb * kSuperBlock;
    if (n_pad == 0) return hipSuccess;
    void *rec = (char *)ws + p.off_rec;
    SubInfo *sub = (SubInfo *)((char *)ws + p.off_sub);
    const int64_t nthr = PREC == S2D_FP64 ? n_pad : n_pad / kSubBlock;
    hipLaunchKernelGGL((prep_records<OP, PREC>), dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, st,
                       p.n_src, n_pad, s->x, s->y, s->nx, s->ny, s->w, s->fx, s->fy, rec, sub);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (OP == S2D_OP_SLP && PREC == S2D_FP32C) {
        hipLaunchKernelGGL(prep_sbsum, dim3((unsigned)((p.n_sb + 3) / 4)), dim3(256), 0, st,
                           p.n_src, p.n_sb, s->w, s->fx, s->fy, (double *)((char *)ws + p.off_sbsum));
        e = hipGetLastError();
    }
    return e;
}

// FP64 records of the sources at p.off_rec64 (FP32C pressures and traction)
template <int OP>
static hipError_t prep_rec64(const Plan &p, const s2d_curves *s, void *ws, hipStream_t st) {
    const int64_t n_pad = p.n_sb * kSuperBlock;
    if (n_pad == 0) return hipSuccess;
    hipLaunchKernelGGL((prep_records<OP, S2D_FP64>), dim3((unsigned)((n_pad + 255) / 256)), dim3(256), 0, st,
                       p.n_src, n_pad, s->x, s->y, s->nx, s->ny, s->w, s->fx, s->fy, (char *)ws + p.off_rec64,
                       (SubInfo *)nullptr);
    return hipGetLastError();
}

hipError_t launch_prep(const Plan &p, const s2d_curves *s, void *ws, hipStream_t st) {
    if (p.mode == S2D_FP32C && near_fp64(p.op)) {
        const hipError_t e = slp_sources(p.op) ? prep_rec64<S2D_OP_SLP_PRESSURE>(p, s, ws, st)
                                               : prep_rec64<S2D_OP_DLP>(p, s, ws, st);
        if (e != hipSuccess) return e;
    }
    if (p.op == S2D_OP_SLP)
        return p.mode == S2D_FP64 ? prep_t<S2D_OP_SLP, S2D_FP64>(p, s, ws, st) : prep_t<S2D_OP_SLP, S2D_FP32C>(p, s, ws, st);
    if (slp_sources(p.op))       // pressure and traction of the single layer: same records, no log sums
        return p.mode == S2D_FP64 ? prep_t<S2D_OP_SLP_PRESSURE, S2D_FP64>(p, s, ws, st)
                                  : prep_t<S2D_OP_SLP_PRESSURE, S2D_FP32C>(p, s, ws, st);
    return p.mode == S2D_FP64 ? prep_t<S2D_OP_DLP, S2D_FP64>(p, s, ws, st) : prep_t<S2D_OP_DLP, S2D_FP32C>(p, s, ws, st);
}

}  // namespace s2d
