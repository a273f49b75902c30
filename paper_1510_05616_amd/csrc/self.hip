// Own-curve terms and the final reduction of a single evaluation (when the
// pair kernel leaves split-group partials, or when there are no sources); the
// per-curve and per-target device code is in self_impl.h.
#include "self_impl.h"

namespace s2d {

__global__ __launch_bounds__(256) void kress_table(const int32_t *__restrict__ off, int32_t n_curves,
                                                   int64_t n_src, double *__restrict__ T) {
    __shared__ double ctab[kCosTab];
    const int c = blockIdx.x;
    if (c >= n_curves) return;
    kress_table_curve(off, c, n_src, T, ctab);
}

__global__ __launch_bounds__(256) void kress_self(int64_t n_trg, int64_t n_src, const int32_t *__restrict__ on_curve,
                                                  const int32_t *__restrict__ on_node,
                                                  const int32_t *__restrict__ off, int32_t n_curves,
                                                  const double *__restrict__ x, const double *__restrict__ y,
                                                  const double *__restrict__ nx, const double *__restrict__ ny,
                                                  const double *__restrict__ w,
                                                  const double *__restrict__ fx, const double *__restrict__ fy,
                                                  const double *__restrict__ T, double *__restrict__ self) {
    __shared__ __attribute__((aligned(16))) double ltab[kLogTabWords];
    fill_log_table(ltab);                           // before any thread returns
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_trg) return;
    double sx, sy;
    kress_self_one(i, n_src, on_curve, on_node, off, n_curves, x, y, nx, ny, w, fx, fy, T, ltab, sx, sy);
    self[i] = sx;
    self[n_trg + i] = sy;
}

__global__ __launch_bounds__(256) void finalize(FinalArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_trg) return;
    double sx = 0.0, sy = 0.0;
    for (int s = 0; s < a.n_parts; ++s) {
        sx += a.part[(int64_t)(2 * s) * a.n_trg + i];
        sy += a.part[(int64_t)(2 * s + 1) * a.n_trg + i];
    }
    final_one(a, i, sx, sy);
}
hipError_t launch_kress(const Plan &p, const s2d_curves *src, const s2d_targets *trg, void *ws,
                        hipStream_t st) {
    double *T = (double *)((char *)ws + p.off_kress);
    double *self = (double *)((char *)ws + p.off_self);
    if (src->n_curves > 0) {
        hipLaunchKernelGGL(kress_table, dim3((unsigned)src->n_curves), dim3(256), 0, st, src->curve_off,
                           src->n_curves, p.n_src, T);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kress_self, dim3((unsigned)((p.n_trg + 255) / 256)), dim3(256), 0, st, p.n_trg,
                       p.n_src, trg->on_curve, trg->on_node, src->curve_off, src->n_curves, src->x, src->y, src->nx,
                       src->ny, src->w, src->fx, src->fy, T, self);
    return hipGetLastError();
}

hipError_t launch_final(const Plan &p, const FinalArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(finalize, dim3((unsigned)((p.n_trg + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace s2d
