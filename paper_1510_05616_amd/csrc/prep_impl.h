#pragma once
// Source preparation (O(N)): turns the caller's FP64 structure-of-arrays
// curve data into the per-source records the pair kernels stream, with the
// trapezoid weight folded in (g = w f for the single layer, nu = w n for the
// double layer; Section 2.3 Nystrom discretisation), zero-density records
// padding the last superblock, and, for the FP32 single layer, each
// superblock's FP64 density sum (used to add back the log of the superblock's
// reference factor).  A padding record sits at the last real source (n_src
// >= 1 whenever there is a superblock): its distance to any target is that of
// a real source, so its terms are finite and exactly zero, and the ragged
// superblock is summed like a full one.  (The one target it coincides with at
// image 0 is that source's own node, whose superblock the exclusion masks.)
#include "s2d_internal.h"

namespace s2d {

// Record j of a padded source array (zero record past n_src), FP64 modes.
template <int OP>
__device__ __forceinline__ void prep_one64(int64_t j, int64_t n_src, const double *__restrict__ x,
                                           const double *__restrict__ y, const double *__restrict__ nx,
                                           const double *__restrict__ ny, const double *__restrict__ w,
                                           const double *__restrict__ fx, const double *__restrict__ fy,
                                           void *rec_out) {
    const bool v = j < n_src;
    const double X = v ? x[j] : x[n_src - 1], Y = v ? y[j] : y[n_src - 1];
    const double W = v ? w[j] : 0.0;
    const double FX = v ? fx[j] : 0.0, FY = v ? fy[j] : 0.0;
    if (slp_sources(OP)) {
        ((RecSlp64 *)rec_out)[j] = RecSlp64{X, Y, W * FX, W * FY};
    } else {
        const double NX = v ? W * nx[j] : 0.0, NY = v ? W * ny[j] : 0.0;
        ((RecDlp64 *)rec_out)[j] = RecDlp64{X, Y, NX, NY, FX, FY};
    }
}

// FP32C sub-block u (kSubBlock records, zero past n_src): origin = its middle
// valid node, radius = largest distance of a valid node from the origin;
// records hold the FP64 node and its FP32 offset from the origin.
template <int OP>
__device__ __forceinline__ void prep_sub32(int64_t u, int64_t n_src, const double *__restrict__ x,
                                           const double *__restrict__ y, const double *__restrict__ nx,
                                           const double *__restrict__ ny, const double *__restrict__ w,
                                           const double *__restrict__ fx, const double *__restrict__ fy,
                                           void *rec_out, SubInfo *sub) {
    const int64_t j0 = u * kSubBlock;
    const int64_t nv = max((int64_t)0, min((int64_t)kSubBlock, n_src - j0));
    double ox = x[n_src - 1], oy = y[n_src - 1], r2 = 0.0;      // origin of an all-padding sub-block
    if (nv > 0) {
        const int64_t jm = j0 + nv / 2;
        ox = x[jm];
        oy = y[jm];
        for (int64_t j = j0; j < j0 + nv; ++j) {
            const double dx = x[j] - ox, dy = y[j] - oy;
            r2 = fmax(r2, dx * dx + dy * dy);
        }
    }
    sub[u] = SubInfo{ox, oy, kFarRadii * kFarRadii * r2};
    for (int64_t j = j0; j < j0 + kSubBlock; ++j) {
        const bool v = j < n_src;
        const double X = v ? x[j] : x[n_src - 1], Y = v ? y[j] : y[n_src - 1];
        const double W = v ? w[j] : 0.0;
        const double FX = v ? fx[j] : 0.0, FY = v ? fy[j] : 0.0;
        const float xl = (float)(X - ox), yl = (float)(Y - oy);
        if (slp_sources(OP)) {
            ((RecSlp32 *)rec_out)[j] = RecSlp32{X, Y, xl, yl, (float)(W * FX), (float)(W * FY)};
        } else {
            const double NX = v ? W * nx[j] : 0.0, NY = v ? W * ny[j] : 0.0;
            ((RecDlp32 *)rec_out)[j] = RecDlp32{X, Y, xl, yl, (float)NX, (float)NY, (float)FX, (float)FY};
        }
    }
}

// FP64 sum of g = w f over superblock sb, by one whole wave: lane l adds
// sources l, l + 64, ... in order, then the lanes are added by a fixed
// butterfly; lane 0 writes (fixed order: deterministic).
__device__ __forceinline__ void sbsum_wave(int64_t sb, int64_t n_src, const double *__restrict__ w,
                                           const double *__restrict__ fx, const double *__restrict__ fy,
                                           double *sbsum, int lane) {
    double sx = 0.0, sy = 0.0;
    const int64_t j0 = sb * kSuperBlock, j1 = min(j0 + (int64_t)kSuperBlock, n_src);
    for (int64_t j = j0 + lane; j < j1; j += kWave) {
        sx += w[j] * fx[j];
        sy += w[j] * fy[j];
    }
#pragma unroll
    for (int m = kWave / 2; m >= 1; m >>= 1) {
        sx += __shfl_xor(sx, m, kWave);
        sy += __shfl_xor(sy, m, kWave);
    }
    if (lane == 0) {
        sbsum[2 * sb] = sx;
        sbsum[2 * sb + 1] = sy;
    }
}

}  // namespace s2d
