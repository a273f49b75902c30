// Internal declarations of the near-field correction kernels (near.hip).
#pragma once
#include "s2d_internal.h"

namespace s2d {

constexpr int kNearFeat = 20;
constexpr int kNearMaxBins = 64;
constexpr int kActStride = 20 + 6 * 64;      // h0 z1 h1 z2 h2 z3 h3 per training sample

// FP32 master parameter vector: standardisation, then W (in x out, row
// major) and b of each layer.
struct MlpOffsets {
    int mu = 0, sd = 20, W1 = 40, b1 = 40 + 1280, W2 = 1384, b2 = 1384 + 4096, W3 = 5544, b3 = 5544 + 4096,
        W4 = 9704, b4 = 9704 + 128, total = 9834;
};

// BF16 inference blob (device): weights as [out][in / 2] bf16 pairs.
struct NearBlob {
    float mu_in[kNearFeat], isd_in[kNearFeat];
    uint32_t W1[64 * kNearFeat / 2];
    float b1[64];
    uint32_t W2[64 * 32];
    float b2[64];
    uint32_t W3[64 * 32];
    float b3[64];
    uint32_t W4[2 * 32];
    float b4[2];
    int32_t n_bins;
    float bin_lo, bin_w;
    float bound[kNearMaxBins];        // network error bound per bin (scaled units)
    float bound_zero[kNearMaxBins];   // plain-rule error bound per bin (scaled units)
};
constexpr int kNearBlobWork = kNearFeat + 64 * kNearFeat / 2 + 2 * 64 * 32 + 2 * 32 + 64;

hipError_t near_launch_upsample(const s2d_curves *c, int P, double *up, hipStream_t st);
// list / list_len (device): when list != NULL only targets list[q],
// q < *list_len, are evaluated; list_len must be NULL otherwise.
hipError_t near_launch_quad(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, const int32_t *list,
                            const int32_t *list_len, int P, const double *up, double mu, double *du, double *dv,
                            hipStream_t st, double *uf = nullptr, double *vf = nullptr, double *uc = nullptr,
                            double *vc = nullptr);
// the targets with flag == 1, in order, into list; their number into
// cnt[ceil(n / 256)] (cnt: ceil(n / 256) + 1 ints of scratch)
hipError_t near_launch_compact(int64_t n, const int32_t *flag, int32_t *cnt, int32_t *list, hipStream_t st);
hipError_t near_launch_features(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, float *X,
                                double *frame, hipStream_t st);
hipError_t near_launch_scale_labels(int64_t n, const double *du, const double *dv, const double *frame, double mu,
                                    float *Y, hipStream_t st);
hipError_t near_launch_wall_features(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, double d,
                                     float *X, double *frame, hipStream_t st);
// The walls' labels and inference reuse the single layer's scale
// h F / (4 pi mu): with the frame's length factor 1 and mu = 1/4 it is the
// double layer's F / pi.
constexpr double kWallMuScale = 0.25;
hipError_t near_launch_infer(int64_t n, const float *X, const double *frame, const NearBlob *nb, double mu,
                             double threshold, int use_bound, double *du, double *dv, int32_t *flag, hipStream_t st);
hipError_t near_launch_pack(const float *prm, const float *bound, const float *bound_zero, int32_t n_bins,
                            float bin_lo, float bin_w, NearBlob *nb, hipStream_t st);
hipError_t near_launch_train_step(int32_t B, const int32_t *idx, const float *X, const float *T, float *prm,
                                  float *m, float *v, int32_t step, float lr, float *grad, float *act, float *dY,
                                  float *lossv, float *loss, int update, hipStream_t st);
hipError_t near_launch_fwd(int64_t n, const float *X, const float *prm, float *Y, hipStream_t st);

constexpr int kUpMaxN = 256;      // coarse nodes per curve for upsampling
constexpr int kUpMaxM = 2048;     // fine nodes per curve

// Spectral upsampling of periodic wall curves (wall.hip).
struct WallArgs {
    int64_t n_nodes;                                    // coarse nodes, all curves
    int32_t n_curves, P;
    const int32_t *off;                                 // [n_curves + 1]
    const double *x, *y, *nx, *ny, *fx, *fy;
    double d;
    int32_t s1, s2;                                     // chunks of the two sums
    double *coef, *part1, *part2;                       // scratch, WallScratch layout
    double *ox, *oy, *onx, *ony, *ow, *ofx, *ofy;       // [P n_nodes]
    int32_t *ooff;                                      // [n_curves + 1] = P off
};
// scratch of the upsampling: coefficients [n_nodes] x 8, partial
// coefficients [s1][n_nodes] x 8, partial fine sums [s2][6][P n_nodes]
// (byte offsets from the scratch base)
struct WallScratch {
    int s1, s2;
    size_t coef, part1, part2, total;
};
WallScratch wall_scratch(int64_t n_nodes, int P);
hipError_t wall_upsample_launch(const WallArgs &a, hipStream_t st);
// t = [uf | vf | uc | vc], each [n]: u (+)= uf - uc, v (+)= vf - vc
hipError_t delta_combine_launch(int64_t n, int accumulate, double *u, double *v, const double *t, hipStream_t st);
// u (+)= tu, v (+)= tv
hipError_t add_or_write_launch(int64_t n, int accumulate, double *u, double *v, const double *tu, const double *tv,
                               hipStream_t st);
// the targets with flag 1 into a list (order unspecified): count[0] = how
// many, list, and their coordinates cx, cy; count must be zero on entry
hipError_t fallback_compact_launch(int64_t n, const int32_t *flag, const double *tx, const double *ty, int32_t *list,
                                   int32_t *count, double *cx, double *cy, hipStream_t st);
// tu[list[j]] = uf[j] - uc[j], tv[list[j]] = vf[j] - vc[j], t4 = [uf|vf|uc|vc] of m
hipError_t fallback_scatter_launch(int64_t m, const int32_t *list, const double *t4, double *tu, double *tv,
                                   hipStream_t st);
hipError_t zero_int_launch(int32_t *p, int n, hipStream_t st);

}  // namespace s2d
