// Internal declarations of the near-field correction kernels (near.hip).
#pragma once
#include "s2d_internal.h"

namespace s2d {

// Learned correction (see near.hip): 14 geometry features per target, a
// frame record of kNearFrame doubles {s, b, t_x, t_y, n_x, n_y, hl, F, sg,
// d_0t, d_0n, ..., d_4t, d_4n, sg kappa hl} (offsets in units of hl, n the normal
// towards the target, sg the sign of the offset along the node normal, d the
// density's node derivatives in the frame, F = sum |d|), and a 64-64-64
// network with 20 outputs dC[p][out][in].
constexpr int kNearFeat = 14;
constexpr int kNearDeriv = 5;
constexpr int kNearOut = 4 * kNearDeriv;
constexpr int kNearFrame = 20;
constexpr int kNearMaxBins = 64;                // bins of log10 b
constexpr int kNearSBins = 5;                   // bins of |s|: width 1/8, the last (|s| >= 1/2) open
constexpr int kNearKBins = 8;                   // bins of log10 |kappa h| from -2, width 3/16, both ends open
constexpr int kNearCell = kNearSBins * kNearKBins;
constexpr int kNearTable = kNearMaxBins * kNearCell;
constexpr int kActStride = kNearFeat + 6 * 64;   // h0 z1 h1 z2 h2 z3 h3 per training sample
// training sample record (floats): d[10] (frame, d_pt at 2p, d_pn at 2p + 1),
// the flat prediction's residual R[2] (frame, units of the layer's scale),
// the loss weight, exp(-2 pi b)
constexpr int kNearTStride = 14;

// FP32 master parameter vector: standardisation, then W (in x out, row
// major) and b of each layer.
struct MlpOffsets {
    static constexpr int mu = 0, sd = kNearFeat, W1 = 2 * kNearFeat, b1 = W1 + kNearFeat * 64, W2 = b1 + 64,
                         b2 = W2 + 4096, W3 = b2 + 64, b3 = W3 + 4096, W4 = b3 + 64, b4 = W4 + 64 * kNearOut,
                         total = b4 + kNearOut;
};

// BF16 inference blob (device): weights as [out][in / 2] bf16 pairs; the
// last layer padded to 32 output rows.
struct NearBlob {
    float mu_in[kNearFeat], isd_in[kNearFeat];
    uint32_t W1[64 * 8];              // first layer: rows padded to 8 input pairs
    float b1[64];
    uint32_t W2[64 * 32];
    float b2[64];
    uint32_t W3[64 * 32];
    float b3[64];
    uint32_t W4[32 * 32];
    float b4[32];
    int32_t n_bins;
    float bin_lo, bin_w;              // bins of log10(b)
    float b_min;                      // smaller normal offsets go to the quadrature
    int32_t P;                        // upsampling factor of the quadrature the network was trained on
    // per bin (log10 b bin k, |s| bin j, |kappa h| bin m at kNearCell k +
    // kNearKBins j + m): the network's error bound and the largest
    // correction, in units of the layer's scale times F
    float bound[kNearTable];
    float bound_zero[kNearTable];
};

hipError_t near_launch_upsample(const s2d_curves *c, int P, double *up, hipStream_t st);
// list / list_len (device): when list != NULL only targets list[q],
// q < *list_len, are evaluated; list_len must be NULL otherwise.
hipError_t near_launch_quad(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, const int32_t *list,
                            const int32_t *list_len, int P, const double *up, double mu, double *du, double *dv,
                            hipStream_t st, double *uf = nullptr, double *vf = nullptr, double *uc = nullptr,
                            double *vc = nullptr);
// the targets with flag == value, in order, into list; their number into
// cnt[ceil(n / 256)] (cnt: ceil(n / 256) + 1 ints of scratch); with list2,
// in the same pass the targets with flag == value2 into list2 (count in
// cnt2 likewise)
hipError_t near_launch_compact(int64_t n, const int32_t *flag, int value, int32_t *cnt, int32_t *list,
                               hipStream_t st, int value2 = 0, int32_t *cnt2 = nullptr, int32_t *list2 = nullptr);
// the density's node derivatives (kNearDeriv x 2 doubles per node, d_p of x
// then y at 2p, 2p + 1), per-node units
// scratch: near_derivs_scratch(c) bytes (256-byte aligned): a flag, and
// when n_nodes > kUpMaxN the large-curve tables
size_t near_derivs_scratch(const s2d_curves *c);
hipError_t near_launch_derivs(const s2d_curves *c, double *dtab, void *scratch, hipStream_t st);
// AUTO's decision inputs: tolerance of target i = curve_tol[tc[i]] when
// curve_tol != NULL (and tc[i] names a curve), else threshold; flag [n]
// receives the decisions (0 learned, 1 quadrature, 2 none; all 0 when
// use_bound == 0), du = dv = 0 is written for decision 2
struct DecideArgs {
    const NearBlob *nb;
    double mu, threshold;
    const double *curve_tol;
    int32_t n_curves, use_bound;
    double *du, *dv;
    int32_t *flag;
};
// near_launch_features writes X and the frame records (training and
// calibration).  The learned and AUTO routes of the vesicles take two
// launches instead: near_launch_scan writes X and the nearest node kstar [n]
// (-1: invalid target) without the density, so it can run beside the
// derivatives; near_launch_head then takes AUTO's decisions and, for every
// target decided learned (all when use_bound == 0), writes the
// straight-line part into du, dv and the network's record into nrec
// [kNetRec floats per target: d_p in the frame (2 p, 2 p + 1), t, n_f,
// scale exp(-2 pi b)].  near_launch_head with kstar == NULL does the search
// as well and writes X (one launch, after the derivatives).  The wall
// feature kernel does both in one launch (fused != NULL; frame unused then).
constexpr int kNetRec = 16;
hipError_t near_launch_features(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, const double *dtab,
                                float *X, double *frame, hipStream_t st);
hipError_t near_launch_scan(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, float *X, int32_t *kstar,
                            hipStream_t st);
hipError_t near_launch_head(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, const double *dtab,
                            const int32_t *kstar, const DecideArgs &da, float *nrec, hipStream_t st,
                            float *X = nullptr);
hipError_t near_launch_wall_features(const s2d_curves *c, const s2d_targets *t, const int32_t *tc, double d,
                                     const double *dtab, float *X, double *frame, hipStream_t st,
                                     const DecideArgs *fused = nullptr, float *nrec = nullptr);
// op: S2D_OP_SLP (vesicles, scale hl / 4 pi mu, side +1) or S2D_OP_DLP
// (walls, scale 1 / pi, side -1)
// the network's part of the learned route, added to du, dv of the targets
// list[q], q < *list_len (device; the learned targets of AUTO compacted by
// near_launch_compact), or of every target when list is NULL
hipError_t near_launch_infer(int op, int64_t n, const float *X, const float *nrec, const NearBlob *nb,
                             const int32_t *list, const int32_t *list_len, double *du, double *dv, hipStream_t st);
hipError_t near_launch_pack(const float *prm, const float *bound, const float *bound_zero, int32_t n_bins,
                            float bin_lo, float bin_w, float b_min, int32_t P, NearBlob *nb, hipStream_t st);
hipError_t near_launch_train_targets(int op, int64_t n, const double *frame, const double *du, const double *dv,
                                     const int32_t *tc, int32_t n_curves, const double *ur, const double *vr,
                                     double mu, int32_t P, float gain, uint32_t *cscale, float *T,
                                     hipStream_t st);
hipError_t near_launch_train_step(int32_t B, const int32_t *idx, const float *X, const float *T, float *prm,
                                  float *m, float *v, int32_t step, float lr, float *grad, float *act, float *dY,
                                  float *lossv, float *loss, int update, hipStream_t st);
hipError_t near_launch_fwd(int64_t n, const float *X, const float *prm, float *Y, hipStream_t st);
hipError_t near_launch_feature_stats(int64_t n, const float *X, float *prm, hipStream_t st);
hipError_t near_launch_calibrate(int op, int64_t n, const double *frame, const double *dup, const double *dvp,
                                 const double *du, const double *dv, double mu, int32_t n_bins, float bin_lo,
                                 float bin_w, float b_min, float margin, float count_margin, uint32_t *bound,
                                 uint32_t *bound_zero, int32_t *count, hipStream_t st);

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
