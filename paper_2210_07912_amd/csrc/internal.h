// Launch interfaces between the C-ABI host code and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace rift {

// Work description shared by the evaluation kernels: items are segments of
// a sample array against one point; tiles are fixed-size runs of samples.
struct ItemsDev {
  const int *point;     // [n_items]
  const int64_t *off;   // [n_items] first column
  const int64_t *cnt;   // [n_items]
  const int *tile0;     // [n_items + 1] prefix of plain tiles
  const int64_t *samp0; // [n_items + 1] prefix of sample counts (flat index space)
  const int *bin0;      // [n_items + 1] prefix of delay bins
  const int *blk0;      // [n_items + 1] prefix of sort blocks (kSortBlock samples)
  const int64_t *hoff;  // [n_items] offset of the point's block histograms
  int n_items;
};

template <typename R>
struct PlainArgsT {
  const PointDev *pts;
  const int *item_point;
  const int64_t *item_off, *item_cnt;
  const int *item_tile0;
  int n_items;
  int64_t stride;
  const R *theta;       // [7][stride]
  R *lnL;               // [stride] or null
  R *lnw;               // [stride] or null: ln L_t + ln_ratio
  const R *ln_ratio;
  const R *gin;         // adjoint: upstream gradient [stride] or null (1)
  R *grad;              // adjoint: [7][stride]
  int rows_cap, nt_cap;
  int dmarg;            // 1: distance-marginalized ln L_tD (theta's distance not read; forward only)
  double dm_lo, dm_hi;  // the distance prior's range
};

template <typename R>
hipError_t plain_launch(const PlainArgsT<R> &a, int TS, int n_tiles, bool bwd, hipStream_t st,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
size_t plain_lds_bytes(int elem, int TS, int rows_cap, int nt_cap, bool bwd);

// ---- FP32 MFMA path -------------------------------------------------------
constexpr int kMaxT = kMaxModes / 2;  // MFMA steps of 4 elements per detector: M_p / 2
constexpr int kMaxClasses = 48;  // one persistent launch per distinct (T = Mp / 2, K)
constexpr int kNtBuckets = 17;   // autotuner key: floor(log2 n_t) of a class's longest window
constexpr int kFeedConfigs = 7;  // launch configurations the autotuner measures per class

constexpr int kSortBlock = 4096;  // samples per sort block
constexpr int kLdsBins = 8192;    // delay bins counted in LDS (more: in global memory)

// one sample at its sorted slot
struct SampleRec {
  float th[7];
  int col;        // column of theta / ln L_t
  int16_t n[3];   // integer row offset per detector
  int16_t flag;   // 0 padding slot, 1 valid, 2 invalid sample
};

// per-tile coefficients written by the coefficient pass (16 samples)
struct CoefTile {
  float B[16];               // quadratic term (FP64, rounded), times log2 e
  float xf[kMaxDet][2][16];  // (D_ref / D) F_k times log2 e (re, im); zero past K
  float mu[kMaxDet][16];     // interpolation fraction
  int n[kMaxDet][16];        // integer row offset (1<<28 for padding / invalid)
  int col[16];               // output column (-1: padding slot)
  int flag[16];              // 0 padding, 1 valid, 2 invalid sample
};

// Up to four tiles of one delay bin, evaluated by one workgroup that stages
// the rows of Q they share in LDS once for all of them.
struct WorkUnit {
  uint32_t tile;    // first tile
  uint32_t ntiles;  // 1..4
  uint32_t key;     // the bin, within its point
};

struct MfmaArgs {
  const PointDev *pts;
  ItemsDev items;
  int64_t stride;
  int64_t total;          // flat samples over all items
  const float *theta;     // [7][stride]
  float *lnL;             // [stride] or null
  float *lnw;             // [stride] or null
  const float *ln_ratio;  // [stride] or null
  // workspace
  uint32_t *key;          // [total] bin of each flat sample within its point
  int16_t *nsh;           // [total][4] integer row offsets n_k (index 3: valid flag)
  uint32_t *count;        // [n_bins]
  uint32_t *bhist;        // per point [sort blocks][bins]: counts, then block offsets
  uint32_t *bin_tile;     // [n_bins] first tile of the bin within its item
  uint32_t *item_tiles;   // [n_items + 1] tile prefix over items (filled on device)
  SampleRec *rec;         // [16 max_tiles] sorted samples (flag 0: padding)
  int *tile_item;         // [max_tiles]
  float *cop;             // per point, per tile [K][2 Mp][16] floats; the coefficient pass fills the first
                          // [2 Mp][16]: Y_m (element 2m + re/im) of the tile's samples
  int64_t *item_cop;      // [n_items] offset of each point's operands in cop
  CoefTile *ctile;        // [max_tiles]
  WorkUnit *unit;         // [max_tiles] work units, bins in order, points in order
  uint32_t *bin_unit;     // [n_bins] first unit of the bin within its item
  uint32_t *item_units;   // [n_items + 1] unit prefix over items (filled on device)
  uint32_t *ctl;          // [0]: number of tiles, [1 + c]: unit counter of class c
  // adjoint (null in the forward pass)
  const float *gin;       // [stride] upstream d/d ln L_t, or null (= 1)
  float *grad;            // [7][stride] gradient of ln L_t (times gin)
  float *gop;             // per point [tiles][K][2 Mp][16]: G_k = sum_r c_k[r] Q_k[r] (cop layout)
  float *hop;             // [tiles][kMaxDet][16]: H_k = sum_j p_j Re(a^dag Qtilde'_k(j))
  int *jrng;              // [16 max_tiles][4] or null: the samples to refine, appended in any order (count in
                          // ctl[kCtlRefine]): sorted slot, then the window blocks whose maximum is within
                          // kRefineNats of the sample's (b0 | b1 << 16, b2 | count << 16)
  // distance marginalization (forward only): a first pass writes each slot's
  // largest window data term, a second integrates over D
  int dmarg;
  float *amax;            // [16 max_tiles] base 2, by sorted slot
  double dm_lo, dm_hi;    // the distance prior's range
  int n_bins;
  int max_item_bins;      // largest bin count of one point
  int n_sort_blocks;
  int max_tiles;
  int grid;               // persistent workgroups
};

// Streams a call may fan out on: the class kernels of one evaluation run
// concurrently on side streams (default priority), forked from and joined
// back to the caller's stream with events, so each class fills the tail of
// the one before it.
constexpr int kSideStreams = 3;
struct Fanout {
  hipStream_t side[kSideStreams];
  hipEvent_t fork;
  hipEvent_t join[kSideStreams];
  int n;  // 0: everything on the caller's stream
};

// ev0/ev1 (or null): recorded around the persistent evaluation kernels
// classes: runs of points with the same MFMA step count T (evaluation
// launches) and with the same mode count M (coefficient launches; mclass_M is
// -M for runs of points that carry a V table, mclass_tiles bounds the tiles
// of each run)
// class_mode (per class, in/out): how the class feeds the matrix cores, 1
// staged through LDS, 2 direct from global memory, 0 not measured yet: with
// tune such a class runs both forms on this call's data, timed (the call
// then waits for them), and gets the faster; without tune it runs staged.
hipError_t mfma_forward(const MfmaArgs &a, const int *class_T, const int *class_K, const int *class_item0, int n_classes,
                        const int *mclass_M, const int *mclass_item0, const int64_t *mclass_tiles, int n_mclasses,
                        int *class_mode, bool tune, hipStream_t st, const Fanout &fo, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);

// the adjoint of the same evaluation: sort, coefficients, then per class the
// two-sweep matrix-core adjoint (G_k, H_k, ln L_t) and per mode class the FP64
// chain rule into grad
hipError_t mfma_backward(const MfmaArgs &a, const int *class_T, const int *class_K, const int *class_item0,
                         int n_classes, const int *mclass_M, const int *mclass_item0, const int64_t *mclass_tiles,
                         int n_mclasses, hipStream_t st, const Fanout &fo, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
// the stream of class c (0: the caller's) and the fork / join around a run
// of classes
inline hipStream_t fan_stream(const Fanout &fo, hipStream_t st, int c) {
  return (fo.n == 0 || c == 0) ? st : fo.side[(c - 1) % fo.n];
}
inline void fan_fork(const Fanout &fo, hipStream_t st, int n_classes) {
  if (fo.n == 0 || n_classes < 2) return;
  (void)hipEventRecord(fo.fork, st);
  for (int i = 0; i < fo.n && i < n_classes - 1; i++) (void)hipStreamWaitEvent(fo.side[i], fo.fork, 0);
}
inline void fan_join(const Fanout &fo, hipStream_t st, int n_classes) {
  if (fo.n == 0 || n_classes < 2) return;
  for (int i = 0; i < fo.n && i < n_classes - 1; i++) {
    (void)hipEventRecord(fo.join[i], fo.side[i]);
    (void)hipStreamWaitEvent(st, fo.join[i], 0);
  }
}
// FP64 re-evaluation of the adjoint over the window blocks that hold each
// sample's softmax mass (samples whose mass lies in at most kRefineBlocks
// blocks of 16 window samples, anywhere in the window); overwrites grad and
// lnL of those samples.  Launched after the
// chain rule on the same stream.
constexpr int kRefineBlocks = 3;
constexpr int kCtlRefine = 1 + kMaxClasses;  // ctl slot of the refinement count
constexpr float kRefineNats = 40.f;
hipError_t refine_backward(const MfmaArgs &a, hipStream_t st);
// the part both share: delay-bin sort, tile records, coefficient pass, work units
hipError_t mfma_prepare(const MfmaArgs &a, const int *mclass_M, const int *mclass_item0, const int64_t *mclass_tiles,
                        int n_mclasses, hipStream_t st);

// ---- sampler / reductions / adaptation -------------------------------------
// Proposal of one point: per parameter d in mask, either the 100-bin
// histogram (cdf) or, with gk > 0, a mixture of gk normals truncated to the
// prior-CDF coordinate's [0, 1] plus a uniform floor geps (gca = Phi(a),
// gz = Phi(b) - Phi(a) of each component; gntr samples fitted so far)
// Correlated pairs (npair of them, parameters pa < pb, disjoint, in mask):
// gk bivariate components in (u_a, u_b) (pcov: xx, xy, yy), drawn from the
// untruncated mixture and rejected outside the unit square; derived: pch
// (Cholesky l11, l21, l22), pic (inverse xx, xy, yy), plog (ln pi - ln 2 pi -
// ln det / 2), pzm (sum_k pi_k Z_k, Z_k the component's mass in the square).
constexpr int kMaxG = 4;
constexpr int kMaxPair = 3;
struct ProposalDev {
  double cdf[7][kNB + 1];
  unsigned mask;
  int gk;
  double geps, gntr;
  double gw[7][kMaxG], gmu[7][kMaxG], gsd[7][kMaxG], gca[7][kMaxG], gz[7][kMaxG];
  int npair;
  int pa[kMaxPair], pb[kMaxPair];
  int pad2_;
  double pw[kMaxPair][kMaxG], pmu[kMaxPair][kMaxG][2], pcov[kMaxPair][kMaxG][3];
  double pch[kMaxPair][kMaxG][3], pic[kMaxPair][kMaxG][3], plog[kMaxPair][kMaxG], pzm[kMaxPair];
};

// pt / pts: the point(s) whose network frame the sky is drawn in, or null for
// the equatorial coordinates; phase: polarization and orbital phase drawn in
// the phase-rotated coordinates (u_s, u_d)
template <typename R>
hipError_t sample_launch(const PointDev *pt, const ProposalDev *prop, int point, uint64_t seed, uint32_t round,
                         int64_t first, int64_t n, int64_t stride, int64_t bin_stride, double d_min, double d_max,
                         double tau_width, R *theta, R *ln_ratio, uint8_t *bins, hipStream_t st,
                         float *ubuf = nullptr, bool mix = true, bool phase = false);
// every point of a round in one launch (blk0: [np + 1] prefix of 256-sample
// blocks; off, cnt: columns and counts of each point; device arrays)
template <typename R>
hipError_t sample_multi_launch(const ProposalDev *props, const PointDev *pts, const int *blk0, int n_blocks, int np,
                               const int64_t *off,
                               const int64_t *cnt, uint64_t seed, uint32_t round, int64_t stride, int64_t bin_stride,
                               double d_min, double d_max, double tau_width, R *theta, R *ln_ratio, uint8_t *bins,
                               hipStream_t st, float *ubuf = nullptr, bool mix = true, bool phase = false);

struct ReduceTuple {
  double m, s1, s2;
  long long n, bad;
  double pad_;
};

// per-segment partial tuples: partials[seg * bps + j]
template <typename R>
hipError_t reduce_partials(const R *lnL, const R *ln_ratio, const int64_t *seg_off, const int64_t *seg_cnt,
                           int n_seg, int bps, ReduceTuple *partials, hipStream_t st);
// merge each segment's partials in order; round_out (or null) receives the
// segment tuple, accum (or null) is replaced by (accumulate ? accum + t : t),
// out (or null) receives the result of accum (or of t without accum)
hipError_t reduce_finish(const ReduceTuple *partials, int n_seg, int bps, ReduceTuple *round_out,
                         ReduceTuple *accum, int accumulate, rift_ile_result *out, hipStream_t st);

// gradient-informed refinement (k_grad.hip)
struct AscentState {
  double best_th[7];
  double best_g[7];
  double best_l;
  double eta;
};
template <typename R>
hipError_t ascent_select(const R *lnw, const R *theta, int64_t stride, const int64_t *seg_off, const int64_t *seg_cnt,
                         int n_seg, int k, int *idx, R *th_a, AscentState *st, hipStream_t s);
template <typename R>
hipError_t ascent_step(R *th_a, const R *grad, const R *lnl, AscentState *st, int n, unsigned mask, double d_min,
                       double d_max, double tw, hipStream_t s);
// pts: the points (one per segment) whose network sky frame the sky
// histograms use, or null for the equatorial coordinates
hipError_t ascent_hist(const AscentState *st, int k, int n_seg, unsigned mask, double d_min, double d_max, double tw,
                       const PointDev *pts, double *ahist, hipStream_t s);

// blocks per segment of the histogram pass (and partial histograms kept)
int hist_blocks(int64_t max_count);
// hist: [n_seg][bps][7][100] 64-bit partial histograms
template <typename R>
hipError_t adapt_launch(const uint8_t *bins, int64_t bin_stride, const R *lnw, const int64_t *seg_off,
                        const int64_t *seg_cnt, const int *seg_prop, int n_seg, int bps,
                        const ReduceTuple *seg_round, unsigned long long *hist, ProposalDev *props,
                        unsigned mask, double floor_eps, hipStream_t st, const double *ahist = nullptr,
                        double ascent_mix = 0.0);

// Gaussian-mixture adaptation of every segment's proposal from the round's
// prior-CDF coordinates ubuf [7][u_stride] (FP32) and ln w: n_iter weighted
// EM iterations from the current mixture (or the initial one when none is
// fitted yet, or its size differs from K), then the online update; part:
// scratch [n_seg][bps][7][kMaxG][3], fit: scratch [2 n_seg] mixtures (the
// current ones, then the EM iterates).
struct GmmDev {
  int k;
  int npair;
  double ntr;
  double w[7][kMaxG], mu[7][kMaxG], sd[7][kMaxG];
  int pa[kMaxPair], pb[kMaxPair];
  double pw[kMaxPair][kMaxG], pmu[kMaxPair][kMaxG][2], pcov[kMaxPair][kMaxG][3];
};
int em_blocks(int64_t max_count);
// pairs: byte i = a | b << 4 (a < b; 0: none); part2: scratch
// [n_seg][bps][kMaxPair][kMaxG][6]; blk0 [n_seg + 1]: prefix of 256-sample blocks
// per segment (wblk in all); wbuf: scratch, one double per sample
template <typename R>
hipError_t gmm_adapt_launch(const float *ubuf, int64_t u_stride, const R *lnw, const int64_t *seg_off,
                            const int64_t *seg_cnt, const int *seg_prop, int n_seg, int bps,
                            const ReduceTuple *seg_round, double *part, double *part2, GmmDev *fit,
                            ProposalDev *props, unsigned mask, unsigned pairs, double floor_eps, int K, int n_iter,
                            const int *blk0, int wblk, double *wbuf, hipStream_t st);
// host: component normalizations gca, gz of a mixture (Phi by erfc)
void gmm_norms(ProposalDev &p);
// derived pair quantities (pch, pic, plog, pzm) of props[p0 .. p0 + n - 1]
hipError_t pair_norm_launch(ProposalDev *props, int p0, int n, hipStream_t st);

hipError_t fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);

// Q/U/V of Eq. (QUV) from frequency-domain inputs, all pointers device
// memory: data [K][N] and modes [M][N] complex (interleaved), psd [K][N];
// X [K][M][N] complex scratch; Q [K][n_rows][M], U and V [K][M][M] complex.
// Ordered on st; returns hipErrorUnknown when the FFT library fails.
hipError_t quv_device(int K, int M, int64_t N, double df, double f_low, const double *data, const double *psd,
                      const double *modes, int64_t row0, int64_t n_rows, double *X, double *Q, double *U, double *V,
                      hipStream_t st);

}  // namespace rift
