// FP32 evaluation of ln L_t on the matrix cores (gfx950).
//
// The data term of App. D Eq. (def:lnL:Decomposed), summed over the window,
// needs for every sample s and detector k the real contraction
//     z_k[r](s) = Re sum_m conj(a_{k,m}(s)) Q_k[r][m]
// over the rows r its arrival time selects.  Over a common run of rows for a
// tile of samples this is a dense product
//     Z_k = Qr_k (rows x 2M) * A_k (2M x samples)
// with the real and imaginary parts of Q and a as the inner dimension, so it
// runs as v_mfma_f32_16x16x4f32 (16 rows x 16 samples per instruction).  The
// rows a sample needs depend on its own delay, so samples are first sorted
// into bins of equal integer delay (per detector, bins of 14 rows); a tile
// holds 16 samples of one bin, whose windows then start within 13 rows of
// each other and share one run of rows (about 3% more rows than the window
// needs at n_t = 820).  Bins are padded to whole tiles, so tile t is sorted
// slots [16 t, 16 t + 16).
//
// Kernels, in launch order:
//   bin_kernel    integer delays n_k, bin key, per-sort-block bin counts
//   colscan       per point: offset of each sort block in each bin
//   tilescan      per point: tiles and work units before each bin
//   item_scan     tiles and units before each point; per-class counters reset
//   scatter       a 40-byte record (theta, column, n_k) at the sorted slot
//   tile_item     point of every tile
//   unit_kernel   the work units: up to 4 tiles of one bin each
//   coef_kernel   one thread per slot, FP64: antenna patterns, harmonics
//                 (polynomial tables), Y_m (rounded to FP32) and x F_k, the
//                 quadratic term B, and the interpolation fraction mu_k
//   mfma_kernel<T,K,DIRECT> persistent, one unit per workgroup, one tile per
//                 wavefront: forms its B operands a_km = x F_k Y_m, walks the
//                 rows in 16-row blocks (T MFMAs per detector and block, the
//                 A operands staged through LDS or loaded directly, per class)
//                 -> a ring of z in LDS -> Catmull-Rom interpolation of the
//                 window samples whose stencils are complete -> a lazy
//                 max-shifted base-2 log-sum-exp.  ell_j never leaves
//                 registers.
#include "common.h"
#include "dmarg.h"
#include "internal.h"
#include "mfma_tile.h"

#include <algorithm>

namespace rift {

// z ring of a detector: 48 logical rows (two 16-row slots and slot 0 again)
// of 16 samples, stored row-major with one pad row after every 4: logical
// row r sits at physical row 5 (r >> 2) + (r & 3), sample s at column s.
// A window read takes 7 consecutive logical rows from r = 4 g + sh_k for
// each lane (g the lane's row group, sh_k its sample's shift): lanes of
// different samples differ in the column's bank, and the two row groups of a
// half-wavefront (4 logical rows apart, 5 physical) differ in the row's
// parity, so the reads are free of bank conflicts whatever the shifts.
// Logical rows 0..47 occupy physical rows 0..58 (the pad after row 47 is
// never stored), which keeps the staged K = 3, T <= 3 instances within a
// third of a compute unit's LDS.
constexpr int kRR = 59;
constexpr int kSortThreads = 1024;  // threads per sort block (kSortBlock samples)
static_assert(kSortBlock % kSortThreads == 0, "a whole number of samples per sort thread");

__device__ __forceinline__ int item_of_flat(const ItemsDev &it, int64_t f) {
  int lo = 0, hi = it.n_items;  // samp0[lo] <= f < samp0[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (it.samp0[mid] <= f) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int item_of_bin(const ItemsDev &it, int b) {
  int lo = 0, hi = it.n_items;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (it.bin0[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

// ---- 1. integer delays, bin keys, per-block bin counts ----------------------
// A sort block is kSortBlock consecutive samples of one point.  Counts go to an
// LDS histogram (the point's bins), then to the block's row of the global
// block histogram; no global atomics, so no contention on busy bins.
__device__ __forceinline__ int block_item(const ItemsDev &it, int b) {
  int lo = 0, hi = it.n_items;  // blk0[lo] <= b < blk0[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (it.blk0[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(kSortThreads) bin_kernel(MfmaArgs a) {
  extern __shared__ uint32_t cnt_l[];
  const int it = block_item(a.items, blockIdx.x);
  const int lb = blockIdx.x - a.items.blk0[it];
  const PointDev &p = a.pts[a.items.point[it]];
  const int nb = a.items.bin0[it + 1] - a.items.bin0[it];
  const bool lds = nb <= kLdsBins;
  uint32_t *cnt = lds ? cnt_l : a.bhist + a.items.hoff[it] + (int64_t)lb * nb;
  for (int i = threadIdx.x; i < nb; i += kSortThreads) cnt[i] = 0u;
  __syncthreads();
  const int64_t n = a.items.cnt[it];
  const int64_t j0 = (int64_t)lb * kSortBlock, j1 = min(n, j0 + kSortBlock);
  // the sort block's samples, kSortBlock / kSortThreads per thread: all
  // their parameters are loaded before any is used, so the loads of a
  // thread's samples are in flight together
  constexpr int U = kSortBlock / kSortThreads;
  float th[U][7];
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int64_t j = j0 + threadIdx.x + (int64_t)u * kSortThreads;
    const int64_t col = a.items.off[it] + (j < j1 ? j : j0);
#pragma unroll
    for (int d = 0; d < 7; d++) th[u][d] = a.theta[d * a.stride + col];
  }
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int64_t j = j0 + threadIdx.x + (int64_t)u * kSortThreads;
    if (j >= j1) break;
    const int64_t f = a.items.samp0[it] + j;
    const double al = th[u][RIFT_ALPHA], de = th[u][RIFT_DELTA], io = th[u][RIFT_IOTA], ph = th[u][RIFT_PHI];
    const double di = th[u][RIFT_DIST], ta = th[u][RIFT_TAU];
    SkyTrig tr = sky_trig(al, de, 0.0, p.gmst);
    Shift sh = shifts(p, tr, ta);
    bool ok = sh.ok && isfinite(io) && isfinite(ph) && (a.dmarg || (isfinite(di) && di > 0.0)) &&
              isfinite((double)th[u][RIFT_PSI]);
    uint32_t key = 0, mul = 1;
    uint32_t nw[2] = {0u, ok ? 1u << 16 : 0u};  // the four int16 of the sample, one 8-byte store
    for (int k = 0; k < p.K; k++) {
      int q = ok ? (sh.n[k] + p.pad) / p.bin_w : 0;
      key += q * mul;
      mul *= p.nq;
      const uint32_t v = (uint16_t)(int16_t)(ok ? sh.n[k] : 0);
      nw[k >> 1] |= (k & 1) ? v << 16 : v;
    }
    *(uint2 *)(a.nsh + f * 4) = make_uint2(nw[0], nw[1]);
    a.key[f] = key;
    atomicAdd(&cnt[key], 1u);
  }
  __syncthreads();
  if (lds) {
    uint32_t *row = a.bhist + a.items.hoff[it] + (int64_t)lb * nb;
    for (int i = threadIdx.x; i < nb; i += kSortThreads) row[i] = cnt_l[i];
  }
}

// ---- 2. per-item scans: block offsets within each bin, tiles before each bin --
// Column scan of the [sort block][bin] histogram of one point: a workgroup
// takes 64 bins; its 16 wavefronts each sum a sixteenth of the sort blocks,
// then rewrite their share as running offsets.  Reads are coalesced along
// the bins, and every point's bins are spread over many workgroups.
constexpr int kScanBins = 64;
constexpr int kScanRanges = 16;  // block ranges per column scan: 1024 threads

__global__ void __launch_bounds__(kScanRanges * kScanBins) colscan_kernel(MfmaArgs a) {
  __shared__ uint32_t part[kScanRanges][kScanBins];
  const int q = threadIdx.x >> 6, bl = threadIdx.x & 63;
  for (int it = blockIdx.y; it < a.items.n_items; it += gridDim.y) {
    const int b0 = a.items.bin0[it], nb = a.items.bin0[it + 1] - b0;
    if ((int)blockIdx.x * kScanBins >= nb) continue;  // uniform over the workgroup
    const int nblk = a.items.blk0[it + 1] - a.items.blk0[it];
    const int lb_per = (nblk + kScanRanges - 1) / kScanRanges;
    const int b = (int)blockIdx.x * kScanBins + bl;
    const int lo = min(nblk, q * lb_per), hi = min(nblk, lo + lb_per);
    uint32_t *h = a.bhist + a.items.hoff[it];
    uint32_t sum = 0;
    if (b < nb)
      for (int lb = lo; lb < hi; lb++) sum += h[(int64_t)lb * nb + b];
    __syncthreads();  // part[] of the previous item fully read
    part[q][bl] = sum;
    __syncthreads();
    uint32_t run = 0;
    for (int i = 0; i < q; i++) run += part[i][bl];
    if (b < nb) {
      for (int lb = lo; lb < hi; lb++) {
        const uint32_t v = h[(int64_t)lb * nb + b];
        h[(int64_t)lb * nb + b] = run;
        run += v;
      }
      if (q == kScanRanges - 1) a.count[b0 + b] = run;
    }
  }
}

// tiles of each bin (bins padded to whole tiles), work units of each bin
// (groups of up to 4 of its tiles), and their prefixes per point
__global__ void __launch_bounds__(256) tilescan_kernel(MfmaArgs a) {
  __shared__ uint32_t pt[256], pu[256];
  const int it = blockIdx.x;
  const int b0 = a.items.bin0[it], nb = a.items.bin0[it + 1] - b0;
  const int per = (nb + 255) / 256;
  const int lo = min(nb, (int)threadIdx.x * per), hi = min(nb, lo + per);
  uint32_t ct = 0, cu = 0;
  for (int b = lo; b < hi; b++) {
    const uint32_t tb = (a.count[b0 + b] + kTS - 1) / kTS;
    ct += tb;
    cu += (tb + 3) / 4;
  }
  pt[threadIdx.x] = ct;
  pu[threadIdx.x] = cu;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t rt = 0, ru = 0;
    for (int i = 0; i < 256; i++) {
      uint32_t y = pt[i], z = pu[i];
      pt[i] = rt;
      pu[i] = ru;
      rt += y;
      ru += z;
    }
    a.item_tiles[it + 1] = (rt + 3u) & ~3u;  // whole groups of 4 tiles per point
    a.item_units[it + 1] = ru;
  }
  __syncthreads();
  uint32_t rt = pt[threadIdx.x], ru = pu[threadIdx.x];
  for (int b = lo; b < hi; b++) {
    const uint32_t tb = (a.count[b0 + b] + kTS - 1) / kTS;
    a.bin_tile[b0 + b] = rt;
    a.bin_unit[b0 + b] = ru;
    rt += tb;
    ru += (tb + 3) / 4;
  }
}

// prefix of tiles over items (one thread); reset of the per-class counters
__global__ void item_scan_kernel(MfmaArgs a) {
  if (threadIdx.x == 0) {
    uint32_t r = 0;
    a.item_tiles[0] = 0;
    for (int i = 0; i < a.items.n_items; i++) {
      r += a.item_tiles[i + 1];
      a.item_tiles[i + 1] = r;
    }
    a.ctl[0] = r;
    for (int c = 0; c < kMaxClasses; c++) a.ctl[1 + c] = 0;
    a.ctl[kCtlRefine] = 0;
    uint32_t u = 0;
    a.item_units[0] = 0;
    for (int i = 0; i < a.items.n_items; i++) {
      u += a.item_units[i + 1];
      a.item_units[i + 1] = u;
    }
    // coefficient storage: K 2Mp 16 floats per tile of each point
    int64_t c = 0;
    for (int i = 0; i < a.items.n_items; i++) {
      a.item_cop[i] = c;
      const PointDev &p = a.pts[a.items.point[i]];
      c += (int64_t)(a.item_tiles[i + 1] - a.item_tiles[i]) * p.K * 2 * p.Mp * kTS;
    }
  }
}

// ---- 3. scatter: one record per sample at its (padded) sorted slot ------------
__global__ void __launch_bounds__(kSortThreads) scatter_kernel(MfmaArgs a) {
  extern __shared__ uint32_t cur_l[];
  const int it = block_item(a.items, blockIdx.x);
  const int lb = blockIdx.x - a.items.blk0[it];
  const int b0 = a.items.bin0[it], nb = a.items.bin0[it + 1] - b0;
  const bool lds = nb <= kLdsBins;
  uint32_t *cur = lds ? cur_l : a.bhist + a.items.hoff[it] + (int64_t)lb * nb;
  if (lds) {
    const uint32_t *row = a.bhist + a.items.hoff[it] + (int64_t)lb * nb;
    for (int i = threadIdx.x; i < nb; i += kSortThreads) cur_l[i] = row[i];
  }
  __syncthreads();
  const int64_t n = a.items.cnt[it];
  const int64_t j0 = (int64_t)lb * kSortBlock, j1 = min(n, j0 + kSortBlock);
  const uint32_t tbase = a.item_tiles[it];
  // kSortBlock / kSortThreads samples per thread, their loads issued together
  constexpr int U = kSortBlock / kSortThreads;
  SampleRec rec[U];
  uint32_t key[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int64_t jj = j0 + threadIdx.x + (int64_t)u * kSortThreads, j = jj < j1 ? jj : j0;
    const int64_t f = a.items.samp0[it] + j;
    const int64_t col = a.items.off[it] + j;
    key[u] = a.key[f];
#pragma unroll
    for (int d = 0; d < 7; d++) rec[u].th[d] = a.theta[d * a.stride + col];
    rec[u].col = (int)col;
    const uint2 nw = *(const uint2 *)(a.nsh + f * 4);
    rec[u].n[0] = (int16_t)(nw.x & 0xffffu);
    rec[u].n[1] = (int16_t)(nw.x >> 16);
    rec[u].n[2] = (int16_t)(nw.y & 0xffffu);
    rec[u].flag = (nw.y >> 16) ? 1 : 2;
  }
#pragma unroll
  for (int u = 0; u < U; u++) {
    if (j0 + threadIdx.x + (int64_t)u * kSortThreads >= j1) break;
    const uint32_t r = atomicAdd(&cur[key[u]], 1u);
    a.rec[kTS * (tbase + a.bin_tile[b0 + key[u]]) + r] = rec[u];
  }
}

// point of every tile (tiles of a point are contiguous)
__global__ void __launch_bounds__(256) tile_item_kernel(MfmaArgs a) {
  int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.ctl[0]) return;
  int lo = 0, hi = a.items.n_items;  // item_tiles[lo] <= t < item_tiles[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (a.item_tiles[mid] <= t) lo = mid; else hi = mid;
  }
  a.tile_item[t] = lo;
}

// work units of every bin: consecutive runs of up to 4 of its tiles.  Also
// the padding slots (flag 0): the rest of the bin's last tile and, for the
// last bin of a point, the tiles that round the point up to groups of 4; the
// scatter fills every other slot of the point's tiles.
__global__ void __launch_bounds__(64) unit_kernel(MfmaArgs a) {
  const int g = blockIdx.x * 64 + threadIdx.x;
  if (g >= a.n_bins) return;
  const int it = item_of_bin(a.items, g);
  const uint32_t cnt = a.count[g];
  const uint32_t tb = (cnt + kTS - 1) / kTS;
  const uint32_t t0 = a.item_tiles[it] + a.bin_tile[g], u0 = a.item_units[it] + a.bin_unit[g];
  for (uint32_t c = 0; 4 * c < tb; c++) {
    WorkUnit w;
    w.tile = t0 + 4 * c;
    w.ntiles = min(4u, tb - 4 * c);
    w.key = (uint32_t)(g - a.items.bin0[it]);
    a.unit[u0 + c] = w;
  }
  SampleRec z;
  for (int d = 0; d < 7; d++) z.th[d] = 0.f;
  z.col = 0;
  z.n[0] = z.n[1] = z.n[2] = 0;
  z.flag = 0;
  const int64_t s0 = (int64_t)kTS * t0;
  int64_t s1 = s0 + (int64_t)kTS * tb;
  if (g == a.items.bin0[it + 1] - 1) s1 = (int64_t)kTS * a.item_tiles[it + 1];
  for (int64_t q = s0 + cnt; q < s1; q++) a.rec[q] = z;
}

// ---- 4. per-sample coefficients (FP64), tile-major ---------------------------
// Quadratic term with the Hermitian (U) and symmetric (V) packing of the
// host: q_k = Y^dag U_k Y = sum_{m <= m'} Re(conj(Y_m) c_{mm'} Y_m'),
// t_k = Y^T V_k Y = sum_{m <= m'} c'_{mm'} Y_m Y_m', with the off-diagonal
// factor 2 folded into c, c'; B = x^2/4 sum_k [|F_k|^2 q_k + Re(F_k^2 t_k)].
// A block is 4 whole tiles of one point, so the point's constants are read
// through the constant address space (scalar loads) and every branch on them
// is uniform.  The packed tables are zero for detectors past K and F_k = 0
// there, so the pair sums run over all kMaxDet detectors without branches.
// Per tile the pass stores Y_m (2 M_p floats per sample, shared by the
// detectors) and x F_k (in the tile record); the evaluation kernels form the
// B operands a_km = x F_k Y_m themselves.
// Harmonics use the polynomial form of the host tables (Horner in
// u = cos^2(iota/2)).  MC > 0: the mode count is a compile-time constant, Y
// lives in registers and the pair sums unroll (table values as scalar
// operands).  MC = 0 is the general form, with Y staged in LDS and the sums
// in loops; points with a V table always take it (the host gives them
// classes of their own: a second unrolled pass would keep every mode product
// of the first alive).  Padding and invalid slots run the same code on a
// harmless angle set and store zeros.
template <int MC>
__global__ void __launch_bounds__(64) coef_kernel(MfmaArgs a, int item_lo, int item_hi) {
  constexpr int YS = MC > 0 ? 1 : 64;
  constexpr int YM = MC > 0 ? 1 : kMaxModes;
  constexpr int YR = MC > 0 ? MC : 1;
  __shared__ double Ys[YS][YM][2];
  const int64_t t_lo = a.item_tiles[item_lo], t_hi = a.item_tiles[item_hi];
  const int64_t t_blk = t_lo + 4 * (int64_t)blockIdx.x;
  if (t_blk >= t_hi) return;  // whole block (items hold whole blocks of 4 tiles)
  const int64_t pos = t_blk * kTS + threadIdx.x;
  const int64_t t = pos / kTS;
  const int s = (int)(pos % kTS);
  const SampleRec rec = a.rec[pos];
  const int it = __builtin_amdgcn_readfirstlane(a.tile_item[t_blk]);
  const int pt = __builtin_amdgcn_readfirstlane(a.items.point[it]);
  const RIFT_CONST PointDev &p = *cp(a.pts + pt);
  const int K = p.K, E = 2 * p.Mp;
  const int M = MC > 0 ? MC : p.M;
  RIFT_GLOBAL float *op = gpw(a.cop + a.item_cop[it] + (int64_t)(t - a.item_tiles[it]) * K * E * kTS + s);
  RIFT_GLOBAL CoefTile *ct = gpw(a.ctile + t);
  const bool pad = rec.flag == 0;
  const bool valid = rec.flag == 1;
  double th[7];
#pragma unroll
  for (int d = 0; d < 7; d++) th[d] = valid ? (double)rec.th[d] : (d == RIFT_DIST ? 1.0 : 0.0);
  const double x = a.dmarg ? 1.0 : p.d_ref / th[RIFT_DIST];  // distance marginalization: the terms at D_ref
  const double xl = valid ? x * kLog2e : 0.0;
  SkyTrig tr = sky_trig(th[RIFT_ALPHA], th[RIFT_DELTA], th[RIFT_PSI], p.gmst);
  double Fr[kMaxDet], Fi[kMaxDet];
#pragma unroll
  for (int k = 0; k < kMaxDet; k++) {
    Fr[k] = Fi[k] = 0.0;
    if (k < K) {
      double D[9], rc[3];
#pragma unroll
      for (int i = 0; i < 9; i++) D[i] = p.D[k][i];
#pragma unroll
      for (int i = 0; i < 3; i++) rc[i] = p.rc[k][i];
      antenna(D, tr, Fr[k], Fi[k]);
      const int n = (int)rec.n[k];
      const double sk = (th[RIFT_TAU] + delay(rc, tr)) * p.f_s;
      ct->mu[k][s] = valid ? (float)(sk - (double)n) : 0.f;
      ct->n[k][s] = valid ? n : 1 << 28;
    } else {
      ct->mu[k][s] = 0.f;
      ct->n[k][s] = 1 << 28;
    }
    // in base-2 units (times log2 e) for the evaluation kernel's exp2/log2
    ct->xf[k][0][s] = (float)(xl * Fr[k]);
    ct->xf[k][1][s] = (float)(xl * Fi[k]);
  }
  // harmonics: Y_m = (sin(iota)/2)^par P_m(cos^2(iota/2)) exp(i m phi), with
  // exp(i m phi) by repeated products of exp(i phi)
  double ci, si, c1, s1;
  sincos(0.5 * th[RIFT_IOTA], &si, &ci);
  sincos(th[RIFT_PHI], &s1, &c1);
  const double u = ci * ci, hs = si * ci;
  double Yr[YR], Yi[YR];
  double (*Yl)[2] = Ys[MC > 0 ? 0 : threadIdx.x];
#pragma unroll
  for (int m = 0; m < (MC > 0 ? MC : kMaxModes); m++) {
    if (m >= M) break;
    double yr, yi;
    harmonic_ym(p, m, u, hs, c1, s1, yr, yi);
    if constexpr (MC > 0) {
      Yr[m] = yr;
      Yi[m] = yi;
    } else {
      Yl[m][0] = yr;
      Yl[m][1] = yi;
    }
    // elements 2m, 2m + 1 of the tile's harmonic block; the evaluation
    // kernels form a_km = (x F_k) Y_m from it and xf
    op[(2 * m) * kTS] = valid ? (float)yr : 0.f;
    op[(2 * m + 1) * kTS] = valid ? (float)yi : 0.f;
  }
  for (int e = 2 * M; e < E; e++) op[e * kTS] = 0.f;
  double q[kMaxDet] = {0.0, 0.0, 0.0}, vr[kMaxDet] = {0.0, 0.0, 0.0}, vi[kMaxDet] = {0.0, 0.0, 0.0};
  // conj(Y_m) Y_m' against U, Y_m Y_m' against V
  auto upair = [&](const auto *T, int idx, double ymr, double ymi, double ypr, double ypi) {
    const double pr = ymr * ypr + ymi * ypi, pi = ymr * ypi - ymi * ypr;
#pragma unroll
    for (int k = 0; k < kMaxDet; k++) {
      const double ur = T[(idx * kMaxDet + k) * 2], ui = T[(idx * kMaxDet + k) * 2 + 1];
      q[k] = fma(-ui, pi, fma(ur, pr, q[k]));
    }
    // unrolled: one wait per four pairs of table loads
    if ((idx & 3) == 3) __builtin_amdgcn_sched_barrier(0);
  };
  auto vpair = [&](const auto *T, int idx, double ymr, double ymi, double ypr, double ypi) {
    const double sr = ymr * ypr - ymi * ypi, s_i = ymr * ypi + ymi * ypr;
#pragma unroll
    for (int k = 0; k < kMaxDet; k++) {
      const double wr = T[(idx * kMaxDet + k) * 2], wi = T[(idx * kMaxDet + k) * 2 + 1];
      vr[k] = fma(-wi, s_i, fma(wr, sr, vr[k]));
      vi[k] = fma(wi, sr, fma(wr, s_i, vi[k]));
    }
  };
  const RIFT_CONST double *Uq = cp(p.Upk);
  if constexpr (MC > 0) {
#pragma unroll
    for (int m = 0; m < MC; m++)
#pragma unroll
      for (int mp = m; mp < MC; mp++) upair(Uq, m * MC - m * (m - 1) / 2 + (mp - m), Yr[m], Yi[m], Yr[mp], Yi[mp]);
  } else {
    int idx = 0;
    for (int m = 0; m < M; m++)
      for (int mp = m; mp < M; mp++, idx++) upair(Uq, idx, Yl[m][0], Yl[m][1], Yl[mp][0], Yl[mp][1]);
    if (p.Vpk) {
      const RIFT_CONST double *Vq = cp(p.Vpk);
      idx = 0;
      for (int m = 0; m < M; m++)
        for (int mp = m; mp < M; mp++, idx++) vpair(Vq, idx, Yl[m][0], Yl[m][1], Yl[mp][0], Yl[mp][1]);
    }
  }
  double b = 0.0;
#pragma unroll
  for (int k = 0; k < kMaxDet; k++) {
    const double f2 = Fr[k] * Fr[k] + Fi[k] * Fi[k];
    const double F2r = Fr[k] * Fr[k] - Fi[k] * Fi[k], F2i = 2.0 * Fr[k] * Fi[k];
    b += f2 * q[k] + (F2r * vr[k] - F2i * vi[k]);
  }
  ct->B[s] = valid ? (float)(0.25 * x * x * b * kLog2e) : 0.f;
  ct->col[s] = pad ? -1 : (int)rec.col;
  ct->flag[s] = valid ? 1 : (pad ? 0 : 2);
}

// ---- 5. persistent MFMA evaluation ------------------------------------------
// One workgroup per work unit: its four wavefronts take the unit's tiles.
// Base row of detector k: the lower edge of the unit's delay bin, so every
// sample's stencil starts 0..bin_w-1 rows above it.  Two ways to feed the
// matrix cores, chosen per (T, K) class by measurement:
//  * staged (DIRECT = false): the rows of blocks b, b + 1 of every detector
//    are loaded once per workgroup, coalesced, into a 4-slot LDS stage (one
//    barrier per two blocks); each wavefront reads its A operands from there
//    (wavefronts past ntiles only help stage);
//  * direct (DIRECT = true): each wavefront loads its own A operands from
//    global memory one block ahead (the four wavefronts of a unit read the
//    same rows, so three of the four reads hit in L1), with no stage and no
//    barrier between blocks; less LDS, so more workgroups per compute unit.
// MODE 0: ln L_t.  Distance marginalization (coefficients at D = D_ref, so
// the window values are the data terms A_j, base 2): MODE 1 writes each
// slot's largest A_j; MODE 2 reads it back, places the slot's nodes x_i over
// D (dmarg.h) and sums exp2(x_i (A_j - A_max)) per node over the window,
// skipping window samples where even the smallest node's term is below
// 2^-(T + 10) log2 e (their n_t terms together are far under the rule's
// error), then combines the nodes in FP64.  Both passes recompute the same
// window values bit for bit.
// WPE: wavefronts per SIMD the register allocation must allow (1: no cap;
// the capped direct forms are extra configurations for the autotuner)
template <int T, int K, bool DIRECT, int MODE, int WPE = 1>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) mfma_kernel(MfmaArgs a, int item_lo,
                                                                                         int item_hi, int cls) {
  constexpr int E = 4 * T, J = T / 4, R = T % 4;
  constexpr int JA = J > 0 ? J : 1, RA = R > 0 ? R : 1;
  constexpr int ES = stage_stride<T>();
  constexpr int SF = K * kTS * ES;  // floats of one staged block
  __shared__ __align__(16) float ring_all[kWaves * K * kRR * kTS];
  __shared__ __align__(16) float stage[DIRECT ? 1 : 4][DIRECT ? 4 : SF];  // staged: block b in slot b % 4
  __shared__ WorkUnit unit_sh;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float *ring = ring_all + wave * (K * kRR * kTS);  // [det][physical row][sample]
  const int s = lane & 15, g = lane >> 4;
  const uint32_t u_lo = a.item_units[item_lo], u_hi = a.item_units[item_hi];
  // staging: thread i < 16 T copies 16-byte group i of the 16 rows x 4 T
  // floats of a detector's block (row i / T, group i % T)
  const int tid = threadIdx.x;
  const bool st_on = tid < 16 * T;
  const uint32_t st_goff = 16u * (uint32_t)tid;                         // bytes into the block
  const int st_loff = (tid / T) * ES + 4 * (tid % T);                   // floats into the stage
  // direct: lane (s, g) reads row s of a block, quads at 64 j + 16 g bytes,
  // tails at 64 J + 16 r + 4 g
  const uint32_t a_row = (uint32_t)(4 * E) * (uint32_t)s;

  for (;;) {
    if constexpr (DIRECT) __syncthreads();  // every wavefront is done with the previous unit
    if (tid == 0) {
      const uint32_t u = u_lo + atomicAdd(&a.ctl[1 + cls], 1u);
      WorkUnit w;
      if (u < u_hi) {
        w = a.unit[u];
      } else {
        w.tile = 0xffffffffu;
        w.ntiles = 0;
        w.key = 0;
      }
      unit_sh = w;
    }
    __syncthreads();
    const uint32_t t0 = __builtin_amdgcn_readfirstlane(unit_sh.tile);
    const int ntiles = __builtin_amdgcn_readfirstlane(unit_sh.ntiles);
    uint32_t key = __builtin_amdgcn_readfirstlane(unit_sh.key);
    if (t0 == 0xffffffffu) break;  // the same for the whole workgroup
    const bool active = wave < ntiles;
    const uint32_t t = t0 + (active ? wave : 0);
    const int it = __builtin_amdgcn_readfirstlane(a.tile_item[t0]);
    const PointDev &p = a.pts[a.items.point[it]];
    const int NT = p.n_t, P = p.pad, Lpad = p.Lpad;
    // detector k of the bin: key digit q_k; lowest integer delay of the bin
    const RIFT_GLOBAL float *qk[K];
    int lo_k[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int q = (int)(key % (uint32_t)p.nq);
      key /= (uint32_t)p.nq;
      lo_k[k] = q * p.bin_w - P;
      qk[k] = gp(uniform_ptr(p.Qm + (size_t)(k * Lpad + P + lo_k[k]) * E));
    }
    const RIFT_GLOBAL CoefTile *ct = gp(a.ctile + t);
    const int flag = active ? ct->flag[s] : 0;
    const int col = ct->col[s];
    const float Bf = active ? ct->B[s] : 0.f;
    const RIFT_GLOBAL float *yop = gp(a.cop + a.item_cop[it] + (int64_t)(t - a.item_tiles[it]) * K * E * kTS + s);
    float Bop[K][T];
    b_operands<T, K>(yop, ct, s, g, active, Bop);
    float w[K][4];
    int sh[K];
    bool valid = flag == 1;
#pragma unroll
    for (int k = 0; k < K; k++) {
      cr_weights<float>(ct->mu[k][s], w[k]);
      sh[k] = valid ? ct->n[k][s] - lo_k[k] : 0;
      if (sh[k] < 0 || sh[k] > kTS - 3) {
        valid = false;
        sh[k] = 0;
      }
    }
    const int JB = (NT + 15) >> 4;
    // z ring: block b in logical rows 16 (b % 2) .. + 15 (slot 0 also in rows
    // 32..47), so the 7 rows a window read needs are consecutive.  Read o of
    // a lane sits 16 (o + ((c + o) >> 2)) floats past its first, c = sh_k & 3:
    // 0, 16 + e3, 32 + e2, 48 + e1, 80, 96 + e3, 112 + e2 with e_i = 16 [c >= i],
    // so four position registers per detector (zb: + 0, e3, e2, e1) and the
    // rest as instruction offsets; slot 1 is 20 physical rows further
    int zb[K][4];
#pragma unroll
    for (int k = 0; k < K; k++) {
      const int c = sh[k] & 3;
      const int b0 = k * kRR * kTS + kTS * (5 * g + sh[k] + (sh[k] >> 2)) + s;
      zb[k][0] = b0;
      zb[k][1] = b0 + (c >= 3 ? kTS : 0);
      zb[k][2] = b0 + (c >= 2 ? kTS : 0);
      zb[k][3] = b0 + (c >= 1 ? kTS : 0);
    }
    float *const wz = ring + kTS * (5 * g) + s;
    const float *const sa = &stage[0][s * ES + 4 * g];       // this lane's quads in slot 0
    const float *const st = &stage[0][s * ES + 16 * J + g];  // and the rest
    const int rem = NT - 16 * (JB - 1);
    float last_pen[4];  // -inf for window samples past n_t in the last block
#pragma unroll
    for (int i = 0; i < 4; i++) last_pen[i] = (4 * g + i < rem) ? 0.f : -INFINITY;

    f4 pre[2][K];
    // global loads of blocks b and b + 1 (clamped to the last block)
    auto stage_load2 = [&](int b) {
      if (st_on) {
#pragma unroll
        for (int hb = 0; hb < 2; hb++) {
          const uint32_t ob = (uint32_t)(64 * E) * (uint32_t)min(b + hb, JB) + st_goff;
#pragma unroll
          for (int k = 0; k < K; k++) pre[hb][k] = *(const RIFT_GLOBAL f4 *)((const RIFT_GLOBAL char *)qk[k] + ob);
        }
      }
    };
    auto stage_store2 = [&](auto slot_c) {
      constexpr int S0 = decltype(slot_c)::value;
      if (st_on) {
#pragma unroll
        for (int hb = 0; hb < 2; hb++)
#pragma unroll
          for (int k = 0; k < K; k++) *(f4 *)(&stage[(S0 + hb) & 3][k * kTS * ES + st_loff]) = pre[hb][k];
      }
    };
    // direct: A operands of blocks in two register sets, one block ahead
    f4 Ad[2][K][JA];
    float Atd[2][K][RA];
    auto load_a = [&](auto buf_c, int b) {
      constexpr int BF = decltype(buf_c)::value;
      const uint32_t ob = (uint32_t)(64 * E) * (uint32_t)min(b, JB) + a_row;
#pragma unroll
      for (int k = 0; k < K; k++) {
        const RIFT_GLOBAL char *base = (const RIFT_GLOBAL char *)qk[k] + ob;
#pragma unroll
        for (int j = 0; j < J; j++) Ad[BF][k][j] = *(const RIFT_GLOBAL f4 *)(base + 64 * j + 16 * g);
#pragma unroll
        for (int r = 0; r < R; r++) Atd[BF][k][r] = *(const RIFT_GLOBAL float *)(base + 64 * J + 16 * r + 4 * g);
      }
    };
    // the block in stage slot S4 (staged) or register set S4 % 2 (direct) on
    // the matrix cores; z_k[base + 16 b + 4 g + v] of sample s -> ring slot S4 % 2
    auto product = [&](auto s4_c) {
      constexpr int S4 = decltype(s4_c)::value;
      f4 Aq[K][JA];
      float At[K][RA];
      if constexpr (DIRECT) {
#pragma unroll
        for (int k = 0; k < K; k++) {
#pragma unroll
          for (int j = 0; j < JA; j++) Aq[k][j] = Ad[S4 & 1][k][j];
#pragma unroll
          for (int r = 0; r < RA; r++) At[k][r] = Atd[S4 & 1][k][r];
        }
      } else {
        const float *sb = sa + S4 * SF;
#pragma unroll
        for (int k = 0; k < K; k++) {
#pragma unroll
          for (int j = 0; j < J; j++) Aq[k][j] = *(const f4 *)(sb + k * kTS * ES + 16 * j);
#pragma unroll
          for (int r = 0; r < R; r++) At[k][r] = st[S4 * SF + k * kTS * ES + 4 * r];
        }
      }
      f4 acc[K];
#pragma unroll
      for (int tt = 0; tt < T; tt++)
#pragma unroll
        for (int k = 0; k < K; k++) {
          const float av = tt < 4 * J ? Aq[k][tt < 4 * J ? tt >> 2 : 0][tt & 3] : At[k][tt < 4 * J ? 0 : tt - 4 * J];
          acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, Bop[k][tt], tt == 0 ? f4{0.f, 0.f, 0.f, 0.f} : acc[k], 0,
                                                        0, 0);
        }
#pragma unroll
      for (int k = 0; k < K; k++) {
#pragma unroll
        for (int i = 0; i < 4; i++) {
          wz[k * kRR * kTS + kTS * (20 * (S4 & 1) + i)] = acc[k][i];
          if constexpr ((S4 & 1) == 0) wz[k * kRR * kTS + kTS * (40 + i)] = acc[k][i];
        }
      }
    };
    // window samples 16 c + 4 g + i (i < 4) of the block in ring slot SL:
    // interpolation, then the log-sum-exp with a lazy reference m_run: sums
    // are kept as exp2(ell + B - m_run), m_run is the first block's maximum
    // and moves only when a value exceeds it by 64, which keeps every sum far
    // from overflow while terms lost below it are under 2^-126 of the sum.
    // The quadratic term B is the same for every window sample, so it stays
    // out of the sums and is subtracted once at the end: the window values
    // then carry the rounding of the data term only, not of B.
    float m_run = 0.f, s_run = 0.f;
    // distance marginalization: the slot's A_max (MODE 2 reads it), its
    // nodes and per-node sums
    constexpr int NQ = MODE == 2 ? kDmGL : 1;
    float am = MODE == 1 ? -INFINITY : 0.f, skip = INFINITY;
    double ta = 0.0, hq = 0.0;  // the nodes' interval in t = ln x
    float xs[NQ], Sq[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) xs[q] = Sq[q] = 0.f;
    if constexpr (MODE == 2) {
      const float av = active ? a.amax[(int64_t)t * kTS + s] : 0.f;
      if (valid && isfinite(av)) {
        am = av;
        // the interval is searched in FP32; an end at the prior's edge takes
        // the edge's FP64 value, so a range much narrower than the FP32
        // spacing of t keeps its exact width (the rule's weights scale with it)
        const double tlo = log(p.d_ref / a.dm_hi), thi = log(p.d_ref / a.dm_lo);
        float taf, tbf;
        dm_interval<float>(av * kLn2f, Bf * kLn2f, (float)tlo, (float)thi, (float)DmRule<float>::T, 24, taf, tbf);
        ta = taf <= (float)tlo ? tlo : (double)taf;
        const double tb = tbf >= (float)thi ? thi : (double)tbf;
        hq = tb - ta;
#pragma unroll
        for (int q = 0; q < NQ; q++) xs[q] = expf((float)(ta + hq * (0.5 + 0.5 * dm_gl_node(q))));
        skip = -(float)((DmRule<float>::T + 10.0) * kLog2e) / xs[0];
      }
    }
    auto window = [&](auto sl_c, bool last, bool first) {
      constexpr int SL = decltype(sl_c)::value;
      const float base = MODE == 0 ? -m_run : 0.f;
      float ell[4];
#pragma unroll
      for (int i = 0; i < 4; i++) ell[i] = last ? base + last_pen[i] : base;
#pragma unroll
      for (int k = 0; k < K; k++) {
        float z[7];
        constexpr int R0 = kTS * 20 * SL;
        z[0] = ring[zb[k][0] + R0];
        z[1] = ring[zb[k][1] + R0 + kTS];
        z[2] = ring[zb[k][2] + R0 + 2 * kTS];
        z[3] = ring[zb[k][3] + R0 + 3 * kTS];
        z[4] = ring[zb[k][0] + R0 + 5 * kTS];
        z[5] = ring[zb[k][1] + R0 + 6 * kTS];
        z[6] = ring[zb[k][2] + R0 + 7 * kTS];
#pragma unroll
        for (int i = 0; i < 4; i++) {
          ell[i] = fmaf(w[k][0], z[i], ell[i]);
          ell[i] = fmaf(w[k][1], z[i + 1], ell[i]);
          ell[i] = fmaf(w[k][2], z[i + 2], ell[i]);
          ell[i] = fmaf(w[k][3], z[i + 3], ell[i]);
        }
      }
      const float cmax = fmaxf(fmaxf(ell[0], ell[1]), fmaxf(ell[2], ell[3]));
      if constexpr (MODE == 1) {
        am = fmaxf(am, cmax);
      } else if constexpr (MODE == 2) {
        float d[4];
#pragma unroll
        for (int i = 0; i < 4; i++) d[i] = ell[i] - am;
        if (fmaxf(fmaxf(d[0], d[1]), fmaxf(d[2], d[3])) >= skip) {
#pragma unroll
          for (int q = 0; q < NQ; q++) {
            float e = 0.f;
#pragma unroll
            for (int i = 0; i < 4; i++) e += __builtin_amdgcn_exp2f(xs[q] * d[i]);
            Sq[q] += e;
          }
        }
      } else {
        if ((first || cmax > 64.f) && cmax > -3.0e38f) {  // rare after the first block
          // (the first block starts from an empty sum; its maximum can be far
          // below zero, where exp2(-cmax) would overflow)
          s_run = first ? 0.f : s_run * __builtin_amdgcn_exp2f(-cmax);
          m_run += cmax;
#pragma unroll
          for (int i = 0; i < 4; i++) ell[i] -= cmax;
        }
#pragma unroll
        for (int i = 0; i < 4; i++) s_run += __builtin_amdgcn_exp2f(ell[i]);
      }
    };
    using C0 = std::integral_constant<int, 0>;
    using C2 = std::integral_constant<int, 2>;
    // block b (stage slot S4 = b % 4): its MFMAs, then the window samples of
    // block b - 1, whose rows (blocks b - 1 and b) are then in the ring
    auto block = [&](auto s4_c, int b) {
      constexpr int S4 = decltype(s4_c)::value;
      product(s4_c);
      wave_sync();
      if (b >= 1) window(std::integral_constant<int, (S4 + 1) & 1>{}, b == JB, b == 1);
    };
    // blocks b, b + 1 (slots S0, S0 + 1) with one barrier; blocks b + 2, b + 3
    // are loaded meanwhile into the other two slots
    auto pair = [&](auto s0_c, int b) {
      constexpr int S0 = decltype(s0_c)::value;
      stage_load2(b + 2);
      if (active) {
        block(std::integral_constant<int, S0>{}, b);
        if (b + 1 <= JB) block(std::integral_constant<int, S0 + 1>{}, b + 1);
      }
      stage_store2(std::integral_constant<int, (S0 + 2) & 3>{});
      __syncthreads();
    };

    if constexpr (DIRECT) {
      // block b (register set and ring slot b % 2): prefetch block b + 1,
      // its MFMAs, then the window samples of block b - 1
      using C1 = std::integral_constant<int, 1>;
      auto dblock = [&](auto s2_c, int b) {
        constexpr int S2 = decltype(s2_c)::value;
        load_a(std::integral_constant<int, S2 ^ 1>{}, b + 1);
        product(s2_c);
        wave_sync();
        if (b >= 1) window(std::integral_constant<int, S2 ^ 1>{}, b == JB, b == 1);
      };
      if (active) {
        load_a(C0{}, 0);
        int b = 0;
        for (; b + 1 <= JB; b += 2) {
          dblock(C0{}, b);
          dblock(C1{}, b + 1);
        }
        if (b <= JB) dblock(C0{}, b);
      }
    } else {
      stage_load2(0);
      stage_store2(C0{});
      __syncthreads();
      int b = 0;
      for (; b + 3 <= JB; b += 4) {
        pair(C0{}, b);
        pair(C2{}, b + 2);
      }
      if (b <= JB) pair(C0{}, b);
      if (b + 2 <= JB) pair(C2{}, b + 2);
    }
    if (active && MODE == 1) {
      // the slot's largest data term over the four lanes of the sample
      float mo = am;
      mo = fmaxf(mo, __shfl_xor(mo, 16));
      mo = fmaxf(mo, __shfl_xor(mo, 32));
      if (g == 0) gpw(a.amax)[(int64_t)t * kTS + s] = valid ? mo : NAN;
    } else if (active && MODE == 2) {
      // per-node sums over the four lanes, then the nodes in FP64:
      // ln L_tD = ln sum_i W_i exp(x_i A_max - x_i^2 B) S_i - ln n_t (nats)
#pragma unroll
      for (int q = 0; q < NQ; q++) {
        Sq[q] += __shfl_xor(Sq[q], 16);
        Sq[q] += __shfl_xor(Sq[q], 32);
      }
      float lt = NAN;
      if (valid && g == 0 && hq > 0.0) {
        const double A = (double)am * (double)kLn2f, Bv = (double)Bf * (double)kLn2f;
        const double c = 3.0 * p.d_ref * p.d_ref * p.d_ref / (a.dm_hi * a.dm_hi * a.dm_hi - a.dm_lo * a.dm_lo * a.dm_lo);
        const double lc = log(0.5 * hq * c);
        double cmax = -INFINITY, acc = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; q++) {
          const double tq = ta + hq * (0.5 + 0.5 * dm_gl_node(q));
          const double xd = (double)xs[q];
          const double ci = lc + log(dm_gl_weight(q)) - 3.0 * tq + xd * A - xd * xd * Bv + log((double)Sq[q]);
          if (ci > cmax) {
            acc = acc * exp(cmax - ci) + 1.0;
            cmax = ci;
          } else {
            acc += exp(ci - cmax);
          }
        }
        lt = (float)(cmax + log(acc) - log((double)NT));
      }
      if (!isfinite(lt)) lt = NAN;
      if (flag != 0 && g == 0) {
        if (a.lnL) gpw(a.lnL)[col] = lt;
        if (a.lnw) gpw(a.lnw)[col] = lt + (a.ln_ratio ? gp(a.ln_ratio)[col] : 0.f);
      }
    } else if (active) {
      // combine the four lanes of each sample (base 2), then ln L_t
      float mo = m_run;
      mo = fmaxf(mo, __shfl_xor(mo, 16));
      mo = fmaxf(mo, __shfl_xor(mo, 32));
      float sc = s_run * __builtin_amdgcn_exp2f(m_run - mo);
      sc += __shfl_xor(sc, 16);
      sc += __shfl_xor(sc, 32);
      float lt = ((mo - Bf) + __log2f(sc)) * kLn2f - __logf((float)NT);
      if (!valid || !isfinite(lt)) lt = NAN;
      if (flag != 0 && g == 0) {
        if (a.lnL) gpw(a.lnL)[col] = lt;
        if (a.lnw) gpw(a.lnw)[col] = lt + (a.ln_ratio ? gp(a.ln_ratio)[col] : 0.f);
      }
    }
  }
}

// persistent grid: as many workgroups as the device keeps resident
// Persistent grid: as many workgroups as the device keeps resident
// (residency 0), or half as many per compute unit, at least one (residency 1:
// fewer workgroups sharing a compute unit's LDS, caches and issue slots).
template <int T, int K, bool D, int MODE, int WPE = 1>
static void launch_tk(const MfmaArgs &a, int lo, int hi, int cls, hipStream_t st, int residency) {
  static int per_cu = 0;
  if (per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mfma_kernel<T, K, D, MODE, WPE>, 256, 0) != hipSuccess ||
        nb < 1)
      nb = 1;
    per_cu = nb;
  }
  const int pc = residency ? std::max(1, per_cu / 2) : per_cu;
  const int grid = std::max(1, a.grid / 4 * pc);  // a.grid = 4 per compute unit
  hipLaunchKernelGGL((mfma_kernel<T, K, D, MODE, WPE>), dim3(grid), dim3(256), 0, st, a, lo, hi, cls);
}

// pass: 0 ln L_t (staged or direct feed); 1, 2 the passes of distance
// marginalization (staged feed)
template <int T, int K>
static void launch_tkm(const MfmaArgs &a, bool direct, int pass, int lo, int hi, int cls, hipStream_t st, int res,
                       int wpe) {
  if (pass == 1) launch_tk<T, K, false, 1>(a, lo, hi, cls, st, res);
  else if (pass == 2) launch_tk<T, K, false, 2>(a, lo, hi, cls, st, res);
  else if (direct && wpe == 3) launch_tk<T, K, true, 0, 3>(a, lo, hi, cls, st, res);
  else if (wpe == 3) launch_tk<T, K, false, 0, 3>(a, lo, hi, cls, st, res);
  else if (direct && wpe == 4) launch_tk<T, K, true, 0, 4>(a, lo, hi, cls, st, res);
  else if (direct) launch_tk<T, K, true, 0>(a, lo, hi, cls, st, res);
  else launch_tk<T, K, false, 0>(a, lo, hi, cls, st, res);
}

template <int T>
static void launch_class(const MfmaArgs &a, int K, bool direct, int pass, int lo, int hi, int cls, hipStream_t st,
                         int res, int wpe) {
  if (K == 1) launch_tkm<T, 1>(a, direct, pass, lo, hi, cls, st, res, wpe);
  else if (K == 2) launch_tkm<T, 2>(a, direct, pass, lo, hi, cls, st, res, wpe);
  else launch_tkm<T, 3>(a, direct, pass, lo, hi, cls, st, res, wpe);
}

// Launch configuration of a class, as the autotuner numbers it: 1 staged,
// 2 direct, 3 staged at half residency, 4 direct at half residency, 5 and 6
// direct with registers capped so that three (5) or four (6) wavefronts fit
// on a SIMD, 7 staged capped for three
static bool cfg_direct(int mode) { return mode == 2 || (mode >= 4 && mode <= 6); }
static int cfg_residency(int mode) { return mode == 3 || mode == 4 ? 1 : 0; }
static int cfg_wpe(int mode) { return mode == 5 || mode == 7 ? 3 : mode == 6 ? 4 : 1; }

static hipError_t launch_mode(const MfmaArgs &a, int T, int K, bool direct, int lo, int hi, int cls, hipStream_t st,
                              int pass = 0, int res = 0, int wpe = 1) {
  switch (T) {
#define RIFT_T_CASE(TT) \
  case TT: launch_class<TT>(a, K, direct, pass, lo, hi, cls, st, res, wpe); break;
    RIFT_T_CASE(1) RIFT_T_CASE(2) RIFT_T_CASE(3) RIFT_T_CASE(4) RIFT_T_CASE(5) RIFT_T_CASE(6) RIFT_T_CASE(7)
    RIFT_T_CASE(8) RIFT_T_CASE(9) RIFT_T_CASE(10) RIFT_T_CASE(11) RIFT_T_CASE(12) RIFT_T_CASE(13)
    RIFT_T_CASE(14) RIFT_T_CASE(15) RIFT_T_CASE(16)
#undef RIFT_T_CASE
    default: return hipErrorInvalidValue;
  }
  return hipSuccess;
}

// Every launch configuration of class c on the call's own data, one after the
// other on st, timed with events (the class's work-unit counter cleared
// before each); the results are bit-identical, so the later runs only
// rewrite the outputs.  The configurations are run in two passes and each is
// judged by the faster of its two runs, so none pays alone for the class's
// first touch of Q and its tile records or for clocks still rising at the
// start of the pass.  The staged form at full residency is kept unless
// another configuration is at least 3 % faster.
static hipError_t tune_class(const MfmaArgs &a, int T, int K, int lo, int hi, int c, hipStream_t st, int &mode) {
  constexpr int kCfg = kFeedConfigs, kPasses = 2, kEv = 2 * kPasses * kCfg;
  hipEvent_t ev[kEv] = {};
  hipError_t e = hipSuccess;
  for (int i = 0; i < kEv && e == hipSuccess; i++) e = hipEventCreate(&ev[i]);
  for (int r = 0; r < kPasses; r++)
    for (int m = 1; m <= kCfg && e == hipSuccess; m++) {
      hipEvent_t *em = ev + 2 * (r * kCfg + m - 1);
      if (r > 0 || m > 1) e = fill_u32(a.ctl + 1 + c, 1, 0u, st);
      if (e == hipSuccess) e = hipEventRecord(em[0], st);
      if (e == hipSuccess) e = launch_mode(a, T, K, cfg_direct(m), lo, hi, c, st, 0, cfg_residency(m), cfg_wpe(m));
      if (e == hipSuccess) e = hipEventRecord(em[1], st);
    }
  if (e == hipSuccess) e = hipEventSynchronize(ev[kEv - 1]);
  float best = 0.f;
  int pick = 1;
  for (int m = 1; m <= kCfg && e == hipSuccess; m++) {
    float t = 0.f;
    for (int r = 0; r < kPasses && e == hipSuccess; r++) {
      const hipEvent_t *em = ev + 2 * (r * kCfg + m - 1);
      float tr = 0.f;
      e = hipEventElapsedTime(&tr, em[0], em[1]);
      t = r == 0 ? tr : std::min(t, tr);
    }
    if (e != hipSuccess) break;
    if (m == 1 || t < 0.97f * best) {
      best = t;
      pick = m;
    }
  }
  if (e == hipSuccess) mode = pick;
  for (int i = 0; i < kEv; i++)
    if (ev[i]) (void)hipEventDestroy(ev[i]);
  return e;
}

hipError_t mfma_prepare(const MfmaArgs &a, const int *mclass_M, const int *mclass_item0, const int64_t *mclass_tiles,
                        int n_mclasses, hipStream_t st) {
  const size_t lds = sizeof(uint32_t) * (size_t)std::min(a.max_item_bins, kLdsBins);
  hipLaunchKernelGGL(bin_kernel, dim3(a.n_sort_blocks), dim3(kSortThreads), lds, st, a);
  hipLaunchKernelGGL(colscan_kernel, dim3((unsigned)((a.max_item_bins + kScanBins - 1) / kScanBins), std::min(a.items.n_items, 65535)),
                     dim3(kScanRanges * kScanBins), 0, st, a);
  hipLaunchKernelGGL(tilescan_kernel, dim3(a.items.n_items), dim3(256), 0, st, a);
  hipLaunchKernelGGL(item_scan_kernel, dim3(1), dim3(64), 0, st, a);
  hipLaunchKernelGGL(scatter_kernel, dim3(a.n_sort_blocks), dim3(kSortThreads), lds, st, a);
  hipLaunchKernelGGL(tile_item_kernel, dim3((unsigned)((a.max_tiles + 255) / 256)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(unit_kernel, dim3((unsigned)((a.n_bins + 63) / 64)), dim3(64), 0, st, a);
  for (int c = 0; c < n_mclasses; c++) {
    const int lo = mclass_item0[c], hi = mclass_item0[c + 1];
    const dim3 grid((unsigned)(((int64_t)kTS * mclass_tiles[c] + 63) / 64));
    switch (mclass_M[c]) {  // negative: points with a V table, general form
      case 2: hipLaunchKernelGGL(coef_kernel<2>, grid, dim3(64), 0, st, a, lo, hi); break;
      case 5: hipLaunchKernelGGL(coef_kernel<5>, grid, dim3(64), 0, st, a, lo, hi); break;
      case 9: hipLaunchKernelGGL(coef_kernel<9>, grid, dim3(64), 0, st, a, lo, hi); break;
      case 21: hipLaunchKernelGGL(coef_kernel<21>, grid, dim3(64), 0, st, a, lo, hi); break;
      default: hipLaunchKernelGGL(coef_kernel<0>, grid, dim3(64), 0, st, a, lo, hi); break;
    }
  }
  return hipGetLastError();
}

hipError_t mfma_forward(const MfmaArgs &a, const int *class_T, const int *class_K, const int *class_item0, int n_classes,
                        const int *mclass_M, const int *mclass_item0, const int64_t *mclass_tiles, int n_mclasses,
                        int *class_mode, bool tune, hipStream_t st, const Fanout &fo, hipEvent_t ev0,
                        hipEvent_t ev1) {
  if (a.total <= 0) return hipSuccess;
  hipError_t e = mfma_prepare(a, mclass_M, mclass_item0, mclass_tiles, n_mclasses, st);
  if (e != hipSuccess) return e;
  uint64_t done = 0;  // classes evaluated while being measured
  if (tune && !a.dmarg)
    for (int c = 0; c < n_classes && c < 64; c++)
      if (class_mode[c] == 0) {
        e = tune_class(a, class_T[c], class_K[c], class_item0[c], class_item0[c + 1], c, st, class_mode[c]);
        if (e != hipSuccess) return e;
        done |= 1ull << c;
      }
  if (ev0) (void)hipEventRecord(ev0, st);
  if (a.dmarg) {
    // distance marginalization: every class's largest data terms, then (the
    // work-unit counters cleared by a fill kernel) the integrals over D
    for (int pass = 1; pass <= 2; pass++) {
      if (pass == 2) {
        e = fill_u32(a.ctl + 1, n_classes, 0u, st);
        if (e != hipSuccess) return e;
      }
      fan_fork(fo, st, n_classes);
      for (int c = 0; c < n_classes; c++) {
        e = launch_mode(a, class_T[c], class_K[c], false, class_item0[c], class_item0[c + 1], c,
                        fan_stream(fo, st, c), pass);
        if (e != hipSuccess) return e;
      }
      e = hipGetLastError();
      fan_join(fo, st, n_classes);
      if (e != hipSuccess) return e;
    }
    if (ev1) (void)hipEventRecord(ev1, st);
    return e;
  }
  fan_fork(fo, st, n_classes);
  for (int c = 0; c < n_classes; c++) {
    if (c < 64 && (done >> c) & 1) continue;
    e = launch_mode(a, class_T[c], class_K[c], cfg_direct(class_mode[c]), class_item0[c], class_item0[c + 1], c,
                    fan_stream(fo, st, c), 0, cfg_residency(class_mode[c]), cfg_wpe(class_mode[c]));
    if (e != hipSuccess) return e;
  }
  e = hipGetLastError();
  fan_join(fo, st, n_classes);
  if (ev1) (void)hipEventRecord(ev1, st);
  return e;
}

}  // namespace rift
