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
// into bins of equal integer delay (per detector, bins of kBinW rows); a tile
// holds 16 samples of one bin, whose windows then start within kBinW-1 rows
// of each other and share one run of rows (about 3% more rows than the
// window needs at n_t = 820).  Bins are padded to whole tiles, so tile t is
// sorted slots [16 t, 16 t + 16).
//
// Kernels, in launch order:
//   bin_kernel    integer delays n_k, bin key, per-sort-block bin counts
//   scan_kernel   per point: offset of each sort block in each bin, tiles
//                 before each bin
//   item_scan     tiles before each point; per-class tile counters reset
//   scatter       a 40-byte record (theta, column, n_k) at the sorted slot
//   tile_item     point of every tile
//   coef_kernel   one thread per slot, FP64: antenna patterns, harmonics,
//                 a_{k,lm} (rounded to FP32, in the MFMA operand layout), the
//                 quadratic term B, and the interpolation fraction mu_k
//   mfma_kernel<T> persistent; each wavefront owns a tile and walks the rows
//                 in 16-row blocks: T MFMAs per detector and block (operands
//                 of the next block already in flight) -> a 32-row ring in
//                 LDS -> Catmull-Rom interpolation of the 16 window samples
//                 whose stencils are complete -> online max-shifted
//                 log-sum-exp.  ell_j never leaves registers.
#include "common.h"
#include "internal.h"

#include <algorithm>

namespace rift {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTS = 16;          // samples per tile (MFMA columns)
constexpr int kRS = 36;          // floats per ring row (32 used, padded for banks)
constexpr int kWaves = 4;        // wavefronts per workgroup
constexpr int kRingFloats = kMaxDet * kTS * kRS;

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

__global__ void __launch_bounds__(256) bin_kernel(MfmaArgs a) {
  extern __shared__ uint32_t cnt_l[];
  const int it = block_item(a.items, blockIdx.x);
  const int lb = blockIdx.x - a.items.blk0[it];
  const PointDev &p = a.pts[a.items.point[it]];
  const int nb = a.items.bin0[it + 1] - a.items.bin0[it];
  const bool lds = nb <= kLdsBins;
  uint32_t *cnt = lds ? cnt_l : a.bhist + a.items.hoff[it] + (int64_t)lb * nb;
  for (int i = threadIdx.x; i < nb; i += 256) cnt[i] = 0u;
  __syncthreads();
  const int64_t n = a.items.cnt[it];
  const int64_t j0 = (int64_t)lb * kSortBlock, j1 = min(n, j0 + kSortBlock);
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) {
    const int64_t f = a.items.samp0[it] + j;
    const int64_t col = a.items.off[it] + j;
    double al = a.theta[RIFT_ALPHA * a.stride + col], de = a.theta[RIFT_DELTA * a.stride + col];
    double io = a.theta[RIFT_IOTA * a.stride + col], ph = a.theta[RIFT_PHI * a.stride + col];
    double di = a.theta[RIFT_DIST * a.stride + col], ta = a.theta[RIFT_TAU * a.stride + col];
    SkyTrig tr = sky_trig(al, de, 0.0, p.gmst);
    Shift sh = shifts(p, tr, ta);
    bool ok = sh.ok && isfinite(io) && isfinite(ph) && isfinite(di) && di > 0.0 &&
              isfinite((double)a.theta[RIFT_PSI * a.stride + col]);
    uint32_t key = 0, mul = 1;
    for (int k = 0; k < p.K; k++) {
      int q = ok ? (sh.n[k] + p.pad) / p.bin_w : 0;
      key += q * mul;
      mul *= p.nq;
      a.nsh[f * 4 + k] = (int16_t)(ok ? sh.n[k] : 0);
    }
    a.nsh[f * 4 + 3] = ok ? 1 : 0;
    a.key[f] = key;
    atomicAdd(&cnt[key], 1u);
  }
  __syncthreads();
  if (lds) {
    uint32_t *row = a.bhist + a.items.hoff[it] + (int64_t)lb * nb;
    for (int i = threadIdx.x; i < nb; i += 256) row[i] = cnt_l[i];
  }
}

// ---- 2. per-item scans: block offsets within each bin, tiles before each bin --
__global__ void __launch_bounds__(256) scan_kernel(MfmaArgs a) {
  __shared__ uint32_t pt[256];
  const int it = blockIdx.x;
  const int b0 = a.items.bin0[it], nb = a.items.bin0[it + 1] - b0;
  const int nblk = a.items.blk0[it + 1] - a.items.blk0[it];
  uint32_t *h = a.bhist + a.items.hoff[it];
  // column scan: offset of each sort block within each bin, and bin totals
  for (int b = threadIdx.x; b < nb; b += 256) {
    uint32_t run = 0;
    for (int lb = 0; lb < nblk; lb++) {
      uint32_t v = h[(int64_t)lb * nb + b];
      h[(int64_t)lb * nb + b] = run;
      run += v;
    }
    a.count[b0 + b] = run;
  }
  __syncthreads();
  const int per = (nb + 255) / 256;
  const int lo = min(nb, (int)threadIdx.x * per), hi = min(nb, lo + per);
  uint32_t ct = 0;
  for (int b = lo; b < hi; b++) ct += (a.count[b0 + b] + kTS - 1) / kTS;
  pt[threadIdx.x] = ct;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t rt = 0;
    for (int i = 0; i < 256; i++) {
      uint32_t y = pt[i];
      pt[i] = rt;
      rt += y;
    }
    a.item_tiles[it + 1] = (rt + 3u) & ~3u;  // whole groups of 4 tiles per point
  }
  __syncthreads();
  uint32_t rt = pt[threadIdx.x];
  for (int b = lo; b < hi; b++) {
    a.bin_tile[b0 + b] = rt;
    rt += (a.count[b0 + b] + kTS - 1) / kTS;
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
__global__ void __launch_bounds__(256) scatter_kernel(MfmaArgs a) {
  extern __shared__ uint32_t cur_l[];
  const int it = block_item(a.items, blockIdx.x);
  const int lb = blockIdx.x - a.items.blk0[it];
  const int b0 = a.items.bin0[it], nb = a.items.bin0[it + 1] - b0;
  const bool lds = nb <= kLdsBins;
  uint32_t *cur = lds ? cur_l : a.bhist + a.items.hoff[it] + (int64_t)lb * nb;
  if (lds) {
    const uint32_t *row = a.bhist + a.items.hoff[it] + (int64_t)lb * nb;
    for (int i = threadIdx.x; i < nb; i += 256) cur_l[i] = row[i];
  }
  __syncthreads();
  const int64_t n = a.items.cnt[it];
  const int64_t j0 = (int64_t)lb * kSortBlock, j1 = min(n, j0 + kSortBlock);
  const uint32_t tbase = a.item_tiles[it];
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) {
    const int64_t f = a.items.samp0[it] + j;
    const int64_t col = a.items.off[it] + j;
    const uint32_t key = a.key[f];
    const uint32_t r = atomicAdd(&cur[key], 1u);
    const uint32_t pos = kTS * (tbase + a.bin_tile[b0 + key]) + r;
    SampleRec rec;
#pragma unroll
    for (int d = 0; d < 7; d++) rec.th[d] = a.theta[d * a.stride + col];
    rec.col = (int)col;
    rec.n[0] = a.nsh[f * 4 + 0];
    rec.n[1] = a.nsh[f * 4 + 1];
    rec.n[2] = a.nsh[f * 4 + 2];
    rec.flag = a.nsh[f * 4 + 3] ? 1 : 2;
    a.rec[pos] = rec;
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

// ---- 4. per-sample coefficients (FP64), tile-major ---------------------------
// Quadratic term with the Hermitian (U) and symmetric (V) packing of the
// host: q_k = Y^dag U_k Y = sum_{m <= m'} Re(conj(Y_m) c_{mm'} Y_m'),
// t_k = Y^T V_k Y = sum_{m <= m'} c'_{mm'} Y_m Y_m', with the off-diagonal
// factor 2 folded into c, c'; B = x^2/4 sum_k [|F_k|^2 q_k + Re(F_k^2 t_k)].
// MC > 0: the mode count is a compile-time constant, Y lives in registers and
// the pair sums unroll (point data then comes through scalar loads); MC = 0
// is the general form, with Y staged in LDS.
template <int MC>
__global__ void __launch_bounds__(64) coef_kernel(MfmaArgs a, int item_lo, int item_hi) {
  constexpr int YS = MC > 0 ? 1 : 64;
  constexpr int YM = MC > 0 ? 1 : kMaxModes;
  constexpr int YR = MC > 0 ? MC : 1;
  __shared__ double Ys[YS][YM][2];
  const int64_t t_lo = a.item_tiles[item_lo], t_hi = a.item_tiles[item_hi];
  const int64_t pos = t_lo * kTS + (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (pos >= t_hi * kTS) return;
  const int64_t t = pos / kTS;
  const int s = (int)(pos % kTS);
  const SampleRec rec = a.rec[pos];
  // a block is 4 whole tiles of one point (tiles are padded per point)
  const int it = __builtin_amdgcn_readfirstlane(a.tile_item[t]);
  const PointDev &p = a.pts[a.items.point[it]];
  const int K = p.K, E = 2 * p.Mp;
  const int M = MC > 0 ? MC : p.M;
  RIFT_GLOBAL float *op = gpw(a.cop + a.item_cop[it] + (int64_t)(t - a.item_tiles[it]) * K * E * kTS + s);
  RIFT_GLOBAL CoefTile *ct = gpw(a.ctile + t);
  bool pad = rec.flag == 0;
  bool valid = rec.flag == 1;
  if (!valid) {
    for (int k = 0; k < K; k++)
      for (int e = 0; e < 2 * p.Mp; e++) op[((size_t)k * E + e) * kTS] = 0.f;
    ct->B[s] = 0.f;
    for (int k = 0; k < kMaxDet; k++) {
      ct->mu[k][s] = 0.f;
      ct->n[k][s] = 1 << 28;
    }
    ct->col[s] = pad ? -1 : rec.col;
    ct->flag[s] = pad ? 0 : 2;
    return;
  }
  const int64_t col = rec.col;
  double th[7];
#pragma unroll
  for (int d = 0; d < 7; d++) th[d] = (double)rec.th[d];
  const double x = p.d_ref / th[RIFT_DIST];
  SkyTrig tr = sky_trig(th[RIFT_ALPHA], th[RIFT_DELTA], th[RIFT_PSI], p.gmst);
  double Fr[kMaxDet], Fi[kMaxDet];
#pragma unroll
  for (int k = 0; k < kMaxDet; k++) {
    Fr[k] = Fi[k] = 0.0;
    if (k < K) {
      antenna(p.D[k], tr, Fr[k], Fi[k]);
      int n = (int)rec.n[k];
      double sk = (th[RIFT_TAU] + delay(p.rc[k], tr)) * p.f_s;
      ct->mu[k][s] = (float)(sk - (double)n);
      ct->n[k][s] = n;
    } else {
      ct->mu[k][s] = 0.f;
      ct->n[k][s] = 1 << 28;
    }
  }
  // harmonics: Y_m = ynorm d(iota) exp(i m phi); exp(i m phi) by repeated
  // products of exp(i phi)
  double ci, si, c1, s1;
  sincos(0.5 * th[RIFT_IOTA], &si, &ci);
  sincos(th[RIFT_PHI], &s1, &c1);
  double Yr[YR], Yi[YR];
  double (*Yl)[2] = Ys[MC > 0 ? 0 : threadIdx.x];
#pragma unroll
  for (int m = 0; m < (MC > 0 ? MC : kMaxModes); m++) {
    if (m >= M) break;
    int em = p.em[m], am = em < 0 ? -em : em;
    double cr = 1.0, cim = 0.0;
    for (int q = 0; q < am; q++) {
      double nr = cr * c1 - cim * s1;
      cim = cr * s1 + cim * c1;
      cr = nr;
    }
    if (em < 0) cim = -cim;
    double yr, yi;
    harmonic(p, m, ci, si, cr, cim, yr, yi);
    if constexpr (MC > 0) {
      Yr[m] = yr;
      Yi[m] = yi;
    } else {
      Yl[m][0] = yr;
      Yl[m][1] = yi;
    }
    // B operand elements 2m (Re a) and 2m+1 (Im a), for every detector
#pragma unroll
    for (int k = 0; k < kMaxDet; k++) {
      if (k < K) {
        double ar = x * (Fr[k] * yr - Fi[k] * yi), ai = x * (Fr[k] * yi + Fi[k] * yr);
        op[((size_t)k * E + 2 * m) * kTS] = (float)ar;
        op[((size_t)k * E + 2 * m + 1) * kTS] = (float)ai;
      }
    }
  }
  for (int k = 0; k < K; k++)
    for (int e = 2 * M; e < 2 * p.Mp; e++) op[((size_t)k * E + e) * kTS] = 0.f;
  double q[kMaxDet] = {0.0, 0.0, 0.0}, vr[kMaxDet] = {0.0, 0.0, 0.0}, vi[kMaxDet] = {0.0, 0.0, 0.0};
  const RIFT_GLOBAL double *Uq = gp(p.Upk);
  const RIFT_GLOBAL double *Vq = p.Vpk ? gp(p.Vpk) : nullptr;
  auto pair = [&](int idx, double ymr, double ymi, double ypr, double ypi) {
    // conj(Y_m) Y_m' and Y_m Y_m'
    const double pr = ymr * ypr + ymi * ypi, pi = ymr * ypi - ymi * ypr;
#pragma unroll
    for (int k = 0; k < kMaxDet; k++) {
      if (k < K) {
        const double ur = Uq[((size_t)idx * kMaxDet + k) * 2], ui = Uq[((size_t)idx * kMaxDet + k) * 2 + 1];
        q[k] += ur * pr - ui * pi;
      }
    }
    if (Vq) {
      const double sr = ymr * ypr - ymi * ypi, s_i = ymr * ypi + ymi * ypr;
#pragma unroll
      for (int k = 0; k < kMaxDet; k++) {
        if (k < K) {
          const double wr = Vq[((size_t)idx * kMaxDet + k) * 2], wi = Vq[((size_t)idx * kMaxDet + k) * 2 + 1];
          vr[k] += wr * sr - wi * s_i;
          vi[k] += wr * s_i + wi * sr;
        }
      }
    }
  };
  if constexpr (MC > 0) {
#pragma unroll
    for (int m = 0; m < MC; m++)
#pragma unroll
      for (int mp = m; mp < MC; mp++) pair(m * MC - m * (m - 1) / 2 + (mp - m), Yr[m], Yi[m], Yr[mp], Yi[mp]);
  } else {
    int idx = 0;
    for (int m = 0; m < M; m++)
      for (int mp = m; mp < M; mp++, idx++) pair(idx, Yl[m][0], Yl[m][1], Yl[mp][0], Yl[mp][1]);
  }
  double b = 0.0;
#pragma unroll
  for (int k = 0; k < kMaxDet; k++) {
    if (k < K) {
      double f2 = Fr[k] * Fr[k] + Fi[k] * Fi[k];
      double F2r = Fr[k] * Fr[k] - Fi[k] * Fi[k], F2i = 2.0 * Fr[k] * Fi[k];
      b += f2 * q[k] + (F2r * vr[k] - F2i * vi[k]);
    }
  }
  ct->B[s] = (float)(0.25 * x * x * b);
  ct->col[s] = (int)col;
  ct->flag[s] = 1;
}

// ---- 5. persistent MFMA evaluation ------------------------------------------
__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int T, int K>
__global__ void __launch_bounds__(256) mfma_kernel(MfmaArgs a, int item_lo, int item_hi, int cls) {
  __shared__ __align__(16) float lds_all[kWaves * kRingFloats];
  const int lane = threadIdx.x & 63;
  float *ring = lds_all + (threadIdx.x >> 6) * kRingFloats;  // [det][16][kRS]
  const int s = lane & 15, g = lane >> 4;
  const uint32_t t_lo = a.item_tiles[item_lo], t_hi = a.item_tiles[item_hi];
  constexpr int E = 4 * T;

  for (;;) {
    uint32_t t = 0;
    if (lane == 0) t = t_lo + atomicAdd(&a.ctl[1 + cls], 1u);
    t = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
    if (t >= t_hi) break;
    const int it = __builtin_amdgcn_readfirstlane(a.tile_item[t]);
    const PointDev &p = a.pts[a.items.point[it]];
    const int NT = p.n_t, P = p.pad, Lpad = p.Lpad;
    const RIFT_GLOBAL CoefTile *ct = gp(a.ctile + t);
    const RIFT_GLOBAL float *op = gp(a.cop + a.item_cop[it] + (int64_t)(t - a.item_tiles[it]) * K * E * kTS);
    const RIFT_GLOBAL float *Qm = gp(p.Qm);
    const int flag = ct->flag[s];
    if (!__any(flag != 0)) continue;  // padding tile
    const int col = ct->col[s];
    const float Bf = ct->B[s];
    // B operands: element e = g T + tt of sample s
    float Bop[K][T];
    float w[K][4];
    int base[K], sh[K];
    bool valid = flag == 1;
#pragma unroll
    for (int k = 0; k < K; k++) {
#pragma unroll
      for (int tt = 0; tt < T; tt++) Bop[k][tt] = op[((size_t)k * E + g * T + tt) * kTS + s];
      const int n = ct->n[k][s];
      cr_weights<float>(ct->mu[k][s], w[k]);
      int nmin = wave_min(n);
      if (nmin >= (1 << 28)) nmin = 0;
      base[k] = __builtin_amdgcn_readfirstlane(P + nmin);
      sh[k] = valid ? n - nmin : 0;
      if (sh[k] < 0 || sh[k] > 13) {
        valid = false;
        sh[k] = 0;
      }
    }
    const int JB = (NT + 15) >> 4;
    // A operands of block b: element e = g T + tt, row base + 16 b + s
    float Acur[K][T], Anext[K][T];
#pragma unroll
    for (int k = 0; k < K; k++) {
      const RIFT_GLOBAL float *qa = Qm + ((size_t)k * E + g * T) * Lpad + base[k] + s;
#pragma unroll
      for (int tt = 0; tt < T; tt++) Acur[k][tt] = qa[(size_t)tt * Lpad];
    }
    float m_run = -INFINITY, s_run = 0.f;
    for (int b = 0; b <= JB; b++) {
      // operands of the next block in flight while this one computes
      if (b < JB) {
#pragma unroll
        for (int k = 0; k < K; k++) {
          const RIFT_GLOBAL float *qa = Qm + ((size_t)k * E + g * T) * Lpad + base[k] + 16 * (b + 1) + s;
#pragma unroll
          for (int tt = 0; tt < T; tt++) Anext[k][tt] = qa[(size_t)tt * Lpad];
        }
      }
#pragma unroll
      for (int k = 0; k < K; k++) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int tt = 0; tt < T; tt++) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Acur[k][tt], Bop[k][tt], acc, 0, 0, 0);
        // acc[v] = z_k[base + 16 b + 4 g + v] of sample s
        *(f4 *)(ring + (k * 16 + s) * kRS + ((16 * b + 4 * g) & 31)) = acc;
      }
      wave_sync();
      if (b >= 1) {
        const int j0 = 16 * (b - 1) + 4 * g;
        float ell[4] = {-Bf, -Bf, -Bf, -Bf};
#pragma unroll
        for (int k = 0; k < K; k++) {
          const float *zr = ring + (k * 16 + s) * kRS;
          float z[7];
#pragma unroll
          for (int o = 0; o < 7; o++) z[o] = zr[(j0 + sh[k] + o) & 31];
#pragma unroll
          for (int i = 0; i < 4; i++)
            ell[i] += w[k][0] * z[i] + w[k][1] * z[i + 1] + w[k][2] * z[i + 2] + w[k][3] * z[i + 3];
        }
        float cmax = -INFINITY;
#pragma unroll
        for (int i = 0; i < 4; i++)
          if (j0 + i < NT) cmax = fmaxf(cmax, ell[i]);
        const float mn = fmaxf(m_run, cmax);
        if (mn > -INFINITY) {
          float acc = (m_run > -INFINITY) ? s_run * __expf(m_run - mn) : 0.f;
#pragma unroll
          for (int i = 0; i < 4; i++)
            if (j0 + i < NT) acc += __expf(ell[i] - mn);
          s_run = acc;
          m_run = mn;
        }
      }
      wave_sync();
#pragma unroll
      for (int k = 0; k < K; k++)
#pragma unroll
        for (int tt = 0; tt < T; tt++) Acur[k][tt] = Anext[k][tt];
    }
    // combine the four lanes of each sample
    float mo = m_run;
    mo = fmaxf(mo, __shfl_xor(mo, 16));
    mo = fmaxf(mo, __shfl_xor(mo, 32));
    float sc = (m_run > -INFINITY) ? s_run * __expf(m_run - mo) : 0.f;
    sc += __shfl_xor(sc, 16);
    sc += __shfl_xor(sc, 32);
    float lt = mo + __logf(sc) - __logf((float)NT);
    if (!valid || !isfinite(lt)) lt = NAN;
    if (flag != 0 && g == 0) {
      if (a.lnL) gpw(a.lnL)[col] = lt;
      if (a.lnw) gpw(a.lnw)[col] = lt + (a.ln_ratio ? gp(a.ln_ratio)[col] : 0.f);
    }
  }
}

template <int T>
static void launch_class(const MfmaArgs &a, int K, int lo, int hi, int cls, hipStream_t st) {
  if (K == 1) hipLaunchKernelGGL((mfma_kernel<T, 1>), dim3(a.grid), dim3(256), 0, st, a, lo, hi, cls);
  else if (K == 2) hipLaunchKernelGGL((mfma_kernel<T, 2>), dim3(a.grid), dim3(256), 0, st, a, lo, hi, cls);
  else hipLaunchKernelGGL((mfma_kernel<T, 3>), dim3(a.grid), dim3(256), 0, st, a, lo, hi, cls);
}

hipError_t mfma_forward(const MfmaArgs &a, const int *class_T, const int *class_K, const int *class_item0, int n_classes,
                        const int *mclass_M, const int *mclass_item0, const int64_t *mclass_tiles, int n_mclasses,
                        hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (a.total <= 0) return hipSuccess;
  hipError_t e = fill_u32((uint32_t *)a.rec, (int64_t)kTS * a.max_tiles * (sizeof(SampleRec) / 4), 0u, st);
  if (e != hipSuccess) return e;
  const size_t lds = sizeof(uint32_t) * (size_t)std::min(a.max_item_bins, kLdsBins);
  hipLaunchKernelGGL(bin_kernel, dim3(a.n_sort_blocks), dim3(256), lds, st, a);
  hipLaunchKernelGGL(scan_kernel, dim3(a.items.n_items), dim3(256), 0, st, a);
  hipLaunchKernelGGL(item_scan_kernel, dim3(1), dim3(64), 0, st, a);
  hipLaunchKernelGGL(scatter_kernel, dim3(a.n_sort_blocks), dim3(256), lds, st, a);
  hipLaunchKernelGGL(tile_item_kernel, dim3((unsigned)((a.max_tiles + 255) / 256)), dim3(256), 0, st, a);
  for (int c = 0; c < n_mclasses; c++) {
    const int lo = mclass_item0[c], hi = mclass_item0[c + 1];
    const dim3 grid((unsigned)(((int64_t)kTS * mclass_tiles[c] + 63) / 64));
    switch (mclass_M[c]) {
      case 2: hipLaunchKernelGGL(coef_kernel<2>, grid, dim3(64), 0, st, a, lo, hi); break;
      case 5: hipLaunchKernelGGL(coef_kernel<5>, grid, dim3(64), 0, st, a, lo, hi); break;
      case 9: hipLaunchKernelGGL(coef_kernel<9>, grid, dim3(64), 0, st, a, lo, hi); break;
      case 21: hipLaunchKernelGGL(coef_kernel<21>, grid, dim3(64), 0, st, a, lo, hi); break;
      default: hipLaunchKernelGGL(coef_kernel<0>, grid, dim3(64), 0, st, a, lo, hi); break;
    }
  }
  if (ev0) (void)hipEventRecord(ev0, st);
  for (int c = 0; c < n_classes; c++) {
    const int lo = class_item0[c], hi = class_item0[c + 1];
    const int K = class_K[c];
    switch (class_T[c]) {
#define RIFT_T_CASE(TT) \
  case TT: launch_class<TT>(a, K, lo, hi, c, st); break;
      RIFT_T_CASE(1) RIFT_T_CASE(2) RIFT_T_CASE(3) RIFT_T_CASE(4) RIFT_T_CASE(5) RIFT_T_CASE(6) RIFT_T_CASE(7)
      RIFT_T_CASE(8) RIFT_T_CASE(9) RIFT_T_CASE(10) RIFT_T_CASE(11) RIFT_T_CASE(12) RIFT_T_CASE(13)
      RIFT_T_CASE(14) RIFT_T_CASE(15) RIFT_T_CASE(16)
#undef RIFT_T_CASE
      default: return hipErrorInvalidValue;
    }
  }
  e = hipGetLastError();
  if (ev1) (void)hipEventRecord(ev1, st);
  return e;
}

}  // namespace rift
