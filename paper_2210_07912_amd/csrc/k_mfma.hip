// FP32 evaluation of ln L_t on the matrix cores (gfx950).
//
// The data term of App. D Eq. (def:lnL:Decomposed), summed over the window,
// needs for every sample s and detector k the real contraction
//     z_k[r](s) = Re sum_m conj(a_{k,m}(s)) Q_k[r][m]
// over the rows r its arrival time selects.  Computed over a common run of
// rows for a tile of samples this is a dense product
//     Z_k = Qr_k (rows x 2M) * A_k (2M x samples),
// with the real and imaginary parts of Q and a as the inner dimension, so it
// runs as v_mfma_f32_16x16x4f32 (16 rows x 16 samples per instruction).  The
// rows a sample needs depend on its own delay, so samples are first sorted
// into bins of equal integer delay (per detector, bins of kBinW rows); a tile
// holds 16 samples of one bin, whose windows then start within kBinW-1 rows
// of each other and share one run of rows (about 3% more rows than the
// window needs at n_t = 820).
//
// Each wavefront owns a tile and walks the rows in blocks of 16:
//   MFMA block b of every detector -> 16x16 outputs -> a 32-row ring in LDS
//   (per detector, per sample) -> the 4-tap Catmull-Rom interpolation of the
//   16 window samples whose stencils are complete -> online max-shifted
//   log-sum-exp.  ell_j never leaves registers; only ln L_t is written.
// Wavefronts pull tiles from a global counter (a persistent launch); tiles
// are ordered so that the costliest points come first.
#include "common.h"
#include "internal.h"

namespace rift {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTS = 16;          // samples per tile (MFMA columns)
constexpr int kBinW = 14;        // delay-bin width in rows: in-tile spread <= 13
constexpr int kTmax = 16;        // MFMA steps per row block: 4 kTmax >= 2 M
constexpr int kRS = 36;          // floats per ring row (32 used, padded for banks)
constexpr int kWaveLDS = 2048;   // floats of LDS per wavefront (ring, or staged Y)
constexpr int kWaves = 4;        // wavefronts per workgroup

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

// ---- 1. integer delays, bin keys and bin counts ---------------------------
__global__ void __launch_bounds__(256) bin_kernel(MfmaArgs a) {
  int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (f >= a.total) return;
  int it = item_of_flat(a.items, f);
  const PointDev &p = a.pts[a.items.point[it]];
  int64_t col = a.items.off[it] + (f - a.items.samp0[it]);
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
  uint32_t gb = a.items.bin0[it] + key;
  a.key[f] = gb;
  atomicAdd(&a.count[gb], 1u);
}

// ---- 2. per-item exclusive scans: bin positions and tile offsets ----------
__global__ void __launch_bounds__(256) scan_kernel(MfmaArgs a) {
  __shared__ uint32_t ps[256], pt[256];
  const int it = blockIdx.x;
  const int b0 = a.items.bin0[it], nb = a.items.bin0[it + 1] - b0;
  const int per = (nb + 255) / 256;
  const int lo = min(nb, (int)threadIdx.x * per), hi = min(nb, lo + per);
  uint32_t cs = 0, ct = 0;
  for (int b = lo; b < hi; b++) {
    uint32_t c = a.count[b0 + b];
    cs += c;
    ct += (c + kTS - 1) / kTS;
  }
  ps[threadIdx.x] = cs;
  pt[threadIdx.x] = ct;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t rs = 0, rt = 0;
    for (int i = 0; i < 256; i++) {
      uint32_t x = ps[i], y = pt[i];
      ps[i] = rs;
      pt[i] = rt;
      rs += x;
      rt += y;
    }
    a.item_tiles[it + 1] = rt;
  }
  __syncthreads();
  uint32_t rs = ps[threadIdx.x], rt = pt[threadIdx.x];
  const uint32_t base = (uint32_t)a.items.samp0[it];
  for (int b = lo; b < hi; b++) {
    uint32_t c = a.count[b0 + b];
    a.bin_pos[b0 + b] = base + rs;
    a.bin_tile[b0 + b] = rt;
    a.cursor[b0 + b] = 0;
    rs += c;
    rt += (c + kTS - 1) / kTS;
  }
}

// prefix of tiles over items (one block), reset of the tile counter
__global__ void item_scan_kernel(MfmaArgs a) {
  if (threadIdx.x == 0) {
    uint32_t r = 0;
    a.item_tiles[0] = 0;
    for (int i = 0; i < a.items.n_items; i++) {
      r += a.item_tiles[i + 1];
      a.item_tiles[i + 1] = r;
    }
    a.ctl[0] = 0;
    a.ctl[1] = r;
  }
}

// ---- 3. scatter to sorted order; tile descriptors -------------------------
__global__ void __launch_bounds__(256) scatter_kernel(MfmaArgs a) {
  int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (f < a.total) {
    uint32_t gb = a.key[f];
    uint32_t pos = a.bin_pos[gb] + atomicAdd(&a.cursor[gb], 1u);
    a.perm[pos] = (uint32_t)f;
  }
  if (f < a.n_bins) {
    int b = (int)f;
    int it = item_of_bin(a.items, b);
    uint32_t c = a.count[b];
    uint32_t t0 = a.item_tiles[it] + a.bin_tile[b];
    for (uint32_t t = 0; t * kTS < c; t++)
      a.tiles[t0 + t] = make_uint4((uint32_t)it, a.bin_pos[b] + t * kTS, min((uint32_t)kTS, c - t * kTS), 0u);
  }
}

// ---- 4. persistent MFMA evaluation -----------------------------------------
__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

__global__ void __launch_bounds__(256) mfma_kernel(MfmaArgs a) {
  __shared__ __align__(16) float lds_all[kWaves * kWaveLDS];
  const int lane = threadIdx.x & 63;
  float *lds = lds_all + (threadIdx.x >> 6) * kWaveLDS;
  const int s = lane & 15, g = lane >> 4;
  const uint32_t n_tiles = a.ctl[1];

  for (;;) {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(&a.ctl[0], 1u);
    t = __builtin_amdgcn_readfirstlane(__shfl(t, 0));
    if (t >= n_tiles) break;
    const uint4 td = a.tiles[t];
    const int it = __builtin_amdgcn_readfirstlane(td.x);
    const int cnt = __builtin_amdgcn_readfirstlane(td.z);
    const PointDev &p = a.pts[a.items.point[it]];
    const int K = p.K, M = p.M, NT = p.n_t, P = p.pad;
    const int T = p.Mp >> 1;  // MFMA steps: 4 T >= 2 M
    const bool act = s < cnt;
    const uint32_t f = act ? a.perm[td.y + s] : 0u;
    const int64_t col = a.items.off[it] + ((int64_t)f - a.items.samp0[it]);
    bool valid = act && a.nsh[(int64_t)f * 4 + 3] != 0;

    // ---- prologue (FP64): geometry, harmonics, coefficients, B ----
    double th[7];
#pragma unroll
    for (int d = 0; d < 7; d++) th[d] = act ? (double)a.theta[d * a.stride + col] : 0.0;
    if (!valid) {
      th[RIFT_DELTA] = 0.0; th[RIFT_ALPHA] = 0.0; th[RIFT_PSI] = 0.0; th[RIFT_IOTA] = 1.0;
      th[RIFT_PHI] = 0.0; th[RIFT_DIST] = 1.0; th[RIFT_TAU] = 0.0;
    }
    const double x = valid ? p.d_ref / th[RIFT_DIST] : 0.0;
    SkyTrig tr = sky_trig(th[RIFT_ALPHA], th[RIFT_DELTA], th[RIFT_PSI], p.gmst);
    double Fr[kMaxDet], Fi[kMaxDet];
    int nk[kMaxDet];
    float w[kMaxDet][4];
#pragma unroll
    for (int k = 0; k < kMaxDet; k++) {
      Fr[k] = Fi[k] = 0.0;
      nk[k] = 0;
      w[k][0] = w[k][1] = w[k][2] = w[k][3] = 0.f;
      if (k < K) {
        antenna(p.D[k], tr, Fr[k], Fi[k]);
        int n = valid ? (int)a.nsh[(int64_t)f * 4 + k] : 0;
        double sk = (th[RIFT_TAU] + delay(p.rc[k], tr)) * p.f_s;
        double mu = valid ? sk - (double)n : 0.0;
        nk[k] = n;
        cr_weights<float>((float)mu, w[k]);
      }
    }
    // harmonics of this lane's quarter of the modes, staged in LDS (FP64)
    double *Y = (double *)lds;  // [16 samples][kMaxModes][2]
    {
      double ci, si, c1, s1;
      sincos(0.5 * th[RIFT_IOTA], &si, &ci);
      sincos(th[RIFT_PHI], &s1, &c1);
      for (int m = g; m < M; m += 4) {
        int em = p.em[m], am = em < 0 ? -em : em;
        double cr = 1.0, cim = 0.0;  // exp(i |m| phi) by repeated products
        for (int q = 0; q < am; q++) {
          double nr = cr * c1 - cim * s1;
          cim = cr * s1 + cim * c1;
          cr = nr;
        }
        if (em < 0) cim = -cim;
        double yr, yi;
        harmonic(p, m, ci, si, cr, cim, yr, yi);
        Y[(s * kMaxModes + m) * 2 + 0] = yr;
        Y[(s * kMaxModes + m) * 2 + 1] = yi;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // quadratic term: B = x^2/4 sum_k [|F_k|^2 Y^dag U_k Y + Re(F_k^2 Y^T V_k Y)],
    // rows m = g, g+4, ... of this lane, summed over the four lanes of a sample
    double Bp = 0.0;
    for (int k = 0; k < K; k++) {
      double uterm = 0.0, vterm_r = 0.0, vterm_i = 0.0;
      for (int m = g; m < M; m += 4) {
        const double *Ur = p.U + ((size_t)k * M + m) * M * 2;
        double ur = 0.0, ui = 0.0;
        for (int mp = 0; mp < M; mp++) {
          double yr = Y[(s * kMaxModes + mp) * 2], yi = Y[(s * kMaxModes + mp) * 2 + 1];
          ur += Ur[2 * mp] * yr - Ur[2 * mp + 1] * yi;
          ui += Ur[2 * mp] * yi + Ur[2 * mp + 1] * yr;
        }
        double ymr = Y[(s * kMaxModes + m) * 2], ymi = Y[(s * kMaxModes + m) * 2 + 1];
        uterm += ymr * ur + ymi * ui;
        if (p.V) {
          const double *Vr = p.V + ((size_t)k * M + m) * M * 2;
          double vr = 0.0, vi = 0.0;
          for (int mp = 0; mp < M; mp++) {
            double yr = Y[(s * kMaxModes + mp) * 2], yi = Y[(s * kMaxModes + mp) * 2 + 1];
            vr += Vr[2 * mp] * yr - Vr[2 * mp + 1] * yi;
            vi += Vr[2 * mp] * yi + Vr[2 * mp + 1] * yr;
          }
          vterm_r += ymr * vr - ymi * vi;
          vterm_i += ymr * vi + ymi * vr;
        }
      }
      double f2 = Fr[k] * Fr[k] + Fi[k] * Fi[k];
      double F2r = Fr[k] * Fr[k] - Fi[k] * Fi[k], F2i = 2.0 * Fr[k] * Fi[k];
      Bp += f2 * uterm + (F2r * vterm_r - F2i * vterm_i);
    }
    Bp += __shfl_xor(Bp, 16);
    Bp += __shfl_xor(Bp, 32);
    const float Bf = (float)(0.25 * x * x * Bp);
    // B operand: element e = g T + t of sample s is Re/Im of a_{k, e/2}
    float Bop[kMaxDet][kTmax];
#pragma unroll
    for (int k = 0; k < kMaxDet; k++) {
#pragma unroll
      for (int tt = 0; tt < kTmax; tt++) {
        float v = 0.f;
        int e = g * T + tt;
        if (k < K && tt < T && e < 2 * M) {
          int m = e >> 1;
          double yr = Y[(s * kMaxModes + m) * 2], yi = Y[(s * kMaxModes + m) * 2 + 1];
          double ar = x * (Fr[k] * yr - Fi[k] * yi), ai = x * (Fr[k] * yi + Fi[k] * yr);
          v = (float)((e & 1) ? ai : ar);
        }
        Bop[k][tt] = v;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // ---- tile row base per detector and per-sample offsets ----
    int base[kMaxDet], sh[kMaxDet];
#pragma unroll
    for (int k = 0; k < kMaxDet; k++) {
      int nmin = wave_min(valid && k < K ? nk[k] : (1 << 29));
      if (nmin == (1 << 29)) nmin = 0;
      base[k] = __builtin_amdgcn_readfirstlane(P + nmin);
      sh[k] = valid ? nk[k] - nmin : 0;
      if (sh[k] > kBinW - 1 || sh[k] < 0) { valid = false; sh[k] = 0; }
    }

    // ---- main loop over 16-row blocks ----
    float *ring = lds;  // [kMaxDet][16][kRS]
    const int JB = (NT + 15) >> 4;
    float m_run = -INFINITY, s_run = 0.f;
    for (int b = 0; b <= JB; b++) {
#pragma unroll
      for (int k = 0; k < kMaxDet; k++) {
        if (k < K) {
          const float *qa = p.Qm + ((size_t)(k * 4 * T + g * T)) * p.Lpad + base[k] + 16 * b + s;
          f4 acc = {0.f, 0.f, 0.f, 0.f};
          float Av[kTmax];
#pragma unroll
          for (int tt = 0; tt < kTmax; tt++)
            if (tt < T) Av[tt] = qa[(size_t)tt * p.Lpad];
#pragma unroll
          for (int tt = 0; tt < kTmax; tt++)
            if (tt < T) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Av[tt], Bop[k][tt], acc, 0, 0, 0);
          // acc[v] = z_k[base + 16 b + 4 g + v] of sample s
          float *dst = ring + (k * 16 + s) * kRS + ((16 * b + 4 * g) & 31);
          *(f4 *)dst = acc;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (b >= 1) {
        const int j0 = 16 * (b - 1) + 4 * g;
        float ell[4] = {-Bf, -Bf, -Bf, -Bf};
#pragma unroll
        for (int k = 0; k < kMaxDet; k++) {
          if (k < K) {
            const float *zr = ring + (k * 16 + s) * kRS;
            float z[7];
#pragma unroll
            for (int o = 0; o < 7; o++) z[o] = zr[(j0 + sh[k] + o) & 31];
#pragma unroll
            for (int i = 0; i < 4; i++)
              ell[i] += w[k][0] * z[i] + w[k][1] * z[i + 1] + w[k][2] * z[i + 2] + w[k][3] * z[i + 3];
          }
        }
        float cmax = -INFINITY;
#pragma unroll
        for (int i = 0; i < 4; i++)
          if (j0 + i < NT) cmax = fmaxf(cmax, ell[i]);
        float mn = fmaxf(m_run, cmax);
        if (mn > -INFINITY) {
          float acc = (m_run > -INFINITY) ? s_run * __expf(m_run - mn) : 0.f;
#pragma unroll
          for (int i = 0; i < 4; i++)
            if (j0 + i < NT) acc += __expf(ell[i] - mn);
          s_run = acc;
          m_run = mn;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // combine the four lanes of each sample
    float mo = m_run;
    mo = fmaxf(mo, __shfl_xor(mo, 16));
    mo = fmaxf(mo, __shfl_xor(mo, 32));
    float sc = (m_run > -INFINITY) ? s_run * __expf(m_run - mo) : 0.f;
    sc += __shfl_xor(sc, 16);
    sc += __shfl_xor(sc, 32);
    bool allvalid = valid;
    allvalid = allvalid && __shfl_xor((int)valid, 16) && __shfl_xor((int)valid, 32);
    float lt = mo + __logf(sc) - __logf((float)NT);
    if (!allvalid || !isfinite(lt)) lt = NAN;
    if (act && g == 0) {
      if (a.lnL) a.lnL[col] = lt;
      if (a.lnw) a.lnw[col] = lt + (a.ln_ratio ? a.ln_ratio[col] : 0.f);
    }
  }
}

hipError_t mfma_forward(const MfmaArgs &a, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (a.total <= 0) return hipSuccess;
  hipError_t e = fill_u32(a.count, a.n_bins, 0u, st);
  if (e != hipSuccess) return e;
  int nb = (int)((a.total + 255) / 256);
  hipLaunchKernelGGL(bin_kernel, dim3(nb), dim3(256), 0, st, a);
  hipLaunchKernelGGL(scan_kernel, dim3(a.items.n_items), dim3(256), 0, st, a);
  hipLaunchKernelGGL(item_scan_kernel, dim3(1), dim3(64), 0, st, a);
  int64_t ns = a.total > a.n_bins ? a.total : a.n_bins;
  hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, a);
  if (ev0) (void)hipEventRecord(ev0, st);
  hipLaunchKernelGGL(mfma_kernel, dim3(a.grid), dim3(256), 0, st, a);
  e = hipGetLastError();
  if (ev1) (void)hipEventRecord(ev1, st);
  return e;
}

}  // namespace rift
