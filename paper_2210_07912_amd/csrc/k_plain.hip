// Plain (VALU) evaluation of the time-marginalized likelihood, forward and
// adjoint, templated on the bulk precision R (float or double).
//
// One 256-thread workgroup takes a tile of TS samples of one point:
//   1. per-sample prologue in FP64 (direction, antenna patterns, delays,
//      harmonics, a_{k,lm} = (D_ref/D) F_k Y_lm, Catmull-Rom weights) and the
//      quadratic term B = 1/4 sum_k [a^dag U a + Re(a^T V a)]
//      (App. D Eq. (def:lnL:Decomposed));
//   2. per detector, the contraction z_k[r] = Re sum_m conj(a_km) Q_k[r][m]
//      over the rows the tile needs (threads over rows, Q read once per tile
//      from L2 and reused across the tile's samples), then the 4-tap
//      interpolation of z (which commutes with the linear contraction) is
//      accumulated into ell_j for the window j = 0..n_t-1;
//   3. ln L_t = max-shifted log-sum-exp over j minus ln n_t (App. D.2); the
//      window sums hold the data term only, and B (the same for every j) is
//      subtracted once at the end, so the sums carry no rounding of B.
// With distance marginalization the prologue takes x = 1 (D = D_ref), so the
// window holds the data terms A_j, and step 3 integrates over D by the
// per-sample rule of dmarg.h (in FP64 for the weights, the sums over j in R).
// The adjoint recomputes ell_j, forms p_j = exp(ell_j - ln L_t - ln n_t) and
// the detector sums G_k = sum_j p_j Qtilde_k(j), H_k = sum_j p_j Re(a^dag
// Qtilde'_k(j)), and applies the chain rule through F, Y, D and the delays.
#include "common.h"
#include "dmarg.h"
#include "internal.h"

namespace rift {

template <typename R>
__device__ __forceinline__ R r_exp(R x);
template <>
__device__ __forceinline__ float r_exp<float>(float x) { return expf(x); }
template <>
__device__ __forceinline__ double r_exp<double>(double x) { return exp(x); }

template <typename R>
__device__ __forceinline__ R r_log(R x);
template <>
__device__ __forceinline__ float r_log<float>(float x) { return logf(x); }
template <>
__device__ __forceinline__ double r_log<double>(double x) { return log(x); }

// bytes of the z rows' space: [TS][rows_cap] in the bulk precision, and in
// the forward at least the (U a), (V a) arrays it also holds (16-byte
// multiple, so the window buffer after it stays aligned)
__host__ __device__ inline size_t plain_zbuf_bytes(int elem, int TS, int rows_cap, bool bwd) {
  size_t z = (size_t)TS * rows_cap * elem;
  const size_t uv = (size_t)2 * TS * kMaxDet * kMaxModes * 2 * 8;
  if (!bwd && uv > z) z = uv;
  return (z + 15) & ~(size_t)15;
}

// maps a flat tile index to (item, first sample, count)
__device__ __forceinline__ int find_item(const int *tile0, int n_items, int t) {
  int lo = 0, hi = n_items;  // tile0[lo] <= t < tile0[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (tile0[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

template <typename R, int TS, bool BWD>
__global__ void __launch_bounds__(256) plain_kernel(PlainArgsT<R> args) {
  static_assert(256 / TS <= 64, "a sample's window reductions must stay within one wavefront");
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int t = blockIdx.x;
  const int it = find_item(args.item_tile0, args.n_items, t);
  const PointDev &p = args.pts[args.item_point[it]];
  const int64_t first = args.item_off[it] + (int64_t)(t - args.item_tile0[it]) * TS;
  const int64_t end = args.item_off[it] + args.item_cnt[it];
  const int ns = (int)min((int64_t)TS, end - first);
  const int K = p.K, M = p.M, NT = p.n_t, P = p.pad;
  const int MM = kMaxModes;

  // LDS carve-up.  (U a) and (V a) are needed by the quadratic term and the
  // adjoint's chain rule only: the forward keeps them in the space the rows
  // of z take later.
  constexpr int AKM = TS * kMaxDet * MM * 2;             // doubles of one [TS][K][MM][2] array
  double *a_d = (double *)smem;                          // [TS][K][MM][2]
  double *gk = a_d + AKM;                                // [TS][K][MM][2]  G_k (adjoint)
  double *ua_b = gk + (BWD ? AKM : 0);                   // adjoint: (U a)_m, (V a)_m
  double *Bs = ua_b + (BWD ? 2 * AKM : 0);               // [TS]
  double *Hk = Bs + TS;                                  // [TS][K]
  double *lnl = Hk + TS * kMaxDet;                       // [TS]
  double *F_l = lnl + TS;                                // [TS][K][2] antenna patterns F+, Fx
  double *sc_l = F_l + TS * kMaxDet * 2;                 // [TS][4] cos, sin of iota/2, phi, x
  R *wq = (R *)(sc_l + TS * 4);                          // [TS][K][4]
  R *wd = wq + TS * kMaxDet * 4;                         // [TS][K][4]
  int *nk = (int *)(wd + TS * kMaxDet * 4);              // [TS][K]
  int *okv = nk + TS * kMaxDet;                          // [TS]
  int *rng = okv + TS;                                   // [K][2] row range
  R *zbuf = (R *)(((uintptr_t)(rng + 2 * kMaxDet) + 15) & ~(uintptr_t)15);  // [TS][rows_cap]
  double *ua = BWD ? ua_b : (double *)zbuf;              // [TS][K][MM][2]  (U a)_m
  double *va = ua + AKM;                                 // [TS][K][MM][2]  (V a)_m
  R *lbuf = (R *)((char *)zbuf + plain_zbuf_bytes(sizeof(R), TS, args.rows_cap, BWD));  // [TS][nt_cap]

  // ---- 1. per-sample prologue (FP64), spread over the workgroup ----
  // 1a. one thread per (sample, detector): geometry, antenna pattern, the
  // row offset and interpolation weights of that detector
  for (int idx = tid; idx < TS * K; idx += blockDim.x) {
    const int s = idx / K, k = idx % K;
    bool ok = false;
    double Fp = 0.0, Fc = 0.0, x = 0.0, mu = 0.0;
    int n = 0;
    if (s < ns) {
      const int64_t i = first + s;
      double th[7];
      for (int d = 0; d < 7; d++) th[d] = (double)args.theta[d * args.stride + i];
      SkyTrig tr = sky_trig(th[RIFT_ALPHA], th[RIFT_DELTA], th[RIFT_PSI], p.gmst);
      Shift sh = shifts(p, tr, th[RIFT_TAU]);
      ok = sh.ok && isfinite(th[RIFT_IOTA]) && isfinite(th[RIFT_PHI]) &&
           (args.dmarg || (th[RIFT_DIST] > 0.0 && isfinite(th[RIFT_DIST])));
      x = args.dmarg ? 1.0 : p.d_ref / th[RIFT_DIST];
      antenna(p.D[k], tr, Fp, Fc);
      mu = sh.mu[k];
      n = sh.n[k];
      if (k == 0) {
        double ci, si;
        sincos(0.5 * th[RIFT_IOTA], &si, &ci);
        sc_l[s * 4 + 0] = ci;
        sc_l[s * 4 + 1] = si;
        sc_l[s * 4 + 2] = th[RIFT_PHI];
        sc_l[s * 4 + 3] = x;
      }
    }
    if (k == 0) okv[s] = ok ? 1 : 0;
    F_l[(s * kMaxDet + k) * 2 + 0] = ok ? Fp : 0.0;
    F_l[(s * kMaxDet + k) * 2 + 1] = ok ? Fc : 0.0;
    R w[4], dw[4];
    cr_weights<R>((R)mu, w);
    cr_dweights<R>((R)mu, dw);
    for (int q = 0; q < 4; q++) {
      wq[(s * kMaxDet + k) * 4 + q] = ok ? w[q] : R(0);
      wd[(s * kMaxDet + k) * 4 + q] = ok ? dw[q] : R(0);
    }
    nk[s * kMaxDet + k] = ok ? n : 0;
  }
  __syncthreads();
  // 1b. one thread per (sample, mode): the harmonic, then a_km = x F_k Y_m
  // for every detector (zero for an invalid sample)
  for (int idx = tid; idx < TS * M; idx += blockDim.x) {
    const int s = idx / M, m = idx % M;
    double yr = 0.0, yi = 0.0, x = 0.0;
    if (okv[s]) {
      double cm, sm;
      sincos(p.em[m] * sc_l[s * 4 + 2], &sm, &cm);
      harmonic(p, m, sc_l[s * 4 + 0], sc_l[s * 4 + 1], cm, sm, yr, yi);
      x = sc_l[s * 4 + 3];
    }
    for (int k = 0; k < K; k++) {
      const double Fp = F_l[(s * kMaxDet + k) * 2 + 0], Fc = F_l[(s * kMaxDet + k) * 2 + 1];
      a_d[((s * kMaxDet + k) * MM + m) * 2 + 0] = x * (Fp * yr - Fc * yi);
      a_d[((s * kMaxDet + k) * MM + m) * 2 + 1] = x * (Fp * yi + Fc * yr);
    }
  }
  __syncthreads();
  // (U a)_m and (V a)_m for every (sample, detector, mode), FP64
  for (int idx = tid; idx < TS * K * M; idx += blockDim.x) {
    int s = idx / (K * M), km = idx % (K * M), k = km / M, m = km % M;
    const RIFT_GLOBAL double *U = gp(p.U) + ((size_t)k * M + m) * M * 2;
    const double *a = a_d + (s * kMaxDet + k) * MM * 2;
    double ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
    for (int mp = 0; mp < M; mp++) {
      double xr = U[2 * mp], xi = U[2 * mp + 1], br = a[2 * mp], bi = a[2 * mp + 1];
      ur += xr * br - xi * bi;
      ui += xr * bi + xi * br;
    }
    if (p.V) {
      const RIFT_GLOBAL double *V = gp(p.V) + ((size_t)k * M + m) * M * 2;
      for (int mp = 0; mp < M; mp++) {
        double xr = V[2 * mp], xi = V[2 * mp + 1], br = a[2 * mp], bi = a[2 * mp + 1];
        vr += xr * br - xi * bi;
        vi += xr * bi + xi * br;
      }
    }
    ua[((s * kMaxDet + k) * MM + m) * 2 + 0] = ur;
    ua[((s * kMaxDet + k) * MM + m) * 2 + 1] = ui;
    va[((s * kMaxDet + k) * MM + m) * 2 + 0] = vr;
    va[((s * kMaxDet + k) * MM + m) * 2 + 1] = vi;
  }
  __syncthreads();
  if (tid < TS) {
    const int s = tid;
    double b = 0.0;
    for (int k = 0; k < K; k++)
      for (int m = 0; m < M; m++) {
        const double *a = a_d + ((s * kMaxDet + k) * MM + m) * 2;
        const double *u = ua + ((s * kMaxDet + k) * MM + m) * 2;
        const double *v = va + ((s * kMaxDet + k) * MM + m) * 2;
        b += a[0] * u[0] + a[1] * u[1];  // Re(conj(a) (U a))
        b += a[0] * v[0] - a[1] * v[1];  // Re(a (V a))
      }
    Bs[s] = 0.25 * b;
  }
  if (tid < K) {
    int lo = 1 << 30, hi = -(1 << 30);
    for (int s = 0; s < TS; s++) {
      int n = nk[s * kMaxDet + tid];
      lo = min(lo, n);
      hi = max(hi, n);
    }
    rng[2 * tid] = P + lo;                 // first row any sample needs (tap q = -1, j = 0)
    rng[2 * tid + 1] = P + hi + NT + 3;    // one past the last
  }
  __syncthreads();

  // ---- 2. contraction and interpolation, detector by detector ----
  const int passes = BWD ? 2 : 1;
  for (int pass = 0; pass < passes; pass++) {
    for (int k = 0; k < K; k++) {
      const int rlo = rng[2 * k], rhi = rng[2 * k + 1];
      const RIFT_GLOBAL R *Qk = gp((const R *)p.Q) + (size_t)k * p.Lpad * M * 2;
      for (int r = rlo + tid; r < rhi; r += blockDim.x) {
        R acc[TS];
#pragma unroll
        for (int s = 0; s < TS; s++) acc[s] = R(0);
        const RIFT_GLOBAL R *qr = Qk + (size_t)r * M * 2;
        for (int m = 0; m < M; m++) {
          R q0 = qr[2 * m], q1 = qr[2 * m + 1];
#pragma unroll
          for (int s = 0; s < TS; s++) {
            const double *a = a_d + ((s * kMaxDet + k) * MM + m) * 2;
            acc[s] += (R)a[0] * q0 + (R)a[1] * q1;
          }
        }
#pragma unroll
        for (int s = 0; s < TS; s++) zbuf[s * args.rows_cap + (r - rlo)] = acc[s];
      }
      __syncthreads();
      if (pass == 0) {
        for (int idx = tid; idx < TS * NT; idx += blockDim.x) {
          int s = idx / NT, j = idx % NT;
          const R *w = wq + (s * kMaxDet + k) * 4;
          int b = P + j + nk[s * kMaxDet + k] - rlo;  // row of tap q = -1
          const R *z = zbuf + s * args.rows_cap + b;
          R v = w[0] * z[0] + w[1] * z[1] + w[2] * z[2] + w[3] * z[3];
          R prev = (k == 0) ? R(0) : lbuf[s * args.nt_cap + j];
          lbuf[s * args.nt_cap + j] = prev + v;
        }
      } else {
        // adjoint: H_k = sum_j p_j sum_q w'_q z[b_j + q]
        constexpr int G = 256 / TS;
        int s = tid / G, g = tid % G;
        double h = 0.0;
        const R *w = wd + (s * kMaxDet + k) * 4;
        const R *z = zbuf + s * args.rows_cap + (P + nk[s * kMaxDet + k] - rlo);
        for (int j = g; j < NT; j += G) {
          R v = w[0] * z[j] + w[1] * z[j + 1] + w[2] * z[j + 2] + w[3] * z[j + 3];
          h += (double)lbuf[s * args.nt_cap + j] * (double)v;
        }
        for (int o = G / 2; o > 0; o >>= 1) h += __shfl_xor(h, o, G);
        if (g == 0) Hk[s * kMaxDet + k] = h;
        __syncthreads();
        // c[r] = sum_q w_q p_{r - b0 - q}, written over z
        for (int idx = tid; idx < TS * (rhi - rlo); idx += blockDim.x) {
          int s2 = idx / (rhi - rlo), rr = idx % (rhi - rlo);
          int j0 = rr - (P + nk[s2 * kMaxDet + k] - rlo);  // j of tap q=-1
          const R *w2 = wq + (s2 * kMaxDet + k) * 4;
          R c = R(0);
          for (int q = 0; q < 4; q++) {
            int j = j0 - q;
            if (j >= 0 && j < NT) c += w2[q] * lbuf[s2 * args.nt_cap + j];
          }
          zbuf[s2 * args.rows_cap + rr] = c;
        }
        __syncthreads();
        // G_k[s][m] = sum_r c[s][r] Q_k[r][m]
        for (int idx = tid; idx < TS * M; idx += blockDim.x) {
          int s2 = idx / M, m = idx % M;
          double gr = 0.0, gi = 0.0;
          const R *c = zbuf + s2 * args.rows_cap;
          for (int r = rlo; r < rhi; r++) {
            double cv = (double)c[r - rlo];
            gr += cv * (double)Qk[((size_t)r * M + m) * 2];
            gi += cv * (double)Qk[((size_t)r * M + m) * 2 + 1];
          }
          gk[((s2 * kMaxDet + k) * MM + m) * 2 + 0] = gr;
          gk[((s2 * kMaxDet + k) * MM + m) * 2 + 1] = gi;
        }
      }
      __syncthreads();
    }
    if (pass == 0) {
      // ---- 3. time marginalization ----
      constexpr int G = 256 / TS;
      int s = tid / G, g = tid % G;
      R mx = R(-INFINITY);
      for (int j = g; j < NT; j += G) mx = fmax(mx, lbuf[s * args.nt_cap + j]);
      for (int o = G / 2; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, G));
      R sum = R(0);
      for (int j = g; j < NT; j += G) sum += r_exp<R>(lbuf[s * args.nt_cap + j] - mx);
      for (int o = G / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, G);
      // the window holds the data term only: the quadratic term B is the
      // same for every window sample and is subtracted once, in FP64
      const R lse = mx + r_log<R>(sum);
      R lt = (R)((double)lse - Bs[s] - log((double)NT));
      if (!BWD && args.dmarg) {
        // over D: nodes x_i on the envelope's interval, S_i = sum_j exp(x_i (A_j - A_max)) in R,
        // the weighted sum over nodes in FP64 (online log-sum-exp)
        using DR = DmRule<R>;
        const double A = (double)mx, Bv = Bs[s];
        const double tlo = log(p.d_ref / args.dm_hi), thi = log(p.d_ref / args.dm_lo);
        double ta, tb;
        dm_interval<double>(A, Bv, tlo, thi, DR::T, 60, ta, tb);
        const double c = 3.0 * p.d_ref * p.d_ref * p.d_ref /
                         (args.dm_hi * args.dm_hi * args.dm_hi - args.dm_lo * args.dm_lo * args.dm_lo);
        const double h = (tb - ta) / DR::P;
        double cmax = -INFINITY, acc = 0.0;
        for (int pp = 0; pp < DR::P; pp++)
          for (int q = 0; q < kDmGL; q++) {
            const double t = ta + h * (pp + 0.5 + 0.5 * dm_gl_node(q));
            const R xr = (R)exp(t);
            R sq = R(0);
            for (int j = g; j < NT; j += G) sq += r_exp<R>(xr * (lbuf[s * args.nt_cap + j] - mx));
            for (int o = G / 2; o > 0; o >>= 1) sq += __shfl_xor(sq, o, G);
            const double xd = (double)xr;
            const double ci = log(0.5 * h * dm_gl_weight(q) * c) - 3.0 * t + xd * A - xd * xd * Bv + log((double)sq);
            if (ci > cmax) {
              acc = acc * exp(cmax - ci) + 1.0;
              cmax = ci;
            } else {
              acc += exp(ci - cmax);
            }
          }
        lt = (R)(cmax + log(acc) - log((double)NT));
      }
      bool ok = okv[s] && isfinite((double)lt);
      if (!ok) lt = R(NAN);
      if (g == 0) {
        lnl[s] = (double)lt;
        if (s < ns) {
          if (args.lnL) args.lnL[first + s] = lt;
          if (args.lnw) args.lnw[first + s] = lt + (args.ln_ratio ? args.ln_ratio[first + s] : R(0));
        }
      }
      if (BWD) {
        __syncthreads();
        // p_j = exp(ell_j + B - lse)
        R sub = ok ? lse : R(0);
        for (int j = g; j < NT; j += G)
          lbuf[s * args.nt_cap + j] = ok ? r_exp<R>(lbuf[s * args.nt_cap + j] - sub) : R(0);
      }
      __syncthreads();
    }
  }

  // ---- 4. adjoint chain rule (FP64), one thread per sample ----
  if (BWD && tid < ns) {
    const int s = tid;
    const int64_t i = first + s;
    double out[7] = {0, 0, 0, 0, 0, 0, 0};
    if (okv[s]) {
      double th[7];
      for (int d = 0; d < 7; d++) th[d] = (double)args.theta[d * args.stride + i];
      SkyTrig tr = sky_trig(th[RIFT_ALPHA], th[RIFT_DELTA], th[RIFT_PSI], p.gmst);
      double x = p.d_ref / th[RIFT_DIST];
      double ci, si;
      sincos(0.5 * th[RIFT_IOTA], &si, &ci);
      double dn_a[3] = {-tr.cd * tr.sh, tr.cd * tr.ch, 0.0};
      double dn_d[3] = {-tr.sd * tr.ch, -tr.sd * tr.sh, tr.cd};
      for (int k = 0; k < K; k++) {
        double Fp, Fc, dFa[2], dFd[2];
        antenna(p.D[k], tr, Fp, Fc, dFa, dFd);
        double H = Hk[s * kMaxDet + k];
        double ddt_a = -(p.rc[k][0] * dn_a[0] + p.rc[k][1] * dn_a[1] + p.rc[k][2] * dn_a[2]);
        double ddt_d = -(p.rc[k][0] * dn_d[0] + p.rc[k][1] * dn_d[1] + p.rc[k][2] * dn_d[2]);
        out[RIFT_ALPHA] += H * p.f_s * ddt_a;
        out[RIFT_DELTA] += H * p.f_s * ddt_d;
        out[RIFT_TAU] += H * p.f_s;
        for (int m = 0; m < M; m++) {
          double yr, yi, dyr, dyi, cm, sm;
          sincos(p.em[m] * th[RIFT_PHI], &sm, &cm);
          harmonic(p, m, ci, si, cm, sm, yr, yi, &dyr, &dyi);
          const double *G = gk + ((s * kMaxDet + k) * MM + m) * 2;
          const double *ua_ = ua + ((s * kMaxDet + k) * MM + m) * 2;
          const double *va_ = va + ((s * kMaxDet + k) * MM + m) * 2;
          const double *a = a_d + ((s * kMaxDet + k) * MM + m) * 2;
          // Re(conj(da) (G - U a / 2)) - Re(da (V a)) / 2
          double er = G[0] - 0.5 * ua_[0], ei = G[1] - 0.5 * ua_[1];
          auto contrib = [&](double dar, double dai) {
            return dar * er + dai * ei - 0.5 * (dar * va_[0] - dai * va_[1]);
          };
          out[RIFT_ALPHA] += contrib(x * (dFa[0] * yr - dFa[1] * yi), x * (dFa[0] * yi + dFa[1] * yr));
          out[RIFT_DELTA] += contrib(x * (dFd[0] * yr - dFd[1] * yi), x * (dFd[0] * yi + dFd[1] * yr));
          // dF/dpsi = -2i F
          double Fpr = 2.0 * Fc, Fpi = -2.0 * Fp;
          out[RIFT_PSI] += contrib(x * (Fpr * yr - Fpi * yi), x * (Fpr * yi + Fpi * yr));
          out[RIFT_IOTA] += contrib(x * (Fp * dyr - Fc * dyi), x * (Fp * dyi + Fc * dyr));
          double iyr = -p.em[m] * yi, iyi = p.em[m] * yr;
          out[RIFT_PHI] += contrib(x * (Fp * iyr - Fc * iyi), x * (Fp * iyi + Fc * iyr));
          out[RIFT_DIST] += contrib(-a[0] / th[RIFT_DIST], -a[1] / th[RIFT_DIST]);
        }
      }
    }
    double g = args.gin ? (double)args.gin[i] : 1.0;
    for (int d = 0; d < 7; d++) args.grad[d * args.stride + i] = okv[s] ? (R)(g * out[d]) : R(NAN);
  }
}

template <typename R, int TS, bool BWD>
static hipError_t launch_ts(const PlainArgsT<R> &a, int n_tiles, size_t lds, hipStream_t st, hipEvent_t ev0,
                            hipEvent_t ev1) {
  auto kern = plain_kernel<R, TS, BWD>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (ev0) (void)hipEventRecord(ev0, st);
  hipLaunchKernelGGL(kern, dim3(n_tiles), dim3(256), lds, st, a);
  hipError_t e = hipGetLastError();
  if (ev1) (void)hipEventRecord(ev1, st);
  return e;
}

size_t plain_lds_bytes(int elem, int TS, int rows_cap, int nt_cap, bool bwd) {
  size_t b = 0;
  b += (size_t)TS * kMaxDet * kMaxModes * 2 * 8 * (bwd ? 4 : 1);
  b += (size_t)TS * 8 * (2 + kMaxDet + 2 * kMaxDet + 4);
  b += (size_t)TS * kMaxDet * 4 * elem * 2;
  b += (size_t)TS * (kMaxDet + 1) * 4 + 2 * kMaxDet * 4 + 16;
  b += plain_zbuf_bytes(elem, TS, rows_cap, bwd) + (size_t)TS * nt_cap * elem;
  return b;
}

template <typename R>
hipError_t plain_launch(const PlainArgsT<R> &a, int TS, int n_tiles, bool bwd, hipStream_t st, hipEvent_t ev0,
                        hipEvent_t ev1) {
  size_t lds = plain_lds_bytes(sizeof(R), TS, a.rows_cap, a.nt_cap, bwd);
  if (n_tiles <= 0) return hipSuccess;
#define RIFT_TS_CASE(T)                                                   \
  case T:                                                                 \
    return bwd ? launch_ts<R, T, true>(a, n_tiles, lds, st, ev0, ev1) : launch_ts<R, T, false>(a, n_tiles, lds, st, ev0, ev1);
  switch (TS) {  // a sample's reductions span 256 / TS <= 64 lanes
    RIFT_TS_CASE(4)
    RIFT_TS_CASE(8)
    RIFT_TS_CASE(16)
    default: return hipErrorInvalidValue;
  }
#undef RIFT_TS_CASE
}

template hipError_t plain_launch<float>(const PlainArgsT<float> &, int, int, bool, hipStream_t, hipEvent_t,
                                        hipEvent_t);
template hipError_t plain_launch<double>(const PlainArgsT<double> &, int, int, bool, hipStream_t, hipEvent_t,
                                         hipEvent_t);

}  // namespace rift
