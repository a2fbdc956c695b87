// FP64 refinement of the FP32 matrix-core adjoint on the window samples that
// hold a sample's softmax mass.
//
// d ln L_t / d theta = sum_j p_j d ell_j / d theta is an average under the
// window softmax p_j (App. D Eq. (def:lnL:Decomposed) differentiated).  For a
// sample whose likelihood is loud, the data term and the quadratic term B
// are both large and nearly cancel in each gradient component, and the FP32
// rounding of the contraction, carried into p_j, G_k and H_k, is then a
// visible fraction of the component.  The mass of such a sample lies in a
// few window samples: the main peak, or, for a loud template at a wrong sky
// position, the top few spikes of the noise.  The FP32 sweep keeps, per
// sample, the three 16-sample window blocks with the largest maxima and the
// largest maximum of all other blocks; when that one is more than
// kRefineNats below the sample's maximum, the blocks within kRefineNats of
// the maximum hold all but n_t e^-kRefineNats of the mass, and this kernel
// redoes the sample over them in FP64 (coefficients, B, the contraction of
// the rows the blocks need, ell_j, p_j, H_k, c_k, G_k and the chain rule),
// overwriting its gradient and ln L_t.  Other samples keep the FP32 result:
// their ell_j come within kRefineNats of the maximum in more than three
// blocks, so the terms of their sums are comparatively small and so is the
// rounding.
//
// The FP32 sweep appends the samples to refine to a list; one persistent
// kernel takes them a wavefront per sample.  Lanes over the five angles for the
// trigonometry, over detectors for the antenna patterns, over modes for the
// harmonics, over (detector, mode) for a, U a, V a, G_k and the chain rule,
// over (block, row) for the contraction z_k[r] = Re sum_m conj(a_km) Q_k[r][m]
// and the transposed interpolation c_k, over (block, window sample) for
// ell_j, p_j and H_k.  Q is read in the handle's plain layout (FP32 values,
// exact in FP64).
#include "common.h"
#include "internal.h"
#include "mfma_tile.h"

#include <algorithm>

namespace rift {

constexpr int kRefWaves = 4;
constexpr int kRefRowsB = kTS + 3;  // rows one window block needs
static_assert(kRefineBlocks * kRefRowsB <= 64, "one (block, row) per lane");

// Wave-wide sum / maximum of a double without LDS: butterflies within each
// 16-lane row by DPP (xor 1, xor 2, half-row mirror, row mirror), then the
// four row results through scalar registers.  All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_d(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}
__device__ __forceinline__ double wsum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}
__device__ __forceinline__ double wmax(double v) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  return fmax(fmax(lane_d(v, 0), lane_d(v, 16)), fmax(lane_d(v, 32), lane_d(v, 48)));
}

// LDS of one wavefront
struct RefineWave {
  double a[kMaxDet * kMaxModes][2];   // a_km
  double ua[kMaxDet * kMaxModes][2];  // (U a)_km
  double va[kMaxDet * kMaxModes][2];  // (V a)_km
  double y[kMaxModes][4];             // Y_m, dY_m / d iota
  double f[kMaxDet][6];               // F+, Fx, dF/dalpha, dF/ddelta
  double z[kMaxDet][64];              // z_k, then c_k, at lane (block, row)
  double p[64];                       // p_j at lane (block, window sample)
};

// one listed sample: entry ent = (sorted slot, b0 | b1 << 16, b2 | count << 16)
__device__ __forceinline__ void refine_one(const MfmaArgs &a, RefineWave &W, int lane, int4 ent) {
  constexpr int MM = kMaxModes;
  const int nb = ent.z >> 16;
  if (nb < 1 || nb > kRefineBlocks) return;
  const int blk[3] = {ent.y & 0xffff, ent.y >> 16, ent.z & 0xffff};
  const int64_t pos = ent.x;
  const SampleRec rec = a.rec[pos];
  if (rec.flag != 1) return;
  const int it = a.tile_item[pos / kTS];
  const PointDev &p = a.pts[a.items.point[it]];
  const int K = p.K, M = p.M, NT = p.n_t, P = p.pad;

  double th[7];
#pragma unroll
  for (int d = 0; d < 7; d++) th[d] = (double)rec.th[d];
  // sin / cos of alpha - gmst, delta, psi, iota / 2, phi: one lane each
  double sv = 0.0, cv = 1.0;
  {
    const double arg = lane == 0 ? th[RIFT_ALPHA] - p.gmst
                       : lane == 1 ? th[RIFT_DELTA]
                       : lane == 2 ? th[RIFT_PSI]
                       : lane == 3 ? 0.5 * th[RIFT_IOTA]
                                   : th[RIFT_PHI];
    if (lane < 5) sincos(arg, &sv, &cv);
  }
  SkyTrig tr;
  tr.sh = lane_d(sv, 0);
  tr.ch = lane_d(cv, 0);
  tr.sd = lane_d(sv, 1);
  tr.cd = lane_d(cv, 1);
  tr.sp = lane_d(sv, 2);
  tr.cp = lane_d(cv, 2);
  const double si = lane_d(sv, 3), ci = lane_d(cv, 3), s1 = lane_d(sv, 4), c1 = lane_d(cv, 4);
  const double x = p.d_ref / th[RIFT_DIST];
  // integer row offsets and Catmull-Rom weights per detector (uniform)
  int nk[kMaxDet];
  double w[kMaxDet][4], wd[kMaxDet][4];
  bool ok = isfinite(th[RIFT_TAU]);
#pragma unroll
  for (int k = 0; k < kMaxDet; k++) {
    nk[k] = 0;
    double mu = 0.0;
    if (k < K) {
      const double sk = (th[RIFT_TAU] + delay(p.rc[k], tr)) * p.f_s;
      const double fl = floor(sk);
      ok = ok && isfinite(sk) && fl >= -P && fl <= P;
      nk[k] = ok ? (int)fl : 0;
      mu = ok ? sk - fl : 0.0;
    }
    cr_weights<double>(mu, w[k]);
    cr_dweights<double>(mu, wd[k]);
  }
  if (!ok) return;

  // ---- antenna patterns (lanes over detectors), harmonics (lanes over modes) ----
  if (lane < K) {
    double D[9];
#pragma unroll
    for (int i = 0; i < 9; i++) D[i] = p.D[lane][i];
    double Fp, Fc, dFa[2], dFd[2];
    antenna(D, tr, Fp, Fc, dFa, dFd);
    W.f[lane][0] = Fp;
    W.f[lane][1] = Fc;
    W.f[lane][2] = dFa[0];
    W.f[lane][3] = dFa[1];
    W.f[lane][4] = dFd[0];
    W.f[lane][5] = dFd[1];
  }
  const double u = ci * ci, hs = si * ci, hc = 0.5 * (ci * ci - si * si);
  for (int m = lane; m < M; m += 64) {
    // Y = s^par P(u) e^{i m phi}, s = sin(iota) / 2, u = cos^2(iota / 2)
    const int deg = p.hdeg[m];
    double Pv = p.hpoly[m][deg], dP = 0.0;
    for (int j = deg - 1; j >= 0; j--) {
      dP = fma(dP, u, Pv);
      Pv = fma(Pv, u, p.hpoly[m][j]);
    }
    double y, dy;
    if (p.hpar[m]) {
      y = hs * Pv;
      dy = hc * Pv - hs * hs * dP;
    } else {
      y = Pv;
      dy = -hs * dP;
    }
    const int em = p.em[m], am = em < 0 ? -em : em;
    double cr = 1.0, cim = 0.0;
    for (int q = 0; q < am; q++) {
      const double nr = cr * c1 - cim * s1;
      cim = cr * s1 + cim * c1;
      cr = nr;
    }
    if (em < 0) cim = -cim;
    W.y[m][0] = y * cr;
    W.y[m][1] = y * cim;
    W.y[m][2] = dy * cr;
    W.y[m][3] = dy * cim;
  }
  wave_sync();
  // ---- a_km = x F_k Y_m ----
  for (int l = lane; l < K * M; l += 64) {
    const int k = l / M, m = l - k * M;
    const double Fp = W.f[k][0], Fc = W.f[k][1], yr = W.y[m][0], yi = W.y[m][1];
    W.a[k * MM + m][0] = x * (Fp * yr - Fc * yi);
    W.a[k * MM + m][1] = x * (Fp * yi + Fc * yr);
  }
  wave_sync();
  // ---- (U a)_km, (V a)_km and B = 1/4 sum_k [a^dag U a + Re(a^T V a)] ----
  double bpart = 0.0;
  for (int l = lane; l < K * M; l += 64) {
    const int k = l / M, m = l - k * M;
    const double *U = p.U + ((size_t)k * M + m) * M * 2;
    double ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
    for (int mp = 0; mp < M; mp++) {
      const double br = W.a[k * MM + mp][0], bi = W.a[k * MM + mp][1];
      ur = fma(U[2 * mp], br, fma(-U[2 * mp + 1], bi, ur));
      ui = fma(U[2 * mp], bi, fma(U[2 * mp + 1], br, ui));
    }
    if (p.V) {
      const double *V = p.V + ((size_t)k * M + m) * M * 2;
      for (int mp = 0; mp < M; mp++) {
        const double br = W.a[k * MM + mp][0], bi = W.a[k * MM + mp][1];
        vr = fma(V[2 * mp], br, fma(-V[2 * mp + 1], bi, vr));
        vi = fma(V[2 * mp], bi, fma(V[2 * mp + 1], br, vi));
      }
    }
    W.ua[k * MM + m][0] = ur;
    W.ua[k * MM + m][1] = ui;
    W.va[k * MM + m][0] = vr;
    W.va[k * MM + m][1] = vi;
    const double ar = W.a[k * MM + m][0], ai = W.a[k * MM + m][1];
    bpart += ar * ur + ai * ui + ar * vr - ai * vi;
  }
  const double B = 0.25 * wsum(bpart);

  // ---- z_k at lane (block i, row r): Q row P + 16 blk[i] + n_k + r ----
  const float *Qf = (const float *)p.Q;
  const int ib = lane / kRefRowsB, rr = lane - ib * kRefRowsB;
  const bool row_on = ib < nb;
  const int row0 = row_on ? P + kTS * blk[ib < 3 ? ib : 0] + rr : 0;
#pragma unroll
  for (int k = 0; k < kMaxDet; k++) {
    if (k < K) {
      double z = 0.0;
      if (row_on) {
        const float *q = Qf + ((size_t)k * p.Lpad + (row0 + nk[k])) * M * 2;
        for (int m = 0; m < M; m++)
          z = fma(W.a[k * MM + m][0], (double)q[2 * m], fma(W.a[k * MM + m][1], (double)q[2 * m + 1], z));
      }
      W.z[k][lane] = z;
    }
  }
  wave_sync();

  // ---- ell_j, p_j, ln L_t, H_k at lane (block i, window sample jj) ----
  const int jb = lane >> 4, jj = lane & 15;
  const int jw = jb < nb ? kTS * blk[jb < 3 ? jb : 0] + jj : NT;  // window index
  const bool win_on = jb < nb && jw < NT;
  double ell = -INFINITY, dk[kMaxDet] = {0.0, 0.0, 0.0};
  if (win_on) {
    ell = -B;
#pragma unroll
    for (int k = 0; k < kMaxDet; k++) {
      if (k < K) {
        const double *z = &W.z[k][jb * kRefRowsB + jj];
        ell += w[k][0] * z[0] + w[k][1] * z[1] + w[k][2] * z[2] + w[k][3] * z[3];
        dk[k] = wd[k][0] * z[0] + wd[k][1] * z[1] + wd[k][2] * z[2] + wd[k][3] * z[3];
      }
    }
  }
  const double mx = wmax(ell);
  const double e = win_on ? exp(ell - mx) : 0.0;
  const double S = wsum(e);
  const double pj = e / S;
  const double lnLt = mx + log(S) - log((double)NT);
  double Hk[kMaxDet];
#pragma unroll
  for (int k = 0; k < kMaxDet; k++) Hk[k] = k < K ? wsum(pj * dk[k]) : 0.0;
  W.p[lane] = pj;
  wave_sync();
  // ---- c_k at lane (block i, row r) = sum_q w_q p_(i, r - q) (overwrites z) ----
#pragma unroll
  for (int k = 0; k < kMaxDet; k++) {
    if (k < K) {
      double c = 0.0;
      if (row_on) {
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const int j = rr - q;
          if (j >= 0 && j < kTS) c = fma(w[k][q], W.p[ib * kTS + j], c);
        }
      }
      W.z[k][lane] = c;
    }
  }
  wave_sync();

  // ---- G_km = sum over (block, row) c_k Q_k[row][m], then the chain rule ----
  double out[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int l = lane; l < K * M; l += 64) {
    const int k = l / M, m = l - k * M;
    const int nkk = k == 0 ? nk[0] : k == 1 ? nk[1] : nk[2];
    double Gr = 0.0, Gi = 0.0;
    for (int i = 0; i < nb; i++) {
      const int bi = i == 0 ? blk[0] : i == 1 ? blk[1] : blk[2];
      const float *q = Qf + ((size_t)k * p.Lpad + (P + kTS * bi + nkk)) * M * 2 + 2 * m;
      for (int r = 0; r < kRefRowsB; r++) {
        const double c = W.z[k][i * kRefRowsB + r];
        Gr = fma(c, (double)q[(size_t)r * M * 2], Gr);
        Gi = fma(c, (double)q[(size_t)r * M * 2 + 1], Gi);
      }
    }
    const double Fp = W.f[k][0], Fc = W.f[k][1];
    const double dFa0 = W.f[k][2], dFa1 = W.f[k][3], dFd0 = W.f[k][4], dFd1 = W.f[k][5];
    const double yr = W.y[m][0], yi = W.y[m][1], dyr = W.y[m][2], dyi = W.y[m][3];
    const double er = Gr - 0.5 * W.ua[k * MM + m][0], ei = Gi - 0.5 * W.ua[k * MM + m][1];
    const double var = W.va[k * MM + m][0], vai = W.va[k * MM + m][1];
    auto contrib = [&](double dar, double dai) { return dar * er + dai * ei - 0.5 * (dar * var - dai * vai); };
    out[RIFT_ALPHA] += contrib(x * (dFa0 * yr - dFa1 * yi), x * (dFa0 * yi + dFa1 * yr));
    out[RIFT_DELTA] += contrib(x * (dFd0 * yr - dFd1 * yi), x * (dFd0 * yi + dFd1 * yr));
    const double Fpr = 2.0 * Fc, Fpi = -2.0 * Fp;  // dF / dpsi = -2 i F
    out[RIFT_PSI] += contrib(x * (Fpr * yr - Fpi * yi), x * (Fpr * yi + Fpi * yr));
    out[RIFT_IOTA] += contrib(x * (Fp * dyr - Fc * dyi), x * (Fp * dyi + Fc * dyr));
    const double iyr = -p.em[m] * yi, iyi = p.em[m] * yr;
    out[RIFT_PHI] += contrib(x * (Fp * iyr - Fc * iyi), x * (Fp * iyi + Fc * iyr));
    const double ar = W.a[k * MM + m][0], ai = W.a[k * MM + m][1];
    out[RIFT_DIST] += contrib(-ar / th[RIFT_DIST], -ai / th[RIFT_DIST]);
  }
#pragma unroll
  for (int d = 0; d < 6; d++) out[d] = wsum(out[d]);
  // arrival times: f_s H_k d(dt_k) / d(alpha, delta) and f_s H_k for tau
  const double dn_a[3] = {-tr.cd * tr.sh, tr.cd * tr.ch, 0.0};
  const double dn_d[3] = {-tr.sd * tr.ch, -tr.sd * tr.sh, tr.cd};
#pragma unroll
  for (int k = 0; k < kMaxDet; k++) {
    if (k < K) {
      const double ddt_a = -(p.rc[k][0] * dn_a[0] + p.rc[k][1] * dn_a[1] + p.rc[k][2] * dn_a[2]);
      const double ddt_d = -(p.rc[k][0] * dn_d[0] + p.rc[k][1] * dn_d[1] + p.rc[k][2] * dn_d[2]);
      out[RIFT_ALPHA] += Hk[k] * p.f_s * ddt_a;
      out[RIFT_DELTA] += Hk[k] * p.f_s * ddt_d;
      out[RIFT_TAU] += Hk[k] * p.f_s;
    }
  }
  if (lane == 0 && isfinite(lnLt)) {
    const int64_t col = rec.col;
    const double gi = a.gin ? (double)a.gin[col] : 1.0;
#pragma unroll
    for (int d = 0; d < 7; d++) a.grad[d * a.stride + col] = (float)(gi * out[d]);
    if (a.lnL) a.lnL[col] = (float)lnLt;
  }
}

// persistent: wavefront w takes list entries w, w + (all wavefronts), ...
__global__ void __launch_bounds__(64 * kRefWaves) refine_bwd_kernel(MfmaArgs a) {
  __shared__ RefineWave sw[kRefWaves];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t n = a.ctl[kCtlRefine];
  const uint32_t stride = gridDim.x * kRefWaves;
  for (uint32_t i = blockIdx.x * kRefWaves + wave; i < n; i += stride) {
    const int4 e = ((const int4 *)a.jrng)[i];
    refine_one(a, sw[wave], lane, e);
    wave_sync();  // the next entry reuses the wavefront's LDS
  }
}

hipError_t refine_backward(const MfmaArgs &a, hipStream_t st) {
  if (a.total <= 0 || !a.jrng) return hipSuccess;
  static int per_cu = 0;
  if (per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, refine_bwd_kernel, 64 * kRefWaves, 0) != hipSuccess || nb < 1)
      nb = 1;
    per_cu = nb;
  }
  // a.grid is 4 workgroups per compute unit
  const int64_t slots = (int64_t)a.max_tiles * kTS;
  const int64_t want = (slots + kRefWaves - 1) / kRefWaves;
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)(a.grid / 4) * per_cu)));
  hipLaunchKernelGGL(refine_bwd_kernel, grid, dim3(64 * kRefWaves), 0, st, a);
  return hipGetLastError();
}

}  // namespace rift
