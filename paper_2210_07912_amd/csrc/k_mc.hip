// Monte Carlo layer: on-device sampling (Sec. III.B: random numbers and the
// likelihood both stay on the GPU), the FP64 importance-sampling reduction
// (Sec. II.A Eq. (lnL:MonteCarlo); n_eff, n_ESS, n_var of App. B) and the
// adaptive 100-bin histogram proposal (Sec. III.B).
//
// Reductions are deterministic: every block reduces a fixed range of samples
// in a fixed order into (max, sum e^{x-max}, sum e^{2(x-max)}) tuples, and the
// tuples of a segment are merged in index order.  Histograms accumulate
// fixed-point weights with 64-bit integer atomics, which are associative.
#include "common.h"
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace rift {

// ---------------------------------------------------------------------------
// sampler
// ---------------------------------------------------------------------------
__device__ __forceinline__ double u01(uint32_t x) { return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0); }
constexpr int kPairTries = 64;  // rejection tries of a correlated pair's draw

// Prior inverse CDFs u -> theta, evaluated in FP64 and rounded once to the
// bulk precision: asin/acos are ill-conditioned near the poles, where FP32
// evaluation would move the drawn angle by far more than its own rounding.
template <typename R>
__device__ __forceinline__ R prior_inv(int d, double u, double d_min, double d_max, double tw) {
  double t;
  switch (d) {
    case RIFT_ALPHA: t = 2.0 * kPi * u; break;
    case RIFT_DELTA: t = asin(2.0 * u - 1.0); break;
    case RIFT_PSI: t = kPi * u; break;
    case RIFT_IOTA: t = acos(2.0 * u - 1.0); break;
    case RIFT_PHI: t = 2.0 * kPi * u; break;
    case RIFT_DIST: {
      double a3 = d_min * d_min * d_min, b3 = d_max * d_max * d_max;
      t = cbrt(a3 + u * (b3 - a3));
      break;
    }
    default: t = (u - 0.5) * tw;
  }
  return (R)t;
}

// Sky in the network frame of the point (rows of fr: x', y', z' in Earth-fixed
// coordinates): phi' = 2 pi u0, cos theta' = 2 u1 - 1 give the direction
// n = sum_i n'_i e'_i, then delta = asin n_z and alpha = atan2(n_y, n_x) + gmst.
// The sky prior is isotropic, so this is the same prior in other coordinates.
__device__ __forceinline__ void frame_sky(const double (*fr)[3], double gmst, double u0, double u1, double &alpha,
                                          double &delta) {
  double sp, cp;
  sincos(2.0 * kPi * u0, &sp, &cp);
  const double ct = 2.0 * u1 - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct));
  const double a = st * cp, b = st * sp;
  const double nx = a * fr[0][0] + b * fr[1][0] + ct * fr[2][0];
  const double ny = a * fr[0][1] + b * fr[1][1] + ct * fr[2][1];
  const double nz = a * fr[0][2] + b * fr[1][2] + ct * fr[2][2];
  delta = asin(fmax(-1.0, fmin(1.0, nz)));
  double al = fmod(atan2(ny, nx) + gmst, 2.0 * kPi);
  alpha = al < 0.0 ? al + 2.0 * kPi : al;
}

// Phase-rotated coordinates of the polarization and orbital phase: the
// uniforms of those two dimensions are u_s = (phi + psi) / 4 pi and
// u_d = (phi - psi) / 4 pi, so that psi = 2 pi (u_s - u_d) mod pi and
// phi = 2 pi (u_s + u_d) mod 2 pi.  A (2, 2) mode depends on (psi, phi) only
// through phi - psi and a (2, -2) mode only through phi + psi (F_k turns as
// exp(-2 i psi), Y_lm as exp(i m phi)), so for a source dominated by either
// the likelihood varies along one coordinate only.  The map is four to one
// with a constant Jacobian: the uniform prior stays uniform in (u_s, u_d),
// and the proposal's ratio keeps its form in those coordinates.
__device__ __forceinline__ void phase_rotated(double us, double ud, double &psi, double &phi) {
  const double x = 2.0 * kPi * (us - ud), y = 2.0 * kPi * (us + ud);
  psi = x - kPi * floor(x / kPi);
  phi = y - 2.0 * kPi * floor(y / (2.0 * kPi));
}

// mixture parameters of a proposal, staged in LDS by the sampling kernels
struct GmmSh {
  int k, npair;
  int pa[kMaxPair], pb[kMaxPair];
  double eps;
  double w[7][kMaxG], mu[7][kMaxG], sd[7][kMaxG], ca[7][kMaxG], z[7][kMaxG];
  double pw[kMaxPair][kMaxG], pmu[kMaxPair][kMaxG][2], pch[kMaxPair][kMaxG][3], pic[kMaxPair][kMaxG][3];
  double plog[kMaxPair][kMaxG], pzm[kMaxPair];
  double pkeep[kMaxPair];  // probability that a pair's rejection keeps a draw: 1 - (1 - pzm)^kPairTries
};
__device__ __forceinline__ void gmm_stage(const ProposalDev *prop, GmmSh &g) {
  if (threadIdx.x == 0) {
    g.k = prop->gk;
    g.eps = prop->geps;
    g.npair = prop->gk > 0 ? prop->npair : 0;
    for (int p = 0; p < kMaxPair; p++) {
      g.pa[p] = prop->pa[p];
      g.pb[p] = prop->pb[p];
      g.pzm[p] = prop->pzm[p];
      g.pkeep[p] = 1.0 - exp((double)kPairTries * log1p(-fmin(prop->pzm[p], 1.0)));
    }
  }
  for (int i = threadIdx.x; i < kMaxPair * kMaxG; i += blockDim.x) {
    const int p = i / kMaxG, c = i % kMaxG;
    g.pw[p][c] = prop->pw[p][c];
    g.plog[p][c] = prop->plog[p][c];
    for (int q = 0; q < 2; q++) g.pmu[p][c][q] = prop->pmu[p][c][q];
    for (int q = 0; q < 3; q++) {
      g.pch[p][c][q] = prop->pch[p][c][q];
      g.pic[p][c][q] = prop->pic[p][c][q];
    }
  }
  for (int i = threadIdx.x; i < 7 * kMaxG; i += blockDim.x) {
    const int d = i / kMaxG, c = i % kMaxG;
    g.w[d][c] = prop->gw[d][c];
    g.mu[d][c] = prop->gmu[d][c];
    g.sd[d][c] = prop->gsd[d][c];
    g.ca[d][c] = prop->gca[d][c];
    g.z[d][c] = prop->gz[d][c];
  }
}

// one draw: Philox words (counter: sample index, 2 round + half, point; key:
// seed) -> seven parameters through the proposal's inverse CDFs in FP64,
// rounded once, their bins and ln p - ln p_s.  pt != null: the sky in the
// point's network frame (u_alpha, u_delta are its azimuth and polar cosine).
// With a mixture proposal (g->k > 0) an adapted parameter draws its
// component from a second Philox block (counter word 2: 2^31 | (2 round +
// half)): below the floor eps the uniform, else component k by the mixture
// weights, then u by the component's truncated-normal inverse CDF at v.
// MIX = false: no point of the launch holds a mixture (the mixture code is
// compiled out, which keeps the common sampler's registers low)
template <typename R, bool MIX>
__device__ __forceinline__ void draw_one(const double (*cdf)[kNB + 1], unsigned mask, const GmmSh *g, uint32_t point,
                                         uint64_t seed, uint32_t round, uint64_t i, double d_min, double d_max,
                                         double tau_width, const PointDev *pt, bool phase, R *theta, int64_t stride,
                                         R *ln_ratio, uint8_t *bins, int64_t bin_stride, int64_t col, float *ubuf) {
  uint32_t r[8], e[8];
  for (int half = 0; half < 2; half++) {
    uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), 2u * round + (uint32_t)half, point};
    philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    for (int q = 0; q < 4; q++) r[4 * half + q] = c[q];
  }
  const int gk = MIX ? g->k : 0;
  if (gk > 0 && mask) {
    for (int half = 0; half < 2; half++) {
      uint32_t c[4] = {(uint32_t)i, (uint32_t)(i >> 32), 0x80000000u | (2u * round + (uint32_t)half), point};
      philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
      for (int q = 0; q < 4; q++) e[4 * half + q] = c[q];
    }
  }
  double lr = 0.0, u_al = 0.0, u_de = 0.0, u_ps = 0.0, u_ph = 0.0;  // uniforms the frame maps read
  unsigned pm = 0u;  // parameters drawn in correlated pairs (after this loop)
  const int npair = MIX ? g->npair : 0;
  for (int p = 0; p < npair; p++) pm |= (1u << g->pa[p]) | (1u << g->pb[p]);
#pragma unroll
  for (int d = 0; d < 7; d++) {
    double v = u01(r[d]);
    double u = v;
    // bin of the raw uniform: floor(v nb), exactly, in integers
    uint32_t bin = (uint32_t)((((uint64_t)(r[d] >> 8) * 2u + 1u) * kNB) >> 25);
    if (((mask >> d) & 1u) && gk > 0 && ((pm >> d) & 1u)) {
      // a pair's parameter: drawn below
    } else if (((mask >> d) & 1u) && gk > 0) {
      const double eps = g->eps, cu = u01(e[d]);
      if (cu >= eps) {
        const double c2 = (cu - eps) / (1.0 - eps);
        int k = 0;
        double acc = g->w[d][0];
        while (k < gk - 1 && c2 >= acc) {
          k++;
          acc += g->w[d][k];
        }
        u = g->mu[d][k] + g->sd[d][k] * normcdfinv(g->ca[d][k] + v * g->z[d][k]);
        u = fmin(fmax(u, 0.0), 1.0 - 0x1p-53);
      }
      double s = 0.0;
      for (int k = 0; k < gk; k++) {
        if (g->w[d][k] > 0.0) {
          const double t = (u - g->mu[d][k]) / g->sd[d][k];
          s += g->w[d][k] * exp(-0.5 * t * t) / (g->sd[d][k] * g->z[d][k] * kSqrt2Pi);
        }
      }
      lr -= log(eps + (1.0 - eps) * s);
      bin = (uint32_t)min((int)(u * kNB), kNB - 1);
    } else if ((mask >> d) & 1u) {
      int lo = 0, hi = kNB;
      while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (cdf[d][mid] <= v) lo = mid; else hi = mid;
      }
      double mass = cdf[d][lo + 1] - cdf[d][lo];
      u = ((double)lo + (v - cdf[d][lo]) / mass) / kNB;
      lr -= log(mass * kNB);
      bin = (uint32_t)lo;
    }
    if (d == RIFT_ALPHA) u_al = u;
    if (d == RIFT_DELTA) u_de = u;
    if (d == RIFT_PSI) u_ps = u;
    if (d == RIFT_PHI) u_ph = u;
    if (ubuf) ubuf[d * bin_stride + col] = (float)u;
    theta[d * stride + col] = prior_inv<R>(d, u, d_min, d_max, tau_width);
    if (bins) bins[d * bin_stride + col] = (uint8_t)bin;
  }
  // correlated pairs: below the floor the raw uniforms, else up to
  // kPairTries draws from the untruncated mixture (Philox counter word 2 =
  // 3 2^30 | round << 10 | pair << 8 | try), the first inside the unit
  // square kept.  None inside (probability (1 - pzm)^kPairTries): the draw
  // is given up and the sample carries zero weight (ln ratio -inf) but stays
  // in the count, and a kept draw's density among all draws is
  // eps + (1 - eps) pkeep T, T the mixture truncated to the square, so that
  // the weights average to 1 over all draws.
  bool discard = false;
  for (int p = 0; p < npair; p++) {
    const int a = g->pa[p], b = g->pb[p];
    double ua = u01(r[a]), ub = u01(r[b]);
    const double eps = g->eps, ca = u01(e[a]);
    if (ca >= eps) {
      const double c0 = (ca - eps) / (1.0 - eps);
      bool ok = false;
      for (int t = 0; t < kPairTries && !ok; t++) {
        uint32_t w4[4] = {(uint32_t)i, (uint32_t)(i >> 32), 0xC0000000u | (round << 10) | ((uint32_t)p << 8) | (uint32_t)t,
                          point};
        philox(w4, (uint32_t)seed, (uint32_t)(seed >> 32));
        const double c = t == 0 ? c0 : ((double)w4[0] + 0.5) * 0x1p-32;
        int k = 0;
        double acc = g->pw[p][0];
        while (k < gk - 1 && c >= acc) {
          k++;
          acc += g->pw[p][k];
        }
        const double u1 = ((double)((((uint64_t)(w4[1] >> 6)) << 27) | (uint64_t)(w4[2] >> 5)) + 0.5) * 0x1p-53;
        const double u2 = ((double)w4[3] + 0.5) * 0x1p-32;
        const double rr = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincos(2.0 * kPi * u2, &sn, &cs);
        const double z1 = rr * cs, z2 = rr * sn;
        const double x = g->pmu[p][k][0] + g->pch[p][k][0] * z1;
        const double y = g->pmu[p][k][1] + g->pch[p][k][1] * z1 + g->pch[p][k][2] * z2;
        if (x >= 0.0 && x < 1.0 && y >= 0.0 && y < 1.0) {
          ua = x;
          ub = y;
          ok = true;
        }
      }
      discard = discard || !ok;
    }
    double sden = 0.0;
    for (int k = 0; k < gk; k++) {
      if (g->pw[p][k] > 0.0) {
        const double dx = ua - g->pmu[p][k][0], dy = ub - g->pmu[p][k][1];
        const double q = g->pic[p][k][0] * dx * dx + 2.0 * g->pic[p][k][1] * dx * dy + g->pic[p][k][2] * dy * dy;
        sden += exp(g->plog[p][k] - 0.5 * q);
      }
    }
    lr -= log(eps + (1.0 - eps) * g->pkeep[p] * sden / g->pzm[p]);
    const int dd[2] = {a, b};
    const double uu[2] = {ua, ub};
    for (int q = 0; q < 2; q++) {
      if (dd[q] == RIFT_ALPHA) u_al = uu[q];
      if (dd[q] == RIFT_DELTA) u_de = uu[q];
      if (dd[q] == RIFT_PSI) u_ps = uu[q];
      if (dd[q] == RIFT_PHI) u_ph = uu[q];
      if (ubuf) ubuf[dd[q] * bin_stride + col] = (float)uu[q];
      theta[dd[q] * stride + col] = prior_inv<R>(dd[q], uu[q], d_min, d_max, tau_width);
      if (bins) bins[dd[q] * bin_stride + col] = (uint8_t)min((int)(uu[q] * kNB), kNB - 1);
    }
  }
  if (discard) lr = -INFINITY;
  if (pt) {
    double al, de;
    frame_sky(pt->frame, pt->gmst, u_al, u_de, al, de);
    theta[RIFT_ALPHA * stride + col] = (R)al;
    theta[RIFT_DELTA * stride + col] = (R)de;
  }
  if (phase) {
    double ps, ph;
    phase_rotated(u_ps, u_ph, ps, ph);
    theta[RIFT_PSI * stride + col] = (R)ps;
    theta[RIFT_PHI * stride + col] = (R)ph;
  }
  if (ln_ratio) ln_ratio[col] = (R)lr;
}

template <typename R, bool MIX>
__global__ void __launch_bounds__(256) sample_kernel(const ProposalDev *prop, const PointDev *pt, uint32_t point,
                                                     uint64_t seed, uint32_t round, int64_t first, int64_t n,
                                                     int64_t stride, int64_t bin_stride, double d_min, double d_max,
                                                     double tau_width, R *theta, R *ln_ratio, uint8_t *bins,
                                                     float *ubuf, int phase) {
  __shared__ double cdf[7][kNB + 1];
  __shared__ GmmSh g;
  // the histogram tables are staged only when some dimension draws from one
  const unsigned mask = prop->mask;
  if (mask)
    for (int i = threadIdx.x; i < 7 * (kNB + 1); i += blockDim.x)
      cdf[i / (kNB + 1)][i % (kNB + 1)] = prop->cdf[i / (kNB + 1)][i % (kNB + 1)];
  if (MIX) gmm_stage(prop, g);
  __syncthreads();
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  draw_one<R, MIX>(cdf, mask, &g, point, seed, round, (uint64_t)(first + j), d_min, d_max, tau_width, pt, phase != 0,
                   theta, stride, ln_ratio, bins, bin_stride, j, ubuf);
}

// every point of a round in one launch: blocks [blk0[p], blk0[p + 1]) draw
// point p's samples into columns off[p] ..
template <typename R, bool MIX>
__global__ void __launch_bounds__(256) sample_multi_kernel(const ProposalDev *props, const PointDev *pts,
                                                           const int *blk0, int np, const int64_t *off,
                                                           const int64_t *cnt, uint64_t seed, uint32_t round,
                                                           int64_t stride, int64_t bin_stride, double d_min,
                                                           double d_max, double tau_width, R *theta, R *ln_ratio,
                                                           uint8_t *bins, float *ubuf, int phase) {
  __shared__ double cdf[7][kNB + 1];
  __shared__ GmmSh g;
  int lo = 0, hi = np;  // blk0[lo] <= blockIdx.x < blk0[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (blk0[mid] <= (int)blockIdx.x) lo = mid; else hi = mid;
  }
  const int p = lo;
  const ProposalDev *prop = props + p;
  // the histogram tables are staged only when some dimension draws from one
  const unsigned mask = prop->mask;
  if (mask)
    for (int i = threadIdx.x; i < 7 * (kNB + 1); i += blockDim.x)
      cdf[i / (kNB + 1)][i % (kNB + 1)] = prop->cdf[i / (kNB + 1)][i % (kNB + 1)];
  if (MIX) gmm_stage(prop, g);
  __syncthreads();
  const int64_t j = (int64_t)(blockIdx.x - blk0[p]) * blockDim.x + threadIdx.x;
  if (j >= cnt[p]) return;
  draw_one<R, MIX>(cdf, mask, &g, (uint32_t)p, seed, round, (uint64_t)j, d_min, d_max, tau_width, pts ? pts + p : nullptr,
                   phase != 0, theta, stride, ln_ratio, bins, bin_stride, off[p] + j, ubuf);
}

template <typename R>
hipError_t sample_launch(const PointDev *pt, const ProposalDev *prop, int point, uint64_t seed, uint32_t round,
                         int64_t first, int64_t n, int64_t stride, int64_t bin_stride, double d_min, double d_max,
                         double tau_width, R *theta, R *ln_ratio, uint8_t *bins, hipStream_t st, float *ubuf,
                         bool mix, bool phase) {
  if (n <= 0) return hipSuccess;
  if (mix)
    hipLaunchKernelGGL((sample_kernel<R, true>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, prop, pt,
                       (uint32_t)point, seed, round, first, n, stride, bin_stride, d_min, d_max, tau_width, theta,
                       ln_ratio, bins, ubuf, (int)phase);
  else
    hipLaunchKernelGGL((sample_kernel<R, false>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, prop, pt,
                       (uint32_t)point, seed, round, first, n, stride, bin_stride, d_min, d_max, tau_width, theta,
                       ln_ratio, bins, ubuf, (int)phase);
  return hipGetLastError();
}

template <typename R>
hipError_t sample_multi_launch(const ProposalDev *props, const PointDev *pts, const int *blk0, int n_blocks, int np,
                               const int64_t *off, const int64_t *cnt, uint64_t seed, uint32_t round, int64_t stride,
                               int64_t bin_stride, double d_min, double d_max, double tau_width, R *theta,
                               R *ln_ratio, uint8_t *bins, hipStream_t st, float *ubuf, bool mix, bool phase) {
  if (n_blocks <= 0) return hipSuccess;
  if (mix)
    hipLaunchKernelGGL((sample_multi_kernel<R, true>), dim3((unsigned)n_blocks), dim3(256), 0, st, props, pts, blk0,
                       np, off, cnt, seed, round, stride, bin_stride, d_min, d_max, tau_width, theta, ln_ratio, bins,
                       ubuf, (int)phase);
  else
    hipLaunchKernelGGL((sample_multi_kernel<R, false>), dim3((unsigned)n_blocks), dim3(256), 0, st, props, pts, blk0,
                       np, off, cnt, seed, round, stride, bin_stride, d_min, d_max, tau_width, theta, ln_ratio, bins,
                       ubuf, (int)phase);
  return hipGetLastError();
}
template hipError_t sample_multi_launch<float>(const ProposalDev *, const PointDev *, const int *, int, int,
                                               const int64_t *,
                                               const int64_t *, uint64_t, uint32_t, int64_t, int64_t, double, double,
                                               double, float *, float *, uint8_t *, hipStream_t, float *, bool, bool);
template hipError_t sample_multi_launch<double>(const ProposalDev *, const PointDev *, const int *, int, int,
                                                const int64_t *,
                                                const int64_t *, uint64_t, uint32_t, int64_t, int64_t, double, double,
                                                double, double *, double *, uint8_t *, hipStream_t, float *, bool, bool);
template hipError_t sample_launch<float>(const PointDev *, const ProposalDev *, int, uint64_t, uint32_t, int64_t,
                                         int64_t, int64_t, int64_t, double, double, double, float *, float *,
                                         uint8_t *, hipStream_t, float *, bool, bool);
template hipError_t sample_launch<double>(const PointDev *, const ProposalDev *, int, uint64_t, uint32_t, int64_t,
                                          int64_t, int64_t, int64_t, double, double, double, double *, double *,
                                          uint8_t *, hipStream_t, float *, bool, bool);

// ---------------------------------------------------------------------------
// FP64 reduction
// ---------------------------------------------------------------------------
__device__ __forceinline__ void tup_add(ReduceTuple &t, double x) {
  if (!(x == x) || x == INFINITY) {  // NaN or +inf
    t.bad++;
    return;
  }
  t.n++;
  if (x == -INFINITY) return;
  // one exponential either way: exp(-|x - m|) rescales the sums to a new
  // maximum or weighs x against the current one (0 when m = -inf)
  const bool up = x > t.m;
  const double e = exp(up ? t.m - x : x - t.m);
  t.s1 = up ? t.s1 * e + 1.0 : t.s1 + e;
  t.s2 = up ? t.s2 * e * e + 1.0 : t.s2 + e * e;
  t.m = up ? x : t.m;
}

__device__ __forceinline__ ReduceTuple tup_merge(const ReduceTuple &a, const ReduceTuple &b) {
  ReduceTuple r;
  r.n = a.n + b.n;
  r.bad = a.bad + b.bad;
  r.pad_ = 0.0;
  r.m = fmax(a.m, b.m);
  if (r.m == -INFINITY) {
    r.s1 = r.s2 = 0.0;
    return r;
  }
  double ea = a.m == -INFINITY ? 0.0 : exp(a.m - r.m);
  double eb = b.m == -INFINITY ? 0.0 : exp(b.m - r.m);
  r.s1 = a.s1 * ea + b.s1 * eb;
  r.s2 = a.s2 * ea * ea + b.s2 * eb * eb;
  return r;
}

__device__ __forceinline__ ReduceTuple tup_zero() {
  ReduceTuple t;
  t.m = -INFINITY;
  t.s1 = t.s2 = 0.0;
  t.n = t.bad = 0;
  t.pad_ = 0.0;
  return t;
}

template <typename R>
__global__ void __launch_bounds__(256) reduce_partials_kernel(const R *lnL, const R *ln_ratio, const int64_t *seg_off,
                                                              const int64_t *seg_cnt, int bps, ReduceTuple *partials) {
  __shared__ ReduceTuple sh[256];
  const int seg = blockIdx.x / bps, j = blockIdx.x % bps;
  const int64_t cnt = seg_cnt[seg], off = seg_off[seg];
  const int64_t chunk = (cnt + bps - 1) / bps;
  const int64_t lo = min(cnt, (int64_t)j * chunk), hi = min(cnt, lo + chunk);
  ReduceTuple t = tup_zero();
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    double x = (double)lnL[off + i];
    if (ln_ratio) x += (double)ln_ratio[off + i];
    tup_add(t, x);
  }
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = tup_merge(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

template <typename R>
hipError_t reduce_partials(const R *lnL, const R *ln_ratio, const int64_t *seg_off, const int64_t *seg_cnt,
                           int n_seg, int bps, ReduceTuple *partials, hipStream_t st) {
  if (n_seg <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_partials_kernel<R>, dim3(n_seg * bps), dim3(256), 0, st, lnL, ln_ratio, seg_off, seg_cnt,
                     bps, partials);
  return hipGetLastError();
}
template hipError_t reduce_partials<float>(const float *, const float *, const int64_t *, const int64_t *, int, int,
                                           ReduceTuple *, hipStream_t);
template hipError_t reduce_partials<double>(const double *, const double *, const int64_t *, const int64_t *, int,
                                            int, ReduceTuple *, hipStream_t);

__device__ void tuple_result(const ReduceTuple &t, rift_ile_result &o) {
  o.n = t.n;
  o.n_nonfinite = t.bad;
  o.max_lnw = t.m;
  if (t.n == 0 || t.m == -INFINITY || !(t.s1 > 0.0)) {
    o.lnL_marg = -INFINITY;
    o.n_eff = o.n_ess = o.n_var = 0.0;
    o.sigma_lnL = INFINITY;
    return;
  }
  double N = (double)t.n;
  o.lnL_marg = t.m + log(t.s1) - log(N);
  o.n_eff = t.s1;
  o.n_ess = t.s1 * t.s1 / t.s2;
  double wbar = t.s1 / N;
  double var = t.n > 1 ? (t.s2 - N * wbar * wbar) / (N - 1.0) : 0.0;
  if (var <= 0.0) {
    o.n_var = INFINITY;
    o.sigma_lnL = 0.0;
  } else {
    o.n_var = N * wbar * wbar / var;
    o.sigma_lnL = 1.0 / sqrt(o.n_var);
  }
}

// One workgroup per segment: lane i merges partials i, i + 64, ... in order,
// then a fixed tree over the lanes; the order depends only on bps.
__global__ void __launch_bounds__(64) reduce_finish_kernel(const ReduceTuple *partials, int n_seg, int bps,
                                                           ReduceTuple *round_out, ReduceTuple *accum,
                                                           int accumulate, rift_ile_result *out) {
  __shared__ ReduceTuple sh[64];
  const int seg = blockIdx.x;
  ReduceTuple t = tup_zero();
  for (int j = threadIdx.x; j < bps; j += 64) t = tup_merge(t, partials[(size_t)seg * bps + j]);
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int o = 32; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = tup_merge(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  t = sh[0];
  if (round_out) round_out[seg] = t;
  if (accum) {
    ReduceTuple a = accumulate ? tup_merge(accum[seg], t) : t;
    accum[seg] = a;
    t = a;
  }
  if (out) tuple_result(t, out[seg]);
}

hipError_t reduce_finish(const ReduceTuple *partials, int n_seg, int bps, ReduceTuple *round_out, ReduceTuple *accum,
                         int accumulate, rift_ile_result *out, hipStream_t st) {
  if (n_seg <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_finish_kernel, dim3(n_seg), dim3(64), 0, st, partials, n_seg, bps, round_out, accum,
                     accumulate, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// adaptation.  Each block histograms at most kHistChunk samples of one
// segment in 64-bit fixed point (w = e^{ln w - max} <= 1 scaled by 2^50, so a
// block's sums stay below 2^63), with integer LDS atomics, which are
// associative; the block histograms are merged in block order in FP64, one
// thread per bin.  The result does not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr double kFix = 1125899906842624.0;  // 2^50
constexpr int kHistChunk = 8192;

template <typename R>
__global__ void __launch_bounds__(256) hist_kernel(const uint8_t *bins, int64_t bin_stride, const R *lnw,
                                                   const int64_t *seg_off, const int64_t *seg_cnt, int bps,
                                                   const ReduceTuple *seg_round, unsigned long long *hist) {
  __shared__ unsigned long long h[7 * kNB];
  for (int i = threadIdx.x; i < 7 * kNB; i += 256) h[i] = 0ull;
  __syncthreads();
  const int seg = blockIdx.x / bps, j = blockIdx.x % bps;
  const int64_t cnt = seg_cnt[seg], off = seg_off[seg];
  const int64_t lo = min(cnt, (int64_t)j * kHistChunk), hi = min(cnt, lo + kHistChunk);
  const double mx = seg_round[seg].m;
  if (mx > -INFINITY) {
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
      double x = (double)lnw[off + i];
      if (!(x == x) || x == INFINITY || x == -INFINITY) continue;
      unsigned long long q = (unsigned long long)llrint(exp(x - mx) * kFix);
      if (q == 0ull) continue;
      for (int d = 0; d < 7; d++) atomicAdd(&h[d * kNB + bins[d * bin_stride + off + i]], q);
    }
  }
  __syncthreads();
  unsigned long long *dst = hist + ((size_t)seg * bps + j) * 7 * kNB;
  for (int i = threadIdx.x; i < 7 * kNB; i += 256) dst[i] = h[i];
}

// h_b = (1 - eps - beta) nb m_b / sum m + beta nb a_b / sum a + eps, with a the
// histogram of the points reached by the gradient ascent (beta = 0 without)
// one thread per (segment, parameter, bin): the block histograms summed in
// block order, in FP64, stored over block 0's entry (read only by this thread)
__global__ void hist_merge_kernel(unsigned long long *hist, int bps, int n_seg) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_seg * 7 * kNB) return;
  const int seg = idx / (7 * kNB), db = idx % (7 * kNB);
  double v = 0.0;
  for (int j = 0; j < bps; j++) v += (double)hist[((size_t)seg * bps + j) * 7 * kNB + db];
  hist[(size_t)seg * bps * 7 * kNB + db] = (unsigned long long)__double_as_longlong(v);
}

__global__ void cdf_kernel(const unsigned long long *hist, int bps, const int *seg_prop, int n_seg,
                           ProposalDev *props, unsigned mask, double floor_eps, const double *ahist, double beta) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_seg * 7) return;
  int seg = idx / 7, d = idx % 7;
  ProposalDev &P = props[seg_prop[seg]];
  double m[kNB];
  double tot = 0.0;
  for (int b = 0; b < kNB; b++) {
    const double v = __longlong_as_double((long long)hist[(size_t)seg * bps * 7 * kNB + d * kNB + b]);
    m[b] = v;
    tot += v;
  }
  bool adapt = ((mask >> d) & 1u) && tot > 0.0;
  const double *ah = ahist ? ahist + ((size_t)seg * 7 + d) * kNB : nullptr;
  double atot = 0.0;
  if (ah)
    for (int b = 0; b < kNB; b++) atot += ah[b];
  const double bw = (ah && atot > 0.0) ? beta : 0.0;
  double c = 0.0;
  P.cdf[d][0] = 0.0;
  for (int b = 0; b < kNB; b++) {
    double hb = adapt ? (1.0 - floor_eps - bw) * kNB * (m[b] / tot) + (bw > 0.0 ? bw * kNB * ah[b] / atot : 0.0) +
                            floor_eps
                      : 1.0;
    c += hb / kNB;
    P.cdf[d][b + 1] = c;
  }
  for (int b = 1; b <= kNB; b++) P.cdf[d][b] /= c;
  if (d == 0) {
    P.mask = mask;
    P.gk = 0;  // histogram proposal
  }
}

int hist_blocks(int64_t max_count) { return (int)std::max<int64_t>(1, (max_count + kHistChunk - 1) / kHistChunk); }

template <typename R>
hipError_t adapt_launch(const uint8_t *bins, int64_t bin_stride, const R *lnw, const int64_t *seg_off,
                        const int64_t *seg_cnt, const int *seg_prop, int n_seg, int bps, const ReduceTuple *seg_round,
                        unsigned long long *hist, ProposalDev *props, unsigned mask, double floor_eps, hipStream_t st,
                        const double *ahist, double ascent_mix) {
  if (n_seg <= 0) return hipSuccess;
  hipLaunchKernelGGL(hist_kernel<R>, dim3(n_seg * bps), dim3(256), 0, st, bins, bin_stride, lnw, seg_off, seg_cnt, bps,
                     seg_round, hist);
  hipLaunchKernelGGL(hist_merge_kernel, dim3((n_seg * 7 * kNB + 255) / 256), dim3(256), 0, st, hist, bps, n_seg);
  hipLaunchKernelGGL(cdf_kernel, dim3((n_seg * 7 + 63) / 64), dim3(64), 0, st, hist, bps, seg_prop, n_seg, props, mask,
                     floor_eps, ahist, ascent_mix);
  return hipGetLastError();
}
template hipError_t adapt_launch<float>(const uint8_t *, int64_t, const float *, const int64_t *, const int64_t *,
                                        const int *, int, int, const ReduceTuple *, unsigned long long *,
                                        ProposalDev *, unsigned, double, hipStream_t, const double *, double);
template hipError_t adapt_launch<double>(const uint8_t *, int64_t, const double *, const int64_t *, const int64_t *,
                                         const int *, int, int, const ReduceTuple *, unsigned long long *,
                                         ProposalDev *, unsigned, double, hipStream_t, const double *, double);

// ---------------------------------------------------------------------------
// Gaussian-mixture adaptation (Sec. III.B; App. A): weighted EM in each
// adapted parameter's prior-CDF coordinate, then the online update.  Sums are
// FP64 in a fixed order (each block a fixed range of samples, a fixed tree
// over its threads, blocks merged in block order), so results do not depend
// on scheduling.
// ---------------------------------------------------------------------------
constexpr int kEmChunk = 2048;
constexpr double kSdMin = 1e-4;
int em_blocks(int64_t max_count) { return (int)std::max<int64_t>(1, (max_count + kEmChunk - 1) / kEmChunk); }

__device__ __forceinline__ double phi_cdf(double x) { return 0.5 * erfc(-x * 0.70710678118654752440); }

// the mixture a round starts from: the point's own when it has K components
// and the same pairs, else the initial one (equal weights, means (k + 1/2) /
// K, sd 1 / (2 K); pairs: means on the diagonal, no correlation)
__global__ void gmm_init_kernel(const ProposalDev *props, const int *seg_prop, int n_seg, int K, unsigned pairs,
                                GmmDev *cur, GmmDev *fit) {
  const int seg = blockIdx.x * blockDim.x + threadIdx.x;
  if (seg >= n_seg) return;
  const ProposalDev &P = props[seg_prop[seg]];
  int np = 0, pa[kMaxPair], pb[kMaxPair];
  for (int i = 0; i < kMaxPair; i++) {
    const unsigned c = (pairs >> (8 * i)) & 0xFFu;
    pa[i] = pb[i] = 0;
    if (c) {
      pa[np] = (int)(c & 15u);
      pb[np] = (int)(c >> 4);
      np++;
    }
  }
  bool own = P.gk == K && P.npair == np;
  for (int i = 0; i < np && own; i++) own = P.pa[i] == pa[i] && P.pb[i] == pb[i];
  GmmDev &c = cur[seg], &f = fit[seg];
  c.k = f.k = K;
  c.npair = f.npair = np;
  c.ntr = f.ntr = own ? P.gntr : 0.0;
  for (int d = 0; d < 7; d++)
    for (int k = 0; k < kMaxG; k++) {
      c.w[d][k] = f.w[d][k] = own ? P.gw[d][k] : (k < K ? 1.0 / K : 0.0);
      c.mu[d][k] = f.mu[d][k] = own ? P.gmu[d][k] : (k + 0.5) / K;
      c.sd[d][k] = f.sd[d][k] = own ? P.gsd[d][k] : 0.5 / K;
    }
  for (int i = 0; i < kMaxPair; i++) {
    c.pa[i] = f.pa[i] = pa[i];
    c.pb[i] = f.pb[i] = pb[i];
    for (int k = 0; k < kMaxG; k++) {
      c.pw[i][k] = f.pw[i][k] = own ? P.pw[i][k] : (k < K ? 1.0 / K : 0.0);
      for (int q = 0; q < 2; q++) c.pmu[i][k][q] = f.pmu[i][k][q] = own ? P.pmu[i][k][q] : (k + 0.5) / K;
      const double v0 = 0.25 / ((double)K * K);
      c.pcov[i][k][0] = f.pcov[i][k][0] = own ? P.pcov[i][k][0] : v0;
      c.pcov[i][k][1] = f.pcov[i][k][1] = own ? P.pcov[i][k][1] : 0.0;
      c.pcov[i][k][2] = f.pcov[i][k][2] = own ? P.pcov[i][k][2] : v0;
    }
  }
}

// E-step and the M-step sums of one block: for each adapted d and component
// k, S0 = sum w r, S1 = sum w r (u - mu_k), S2 = sum w r (u - mu_k)^2 with
// w = e^{ln w - max ln w} and r the responsibility (untruncated normals)
__global__ void __launch_bounds__(256) em_partials_kernel(const float *ub, int64_t us, const double *wbuf,
                                                          const int64_t *seg_off, const int64_t *seg_cnt, int bps,
                                                          const ReduceTuple *seg_round, const GmmDev *fit,
                                                          unsigned mask, double *part) {
  __shared__ double red[256][3 * kMaxG];
  const int seg = blockIdx.x / bps, j = blockIdx.x % bps;
  const int64_t cnt = seg_cnt[seg], off = seg_off[seg];
  const int64_t lo = min(cnt, (int64_t)j * kEmChunk), hi = min(cnt, lo + kEmChunk);
  const double mx = seg_round[seg].m;
  const GmmDev &F = fit[seg];
  const int K = F.k;
  for (int d = 0; d < 7; d++) {
    if (!((mask >> d) & 1u)) continue;
    double acc[3 * kMaxG];
    double lw[kMaxG], mu[kMaxG], isd[kMaxG];
#pragma unroll
    for (int q = 0; q < 3 * kMaxG; q++) acc[q] = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxG; k++) {
      lw[k] = (k < K && F.w[d][k] > 0.0) ? log(F.w[d][k]) - log(F.sd[d][k]) : -INFINITY;
      mu[k] = F.mu[d][k];
      isd[k] = 1.0 / F.sd[d][k];
    }
    if (mx > -INFINITY) {
      for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
        const double wt = wbuf[off + i];
        if (!(wt > 0.0)) continue;
        const double uu = (double)ub[d * us + off + i];
        double lp[kMaxG], m = -INFINITY;
#pragma unroll
        for (int k = 0; k < kMaxG; k++) {
          const double t = (uu - mu[k]) * isd[k];
          lp[k] = lw[k] - 0.5 * t * t;
          m = fmax(m, lp[k]);
        }
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxG; k++) {
          lp[k] = lw[k] == -INFINITY ? 0.0 : exp(lp[k] - m);
          sum += lp[k];
        }
#pragma unroll
        for (int k = 0; k < kMaxG; k++) {
          const double r = wt * (lp[k] / sum), dk = uu - mu[k];
          acc[3 * k] += r;
          acc[3 * k + 1] += r * dk;
          acc[3 * k + 2] += r * dk * dk;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 3 * kMaxG; q++) red[threadIdx.x][q] = acc[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o)
#pragma unroll
        for (int q = 0; q < 3 * kMaxG; q++) red[threadIdx.x][q] += red[threadIdx.x + o][q];
      __syncthreads();
    }
    if (threadIdx.x < 3 * kMaxG) part[(((size_t)seg * bps + j) * 7 + d) * 3 * kMaxG + threadIdx.x] = red[0][threadIdx.x];
    __syncthreads();
  }
}

// the round's weights w = e^{ln w - max ln w} (0 for non-finite ln w), once
// per adaptation for all EM iterations
template <typename R>
__global__ void __launch_bounds__(256) em_weight_kernel(const R *lnw, const int64_t *seg_off, const int64_t *seg_cnt,
                                                        const int *blk0, int n_seg, const ReduceTuple *seg_round,
                                                        double *wbuf) {
  int lo = 0, hi = n_seg;  // blk0[lo] <= blockIdx.x < blk0[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (blk0[mid] <= (int)blockIdx.x) lo = mid; else hi = mid;
  }
  const int seg = lo;
  const int64_t i = (int64_t)(blockIdx.x - blk0[seg]) * 256 + threadIdx.x;
  if (i >= seg_cnt[seg]) return;
  const int64_t c = seg_off[seg] + i;
  const double x = (double)lnw[c], mx = seg_round[seg].m;
  wbuf[c] = (!(x == x) || x == INFINITY || x == -INFINITY || !(mx > -INFINITY)) ? 0.0 : exp(x - mx);
}

// the blocks' partial sums [n_seg][bps][X] merged in block order, one
// thread per (segment, entry), into block 0's entry (read only by this thread)
__global__ void sum_blocks_kernel(double *part, int n_seg, int bps, int X) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_seg * X) return;
  const int seg = idx / X, x = idx % X;
  double v = 0.0;
  for (int j = 0; j < bps; j++) v += part[((size_t)seg * bps + j) * X + x];
  part[(size_t)seg * bps * X + x] = v;
}

// M-step: the summed moments -> new weights, means, sds
__global__ void em_update_kernel(const double *part, int n_seg, int bps, GmmDev *fit, unsigned mask) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_seg * 7) return;
  const int seg = idx / 7, d = idx % 7;
  if (!((mask >> d) & 1u)) return;
  GmmDev &F = fit[seg];
  const int K = F.k;
  double S[3 * kMaxG];  // the blocks' sums, merged into block 0 by sum_blocks_kernel
  for (int q = 0; q < 3 * kMaxG; q++) S[q] = part[((size_t)seg * bps * 7 + d) * 3 * kMaxG + q];
  double tot = 0.0;
  for (int k = 0; k < K; k++) tot += S[3 * k];
  if (!(tot > 0.0)) return;
  for (int k = 0; k < K; k++) {
    const double s0 = S[3 * k];
    if (s0 > 0.0) {
      const double m1 = S[3 * k + 1] / s0, m2 = S[3 * k + 2] / s0;
      F.mu[d][k] += m1;
      F.sd[d][k] = fmax(sqrt(fmax(m2 - m1 * m1, 0.0)), kSdMin);
    }
    F.w[d][k] = s0 / tot;
  }
}

// sd >= kSdMin per axis, |correlation| <= kRhoMax
constexpr double kRhoMax = 0.99;
__device__ __forceinline__ void regularize(double &xx, double &xy, double &yy) {
  xx = fmax(xx, kSdMin * kSdMin);
  yy = fmax(yy, kSdMin * kSdMin);
  const double cm = kRhoMax * sqrt(xx * yy);
  xy = fmin(fmax(xy, -cm), cm);
}

// pairs: E-step and sums of one block, per pair and component S0, Sx, Sy,
// Sxx, Sxy, Syy (moments about the component's current mean)
__global__ void __launch_bounds__(256) em_pair_partials_kernel(const float *ub, int64_t us, const double *wbuf,
                                                               const int64_t *seg_off, const int64_t *seg_cnt,
                                                               int bps, const ReduceTuple *seg_round,
                                                               const GmmDev *fit, double *part2) {
  __shared__ double red[256][6 * kMaxG];
  const int seg = blockIdx.x / bps, j = blockIdx.x % bps;
  const int64_t cnt = seg_cnt[seg], off = seg_off[seg];
  const int64_t lo = min(cnt, (int64_t)j * kEmChunk), hi = min(cnt, lo + kEmChunk);
  const double mx = seg_round[seg].m;
  const GmmDev &F = fit[seg];
  const int K = F.k;
  for (int p = 0; p < F.npair; p++) {
    const int a = F.pa[p], b = F.pb[p];
    double acc[6 * kMaxG];
    double lw[kMaxG], m0[kMaxG], m1[kMaxG], i0[kMaxG], i1[kMaxG], i2[kMaxG];
#pragma unroll
    for (int q = 0; q < 6 * kMaxG; q++) acc[q] = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxG; k++) {
      const double c0 = F.pcov[p][k][0], c1 = F.pcov[p][k][1], c2 = F.pcov[p][k][2];
      const double det = c0 * c2 - c1 * c1;
      i0[k] = c2 / det;
      i1[k] = -c1 / det;
      i2[k] = c0 / det;
      lw[k] = (k < K && F.pw[p][k] > 0.0) ? log(F.pw[p][k]) - 0.5 * log(det) : -INFINITY;
      m0[k] = F.pmu[p][k][0];
      m1[k] = F.pmu[p][k][1];
    }
    if (mx > -INFINITY) {
      for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
        const double wt = wbuf[off + i];
        if (!(wt > 0.0)) continue;
        const double ux = (double)ub[a * us + off + i], uy = (double)ub[b * us + off + i];
        double lp[kMaxG], m = -INFINITY;
#pragma unroll
        for (int k = 0; k < kMaxG; k++) {
          const double dx = ux - m0[k], dy = uy - m1[k];
          lp[k] = lw[k] - 0.5 * (i0[k] * dx * dx + 2.0 * i1[k] * dx * dy + i2[k] * dy * dy);
          m = fmax(m, lp[k]);
        }
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxG; k++) {
          lp[k] = lw[k] == -INFINITY ? 0.0 : exp(lp[k] - m);
          sum += lp[k];
        }
#pragma unroll
        for (int k = 0; k < kMaxG; k++) {
          const double r = wt * (lp[k] / sum), dx = ux - m0[k], dy = uy - m1[k];
          acc[6 * k] += r;
          acc[6 * k + 1] += r * dx;
          acc[6 * k + 2] += r * dy;
          acc[6 * k + 3] += r * dx * dx;
          acc[6 * k + 4] += r * dx * dy;
          acc[6 * k + 5] += r * dy * dy;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 6 * kMaxG; q++) red[threadIdx.x][q] = acc[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o)
#pragma unroll
        for (int q = 0; q < 6 * kMaxG; q++) red[threadIdx.x][q] += red[threadIdx.x + o][q];
      __syncthreads();
    }
    if (threadIdx.x < 6 * kMaxG)
      part2[(((size_t)seg * bps + j) * kMaxPair + p) * 6 * kMaxG + threadIdx.x] = red[0][threadIdx.x];
    __syncthreads();
  }
}

__global__ void em_pair_update_kernel(const double *part2, int n_seg, int bps, GmmDev *fit) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_seg * kMaxPair) return;
  const int seg = idx / kMaxPair, p = idx % kMaxPair;
  GmmDev &F = fit[seg];
  if (p >= F.npair) return;
  const int K = F.k;
  double S[6 * kMaxG];  // the blocks' sums, merged into block 0 by sum_blocks_kernel
  for (int q = 0; q < 6 * kMaxG; q++) S[q] = part2[((size_t)seg * bps * kMaxPair + p) * 6 * kMaxG + q];
  double tot = 0.0;
  for (int k = 0; k < K; k++) tot += S[6 * k];
  if (!(tot > 0.0)) return;
  for (int k = 0; k < K; k++) {
    const double s0 = S[6 * k];
    if (s0 > 0.0) {
      const double mx = S[6 * k + 1] / s0, my = S[6 * k + 2] / s0;
      double xx = S[6 * k + 3] / s0 - mx * mx, xy = S[6 * k + 4] / s0 - mx * my, yy = S[6 * k + 5] / s0 - my * my;
      F.pmu[p][k][0] += mx;
      F.pmu[p][k][1] += my;
      regularize(xx, xy, yy);
      F.pcov[p][k][0] = xx;
      F.pcov[p][k][1] = xy;
      F.pcov[p][k][2] = yy;
    }
    F.pw[p][k] = s0 / tot;
  }
}

__device__ __forceinline__ double maha(double dx, double dy, const double *c) {
  const double det = c[0] * c[2] - c[1] * c[1];
  return sqrt(fmax((c[2] * dx * dx - 2.0 * c[1] * dx * dy + c[0] * dy * dy) / det, 0.0));
}

__device__ bool next_perm(int *p, int n);

// pairs: online update (App. A) with the text's symmetric Mahalanobis
// distances, each component's own covariance
__global__ void gmm_pair_merge_kernel(const GmmDev *cur, const GmmDev *fit, int n_seg, const int *seg_prop,
                                      const ReduceTuple *seg_round, ProposalDev *props) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_seg * kMaxPair) return;
  const int seg = idx / kMaxPair, p = idx % kMaxPair;
  const GmmDev &C = cur[seg], &F = fit[seg];
  ProposalDev &P = props[seg_prop[seg]];
  if (p >= C.npair) return;
  const int K = C.k;
  const bool any = seg_round[seg].m > -INFINITY;
  const double N = C.ntr, M = (double)seg_round[seg].n;
  const bool take_new = any && !(N > 0.0);
  for (int k = 0; k < kMaxG; k++) {
    const GmmDev &S = (take_new && k < K) ? F : C;
    P.pw[p][k] = S.pw[p][k];
    for (int q = 0; q < 2; q++) P.pmu[p][k][q] = S.pmu[p][k][q];
    for (int q = 0; q < 3; q++) P.pcov[p][k][q] = S.pcov[p][k][q];
  }
  if (!any || take_new) return;
  int pr[kMaxG], bp[kMaxG];
  for (int k = 0; k < K; k++) pr[k] = bp[k] = k;
  double best = INFINITY;
  do {
    double s = 0.0;
    for (int i = 0; i < K; i++) {
      const int jj = pr[i];
      const double dx = C.pmu[p][jj][0] - F.pmu[p][i][0], dy = C.pmu[p][jj][1] - F.pmu[p][i][1];
      s += maha(dx, dy, F.pcov[p][i]) + maha(dx, dy, C.pcov[p][jj]);
    }
    if (s < best) {
      best = s;
      for (int k = 0; k < K; k++) bp[k] = pr[k];
    }
  } while (next_perm(pr, K));
  for (int i = 0; i < K; i++) {
    const int jj = bp[i];
    const double a = N * C.pw[p][jj], b = M * F.pw[p][i];
    if (!(a + b > 0.0)) {
      P.pw[p][jj] = 0.0;
      continue;
    }
    const double dx = C.pmu[p][jj][0] - F.pmu[p][i][0], dy = C.pmu[p][jj][1] - F.pmu[p][i][1];
    const double f = a * b / ((a + b) * (a + b));
    P.pmu[p][jj][0] = (a * C.pmu[p][jj][0] + b * F.pmu[p][i][0]) / (a + b);
    P.pmu[p][jj][1] = (a * C.pmu[p][jj][1] + b * F.pmu[p][i][1]) / (a + b);
    double xx = (a * C.pcov[p][jj][0] + b * F.pcov[p][i][0]) / (a + b) + f * dx * dx;
    double xy = (a * C.pcov[p][jj][1] + b * F.pcov[p][i][1]) / (a + b) + f * dx * dy;
    double yy = (a * C.pcov[p][jj][2] + b * F.pcov[p][i][2]) / (a + b) + f * dy * dy;
    regularize(xx, xy, yy);
    P.pcov[p][jj][0] = xx;
    P.pcov[p][jj][1] = xy;
    P.pcov[p][jj][2] = yy;
    P.pw[p][jj] = (a + b) / (N + M);
  }
}

// derived pair quantities, one 256-thread block per (point, pair): thread
// (k, q) integrates panel q of 64 of component k's mass in the unit square,
// Z = int_0^1 N(x; mx, sx) [Phi((1 - m(x)) / s) - Phi(-m(x) / s)] dx with
// m(x) the conditional mean of y and s its sd, over [mx - 9 sx, mx + 9 sx]
// clipped to [0, 1], 8-point Gauss-Legendre per panel; a fixed tree sums
__global__ void __launch_bounds__(256) pair_norm_kernel(ProposalDev *props, int p0) {
  __shared__ double red[256];
  ProposalDev &P = props[p0 + blockIdx.x / kMaxPair];
  const int p = blockIdx.x % kMaxPair;
  if (P.gk <= 0 || p >= P.npair) return;  // uniform over the block
  const int K = P.gk, k = threadIdx.x / 64, q = threadIdx.x % 64;
  double zq = 0.0;
  if (k < K) {
    const double mx = P.pmu[p][k][0], my = P.pmu[p][k][1];
    const double cxx = P.pcov[p][k][0], cxy = P.pcov[p][k][1], cyy = P.pcov[p][k][2];
    const double sx = sqrt(cxx), bc = cxy / cxx, sc = sqrt(fmax(cyy - cxy * cxy / cxx, 0.0));
    const double lo = fmax(0.0, mx - 9.0 * sx), hi = fmin(1.0, mx + 9.0 * sx);
    if (hi > lo) {
      const double gx[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
      const double gw[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
      const double h = (hi - lo) / 64.0, c = lo + (q + 0.5) * h;
      for (int n = 0; n < 8; n++) {
        const double x = c + 0.5 * h * (n < 4 ? -gx[3 - n] : gx[n - 4]);
        const double wgt = n < 4 ? gw[3 - n] : gw[n - 4];
        const double m = my + bc * (x - mx), A = -m / sc, B = (1.0 - m) / sc;
        const double d = A > 0.0 ? 0.5 * (erfc(A * 0.70710678118654752440) - erfc(B * 0.70710678118654752440))
                                 : 0.5 * (erfc(-B * 0.70710678118654752440) - erfc(-A * 0.70710678118654752440));
        const double t = (x - mx) / sx;
        zq += wgt * exp(-0.5 * t * t) / (sx * kSqrt2Pi) * d;
      }
      zq *= 0.5 * h;
    }
  }
  red[threadIdx.x] = zq;
  __syncthreads();
  // per component: a fixed tree over its 64 panels
  for (int o = 32; o > 0; o >>= 1) {
    if (q < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double zm = 0.0;
  for (int kk = 0; kk < kMaxG; kk++) {
    const double c0 = P.pcov[p][kk][0], c1 = P.pcov[p][kk][1], c2 = P.pcov[p][kk][2];
    const double det = c0 * c2 - c1 * c1;
    const double l11 = sqrt(c0), l21 = c1 / l11;
    P.pch[p][kk][0] = l11;
    P.pch[p][kk][1] = l21;
    P.pch[p][kk][2] = sqrt(fmax(c2 - l21 * l21, 0.0));
    P.pic[p][kk][0] = c2 / det;
    P.pic[p][kk][1] = -c1 / det;
    P.pic[p][kk][2] = c0 / det;
    const bool on = kk < K && P.pw[p][kk] > 0.0;
    P.plog[p][kk] = on ? log(P.pw[p][kk]) - log(2.0 * kPi) - 0.5 * log(det) : -INFINITY;
    if (on) zm += P.pw[p][kk] * red[64 * kk];
  }
  P.pzm[p] = zm;
}

hipError_t pair_norm_launch(ProposalDev *props, int p0, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(pair_norm_kernel, dim3(n * kMaxPair), dim3(256), 0, st, props, p0);
  return hipGetLastError();
}

__device__ bool next_perm(int *p, int n) {
  int i = n - 2;
  while (i >= 0 && p[i] >= p[i + 1]) i--;
  if (i < 0) return false;
  int j = n - 1;
  while (p[j] <= p[i]) j--;
  int t = p[i];
  p[i] = p[j];
  p[j] = t;
  for (int a = i + 1, b = n - 1; a < b; a++, b--) {
    t = p[a];
    p[a] = p[b];
    p[b] = t;
  }
  return true;
}

// online update (App. A): new component i is matched to old component p[i]
// by the smallest summed symmetric Mahalanobis distance over all
// permutations (the first minimum in lexicographic order), then combined
// with the sample counts N (earlier rounds) and M (this round)
__global__ void gmm_merge_kernel(const GmmDev *cur, const GmmDev *fit, int n_seg, const int *seg_prop,
                                 const ReduceTuple *seg_round, ProposalDev *props, unsigned mask, unsigned mask_all,
                                 double eps) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // one thread per (segment, parameter)
  if (idx >= n_seg * 7) return;
  const int seg = idx / 7, d = idx % 7;
  const GmmDev &C = cur[seg], &F = fit[seg];
  ProposalDev &P = props[seg_prop[seg]];
  const int K = C.k;
  const bool any = seg_round[seg].m > -INFINITY;
  const double N = C.ntr, M = (double)seg_round[seg].n;
  for (int k = 0; k < kMaxG; k++) {
    P.gw[d][k] = C.w[d][k];
    P.gmu[d][k] = C.mu[d][k];
    P.gsd[d][k] = C.sd[d][k];
  }
  if (any && ((mask >> d) & 1u) && !(N > 0.0)) {
    for (int k = 0; k < K; k++) {
      P.gw[d][k] = F.w[d][k];
      P.gmu[d][k] = F.mu[d][k];
      P.gsd[d][k] = F.sd[d][k];
    }
  } else if (any && ((mask >> d) & 1u)) {
    int p[kMaxG], bp[kMaxG];
    for (int k = 0; k < K; k++) p[k] = bp[k] = k;
    double best = INFINITY;
    do {
      double s = 0.0;
      for (int i = 0; i < K; i++) {
        const double dd = fabs(F.mu[d][i] - C.mu[d][p[i]]);
        s += dd / F.sd[d][i] + dd / C.sd[d][p[i]];
      }
      if (s < best) {
        best = s;
        for (int k = 0; k < K; k++) bp[k] = p[k];
      }
    } while (next_perm(p, K));
    for (int i = 0; i < K; i++) {
      const int jj = bp[i];
      const double a = N * C.w[d][jj], b = M * F.w[d][i];
      if (!(a + b > 0.0)) {
        P.gw[d][jj] = 0.0;
        continue;
      }
      const double mu = (a * C.mu[d][jj] + b * F.mu[d][i]) / (a + b), dm = C.mu[d][jj] - F.mu[d][i];
      const double var = (a * C.sd[d][jj] * C.sd[d][jj] + b * F.sd[d][i] * F.sd[d][i]) / (a + b) +
                         a * b * dm * dm / ((a + b) * (a + b));
      P.gmu[d][jj] = mu;
      P.gsd[d][jj] = fmax(sqrt(var), kSdMin);
      P.gw[d][jj] = (a + b) / (N + M);
    }
  }
  for (int k = 0; k < kMaxG; k++) {
    const double ca = phi_cdf(-P.gmu[d][k] / P.gsd[d][k]);
    P.gca[d][k] = ca;
    P.gz[d][k] = phi_cdf((1.0 - P.gmu[d][k]) / P.gsd[d][k]) - ca;
  }
  if (d == 0) {  // the segment's scalars (no thread reads them here)
    P.gk = K;
    P.gntr = any ? N + M : N;
    P.geps = eps;
    P.mask = mask_all;
    P.npair = C.npair;
    for (int i = 0; i < kMaxPair; i++) {
      P.pa[i] = C.pa[i];
      P.pb[i] = C.pb[i];
    }
  }
}

template <typename R>
hipError_t gmm_adapt_launch(const float *ubuf, int64_t u_stride, const R *lnw, const int64_t *seg_off,
                            const int64_t *seg_cnt, const int *seg_prop, int n_seg, int bps,
                            const ReduceTuple *seg_round, double *part, double *part2, GmmDev *fit,
                            ProposalDev *props, unsigned mask, unsigned pairs, double floor_eps, int K, int n_iter,
                            const int *blk0, int wblk, double *wbuf, hipStream_t st) {
  if (n_seg <= 0) return hipSuccess;
  unsigned pm = 0u;  // parameters in pairs: not fitted one by one
  for (int i = 0; i < kMaxPair; i++) {
    const unsigned c = (pairs >> (8 * i)) & 0xFFu;
    if (c) pm |= (1u << (c & 15u)) | (1u << (c >> 4));
  }
  const unsigned m1 = mask & ~pm;
  const dim3 g1((n_seg + 63) / 64), g7((n_seg * 7 + 63) / 64), g3((n_seg * kMaxPair + 63) / 64);
  hipLaunchKernelGGL(gmm_init_kernel, g1, dim3(64), 0, st, props, seg_prop, n_seg, K, pairs, fit, fit + n_seg);
  if (wblk > 0)
    hipLaunchKernelGGL(em_weight_kernel<R>, dim3(wblk), dim3(256), 0, st, lnw, seg_off, seg_cnt, blk0, n_seg,
                       seg_round, wbuf);
  for (int it = 0; it < n_iter; it++) {
    if (m1) {
      hipLaunchKernelGGL(em_partials_kernel, dim3(n_seg * bps), dim3(256), 0, st, ubuf, u_stride, wbuf, seg_off,
                         seg_cnt, bps, seg_round, fit + n_seg, m1, part);
      hipLaunchKernelGGL(sum_blocks_kernel, dim3((n_seg * 7 * 3 * kMaxG + 255) / 256), dim3(256), 0, st, part, n_seg,
                         bps, 7 * 3 * kMaxG);
      hipLaunchKernelGGL(em_update_kernel, g7, dim3(64), 0, st, part, n_seg, bps, fit + n_seg, m1);
    }
    if (pairs) {
      hipLaunchKernelGGL(em_pair_partials_kernel, dim3(n_seg * bps), dim3(256), 0, st, ubuf, u_stride, wbuf,
                         seg_off, seg_cnt, bps, seg_round, fit + n_seg, part2);
      hipLaunchKernelGGL(sum_blocks_kernel, dim3((n_seg * kMaxPair * 6 * kMaxG + 255) / 256), dim3(256), 0, st, part2,
                         n_seg, bps, kMaxPair * 6 * kMaxG);
      hipLaunchKernelGGL(em_pair_update_kernel, g3, dim3(64), 0, st, part2, n_seg, bps, fit + n_seg);
    }
  }
  hipLaunchKernelGGL(gmm_merge_kernel, g7, dim3(64), 0, st, fit, fit + n_seg, n_seg, seg_prop, seg_round, props, m1,
                     mask, floor_eps);
  hipLaunchKernelGGL(gmm_pair_merge_kernel, g3, dim3(64), 0, st, fit, fit + n_seg, n_seg, seg_prop, seg_round, props);
  return hipGetLastError();
}
template hipError_t gmm_adapt_launch<float>(const float *, int64_t, const float *, const int64_t *, const int64_t *,
                                            const int *, int, int, const ReduceTuple *, double *, double *, GmmDev *,
                                            ProposalDev *, unsigned, unsigned, double, int, int, const int *, int,
                                            double *, hipStream_t);
template hipError_t gmm_adapt_launch<double>(const float *, int64_t, const double *, const int64_t *,
                                             const int64_t *, const int *, int, int, const ReduceTuple *, double *,
                                             double *, GmmDev *, ProposalDev *, unsigned, unsigned, double, int, int,
                                             const int *, int, double *, hipStream_t);

// host: the same normalizations for a mixture set by the caller
void gmm_norms(ProposalDev &p) {
  for (int d = 0; d < 7; d++)
    for (int k = 0; k < kMaxG; k++) {
      const double ca = 0.5 * std::erfc(p.gmu[d][k] / p.gsd[d][k] * 0.70710678118654752440);
      p.gca[d][k] = ca;
      p.gz[d][k] = 0.5 * std::erfc(-(1.0 - p.gmu[d][k]) / p.gsd[d][k] * 0.70710678118654752440) - ca;
    }
}

// ---------------------------------------------------------------------------
__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace rift
