// Distance marginalization (Sec. III.B, distance marginalization; the
// production configuration of Sec. III pairs it with the adaptive
// integrator).  The paper cites the technique without formulas; the form
// built here integrates the time-marginalized likelihood against the
// sampler's distance prior p(D) = 3 D^2 / (d_max^3 - d_min^3):
//   L_tD = int p(D) (1/n_t) sum_j exp(ell_j(D)) dD.
// a_km scales as 1/D and B as 1/D^2 (App. D Eq. (def:lnL:Decomposed)), so
// with x = D_ref / D every window value is ell_j = x A_j - x^2 B, where A_j is
// the data term and B the quadratic term at D = D_ref.  One evaluation at
// D_ref gives every A_j; the integral over D is then a one-dimensional
// quadrature per sample, in t = ln x, where p(D) dD = c x^-3 dt with
// c = 3 D_ref^3 / (d_max^3 - d_min^3):
//   L_tD = (1/n_t) sum_i W_i exp(x_i A_max - x_i^2 B) S_i,
//   S_i = sum_j exp(x_i (A_j - A_max)),   W_i = c x_i^-3 (quadrature weight),
// A_max = max_j A_j (so every term of S_i is at most 1 and the largest is 1).
// Nodes: Gauss-Legendre in t on the interval where the envelope
// E(t) = x A_max - x^2 B - 3 t (an upper bound of every term's log) is within
// T of its largest value on the prior's range; outside it the n_t terms
// together are below n_t e^-T of the peak.  E has at most two stationary
// points (roots of 2 B x^2 - A x + 3 = 0), so the range splits into at most
// three monotone pieces and each end of the interval is found by bisection on
// one of them.
#pragma once
#include "common.h"

namespace rift {

// 24-point Gauss-Legendre rule on [-1, 1], positive half (nodes ascending);
// the published values (Abramowitz and Stegun, Table 25.4)
constexpr int kDmGL = 24;
constexpr double kDmNode[12] = {0.0640568928626056, 0.1911188674736163, 0.3150426796961634, 0.4337935076260451,
                                0.5454214713888395, 0.6480936519369756, 0.7401241915785544, 0.8200019859739029,
                                0.8864155270044011, 0.9382745520027328, 0.9747285559713095, 0.9951872199970214};
constexpr double kDmWeight[12] = {0.1279381953467522, 0.1258374563468283, 0.1216704729278034, 0.1155056680537256,
                                  0.1074442701159656, 0.0976186521041139, 0.0861901615319533, 0.0733464814110803,
                                  0.0592985849154368, 0.0442774388174198, 0.0285313886289337, 0.0123412297999872};

// node q of the 24 on [-1, 1], ascending, and its weight
__host__ __device__ constexpr double dm_gl_node(int q) { return q < 12 ? -kDmNode[11 - q] : kDmNode[q - 12]; }
__host__ __device__ constexpr double dm_gl_weight(int q) { return q < 12 ? kDmWeight[11 - q] : kDmWeight[q - 12]; }

// Rule per bulk precision: panels of 24 nodes and the envelope threshold T
// (nats).  FP32: one panel, T = 30 (quadrature error below 1e-5 in ln L_tD,
// under the FP32 rounding of the window values of a loud sample); FP64: three
// panels, T = 50 (below 1e-10).
template <typename R>
struct DmRule;
template <>
struct DmRule<float> {
  static constexpr int P = 1;
  static constexpr double T = 30.0;
};
template <>
struct DmRule<double> {
  static constexpr int P = 3;
  static constexpr double T = 50.0;
};

template <typename F>
__device__ __forceinline__ F dm_exp(F v);
template <>
__device__ __forceinline__ float dm_exp<float>(float v) { return expf(v); }
template <>
__device__ __forceinline__ double dm_exp<double>(double v) { return exp(v); }
template <typename F>
__device__ __forceinline__ F dm_log(F v);
template <>
__device__ __forceinline__ float dm_log<float>(float v) { return logf(v); }
template <>
__device__ __forceinline__ double dm_log<double>(double v) { return log(v); }

// Interval [ta, tb] of t = ln x (within [t_lo, t_hi]) where
// E(t) = x A - x^2 B - 3 t >= max E - T.  A, B in nats (B >= 0 for physical
// inputs; B < 0 only moves the maximum to an end).  iters bisection steps.
// The breakpoints are the ends and the stationary points clamped to the range
// (missing ones repeat an end), so every loop has a fixed trip count and the
// arrays stay in registers.
template <typename F>
__device__ inline void dm_interval(F A, F B, F t_lo, F t_hi, F T, int iters, F &ta, F &tb) {
  auto E = [&](F t) {
    const F x = dm_exp<F>(t);
    return x * A - x * x * B - F(3) * t;
  };
  // stationary points: positive roots x of 2 B x^2 - A x + 3 = 0
  F x0 = F(-1), x1 = F(-1);
  if (B == F(0)) {
    if (A > F(0)) x0 = F(3) / A;
  } else {
    const F disc = A * A - F(24) * B;
    if (disc >= F(0)) {
      // stable roots: q = (A + sign(A) sqrt(disc)) / 2, x = q / 2B and 3 / q
      const F sq = sqrt(disc);
      const F q = F(0.5) * (A + (A >= F(0) ? sq : -sq));
      if (q != F(0)) {
        x0 = q / (F(2) * B);
        x1 = F(3) / q;
      }
    }
  }
  F s0 = x0 > F(0) ? fmin(fmax(dm_log<F>(x0), t_lo), t_hi) : t_lo;
  F s1 = x1 > F(0) ? fmin(fmax(dm_log<F>(x1), t_lo), t_hi) : t_lo;
  if (s1 < s0) {
    const F tmp = s0;
    s0 = s1;
    s1 = tmp;
  }
  const F br[4] = {t_lo, s0, s1, t_hi};
  F Eb[4];
  F emax = -INFINITY;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    Eb[i] = E(br[i]);
    emax = fmax(emax, Eb[i]);
  }
  const F thr = emax - T;
  // E is monotone between consecutive breakpoints.  Left end: the first
  // breakpoint at or above thr, or the crossing inside the piece before it.
  F u = t_lo, v = t_lo;
  bool done = false, cross = false;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    if (!done && Eb[i] >= thr) {
      done = true;
      if (i > 0) {
        u = br[i - 1];
        v = br[i];
        cross = true;
      } else {
        v = br[0];
      }
    }
  }
  if (cross) {
    for (int k = 0; k < iters; k++) {
      const F m = F(0.5) * (u + v);
      if (E(m) >= thr) v = m; else u = m;
    }
    ta = u;
  } else {
    ta = v;
  }
  // right end: the last breakpoint at or above thr, or the crossing after it
  u = t_hi;
  v = t_hi;
  done = false;
  cross = false;
#pragma unroll
  for (int i = 3; i >= 0; i--) {
    if (!done && Eb[i] >= thr) {
      done = true;
      if (i < 3) {
        u = br[i];
        v = br[i + 1];
        cross = true;
      } else {
        u = br[3];
      }
    }
  }
  if (cross) {
    for (int k = 0; k < iters; k++) {
      const F m = F(0.5) * (u + v);
      if (E(m) >= thr) u = m; else v = m;
    }
    tb = v;
  } else {
    tb = u;
  }
  if (!(tb > ta)) {  // a single point (or a non-finite envelope): the whole range
    ta = t_lo;
    tb = t_hi;
  }
}

}  // namespace rift
