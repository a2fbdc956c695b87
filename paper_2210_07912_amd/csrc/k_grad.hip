// Gradient-informed refinement of the histogram proposal.
//
// Between rounds, the samples of largest ln w of each point climb ln L_t
// along its gradient (the adjoint of the likelihood: k_bwd.hip on the
// matrix cores for FP32 handles, k_plain.hip for FP64) in the
// prior-CDF coordinates u of the adapted parameters, where the prior is
// uniform on the unit cube.  Steps are normalized, u <- u + eta g_u/|g_u|,
// and kept only when ln L_t rises (eta grows by 1.25 on success, halves on
// failure).  The points reached then carry a fraction of the next round's
// histogram mass.  This chooses the proposal only; the importance weights
// of the next round use that proposal's exact density.
#include "common.h"
#include "internal.h"

namespace rift {

// prior-CDF coordinate u(theta_d) and the Jacobian d theta_d / d u
__device__ __forceinline__ double prior_u(int d, double t, double d_min, double d_max, double tw) {
  switch (d) {
    case RIFT_ALPHA: return t / (2.0 * kPi);
    case RIFT_DELTA: return 0.5 * (sin(t) + 1.0);
    case RIFT_PSI: return t / kPi;
    case RIFT_IOTA: return 0.5 * (1.0 + cos(t));
    case RIFT_PHI: return t / (2.0 * kPi);
    case RIFT_DIST: {
      double a3 = d_min * d_min * d_min, b3 = d_max * d_max * d_max;
      return (t * t * t - a3) / (b3 - a3);
    }
    default: return tw > 0.0 ? t / tw + 0.5 : 0.5;
  }
}

__device__ __forceinline__ double dtheta_du(int d, double t, double d_min, double d_max, double tw) {
  switch (d) {
    case RIFT_ALPHA: return 2.0 * kPi;
    case RIFT_DELTA: return 2.0 / fmax(cos(t), 1e-12);
    case RIFT_PSI: return kPi;
    case RIFT_IOTA: return -2.0 / fmax(sin(t), 1e-12);
    case RIFT_PHI: return 2.0 * kPi;
    case RIFT_DIST: {
      double a3 = d_min * d_min * d_min, b3 = d_max * d_max * d_max;
      return (b3 - a3) / (3.0 * t * t);
    }
    default: return tw;
  }
}

__device__ __forceinline__ double theta_of_u(int d, double u, double d_min, double d_max, double tw) {
  switch (d) {
    case RIFT_ALPHA: return 2.0 * kPi * u;
    case RIFT_DELTA: return asin(2.0 * u - 1.0);
    case RIFT_PSI: return kPi * u;
    case RIFT_IOTA: return acos(2.0 * u - 1.0);
    case RIFT_PHI: return 2.0 * kPi * u;
    case RIFT_DIST: {
      double a3 = d_min * d_min * d_min, b3 = d_max * d_max * d_max;
      return cbrt(a3 + u * (b3 - a3));
    }
    default: return (u - 0.5) * tw;
  }
}

// alpha, psi and phi are periodic over their prior range (psi with period pi)
__device__ __forceinline__ bool periodic(int d) { return d == RIFT_ALPHA || d == RIFT_PSI || d == RIFT_PHI; }

// ---- top-k samples of each segment by ln w --------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) topk_kernel(const R *lnw, const int64_t *seg_off, const int64_t *seg_cnt,
                                                   int k, int *out) {
  constexpr int L = 4;  // candidates per thread
  __shared__ double v[256 * L];
  __shared__ int ix[256 * L];
  const int seg = blockIdx.x;
  const int64_t off = seg_off[seg], cnt = seg_cnt[seg];
  double bv[L];
  int bi[L];
  for (int q = 0; q < L; q++) {
    bv[q] = -INFINITY;
    bi[q] = -1;
  }
  for (int64_t i = threadIdx.x; i < cnt; i += 256) {
    double x = (double)lnw[off + i];
    if (!(x > -INFINITY) || x == INFINITY) continue;  // NaN, -inf, +inf
    if (x > bv[L - 1]) {
      int q = L - 1;
      while (q > 0 && bv[q - 1] < x) {
        bv[q] = bv[q - 1];
        bi[q] = bi[q - 1];
        q--;
      }
      bv[q] = x;
      bi[q] = (int)i;
    }
  }
  for (int q = 0; q < L; q++) {
    v[threadIdx.x * L + q] = bv[q];
    ix[threadIdx.x * L + q] = bi[q];
  }
  __syncthreads();
  // bitonic sort of the 1024 candidates, descending
  constexpr int N = 256 * L;
  for (int size = 2; size <= N; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < N / 2; t += 256) {
        int lo = 2 * t - (t & (stride - 1));
        int hi = lo + stride;
        bool desc = ((lo & size) == 0);
        double a = v[lo], b = v[hi];
        if ((a < b) == desc) {
          v[lo] = b;
          v[hi] = a;
          int ti = ix[lo];
          ix[lo] = ix[hi];
          ix[hi] = ti;
        }
      }
      __syncthreads();
    }
  }
  for (int j = threadIdx.x; j < k; j += 256) out[seg * k + j] = (j < N && v[j] > -INFINITY) ? ix[j] : -1;
}

// ---- ascent state ------------------------------------------------------------------
template <typename R>
__global__ void ascent_init_kernel(const R *theta, int64_t stride, const int64_t *seg_off, const int *idx, int k,
                                   int n, R *th_a, AscentState *st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int seg = i / k;
  int j = idx[i];
  if (j < 0) j = idx[seg * k];  // fewer finite samples than k: repeat the best
  AscentState &S = st[i];
  if (j < 0) {  // no finite sample at all: a point that never moves
    for (int d = 0; d < 7; d++) th_a[d * n + i] = (R)0;
    th_a[RIFT_DIST * n + i] = (R)1e30;  // evaluates to ln L_t = NaN
    S.eta = 0.0;
  } else {
    for (int d = 0; d < 7; d++) th_a[d * n + i] = theta[d * stride + seg_off[seg] + j];
    S.eta = 0.01;
  }
  S.best_l = -INFINITY;
  for (int d = 0; d < 7; d++) {
    S.best_th[d] = (double)th_a[d * n + i];
    S.best_g[d] = 0.0;
  }
}

template <typename R>
__global__ void ascent_step_kernel(R *th_a, const R *grad, const R *lnl, AscentState *st, int n, unsigned mask,
                                   double d_min, double d_max, double tw) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  AscentState &S = st[i];
  const double l = (double)lnl[i];
  if (l == l && l > S.best_l && fabs(l) < INFINITY) {
    S.best_l = l;
    for (int d = 0; d < 7; d++) {
      S.best_th[d] = (double)th_a[d * n + i];
      S.best_g[d] = (double)grad[d * n + i];
    }
    S.eta = fmin(S.eta * 1.25, 0.05);
  } else {
    S.eta *= 0.5;
  }
  // next trial point: from the best point along its gradient, in u
  double gu[7], nrm = 0.0;
  for (int d = 0; d < 7; d++) {
    gu[d] = 0.0;
    if ((mask >> d) & 1u) {
      gu[d] = S.best_g[d] * dtheta_du(d, S.best_th[d], d_min, d_max, tw);
      nrm += gu[d] * gu[d];
    }
  }
  nrm = sqrt(nrm);
  for (int d = 0; d < 7; d++) {
    double t = S.best_th[d];
    if (((mask >> d) & 1u) && nrm > 0.0 && isfinite(nrm) && S.eta > 0.0) {
      double u = prior_u(d, t, d_min, d_max, tw) + S.eta * gu[d] / nrm;
      if (periodic(d)) u -= floor(u);
      else u = fmin(fmax(u, 1e-9), 1.0 - 1e-9);
      t = theta_of_u(d, u, d_min, d_max, tw);
    }
    th_a[d * n + i] = (R)t;
  }
}

// ---- histogram of the points reached (per segment, deterministic) ------------------
// (alpha, delta) -> the prior-CDF coordinates of the point's network sky frame
// (azimuth / 2 pi, (cos theta' + 1) / 2)
__device__ __forceinline__ double frame_u(const PointDev &p, int d, double alpha, double delta) {
  double sh, ch, sd, cd;
  sincos(alpha - p.gmst, &sh, &ch);
  sincos(delta, &sd, &cd);
  const double n[3] = {cd * ch, cd * sh, sd};
  const double x = p.frame[0][0] * n[0] + p.frame[0][1] * n[1] + p.frame[0][2] * n[2];
  const double y = p.frame[1][0] * n[0] + p.frame[1][1] * n[1] + p.frame[1][2] * n[2];
  const double z = p.frame[2][0] * n[0] + p.frame[2][1] * n[1] + p.frame[2][2] * n[2];
  if (d == RIFT_ALPHA) {
    const double a = atan2(y, x);
    return (a < 0.0 ? a + 2.0 * kPi : a) / (2.0 * kPi);
  }
  return 0.5 * (fmax(-1.0, fmin(1.0, z)) + 1.0);
}

// pts != null: the sky histograms live in each point's network frame
__global__ void ascent_hist_kernel(const AscentState *st, int k, int n_seg, unsigned mask, double d_min,
                                   double d_max, double tw, const PointDev *pts, double *ahist) {
  const int seg = blockIdx.x, d = threadIdx.x;
  if (d >= 7) return;
  double *h = ahist + ((size_t)seg * 7 + d) * kNB;
  for (int b = 0; b < kNB; b++) h[b] = 0.0;
  if (!((mask >> d) & 1u)) return;
  double mx = -INFINITY;
  for (int j = 0; j < k; j++) mx = fmax(mx, st[seg * k + j].best_l);
  if (!(mx > -INFINITY)) return;
  for (int j = 0; j < k; j++) {
    const AscentState &S = st[seg * k + j];
    if (!(S.best_l > -INFINITY)) continue;
    const double w = exp(S.best_l - mx);
    const double u = (pts && d < 2) ? frame_u(pts[seg], d, S.best_th[RIFT_ALPHA], S.best_th[RIFT_DELTA])
                                    : prior_u(d, S.best_th[d], d_min, d_max, tw);
    int b = (int)floor(u * kNB);
    b = b < 0 ? 0 : (b >= kNB ? kNB - 1 : b);
    int bl = b - 1, br = b + 1;
    if (periodic(d)) {
      bl = (bl + kNB) % kNB;
      br = br % kNB;
    } else {
      bl = bl < 0 ? b : bl;
      br = br >= kNB ? b : br;
    }
    h[b] += 0.5 * w;
    h[bl] += 0.25 * w;
    h[br] += 0.25 * w;
  }
}

template <typename R>
hipError_t ascent_select(const R *lnw, const R *theta, int64_t stride, const int64_t *seg_off, const int64_t *seg_cnt,
                         int n_seg, int k, int *idx, R *th_a, AscentState *st, hipStream_t s) {
  hipLaunchKernelGGL(topk_kernel<R>, dim3(n_seg), dim3(256), 0, s, lnw, seg_off, seg_cnt, k, idx);
  const int n = n_seg * k;
  hipLaunchKernelGGL(ascent_init_kernel<R>, dim3((n + 63) / 64), dim3(64), 0, s, theta, stride, seg_off, idx, k, n,
                     th_a, st);
  return hipGetLastError();
}

template <typename R>
hipError_t ascent_step(R *th_a, const R *grad, const R *lnl, AscentState *st, int n, unsigned mask, double d_min,
                       double d_max, double tw, hipStream_t s) {
  hipLaunchKernelGGL(ascent_step_kernel<R>, dim3((n + 63) / 64), dim3(64), 0, s, th_a, grad, lnl, st, n, mask, d_min,
                     d_max, tw);
  return hipGetLastError();
}

hipError_t ascent_hist(const AscentState *st, int k, int n_seg, unsigned mask, double d_min, double d_max, double tw,
                       const PointDev *pts, double *ahist, hipStream_t s) {
  hipLaunchKernelGGL(ascent_hist_kernel, dim3(n_seg), dim3(64), 0, s, st, k, n_seg, mask, d_min, d_max, tw, pts,
                     ahist);
  return hipGetLastError();
}

#define RIFT_INST(R)                                                                                            \
  template hipError_t ascent_select<R>(const R *, const R *, int64_t, const int64_t *, const int64_t *, int, int, \
                                       int *, R *, AscentState *, hipStream_t);                                   \
  template hipError_t ascent_step<R>(R *, const R *, const R *, AscentState *, int, unsigned, double, double,     \
                                     double, hipStream_t);
RIFT_INST(float)
RIFT_INST(double)
#undef RIFT_INST

}  // namespace rift
