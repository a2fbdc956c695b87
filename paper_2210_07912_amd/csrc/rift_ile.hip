// Host side of the C ABI declared in include/rift_ile.h: argument checks,
// device layouts of the per-point data, workspace management and the order
// of kernel launches for each entry point.  No exception crosses the ABI.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "common.h"
#include "internal.h"

using namespace rift;

namespace {

thread_local std::string g_create_error;

struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
  std::vector<char> last;  // bytes of the last upload into p (kernels never write these buffers)
};

}  // namespace

struct rift_ile {
  int precision = RIFT_FP32;
  unsigned flags = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  int n_points = 0;
  double d_min = 10.0, d_max = 1000.0, tau_width = 0.0;
  bool any_mix = false;  // some point may hold a Gaussian-mixture proposal (sampler variant)
  bool have_accum = false;  // the pooled-estimate accumulators hold a run (resume allowed)
  std::vector<PointDev> hp;       // host copies (device pointers inside)
  std::vector<void *> owned;      // per-point allocations
  PointDev *d_pts = nullptr;
  ProposalDev *d_props = nullptr;
  int max_L = 0, max_nt = 0;
  int n_cu = 0;
  int lds_max = 65536;
  // grow-only workspace, indexed by name
  DevBuf ws[48];
  // side streams for concurrent class kernels, and the workspace budget
  Fanout fan{};
  // captured evaluation runs: key (launch arguments and class layout) -> graph
  bool use_graph = false;
  std::vector<std::pair<std::vector<char>, hipGraphExec_t>> graphs;
  hipStream_t gstream = nullptr;  // graph stream when the handle's stream is the null stream
  hipEvent_t gfork = nullptr, gjoin = nullptr;
  int64_t n_captures = 0, n_replays = 0;
  // sky drawn in each point's network frame (rift_ile_set_network_frame)
  bool net_frame = false;
  bool phase_rot = false;  // polarization and phase in phase-rotated coordinates
  bool dmarg = false;      // distance-marginalized ln L_tD (theta's distance not read)
  // launch configuration of each class (1 staged, 2 direct, 3 and 4 the same
  // at half residency, 5 and 6 direct with registers capped for three or four
  // wavefronts per SIMD, 7 staged capped for three; 0 not measured), by (T, K,
  // n_t bucket = floor(log2 of the class's longest window)); kmode: the
  // configuration each (T, K) ran last.  feed: 1 measure on first use, 0 all
  // staged, 2 all direct, 3 and 4 all direct with registers capped for three
  // or four wavefronts per SIMD, 5 all staged capped for three.
  // tune_path: a file the measurements are read from and appended to.
  int feed = 1;
  int kmode[kMaxT + 1][kMaxDet + 1] = {};
  int tune[kMaxT + 1][kMaxDet + 1][kNtBuckets] = {};
  std::string tune_path;
  std::string arch;
  double ws_budget = 6.0e9;
  // FP64 refinement of the matrix-core adjoint (rift_ile_set_grad_refine)
  bool refine = true;
  // this device's copy of the no-allocation scratch (rift_ile_reduce_noalloc)
  void *scratch = nullptr;
  // optional timing of the dominant evaluation kernel
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
};

namespace {

enum WsId {
  W_ITEM_POINT, W_ITEM_OFF, W_ITEM_CNT, W_ITEM_TILE0, W_ITEM_SAMP0, W_ITEM_BIN0,
  W_KEY, W_NSH, W_COUNT, W_CURSOR, W_COP, W_BINTILE, W_ITEMTILES, W_PERM, W_TILES, W_CTL, W_CTILE,
  W_PARTIALS, W_ROUND, W_ACCUM, W_RESULT, W_HIST, W_THETA, W_LNW, W_AUX, W_RATIO, W_BINS, W_ITEM_BLK0,
  W_ITEM_HOFF, W_ITEM_COP, W_SEG_OFF, W_SEG_CNT, W_ASC, W_AHIST, W_UNIT, W_BINUNIT, W_ITEMUNITS, W_GOP, W_HOP, W_SEG_BLK, W_UBUF, W_EMPART, W_EMPART2, W_GMMFIT, W_EMWT, W_JRNG, W_AMAX, W_COUNT_IDS
};
static_assert(W_COUNT_IDS <= 48, "workspace table too small");

// Scratch of rift_ile_reduce_noalloc, for callers that cannot allocate:
// the partial FP64 tuples of the reduction, the segment's offset and count,
// the merged tuple and the result.  A file-scope device array: every device
// the library runs on holds one copy until the process ends.  Host code never
// uses the array's name as an address: rift_ile_create takes this device's
// address once with hipGetSymbolAddress and the entry point passes that.
constexpr int kNoAllocPartials = 1024;                 // partial tuples (blocks of the reduction)
constexpr int64_t kNoAllocMaxN = (int64_t)1 << 40;     // samples per call
struct NoAllocScratch {
  ReduceTuple partials[kNoAllocPartials];
  ReduceTuple merged;
  int64_t seg[2];  // offset, count
  rift_ile_result result;
};
__device__ __align__(256) unsigned char scratch[sizeof(NoAllocScratch)];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// blocks of the reduction for a segment of at most mx samples (both reduce
// entry points use this, so their results are identical)
int reduce_bps(int64_t mx) { return (int)std::min<int64_t>(kNoAllocPartials, (std::max<int64_t>(mx, 1) + 2047) / 2048); }

rift_status fail(rift_ile *h, rift_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (h) h->err = buf; else g_create_error = buf;
  return s;
}

rift_status hip_fail(rift_ile *h, hipError_t e, const char *what) {
  return fail(h, e == hipErrorOutOfMemory ? RIFT_E_OOM : RIFT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(h, expr)                                   \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return hip_fail((h), e_, #expr); \
  } while (0)

rift_status ws_get(rift_ile *h, WsId id, size_t bytes, void **out) {
  DevBuf &b = h->ws[id];
  if (bytes == 0) bytes = 16;
  if (b.n < bytes) {
    if (b.p) {
      hipError_t e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
      (void)hipFree(b.p);
      b.p = nullptr;
      b.n = 0;
    }
    b.last.clear();
    size_t want = bytes + bytes / 4;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(h, RIFT_E_OOM, "workspace allocation of %zu bytes failed", want);
    }
    b.n = want;
  }
  *out = b.p;
  return RIFT_OK;
}

template <typename T>
rift_status upload(rift_ile *h, WsId id, const std::vector<T> &v, T **out) {
  void *p;
  rift_status s = ws_get(h, id, sizeof(T) * std::max<size_t>(v.size(), 1), &p);
  if (s != RIFT_OK) return s;
  // a copy from pageable memory makes the host wait for the stream, so an
  // array identical to the one already in the buffer is not sent again
  DevBuf &b = h->ws[id];
  const size_t bytes = sizeof(T) * v.size();
  if (!v.empty() && !(b.last.size() == bytes && std::memcmp(b.last.data(), v.data(), bytes) == 0)) {
    HIPCHK(h, hipMemcpyAsync(p, v.data(), bytes, hipMemcpyHostToDevice, h->stream));
    b.last.assign((const char *)v.data(), (const char *)v.data() + bytes);
  }
  *out = (T *)p;
  return RIFT_OK;
}

double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; i++) f *= i;
  return f;
}

bool finite_all(const double *p, size_t n) {
  for (size_t i = 0; i < n; i++)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Wigner-d sum for spin weight -2 (Goldberg et al. 1967): term k has
// coefficient (-1)^k sqrt((l+m)!(l-m)!(l+2)!(l-2)!) / ((l+m-k)!(l-2-k)! k! (k+2-m)!)
// and powers cos(iota/2)^(2l+m-2-2k), sin(iota/2)^(2k+2-m).
void harmonic_table(PointDev &p, int m_idx, int l, int m) {
  int kmin = std::max(0, m - 2), kmax = std::min(l + m, l - 2);
  double nrm = std::sqrt(factorial(l + m) * factorial(l - m) * factorial(l + 2) * factorial(l - 2));
  int n = 0;
  for (int k = kmin; k <= kmax; k++, n++) {
    double den = factorial(l + m - k) * factorial(l - 2 - k) * factorial(k) * factorial(k + 2 - m);
    p.ycoef[m_idx][n] = ((k & 1) ? -1.0 : 1.0) * nrm / den;
    p.ypc[m_idx][n] = 2 * l + m - 2 - 2 * k;
    p.yps[m_idx][n] = 2 * k + 2 - m;
  }
  p.nterm[m_idx] = n;
  p.ynorm[m_idx] = std::sqrt((2.0 * l + 1.0) / (4.0 * kPi));
  p.em[m_idx] = m;
  // Polynomial form: with c = cos(iota/2), s = sin(iota/2) and par = |m| mod 2,
  // c^A s^B = (s c)^par u^((A - par)/2) (1 - u)^((B - par)/2), u = c^2;
  // expanding (1 - u)^n binomially gives a polynomial in u of degree l - par.
  const int par = m & 1;
  const int deg = l - par;
  for (int j = 0; j <= kMaxHDeg; j++) p.hpoly[m_idx][j] = 0.0;
  for (int t = 0; t < n; t++) {
    const int a = (p.ypc[m_idx][t] - par) / 2, nb = (p.yps[m_idx][t] - par) / 2;
    double binom = 1.0;  // C(nb, i)
    for (int i = 0; i <= nb; i++) {
      p.hpoly[m_idx][a + i] += p.ynorm[m_idx] * p.ycoef[m_idx][t] * ((i & 1) ? -binom : binom);
      binom = binom * (nb - i) / (i + 1);
    }
  }
  p.hdeg[m_idx] = deg;
  p.hpar[m_idx] = par;
}

// Network sky frame of the point (Sec. II.A, rotated detector-network-frame
// sky coordinates): z' the unit vector from detector 0 to detector 1,
// x' = normalize(e_z x z') (e_x x z' when the baseline is along e_z),
// y' = z' x x'.  One detector: the equatorial axes.
void network_frame(const rift_ile_point &q, PointDev &p) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) p.frame[i][j] = i == j ? 1.0 : 0.0;
  if (q.n_det < 2) return;
  auto unit = [](double v[3]) {
    const double n = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int i = 0; i < 3; i++) v[i] /= n;
  };
  auto cross = [](const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
  };
  double z[3], x[3], y[3];
  for (int i = 0; i < 3; i++) z[i] = q.det_pos[3 + i] - q.det_pos[i];
  unit(z);
  const double ez[3] = {0.0, 0.0, 1.0}, ex[3] = {1.0, 0.0, 0.0};
  cross(ez, z, x);
  if (std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) < 1e-6) cross(ex, z, x);
  unit(x);
  cross(z, x, y);
  for (int i = 0; i < 3; i++) {
    p.frame[0][i] = x[i];
    p.frame[1][i] = y[i];
    p.frame[2][i] = z[i];
  }
}

rift_status check_point(const rift_ile_point &q, int idx, double tau_width) {
  if (q.n_det < 1 || q.n_det > RIFT_MAX_DET)
    return fail(nullptr, RIFT_E_SHAPE, "point %d: n_det=%d outside 1..%d", idx, q.n_det, RIFT_MAX_DET);
  if (q.n_modes < 1 || q.n_modes > RIFT_MAX_MODES)
    return fail(nullptr, RIFT_E_SHAPE, "point %d: n_modes=%d outside 1..%d", idx, q.n_modes, RIFT_MAX_MODES);
  if (q.n_t < 1 || q.n_t > (1 << 20)) return fail(nullptr, RIFT_E_SHAPE, "point %d: n_t=%d", idx, q.n_t);
  // (the matrix-core path stores row offsets in -pad..pad as 16-bit integers)
  if (q.pad < 0 || q.pad > 32767) return fail(nullptr, RIFT_E_SHAPE, "point %d: pad=%d (at most 32767)", idx, q.pad);
  if (!q.ell || !q.em || !q.det_pos || !q.det_resp || !q.Q || !q.U)
    return fail(nullptr, RIFT_E_INVALID, "point %d: NULL array", idx);
  for (int m = 0; m < q.n_modes; m++)
    if (q.ell[m] < 2 || q.ell[m] > 8 || q.em[m] < -q.ell[m] || q.em[m] > q.ell[m])
      return fail(nullptr, RIFT_E_INVALID, "point %d: mode %d = (%d,%d) unsupported", idx, m, q.ell[m], q.em[m]);
  if (!(q.f_s > 0) || !std::isfinite(q.f_s) || !(q.d_ref > 0) || !std::isfinite(q.d_ref) || !std::isfinite(q.gmst))
    return fail(nullptr, RIFT_E_NONFINITE, "point %d: f_s, d_ref or gmst invalid", idx);
  const int K = q.n_det, M = q.n_modes;
  const size_t L = (size_t)q.n_t + 2 * (size_t)q.pad + 3;
  if (!finite_all(q.det_pos, 3 * K) || !finite_all(q.det_resp, 9 * K))
    return fail(nullptr, RIFT_E_NONFINITE, "point %d: detector constants not finite", idx);
  if (!finite_all(q.Q, 2 * (size_t)K * L * M)) return fail(nullptr, RIFT_E_NONFINITE, "point %d: Q not finite", idx);
  if (!finite_all(q.U, 2 * (size_t)K * M * M)) return fail(nullptr, RIFT_E_NONFINITE, "point %d: U not finite", idx);
  if (q.V && !finite_all(q.V, 2 * (size_t)K * M * M))
    return fail(nullptr, RIFT_E_NONFINITE, "point %d: V not finite", idx);
  for (int k = 0; k < K; k++) {
    const double *U = q.U + 2 * (size_t)k * M * M;
    double mx = 0.0;
    for (int i = 0; i < M * M; i++) mx = std::max(mx, std::hypot(U[2 * i], U[2 * i + 1]));
    for (int i = 0; i < M; i++)
      for (int j = 0; j < M; j++) {
        const double *a = U + 2 * (i * M + j), *b = U + 2 * (j * M + i);
        if (std::fabs(a[0] - b[0]) > 1e-6 * mx || std::fabs(a[1] + b[1]) > 1e-6 * mx)
          return fail(nullptr, RIFT_E_NOT_HERMITIAN, "point %d: U_%d not Hermitian at (%d,%d)", idx, k, i, j);
      }
    if (q.V) {
      const double *V = q.V + 2 * (size_t)k * M * M;
      double vx = 0.0;
      for (int i = 0; i < M * M; i++) vx = std::max(vx, std::hypot(V[2 * i], V[2 * i + 1]));
      for (int i = 0; i < M; i++)
        for (int j = 0; j < M; j++) {
          const double *a = V + 2 * (i * M + j), *b = V + 2 * (j * M + i);
          if (std::fabs(a[0] - b[0]) > 1e-6 * vx || std::fabs(a[1] - b[1]) > 1e-6 * vx)
            return fail(nullptr, RIFT_E_NOT_HERMITIAN, "point %d: V_%d not symmetric at (%d,%d)", idx, k, i, j);
        }
    }
    const double *D = q.det_resp + 9 * k;
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++)
        if (std::fabs(D[3 * i + j] - D[3 * j + i]) > 1e-9)
          return fail(nullptr, RIFT_E_INVALID, "point %d: response tensor %d not symmetric", idx, k);
  }
  double rmax = 0.0;
  for (int k = 0; k < K; k++)
    rmax = std::max(rmax, std::sqrt(q.det_pos[3 * k] * q.det_pos[3 * k] + q.det_pos[3 * k + 1] * q.det_pos[3 * k + 1] +
                                    q.det_pos[3 * k + 2] * q.det_pos[3 * k + 2]));
  double need = q.f_s * (rmax / kC + 0.5 * tau_width);
  if ((double)q.pad < need)
    return fail(nullptr, RIFT_E_WINDOW, "point %d: pad=%d rows < %.3f needed for light travel time and tau", idx,
                q.pad, need);
  return RIFT_OK;
}

template <typename R>
rift_status build_point(rift_ile *h, const rift_ile_point &q, PointDev &p) {
  const int K = q.n_det, M = q.n_modes;
  std::memset(&p, 0, sizeof(p));
  p.K = K;
  p.M = M;
  p.n_t = q.n_t;
  p.pad = q.pad;
  p.L = q.n_t + 2 * q.pad + 3;
  p.Lpad = p.L + 32;
  p.f_s = q.f_s;
  p.d_ref = q.d_ref;
  p.gmst = q.gmst;
  p.Mp = (M + 1) & ~1;
  p.bin_w = 14;
  p.nq = (2 * q.pad) / p.bin_w + 1;
  long long nb = 1;
  for (int k = 0; k < K; k++) nb *= p.nq;
  p.n_bins_key = (int)std::min<long long>(nb, 1 << 30);
  for (int k = 0; k < K; k++) {
    for (int i = 0; i < 3; i++) p.rc[k][i] = q.det_pos[3 * k + i] / kC;
    for (int i = 0; i < 9; i++) p.D[k][i] = q.det_resp[9 * k + i];
  }
  network_frame(q, p);
  for (int m = 0; m < M; m++) harmonic_table(p, m, q.ell[m], q.em[m]);
  // U (and V) in FP64, holding the values rounded to the bulk precision
  std::vector<double> u(2 * (size_t)K * M * M);
  for (size_t i = 0; i < u.size(); i++) u[i] = (double)(R)q.U[i];
  void *d;
  HIPCHK(h, hipMalloc(&d, sizeof(double) * u.size()));
  h->owned.push_back(d);
  HIPCHK(h, hipMemcpy(d, u.data(), sizeof(double) * u.size(), hipMemcpyHostToDevice));
  p.U = (const double *)d;
  if (q.V) {
    for (size_t i = 0; i < u.size(); i++) u[i] = (double)(R)q.V[i];
    HIPCHK(h, hipMalloc(&d, sizeof(double) * u.size()));
    h->owned.push_back(d);
    HIPCHK(h, hipMemcpy(d, u.data(), sizeof(double) * u.size(), hipMemcpyHostToDevice));
    p.V = (const double *)d;
  }
  // U and V packed over pairs m <= m' (off-diagonal doubled) for the quadratic
  // term of the coefficient pass: [pair][kMaxDet][2]
  {
    const int npair = M * (M + 1) / 2;
    std::vector<double> up((size_t)npair * kMaxDet * 2, 0.0), vp((size_t)npair * kMaxDet * 2, 0.0);
    int idx = 0;
    for (int m = 0; m < M; m++)
      for (int mp = m; mp < M; mp++, idx++)
        for (int k = 0; k < K; k++) {
          double f = (m == mp) ? 1.0 : 2.0;
          size_t src = (((size_t)k * M + m) * M + mp) * 2;
          up[((size_t)idx * kMaxDet + k) * 2] = f * (double)(R)q.U[src];
          up[((size_t)idx * kMaxDet + k) * 2 + 1] = f * (double)(R)q.U[src + 1];
          if (q.V) {
            vp[((size_t)idx * kMaxDet + k) * 2] = f * (double)(R)q.V[src];
            vp[((size_t)idx * kMaxDet + k) * 2 + 1] = f * (double)(R)q.V[src + 1];
          }
        }
    HIPCHK(h, hipMalloc(&d, sizeof(double) * up.size()));
    h->owned.push_back(d);
    HIPCHK(h, hipMemcpy(d, up.data(), sizeof(double) * up.size(), hipMemcpyHostToDevice));
    p.Upk = (const double *)d;
    if (q.V) {
      HIPCHK(h, hipMalloc(&d, sizeof(double) * vp.size()));
      h->owned.push_back(d);
      HIPCHK(h, hipMemcpy(d, vp.data(), sizeof(double) * vp.size(), hipMemcpyHostToDevice));
      p.Vpk = (const double *)d;
    }
  }
  // Q, row layout [K][Lpad][M][2] with zero rows past L
  {
    std::vector<R> qv((size_t)K * p.Lpad * M * 2, R(0));
    for (int k = 0; k < K; k++)
      for (int r = 0; r < p.L; r++)
        for (int i = 0; i < 2 * M; i++)
          qv[((size_t)k * p.Lpad + r) * M * 2 + i] = (R)q.Q[((size_t)k * p.L + r) * M * 2 + i];
    HIPCHK(h, hipMalloc(&d, sizeof(R) * qv.size()));
    h->owned.push_back(d);
    HIPCHK(h, hipMemcpy(d, qv.data(), sizeof(R) * qv.size(), hipMemcpyHostToDevice));
    p.Q = d;
  }
  // Q for the matrix cores (FP32 handles): [K][Lpad][2 Mp], element e = 2m + part,
  // zero past M and past L
  if (sizeof(R) == 4) {
    const int E = 2 * p.Mp;
    std::vector<float> qm((size_t)K * E * p.Lpad, 0.f);
    for (int k = 0; k < K; k++)
      for (int r = 0; r < p.L; r++)
        for (int e = 0; e < 2 * M; e++)
          qm[((size_t)k * p.Lpad + r) * E + e] = (float)q.Q[((size_t)k * p.L + r) * M * 2 + e];
    HIPCHK(h, hipMalloc(&d, sizeof(float) * qm.size()));
    h->owned.push_back(d);
    HIPCHK(h, hipMemcpy(d, qm.data(), sizeof(float) * qm.size(), hipMemcpyHostToDevice));
    p.Qm = (const float *)d;
  }
  return RIFT_OK;
}

void uniform_proposal(ProposalDev &pr) {
  std::memset(&pr, 0, sizeof pr);  // no mixture (gk = 0)
  for (int d = 0; d < 7; d++)
    for (int b = 0; b <= kNB; b++) pr.cdf[d][b] = (double)b / kNB;
}

// ---- evaluation -------------------------------------------------------------
struct Items {
  std::vector<int> point;
  std::vector<int64_t> off, cnt;
};

rift_status check_items(rift_ile *h, int n_items, const rift_ile_item *items, int64_t stride) {
  if (n_items < 0 || (n_items > 0 && !items) || stride < 0) return fail(h, RIFT_E_INVALID, "bad item list");
  for (int i = 0; i < n_items; i++) {
    const rift_ile_item &it = items[i];
    if (it.point < 0 || it.point >= h->n_points) return fail(h, RIFT_E_INVALID, "item %d: point %d", i, it.point);
    if (it.offset < 0 || it.count < 0 || it.offset + it.count > stride)
      return fail(h, RIFT_E_INVALID, "item %d: columns [%lld, %lld) outside stride %lld", i, (long long)it.offset,
                  (long long)(it.offset + it.count), (long long)stride);
  }
  return RIFT_OK;
}

template <typename R>
rift_status run_plain(rift_ile *h, const Items &it, int64_t stride, const R *theta, R *lnL, R *lnw,
                      const R *ln_ratio, const R *gin, R *grad, bool bwd) {
  const int n = (int)it.point.size();
  // samples per workgroup (4, 8 or 16: each sample's window reductions take
  // 256 / TS lanes of one wavefront): the most that still let two workgroups
  // share a compute unit's LDS, else the most that fit at all
  auto lds = [&](int ts) { return plain_lds_bytes(sizeof(R), ts, h->max_L, h->max_nt, bwd); };
  int TS = 16;
  while (TS > 4 && lds(TS) > (size_t)h->lds_max / 2) TS >>= 1;
  if (lds(TS) > (size_t)h->lds_max / 2) {
    TS = 16;
    while (TS > 4 && lds(TS) > (size_t)h->lds_max) TS >>= 1;
  }
  if (lds(TS) > (size_t)h->lds_max) return fail(h, RIFT_E_SHAPE, "window too long for the plain kernel's LDS");
  std::vector<int> tile0(n + 1, 0);
  for (int i = 0; i < n; i++) tile0[i + 1] = tile0[i] + (int)((it.cnt[i] + TS - 1) / TS);
  if (tile0[n] == 0) return RIFT_OK;
  int *d_point, *d_tile0;
  int64_t *d_off, *d_cnt;
  rift_status s;
  if ((s = upload(h, W_ITEM_POINT, it.point, &d_point)) != RIFT_OK) return s;
  if ((s = upload(h, W_ITEM_OFF, it.off, &d_off)) != RIFT_OK) return s;
  if ((s = upload(h, W_ITEM_CNT, it.cnt, &d_cnt)) != RIFT_OK) return s;
  if ((s = upload(h, W_ITEM_TILE0, tile0, &d_tile0)) != RIFT_OK) return s;
  PlainArgsT<R> a;
  a.pts = h->d_pts;
  a.item_point = d_point;
  a.item_off = d_off;
  a.item_cnt = d_cnt;
  a.item_tile0 = d_tile0;
  a.n_items = n;
  a.stride = stride;
  a.theta = theta;
  a.lnL = lnL;
  a.lnw = lnw;
  a.ln_ratio = ln_ratio;
  a.gin = gin;
  a.grad = grad;
  a.rows_cap = h->max_L;
  a.nt_cap = h->max_nt;
  a.dmarg = h->dmarg && !bwd ? 1 : 0;
  a.dm_lo = h->d_min;
  a.dm_hi = h->d_max;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->prof) {
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    h->prof_ev.emplace_back(e0, e1);
  }
  HIPCHK(h, plain_launch<R>(a, TS, tile0[n], bwd, h->stream, e0, e1));
  return RIFT_OK;
}

// The evaluation launches of one run from a captured graph: the key is the
// bytes of the launch arguments and of the class layout, so a replay happens
// only when every kernel would see the same arguments.
template <typename V>
void key_add(std::vector<char> &k, const V &v) {
  const char *b = (const char *)v.data();
  k.insert(k.end(), b, b + sizeof(v[0]) * v.size());
  k.push_back('|');
}

rift_status launch_graph(rift_ile *h, const MfmaArgs &a, const std::vector<int> &class_T,
                         const std::vector<int> &class_K, const std::vector<int> &class_item0,
                         const std::vector<int> &mclass_M, const std::vector<int> &mclass_item0,
                         const std::vector<int64_t> &mclass_tiles, std::vector<int> &class_mode) {
  std::vector<char> key((const char *)&a, (const char *)&a + sizeof(a));
  key_add(key, class_mode);
  key_add(key, class_T);
  key_add(key, class_K);
  key_add(key, class_item0);
  key_add(key, mclass_M);
  key_add(key, mclass_item0);
  key_add(key, mclass_tiles);
  // the null stream cannot be captured: then the graph runs on the handle's
  // own stream, ordered after and before the caller's work by events
  hipStream_t gs = h->stream;
  if (!gs) {
    if (!h->gstream) {
      HIPCHK(h, hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking));
      HIPCHK(h, hipEventCreateWithFlags(&h->gfork, hipEventDisableTiming));
      HIPCHK(h, hipEventCreateWithFlags(&h->gjoin, hipEventDisableTiming));
    }
    gs = h->gstream;
    HIPCHK(h, hipEventRecord(h->gfork, h->stream));
    HIPCHK(h, hipStreamWaitEvent(gs, h->gfork, 0));
  }
  auto join = [&]() -> rift_status {
    if (gs != h->stream) {
      HIPCHK(h, hipEventRecord(h->gjoin, gs));
      HIPCHK(h, hipStreamWaitEvent(h->stream, h->gjoin, 0));
    }
    return RIFT_OK;
  };
  for (auto &g : h->graphs)
    if (g.first == key) {
      HIPCHK(h, hipGraphLaunch(g.second, gs));
      h->n_replays++;
      return join();
    }
  hipGraph_t graph = nullptr;
  HIPCHK(h, hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
  hipError_t e = mfma_forward(a, class_T.data(), class_K.data(), class_item0.data(), (int)class_T.size(),
                              mclass_M.data(), mclass_item0.data(), mclass_tiles.data(), (int)mclass_M.size(),
                              class_mode.data(), false, gs, h->fan, nullptr, nullptr);
  hipError_t e2 = hipStreamEndCapture(gs, &graph);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(h, e != hipSuccess ? e : e2, "capturing the evaluation graph");
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(h, e, "instantiating the evaluation graph");
  if (h->graphs.size() >= 16) {  // keep the most recent runs
    (void)hipGraphExecDestroy(h->graphs.front().second);
    h->graphs.erase(h->graphs.begin());
  }
  h->graphs.emplace_back(std::move(key), exec);
  h->n_captures++;
  HIPCHK(h, hipGraphLaunch(exec, gs));
  return join();
}

// One group of points (already in evaluation order) through the sort, the
// coefficient pass and the persistent MFMA launches.
rift_status run_mfma_group(rift_ile *h, const Items &it, int64_t stride, const float *theta, float *lnL, float *lnw,
                           const float *ln_ratio, const float *gin = nullptr, float *grad = nullptr) {
  std::vector<int64_t> samp0(1, 0), mclass_tiles, hoff;
  std::vector<int> bin0(1, 0), blk0(1, 0), class_T, class_K, class_item0, mclass_M, mclass_item0;
  int64_t hist_total = 0, cop_floats = 0;
  int max_item_bins = 1;
  int64_t max_tiles = 0;
  for (size_t i = 0; i < it.point.size(); i++) {
    const PointDev &p = h->hp[it.point[i]];
    const int T = p.Mp >> 1;
    if (class_T.empty() || class_T.back() != T || class_K.back() != p.K) {
      class_T.push_back(T);
      class_K.push_back(p.K);
      class_item0.push_back((int)i);
    }
    const int64_t tiles_i = (it.cnt[i] + 15) / 16 + p.n_bins_key + 4;
    const int mkey = p.Vpk ? -p.M : p.M;  // V tables: the general coefficient kernel
    if (mclass_M.empty() || mclass_M.back() != mkey) {
      mclass_M.push_back(mkey);
      mclass_item0.push_back((int)i);
      mclass_tiles.push_back(0);
    }
    mclass_tiles.back() += tiles_i;
    samp0.push_back(samp0.back() + it.cnt[i]);
    long long nb = (long long)bin0.back() + p.n_bins_key;
    if (nb > (1 << 28)) return fail(h, RIFT_E_SHAPE, "too many delay bins in one call");
    bin0.push_back((int)nb);
    const int nblk = (int)((it.cnt[i] + kSortBlock - 1) / kSortBlock);
    blk0.push_back(blk0.back() + nblk);
    hoff.push_back(hist_total);
    hist_total += (int64_t)nblk * p.n_bins_key;
    max_item_bins = std::max(max_item_bins, p.n_bins_key);
    max_tiles += tiles_i;
    cop_floats += tiles_i * p.K * 2 * p.Mp * 16;
  }
  const int ni = (int)it.point.size();
  class_item0.push_back(ni);
  mclass_item0.push_back(ni);
  const int64_t total = samp0.back();
  if (ni == 0) return RIFT_OK;
  if (total == 0) return RIFT_OK;
  if (total >= (int64_t)1 << 31 || max_tiles >= (int64_t)1 << 26)
    return fail(h, RIFT_E_SHAPE, "more than 2^31 samples in one call");
  MfmaArgs a;
  std::memset(&a, 0, sizeof(a));
  rift_status s;
  int *d_point, *d_bin0, *d_blk0;
  int64_t *d_off, *d_cnt, *d_samp0, *d_hoff;
  if ((s = upload(h, W_ITEM_POINT, it.point, &d_point)) != RIFT_OK) return s;
  if ((s = upload(h, W_ITEM_OFF, it.off, &d_off)) != RIFT_OK) return s;
  if ((s = upload(h, W_ITEM_CNT, it.cnt, &d_cnt)) != RIFT_OK) return s;
  if ((s = upload(h, W_ITEM_SAMP0, samp0, &d_samp0)) != RIFT_OK) return s;
  if ((s = upload(h, W_ITEM_BIN0, bin0, &d_bin0)) != RIFT_OK) return s;
  if ((s = upload(h, W_ITEM_BLK0, blk0, &d_blk0)) != RIFT_OK) return s;
  if ((s = upload(h, W_ITEM_HOFF, hoff, &d_hoff)) != RIFT_OK) return s;
  a.pts = h->d_pts;
  a.items.blk0 = d_blk0;
  a.items.hoff = d_hoff;
  a.n_sort_blocks = blk0.back();
  a.max_item_bins = max_item_bins;
  a.items.point = d_point;
  a.items.off = d_off;
  a.items.cnt = d_cnt;
  a.items.samp0 = d_samp0;
  a.items.bin0 = d_bin0;
  a.items.tile0 = nullptr;
  a.items.n_items = ni;
  a.stride = stride;
  a.total = total;
  a.theta = theta;
  a.lnL = lnL;
  a.lnw = lnw;
  a.ln_ratio = ln_ratio;
  a.n_bins = bin0.back();
  a.max_tiles = (int)max_tiles;
  void *p;
  if ((s = ws_get(h, W_KEY, 4 * total, &p)) != RIFT_OK) return s;
  a.key = (uint32_t *)p;
  if ((s = ws_get(h, W_NSH, 8 * total, &p)) != RIFT_OK) return s;
  a.nsh = (int16_t *)p;
  if ((s = ws_get(h, W_COUNT, 4 * (size_t)a.n_bins, &p)) != RIFT_OK) return s;
  a.count = (uint32_t *)p;
  if ((s = ws_get(h, W_CURSOR, 4 * (size_t)std::max<int64_t>(hist_total, 1), &p)) != RIFT_OK) return s;
  a.bhist = (uint32_t *)p;
  if ((s = ws_get(h, W_BINTILE, 4 * (size_t)a.n_bins, &p)) != RIFT_OK) return s;
  a.bin_tile = (uint32_t *)p;
  if ((s = ws_get(h, W_ITEMTILES, 4 * (size_t)(ni + 1), &p)) != RIFT_OK) return s;
  a.item_tiles = (uint32_t *)p;
  if ((s = ws_get(h, W_PERM, sizeof(SampleRec) * 16 * (size_t)max_tiles, &p)) != RIFT_OK) return s;
  a.rec = (SampleRec *)p;
  if ((s = ws_get(h, W_TILES, 4 * (size_t)max_tiles, &p)) != RIFT_OK) return s;
  a.tile_item = (int *)p;
  if ((s = ws_get(h, W_COP, sizeof(float) * (size_t)cop_floats, &p)) != RIFT_OK) return s;
  a.cop = (float *)p;
  if (grad) {  // the adjoint's per-tile G_k (cop layout) and H_k
    if ((s = ws_get(h, W_GOP, sizeof(float) * (size_t)cop_floats, &p)) != RIFT_OK) return s;
    a.gop = (float *)p;
    if ((s = ws_get(h, W_HOP, sizeof(float) * kMaxDet * 16 * (size_t)max_tiles, &p)) != RIFT_OK) return s;
    a.hop = (float *)p;
    if (h->refine) {
      if ((s = ws_get(h, W_JRNG, 4 * sizeof(int) * 16 * (size_t)max_tiles, &p)) != RIFT_OK) return s;
      a.jrng = (int *)p;
    }
    a.gin = gin;
    a.grad = grad;
  }
  if (h->dmarg && !grad) {  // distance marginalization: each slot's largest data term
    if ((s = ws_get(h, W_AMAX, sizeof(float) * 16 * (size_t)max_tiles, &p)) != RIFT_OK) return s;
    a.amax = (float *)p;
    a.dmarg = 1;
    a.dm_lo = h->d_min;
    a.dm_hi = h->d_max;
  }
  if ((s = ws_get(h, W_ITEM_COP, sizeof(int64_t) * (size_t)ni, &p)) != RIFT_OK) return s;
  a.item_cop = (int64_t *)p;
  if ((s = ws_get(h, W_CTILE, sizeof(CoefTile) * (size_t)max_tiles, &p)) != RIFT_OK) return s;
  a.ctile = (CoefTile *)p;
  if ((s = ws_get(h, W_UNIT, sizeof(WorkUnit) * (size_t)max_tiles, &p)) != RIFT_OK) return s;
  a.unit = (WorkUnit *)p;
  if ((s = ws_get(h, W_BINUNIT, 4 * (size_t)a.n_bins, &p)) != RIFT_OK) return s;
  a.bin_unit = (uint32_t *)p;
  if ((s = ws_get(h, W_ITEMUNITS, 4 * (size_t)(ni + 1), &p)) != RIFT_OK) return s;
  a.item_units = (uint32_t *)p;
  if ((s = ws_get(h, W_CTL, 4 * (1 + kMaxClasses) + 64, &p)) != RIFT_OK) return s;
  a.ctl = (uint32_t *)p;
  a.grid = h->n_cu * 4;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->prof) {
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    h->prof_ev.emplace_back(e0, e1);
  }
  // launch configuration of each class (measured on first use when autotuning)
  std::vector<int> class_mode(class_T.size()), class_ntb(class_T.size(), 0);
  for (size_t c = 0; c < class_T.size(); c++) {
    int nt = 1;
    for (int i = class_item0[c]; i < class_item0[c + 1]; i++) nt = std::max(nt, h->hp[it.point[i]].n_t);
    int b = 0;
    while (b + 1 < kNtBuckets && (nt >> (b + 1)) > 0) b++;
    class_ntb[c] = b;
  }
  bool measured = true;
  for (size_t c = 0; c < class_T.size(); c++) {
    // feed 0: staged, 1: measured, 2: direct, 3 and 4: direct with registers
    // capped for three or four wavefronts per SIMD (configurations 5, 6),
    // 5: staged capped for three (configuration 7)
    class_mode[c] = h->feed == 1 ? h->tune[class_T[c]][class_K[c]][class_ntb[c]]
                    : h->feed == 0 ? 1
                    : h->feed == 2 ? 2
                                   : h->feed + 2;
    measured = measured && class_mode[c] != 0;
  }
  if (!grad && h->use_graph && !h->prof && measured) {
    for (size_t c = 0; c < class_T.size(); c++) h->kmode[class_T[c]][class_K[c]] = class_mode[c];
    return launch_graph(h, a, class_T, class_K, class_item0, mclass_M, mclass_item0, mclass_tiles, class_mode);
  }
  if (grad)
    HIPCHK(h, mfma_backward(a, class_T.data(), class_K.data(), class_item0.data(), (int)class_T.size(),
                            mclass_M.data(), mclass_item0.data(), mclass_tiles.data(), (int)mclass_M.size(), h->stream,
                            h->fan, e0, e1));
  else {
    HIPCHK(h, mfma_forward(a, class_T.data(), class_K.data(), class_item0.data(), (int)class_T.size(),
                           mclass_M.data(), mclass_item0.data(), mclass_tiles.data(), (int)mclass_M.size(),
                           class_mode.data(), h->feed == 1, h->stream, h->fan, e0, e1));
    std::string lines;
    for (size_t c = 0; c < class_T.size(); c++) {
      if (class_mode[c] == 0) continue;  // distance marginalization: the fixed passes
      h->kmode[class_T[c]][class_K[c]] = class_mode[c];
      int &slot = h->tune[class_T[c]][class_K[c]][class_ntb[c]];
      if (h->feed == 1 && slot == 0) {
        slot = class_mode[c];
        char ln[96];
        std::snprintf(ln, sizeof ln, "%s %d %d %d %d\n", h->arch.c_str(), class_T[c], class_K[c], class_ntb[c],
                      class_mode[c]);
        lines += ln;
      }
    }
    if (!lines.empty() && !h->tune_path.empty()) {
      // appended in one write; a cache that cannot be written is skipped
      if (FILE *f = std::fopen(h->tune_path.c_str(), "a")) {
        (void)std::fwrite(lines.data(), 1, lines.size(), f);
        std::fclose(f);
      }
    }
  }
  return RIFT_OK;
}

// Points grouped by MFMA step count T (one persistent launch per group),
// then mode count, costliest first: the kernels take tiles in this order.
// The points are evaluated in runs whose workspace stays under a budget.
rift_status run_mfma(rift_ile *h, const Items &it_in, int64_t stride, const float *theta, float *lnL, float *lnw,
                     const float *ln_ratio, const float *gin = nullptr, float *grad = nullptr) {
  const int n = (int)it_in.point.size();
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  auto Tof = [&](int i) { return h->hp[it_in.point[i]].Mp >> 1; };
  auto Mof = [&](int i) { return h->hp[it_in.point[i]].M; };
  auto cost = [&](int i) {
    const PointDev &p = h->hp[it_in.point[i]];
    return (double)p.K * (p.Mp + 4) * p.n_t;
  };
  auto Kof = [&](int i) { return h->hp[it_in.point[i]].K; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (Tof(a) != Tof(b)) return Tof(a) > Tof(b);
    if (Kof(a) != Kof(b)) return Kof(a) > Kof(b);
    if (Mof(a) != Mof(b)) return Mof(a) > Mof(b);
    return cost(a) > cost(b);
  });
  const double budget = h->ws_budget;  // bytes of per-sample workspace per run
  Items grp;
  double used = 0.0;
  for (int oi : order) {
    if (it_in.cnt[oi] == 0) continue;
    const PointDev &p = h->hp[it_in.point[oi]];
    int64_t remaining = it_in.cnt[oi], off = it_in.off[oi];
    while (remaining > 0) {
      const double per = 4.0 + 8.0 + 44.0 + 40.0 + (double)p.K * 2 * p.Mp * 4 * 1.1 * (grad ? 2.0 : 1.0) +
                         (h->dmarg ? 4.4 : 0.0);
      int64_t take = remaining;
      if (used + per * take > budget) {
        if (!grp.point.empty()) {
          rift_status s = run_mfma_group(h, grp, stride, theta, lnL, lnw, ln_ratio, gin, grad);
          if (s != RIFT_OK) return s;
          grp = Items();
          used = 0.0;
        }
        take = std::min<int64_t>(remaining, std::max<int64_t>(4096, (int64_t)(budget / per)));
      }
      grp.point.push_back(it_in.point[oi]);
      grp.off.push_back(off);
      grp.cnt.push_back(take);
      used += per * take;
      off += take;
      remaining -= take;
    }
  }
  if (!grp.point.empty()) return run_mfma_group(h, grp, stride, theta, lnL, lnw, ln_ratio, gin, grad);
  return RIFT_OK;
}

Items make_items(int n_items, const rift_ile_item *items) {
  Items it;
  for (int i = 0; i < n_items; i++) {
    it.point.push_back(items[i].point);
    it.off.push_back(items[i].offset);
    it.cnt.push_back(items[i].count);
  }
  return it;
}

template <typename R>
rift_status eval(rift_ile *h, const Items &it, int64_t stride, const R *theta, R *lnL, R *lnw, const R *ln_ratio) {
  if (sizeof(R) == 4 && !(h->flags & 1u))
    return run_mfma(h, it, stride, (const float *)theta, (float *)lnL, (float *)lnw, (const float *)ln_ratio);
  return run_plain<R>(h, it, stride, theta, lnL, lnw, ln_ratio, nullptr, nullptr, false);
}

// ln L_t and its gradient (times gin): the matrix-core adjoint for FP32
// handles, the plain adjoint otherwise
template <typename R>
rift_status eval_grad(rift_ile *h, const Items &it, int64_t stride, const R *theta, R *lnL, const R *gin, R *grad) {
  if (sizeof(R) == 4 && !(h->flags & 1u))
    return run_mfma(h, it, stride, (const float *)theta, (float *)lnL, nullptr, nullptr, (const float *)gin,
                    (float *)grad);
  return run_plain<R>(h, it, stride, theta, lnL, nullptr, nullptr, gin, grad, true);
}

template <typename R>
rift_status reduce_segments(rift_ile *h, const R *lnL, const R *ln_ratio, const std::vector<int64_t> &off,
                            const std::vector<int64_t> &cnt, ReduceTuple **round_out, ReduceTuple *accum,
                            int accumulate, rift_ile_result *d_out) {
  const int ns = (int)off.size();
  int64_t mx = 1;
  for (auto c : cnt) mx = std::max(mx, c);
  // enough blocks per segment to spread a large segment over the device
  const int bps = reduce_bps(mx);
  int64_t *d_off, *d_cnt;
  rift_status s;
  if ((s = upload(h, W_ITEM_OFF, off, &d_off)) != RIFT_OK) return s;
  if ((s = upload(h, W_ITEM_CNT, cnt, &d_cnt)) != RIFT_OK) return s;
  void *pp, *pr;
  if ((s = ws_get(h, W_PARTIALS, sizeof(ReduceTuple) * (size_t)ns * bps, &pp)) != RIFT_OK) return s;
  if ((s = ws_get(h, W_ROUND, sizeof(ReduceTuple) * (size_t)ns, &pr)) != RIFT_OK) return s;
  HIPCHK(h, reduce_partials<R>(lnL, ln_ratio, d_off, d_cnt, ns, bps, (ReduceTuple *)pp, h->stream));
  HIPCHK(h, reduce_finish((ReduceTuple *)pp, ns, bps, (ReduceTuple *)pr, accum, accumulate, d_out, h->stream));
  if (round_out) *round_out = (ReduceTuple *)pr;
  return RIFT_OK;
}

// pairs code: byte i = a | b << 4, a < b < 7, both in mask, pairs disjoint
rift_status check_pairs(rift_ile *h, unsigned pairs, unsigned mask) {
  if (pairs >> (8 * kMaxPair)) return fail(h, RIFT_E_INVALID, "pairs 0x%x: at most %d", pairs, kMaxPair);
  unsigned used = 0u;
  for (int i = 0; i < kMaxPair; i++) {
    const unsigned c = (pairs >> (8 * i)) & 0xFFu;
    if (!c) continue;
    const unsigned a = c & 15u, b = c >> 4;
    if (!(a < b) || b >= 7u || !((mask >> a) & 1u) || !((mask >> b) & 1u) || ((used >> a) & 1u) || ((used >> b) & 1u))
      return fail(h, RIFT_E_INVALID, "pair %d (%u, %u): need a < b < 7, both adapted, pairs disjoint", i, a, b);
    used |= (1u << a) | (1u << b);
  }
  return RIFT_OK;
}

template <typename R>
rift_status marginalize_impl(rift_ile *h, const rift_ile_mc *mc, rift_ile_result *out, R *theta_out,
                                    R *lnw_out) {
  const int np = h->n_points;
  std::vector<int64_t> cnt(np), off(np);
  std::vector<int> seg_prop(np);
  int64_t per_round = 0;
  for (int p = 0; p < np; p++) {
    cnt[p] = mc->n_per_point ? mc->n_per_point[p] : mc->n_per_round;
    if (cnt[p] < 0) return fail(h, RIFT_E_INVALID, "negative sample count for point %d", p);
    if (mc->adapt_mask && cnt[p] > (1 << 23)) return fail(h, RIFT_E_INVALID, "more than 2^23 samples per round");
    off[p] = per_round;
    per_round += cnt[p];
    seg_prop[p] = p;
  }
  const int64_t total = per_round * mc->n_rounds;
  const int64_t nr = std::max<int64_t>(per_round, 1);
  rift_status s;
  // every argument is checked before the handle's state changes
  // gradient-informed refinement: ascent set of k points per point
  const bool grad = (mc->flags & RIFT_MC_GRADIENT) && mc->adapt_mask;
  const int ka = mc->n_ascent > 0 ? mc->n_ascent : 64;
  const int steps = mc->ascent_steps > 0 ? mc->ascent_steps : 12;
  const double beta = mc->ascent_mix > 0.0 ? mc->ascent_mix : 0.3;
  if (grad && (ka > 256 || !(beta + mc->floor_eps < 1.0)))
    return fail(h, RIFT_E_INVALID, "n_ascent %d (<= 256) or ascent_mix %g (< 1 - floor_eps)", ka, beta);
  // the ascent places its points in the histograms by the prior-CDF
  // coordinates of (psi, phi), which the four-to-one phase rotation does not
  // give back
  if (grad && h->phase_rot)
    return fail(h, RIFT_E_INVALID, "the gradient refinement is not combined with phase-rotated coordinates");
  // with distance marginalization D is integrated per sample, not sampled:
  // no proposal over it, and no adjoint for the ascent
  if (h->dmarg && (grad || ((mc->adapt_mask >> RIFT_DIST) & 1u)))
    return fail(h, RIFT_E_INVALID, "distance marginalization: adapt_mask must leave out the distance (bit %d) and "
                "the gradient refinement is not available", RIFT_DIST);
  // Gaussian-mixture proposal: prior-CDF coordinates of every sample, EM sums
  // and the mixtures being fitted
  const int gk = mc->gmm_components;
  const int giter = mc->gmm_iters > 0 ? mc->gmm_iters : 10;
  if (gk < 0 || gk > kMaxG || mc->gmm_iters < 0 || mc->gmm_iters > 1000 || (gk > 0 && grad))
    return fail(h, RIFT_E_INVALID, "gmm_components %d (0..%d), gmm_iters %d (0..1000), or both a mixture and the "
                "gradient refinement", gk, kMaxG, mc->gmm_iters);
  if ((s = check_pairs(h, mc->gmm_pairs, mc->adapt_mask)) != RIFT_OK) return s;
  if (mc->gmm_pairs && gk == 0) return fail(h, RIFT_E_INVALID, "correlated pairs need gmm_components > 0");
  if (h->dmarg && !mc->reset_proposal) {
    // the proposals a run continues from must leave the distance to the prior
    std::vector<ProposalDev> props(np);
    HIPCHK(h, hipMemcpyAsync(props.data(), h->d_props, sizeof(ProposalDev) * np, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int p = 0; p < np; p++)
      if ((props[p].mask >> RIFT_DIST) & 1u)
        return fail(h, RIFT_E_INVALID, "distance marginalization: the proposal of point %d adapts the distance", p);
  }
  if (mc->reset_proposal) {
    std::vector<ProposalDev> props(np);
    for (auto &p : props) uniform_proposal(p);
    HIPCHK(h, hipMemcpyAsync(h->d_props, props.data(), sizeof(ProposalDev) * np, hipMemcpyHostToDevice, h->stream));
    h->any_mix = false;
  }
  void *accum, *d_res, *bins, *hist, *ratio, *th_ws = nullptr, *lw_ws = nullptr;
  if ((s = ws_get(h, W_ACCUM, sizeof(ReduceTuple) * np, &accum)) != RIFT_OK) return s;
  if ((s = ws_get(h, W_RESULT, sizeof(rift_ile_result) * np, &d_res)) != RIFT_OK) return s;
  if ((s = ws_get(h, W_BINS, 7 * (size_t)nr, &bins)) != RIFT_OK) return s;
  int64_t mxc = 1;
  for (auto c : cnt) mxc = std::max(mxc, c);
  const int hbps = hist_blocks(mxc);
  if ((s = ws_get(h, W_HIST, sizeof(unsigned long long) * 7 * kNB * np * (size_t)hbps, &hist)) != RIFT_OK) return s;
  if ((s = ws_get(h, W_RATIO, sizeof(R) * (size_t)nr, &ratio)) != RIFT_OK) return s;
  if (!theta_out && (s = ws_get(h, W_THETA, 7 * sizeof(R) * (size_t)nr, &th_ws)) != RIFT_OK) return s;
  if (!lnw_out && (s = ws_get(h, W_LNW, sizeof(R) * (size_t)nr, &lw_ws)) != RIFT_OK) return s;
  int *d_prop;
  if ((s = upload(h, W_AUX, seg_prop, &d_prop)) != RIFT_OK) return s;
  int64_t *d_soff, *d_scnt;
  if ((s = upload(h, W_SEG_OFF, off, &d_soff)) != RIFT_OK) return s;
  if ((s = upload(h, W_SEG_CNT, cnt, &d_scnt)) != RIFT_OK) return s;
  // sampling blocks of 256 per point, for one launch per round
  std::vector<int> sblk(np + 1, 0);
  for (int p = 0; p < np; p++) sblk[p + 1] = sblk[p] + (int)((cnt[p] + 255) / 256);
  int *d_sblk;
  if ((s = upload(h, W_SEG_BLK, sblk, &d_sblk)) != RIFT_OK) return s;
  const int64_t th_stride = theta_out ? total : nr;
  const bool gmm = gk > 0 && mc->adapt_mask;
  float *ubuf = nullptr;
  double *em_part = nullptr, *em_part2 = nullptr, *em_wt = nullptr;
  GmmDev *em_fit = nullptr;
  const int ebps = em_blocks(mxc);
  if (gmm) {
    void *pu, *pp, *pp2, *pf, *pw;
    if ((s = ws_get(h, W_EMWT, sizeof(double) * (size_t)nr, &pw)) != RIFT_OK) return s;
    em_wt = (double *)pw;
    if ((s = ws_get(h, W_UBUF, 7 * sizeof(float) * (size_t)nr, &pu)) != RIFT_OK) return s;
    if ((s = ws_get(h, W_EMPART, sizeof(double) * 7 * 3 * kMaxG * (size_t)np * ebps, &pp)) != RIFT_OK) return s;
    if ((s = ws_get(h, W_EMPART2, sizeof(double) * kMaxPair * 6 * kMaxG * (size_t)np * ebps, &pp2)) != RIFT_OK)
      return s;
    if ((s = ws_get(h, W_GMMFIT, 2 * sizeof(GmmDev) * (size_t)np, &pf)) != RIFT_OK) return s;
    ubuf = (float *)pu;
    em_part = (double *)pp;
    em_part2 = (double *)pp2;
    em_fit = (GmmDev *)pf;
    h->any_mix = true;
  }
  const int na = np * ka;
  int *a_idx = nullptr;
  R *a_th = nullptr, *a_g = nullptr, *a_l = nullptr;
  AscentState *a_st = nullptr;
  double *ahist = nullptr;
  Items ita;
  if (grad) {
    void *pa;
    const size_t bytes = sizeof(int) * na + sizeof(R) * (size_t)na * 15 + sizeof(AscentState) * na + 256;
    if ((s = ws_get(h, W_ASC, bytes, &pa)) != RIFT_OK) return s;
    char *c = (char *)pa;
    a_st = (AscentState *)c;
    c += sizeof(AscentState) * na;
    a_th = (R *)c;
    c += sizeof(R) * 7 * (size_t)na;
    a_g = (R *)c;
    c += sizeof(R) * 7 * (size_t)na;
    a_l = (R *)c;
    c += sizeof(R) * (size_t)na;
    a_idx = (int *)c;
    void *ph;
    if ((s = ws_get(h, W_AHIST, sizeof(double) * 7 * kNB * np, &ph)) != RIFT_OK) return s;
    ahist = (double *)ph;
    for (int p = 0; p < np; p++) {
      ita.point.push_back(p);
      ita.off.push_back((int64_t)p * ka);
      ita.cnt.push_back(ka);
    }
  }
  Items it;
  for (int p = 0; p < np; p++) {
    it.point.push_back(p);
    it.off.push_back(off[p]);
    it.cnt.push_back(cnt[p]);
  }
  // trace ranges (rocprofv3 --marker-trace): one per round, nested ones per phase
  struct Range {
    explicit Range(const char *m) { roctxRangePushA(m); }
    ~Range() { roctxRangePop(); }
  };
  Range run_range("rift_ile_marginalize");
  for (int r = 0; r < mc->n_rounds; r++) {
    char rname[48];
    std::snprintf(rname, sizeof rname, "round %d", mc->first_round + r);
    Range round_range(rname);
    const int64_t cb = theta_out ? (int64_t)r * per_round : 0;
    R *th = theta_out ? theta_out + cb : (R *)th_ws;
    R *lw = lnw_out ? lnw_out + (int64_t)r * per_round : (R *)lw_ws;
    HIPCHK(h, sample_multi_launch<R>(h->d_props, h->net_frame ? h->d_pts : nullptr, d_sblk, sblk[np], np, d_soff,
                                     d_scnt, mc->seed, (uint32_t)(mc->first_round + r),
                                     th_stride, nr, h->d_min, h->d_max, h->tau_width, th, (R *)ratio,
                                     // bins only for the histogram adaptation that reads them
                                     mc->adapt_mask && !gmm ? (uint8_t *)bins : nullptr, h->stream, ubuf,
                                     h->any_mix, h->phase_rot));
    {
      Range ph("evaluate");
      if ((s = eval<R>(h, it, th_stride, th, nullptr, lw, (const R *)ratio)) != RIFT_OK) return s;
    }
    ReduceTuple *round;
    const bool last = r + 1 == mc->n_rounds;
    if ((s = reduce_segments<R>(h, lw, nullptr, off, cnt, &round, (ReduceTuple *)accum, r > 0 || mc->first_round > 0,
                                last ? (rift_ile_result *)d_res : nullptr)) != RIFT_OK)
      return s;
    // adapted after every round, the last included, so the proposals a run
    // leaves (and a checkpoint holds) are the next round's
    if (mc->adapt_mask) {
      Range ph("adapt");
      if (grad) {
        HIPCHK(h, ascent_select<R>(lw, th, th_stride, d_soff, d_scnt, np, ka, a_idx, a_th, a_st, h->stream));
        const bool prof = h->prof;  // the timing hook follows the evaluation launches only
        h->prof = false;
        for (int it_s = 0; it_s <= steps; it_s++) {
          if ((s = eval_grad<R>(h, ita, na, a_th, a_l, nullptr, a_g)) != RIFT_OK) {
            h->prof = prof;
            return s;
          }
          HIPCHK(h, ascent_step<R>(a_th, a_g, a_l, a_st, na, mc->adapt_mask, h->d_min, h->d_max, h->tau_width,
                                   h->stream));
        }
        h->prof = prof;
        HIPCHK(h, ascent_hist(a_st, ka, np, mc->adapt_mask, h->d_min, h->d_max, h->tau_width,
                              h->net_frame ? h->d_pts : nullptr, ahist, h->stream));
      }
      if (gmm) {
        HIPCHK(h, gmm_adapt_launch<R>(ubuf, nr, lw, d_soff, d_scnt, d_prop, np, ebps, round, em_part, em_part2,
                                      em_fit, h->d_props, mc->adapt_mask, mc->gmm_pairs, mc->floor_eps, gk, giter,
                                      d_sblk, sblk[np], em_wt, h->stream));
        HIPCHK(h, pair_norm_launch(h->d_props, 0, np, h->stream));
      } else
        HIPCHK(h, adapt_launch<R>((const uint8_t *)bins, nr, lw, d_soff, d_scnt, d_prop, np, hbps, round,
                                  (unsigned long long *)hist, h->d_props, mc->adapt_mask, mc->floor_eps, h->stream,
                                  grad ? ahist : nullptr, grad ? beta : 0.0));
    }
  }
  HIPCHK(h, hipMemcpyAsync(out, d_res, sizeof(rift_ile_result) * np, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->have_accum = true;
  return RIFT_OK;
}

}  // namespace

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

int rift_ile_abi_version(void) { return RIFT_ILE_ABI_VERSION; }

const char *rift_ile_status_string(int s) {
  switch (s) {
    case RIFT_OK: return "ok";
    case RIFT_E_INVALID: return "invalid argument";
    case RIFT_E_SHAPE: return "inconsistent or unsupported shape";
    case RIFT_E_NOT_HERMITIAN: return "U not Hermitian or V not symmetric";
    case RIFT_E_WINDOW: return "pad too small for the light travel time";
    case RIFT_E_NONFINITE: return "non-finite input";
    case RIFT_E_OOM: return "device allocation failed";
    case RIFT_E_DEVICE: return "HIP runtime error";
    case RIFT_E_STATE: return "invalid state";
  }
  return "unknown status";
}

const char *rift_ile_last_error(const rift_ile *h) { return h ? h->err.c_str() : g_create_error.c_str(); }

void rift_ile_destroy(rift_ile *h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  for (auto &pe : h->prof_ev) {
    (void)hipEventDestroy(pe.first);
    (void)hipEventDestroy(pe.second);
  }
  for (auto &g : h->graphs) (void)hipGraphExecDestroy(g.second);
  if (h->gstream) {
    (void)hipStreamSynchronize(h->gstream);
    (void)hipStreamDestroy(h->gstream);
  }
  if (h->gfork) (void)hipEventDestroy(h->gfork);
  if (h->gjoin) (void)hipEventDestroy(h->gjoin);
  for (int i = 0; i < h->fan.n; i++) {
    (void)hipStreamSynchronize(h->fan.side[i]);
    (void)hipStreamDestroy(h->fan.side[i]);
    (void)hipEventDestroy(h->fan.join[i]);
  }
  if (h->fan.n) (void)hipEventDestroy(h->fan.fork);
  for (void *p : h->owned) (void)hipFree(p);
  for (auto &b : h->ws)
    if (b.p) (void)hipFree(b.p);
  if (h->d_pts) (void)hipFree(h->d_pts);
  if (h->d_props) (void)hipFree(h->d_props);
  delete h;
}

rift_status rift_ile_create(rift_ile **out, const rift_ile_desc *desc, void *stream) {
  g_create_error.clear();
  if (!out) return fail(nullptr, RIFT_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!desc || desc->n_points < 1 || !desc->points) return fail(nullptr, RIFT_E_INVALID, "no points");
  if (desc->precision != RIFT_FP32 && desc->precision != RIFT_FP64)
    return fail(nullptr, RIFT_E_INVALID, "precision %d", desc->precision);
  if (!(desc->d_min > 0) || !(desc->d_max > desc->d_min) || !std::isfinite(desc->d_max))
    return fail(nullptr, RIFT_E_INVALID, "distance prior [%g, %g]", desc->d_min, desc->d_max);
  if (!(desc->tau_width >= 0) || !std::isfinite(desc->tau_width))
    return fail(nullptr, RIFT_E_INVALID, "tau_width %g", desc->tau_width);
  for (int i = 0; i < desc->n_points; i++) {
    rift_status s = check_point(desc->points[i], i, desc->tau_width);
    if (s != RIFT_OK) return s;
  }
  rift_ile *h = new (std::nothrow) rift_ile();
  if (!h) return fail(nullptr, RIFT_E_OOM, "host allocation");
  h->precision = desc->precision;
  h->flags = 0;
  if (const char *e = getenv("RIFT_ILE_FP32_KERNEL"))
    if (!strcmp(e, "plain")) h->flags |= 1u;
  h->stream = (hipStream_t)stream;
  h->n_points = desc->n_points;
  h->d_min = desc->d_min;
  h->d_max = desc->d_max;
  h->tau_width = desc->tau_width;
  auto bail = [&](rift_status s) {
    std::string msg = h->err;
    rift_ile_destroy(h);
    g_create_error = msg;
    return s;
  };
  if (hipGetDevice(&h->device) != hipSuccess) return bail(fail(h, RIFT_E_DEVICE, "no HIP device"));
  {
    // this device's address of the no-allocation scratch, taken once per device
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (h->device < 0 || h->device >= kMaxDevices) return bail(fail(h, RIFT_E_DEVICE, "device %d", h->device));
    if (!g_scratch_dev[h->device]) {
      void *ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) return bail(hip_fail(h, e != hipSuccess ? e : hipErrorUnknown, "hipGetSymbolAddress"));
      g_scratch_dev[h->device] = ptr;
    }
    h->scratch = g_scratch_dev[h->device];
  }
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess && v > 0) h->n_cu = v;
  else h->n_cu = 256;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) {
      std::string an(prop.gcnArchName);
      h->arch = an.substr(0, an.find(':'));
    }
    if (h->arch.empty()) h->arch = "unknown";
  }
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) == hipSuccess && v > 0)
    h->lds_max = std::min(v, 160 * 1024) - 1024;
  // per-sample workspace of one evaluation run: a third of the free device
  // memory, between 2 and 64 GB (fewer, larger runs on a 288 GB device)
  size_t mfree = 0, mtot = 0;
  if (hipMemGetInfo(&mfree, &mtot) == hipSuccess && mfree > 0)
    h->ws_budget = std::min(64.0e9, std::max(2.0e9, (double)mfree / 3.0));
  if (h->precision == RIFT_FP32) {
    bool ok = hipEventCreateWithFlags(&h->fan.fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < kSideStreams; i++) {
      ok = hipStreamCreateWithFlags(&h->fan.side[i], hipStreamNonBlocking) == hipSuccess;
      if (ok && hipEventCreateWithFlags(&h->fan.join[i], hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(h->fan.side[i]);
        ok = false;
      }
      if (ok) h->fan.n = i + 1;
    }
    if (h->fan.n == 0 && h->fan.fork) {
      (void)hipEventDestroy(h->fan.fork);
      h->fan.fork = nullptr;
    }
  }
  h->hp.resize(h->n_points);
  for (int i = 0; i < h->n_points; i++) {
    rift_status s = h->precision == RIFT_FP32 ? build_point<float>(h, desc->points[i], h->hp[i])
                                              : build_point<double>(h, desc->points[i], h->hp[i]);
    if (s != RIFT_OK) return bail(s);
    h->max_L = std::max(h->max_L, h->hp[i].L);
    h->max_nt = std::max(h->max_nt, h->hp[i].n_t);
  }
  hipError_t e = hipMalloc(&h->d_pts, sizeof(PointDev) * h->n_points);
  if (e != hipSuccess) return bail(hip_fail(h, e, "hipMalloc points"));
  e = hipMemcpy(h->d_pts, h->hp.data(), sizeof(PointDev) * h->n_points, hipMemcpyHostToDevice);
  if (e != hipSuccess) return bail(hip_fail(h, e, "hipMemcpy points"));
  std::vector<ProposalDev> props(h->n_points);
  for (auto &p : props) uniform_proposal(p);
  e = hipMalloc(&h->d_props, sizeof(ProposalDev) * h->n_points);
  if (e != hipSuccess) return bail(hip_fail(h, e, "hipMalloc proposals"));
  e = hipMemcpy(h->d_props, props.data(), sizeof(ProposalDev) * h->n_points, hipMemcpyHostToDevice);
  if (e != hipSuccess) return bail(hip_fail(h, e, "hipMemcpy proposals"));
  *out = h;
  return RIFT_OK;
}

rift_status rift_ile_profile(rift_ile *h, int enable, double *ms_total, int64_t *launches) {
  if (!h) return RIFT_E_INVALID;
  double tot = 0.0;
  int64_t n = 0;
  if (!h->prof_ev.empty()) HIPCHK(h, hipStreamSynchronize(h->stream));
  for (auto &pe : h->prof_ev) {
    float ms = 0.f;
    HIPCHK(h, hipEventElapsedTime(&ms, pe.first, pe.second));
    tot += ms;
    n++;
    (void)hipEventDestroy(pe.first);
    (void)hipEventDestroy(pe.second);
  }
  h->prof_ev.clear();
  h->prof = enable != 0;
  if (ms_total) *ms_total = tot;
  if (launches) *launches = n;
  return RIFT_OK;
}

rift_status rift_ile_set_graph(rift_ile *h, int enable) {
  if (!h) return RIFT_E_INVALID;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (!enable) {
    for (auto &g : h->graphs) (void)hipGraphExecDestroy(g.second);
    h->graphs.clear();
  }
  h->use_graph = enable != 0;
  return RIFT_OK;
}

rift_status rift_ile_graph_stats(const rift_ile *h, int64_t *captures, int64_t *replays) {
  if (!h) return RIFT_E_INVALID;
  if (captures) *captures = h->n_captures;
  if (replays) *replays = h->n_replays;
  return RIFT_OK;
}

rift_status rift_ile_precompute(const rift_ile_fd_point *in, int64_t row0, int64_t n_rows, double *Q, double *U,
                                double *V) {
  if (!in || !in->data || !in->psd || !in->modes || !U || !V || (n_rows > 0 && !Q))
    return fail(nullptr, RIFT_E_INVALID, "precompute: NULL argument");
  const int K = in->n_det, M = in->n_modes;
  const int64_t N = in->n_f;
  if (K < 1 || K > RIFT_MAX_DET || M < 1 || M > RIFT_MAX_MODES || N < 2 || N > ((int64_t)1 << 30) || n_rows < 0 ||
      n_rows > ((int64_t)1 << 30))
    return fail(nullptr, RIFT_E_SHAPE, "precompute: K=%d M=%d N=%lld n_rows=%lld out of range", K, M, (long long)N,
                (long long)n_rows);
  if (!(in->df > 0.0) || !std::isfinite(in->df) || !(in->f_low >= 0.0) || !std::isfinite(in->f_low))
    return fail(nullptr, RIFT_E_INVALID, "precompute: df or f_low invalid");
  if (!finite_all(in->data, 2 * (size_t)K * N) || !finite_all(in->modes, 2 * (size_t)M * N))
    return fail(nullptr, RIFT_E_NONFINITE, "precompute: data or modes not finite");
  for (int64_t i = 0; i < N; i++) {
    const double f = (double)(i < (N + 1) / 2 ? i : i - N) * in->df;
    if (std::fabs(f) <= in->f_low) continue;
    for (int k = 0; k < K; k++) {
      const double S = in->psd[(size_t)k * N + i];
      if (!(S > 0.0) || !std::isfinite(S))
        return fail(nullptr, RIFT_E_NONFINITE, "precompute: psd[%d][%lld] = %g in band", k, (long long)i, S);
    }
  }
  const size_t nd = 2 * (size_t)K * N, np_ = (size_t)K * N, nm = 2 * (size_t)M * N, nx = 2 * (size_t)K * M * N;
  const size_t nq = 2 * (size_t)K * n_rows * M, nu = 2 * (size_t)K * M * M;
  std::vector<void *> bufs;
  auto release = [&]() {
    for (void *b : bufs) (void)hipFree(b);
  };
  auto alloc = [&](size_t n, double **p) -> bool {
    void *v = nullptr;
    if (hipMalloc(&v, sizeof(double) * std::max<size_t>(n, 1)) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    bufs.push_back(v);
    *p = (double *)v;
    return true;
  };
  double *dd, *dp, *dm, *dx, *dq, *du, *dv;
  if (!alloc(nd, &dd) || !alloc(np_, &dp) || !alloc(nm, &dm) || !alloc(nx, &dx) || !alloc(nq, &dq) ||
      !alloc(nu, &du) || !alloc(nu, &dv)) {
    release();
    return fail(nullptr, RIFT_E_OOM, "precompute: device allocation failed");
  }
  hipError_t e = hipMemcpy(dd, in->data, sizeof(double) * nd, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dp, in->psd, sizeof(double) * np_, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dm, in->modes, sizeof(double) * nm, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = quv_device(K, M, N, in->df, in->f_low, dd, dp, dm, row0, n_rows, dx, dq, du, dv, nullptr);
  if (e == hipSuccess && n_rows > 0) e = hipMemcpy(Q, dq, sizeof(double) * nq, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(U, du, sizeof(double) * nu, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(V, dv, sizeof(double) * nu, hipMemcpyDeviceToHost);
  release();
  if (e != hipSuccess) return hip_fail(nullptr, e, "precompute");
  return RIFT_OK;
}

rift_status rift_ile_set_network_frame(rift_ile *h, int enable) {
  if (!h) return RIFT_E_INVALID;
  h->net_frame = enable != 0;
  return RIFT_OK;
}

rift_status rift_ile_set_phase_rotation(rift_ile *h, int enable) {
  if (!h) return RIFT_E_INVALID;
  h->phase_rot = enable != 0;
  return RIFT_OK;
}

rift_status rift_ile_set_distance_marginalization(rift_ile *h, int enable) {
  if (!h) return RIFT_E_INVALID;
  h->dmarg = enable != 0;
  return RIFT_OK;
}

rift_status rift_ile_set_grad_refine(rift_ile *h, int enable) {
  if (!h) return RIFT_E_INVALID;
  h->refine = enable != 0;
  return RIFT_OK;
}

rift_status rift_ile_set_autotune(rift_ile *h, int mode) {
  if (!h || mode < 0 || mode > 5) return RIFT_E_INVALID;
  h->feed = mode;
  return RIFT_OK;
}

rift_status rift_ile_set_autotune_cache(rift_ile *h, const char *path) {
  if (!h) return RIFT_E_INVALID;
  if (!path) {
    h->tune_path.clear();
    return RIFT_OK;
  }
  FILE *f = std::fopen(path, "r");
  if (!f) {
    if (errno != ENOENT) return fail(h, RIFT_E_INVALID, "cannot read the autotune cache %s", path);
  } else {
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
      char arch[96];
      int T, K, b, m;
      if (std::sscanf(line, "%95s %d %d %d %d", arch, &T, &K, &b, &m) != 5) continue;
      if (h->arch != arch || T < 1 || T > kMaxT || K < 1 || K > kMaxDet || b < 0 || b >= kNtBuckets || m < 1 ||
          m > kFeedConfigs)
        continue;
      h->tune[T][K][b] = m;  // later lines win
    }
    std::fclose(f);
  }
  h->tune_path = path;
  return RIFT_OK;
}

rift_status rift_ile_autotune_table(const rift_ile *h, int *modes) {
  if (!h || !modes) return RIFT_E_INVALID;
  for (int T = 1; T <= kMaxT; T++)
    for (int K = 1; K <= kMaxDet; K++) modes[(T - 1) * kMaxDet + (K - 1)] = h->kmode[T][K];
  return RIFT_OK;
}

rift_status rift_ile_set_stream(rift_ile *h, void *stream) {
  if (!h) return RIFT_E_INVALID;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->stream = (hipStream_t)stream;
  return RIFT_OK;
}

rift_status rift_ile_sample(rift_ile *h, int point, uint64_t seed, uint32_t round, int64_t first, int64_t n,
                            void *theta, void *ln_ratio, uint8_t *bins) {
  if (!h) return RIFT_E_INVALID;
  if (point < 0 || point >= h->n_points) return fail(h, RIFT_E_INVALID, "point %d", point);
  if (n < 0 || first < 0 || (n > 0 && !theta)) return fail(h, RIFT_E_INVALID, "bad sample range or NULL theta");
  hipError_t e = h->precision == RIFT_FP32
                     ? sample_launch<float>(h->net_frame ? h->d_pts + point : nullptr, h->d_props + point, point, seed,
                                            round, first, n, n, n, h->d_min,
                                            h->d_max, h->tau_width, (float *)theta, (float *)ln_ratio, bins, h->stream,
                                            nullptr, h->any_mix, h->phase_rot)
                     : sample_launch<double>(h->net_frame ? h->d_pts + point : nullptr, h->d_props + point, point, seed,
                                             round, first, n, n, n, h->d_min,
                                             h->d_max, h->tau_width, (double *)theta, (double *)ln_ratio, bins,
                                             h->stream, nullptr, h->any_mix, h->phase_rot);
  if (e != hipSuccess) return hip_fail(h, e, "sample");
  return RIFT_OK;
}

rift_status rift_ile_lnL(rift_ile *h, int n_items, const rift_ile_item *items, int64_t stride, const void *theta,
                         void *lnL_t) {
  if (!h) return RIFT_E_INVALID;
  rift_status s = check_items(h, n_items, items, stride);
  if (s != RIFT_OK) return s;
  if (n_items > 0 && stride > 0 && (!theta || !lnL_t)) return fail(h, RIFT_E_INVALID, "NULL theta or lnL_t");
  Items it = make_items(n_items, items);
  if (h->precision == RIFT_FP32)
    return eval<float>(h, it, stride, (const float *)theta, (float *)lnL_t, nullptr, nullptr);
  return eval<double>(h, it, stride, (const double *)theta, (double *)lnL_t, nullptr, nullptr);
}

rift_status rift_ile_reduce(rift_ile *h, int64_t n, const void *lnL_t, const void *ln_ratio, rift_ile_result *out) {
  if (!h) return RIFT_E_INVALID;
  if (n < 0 || (n > 0 && !lnL_t) || !out) return fail(h, RIFT_E_INVALID, "bad reduce arguments");
  void *d_res;
  rift_status s = ws_get(h, W_RESULT, sizeof(rift_ile_result), &d_res);
  if (s != RIFT_OK) return s;
  std::vector<int64_t> off(1, 0), cnt(1, n);
  if (h->precision == RIFT_FP32)
    s = reduce_segments<float>(h, (const float *)lnL_t, (const float *)ln_ratio, off, cnt, nullptr, nullptr, 0,
                               (rift_ile_result *)d_res);
  else
    s = reduce_segments<double>(h, (const double *)lnL_t, (const double *)ln_ratio, off, cnt, nullptr, nullptr, 0,
                                (rift_ile_result *)d_res);
  if (s != RIFT_OK) return s;
  HIPCHK(h, hipMemcpyAsync(out, d_res, sizeof(rift_ile_result), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return RIFT_OK;
}

rift_status rift_ile_reduce_noalloc(rift_ile *h, int64_t n, const void *lnL_t, const void *ln_ratio,
                                   rift_ile_result *out) {
  if (!h) return RIFT_E_INVALID;
  if (n < 0 || (n > 0 && !lnL_t) || !out) return fail(h, RIFT_E_INVALID, "bad reduce arguments");
  if (n > kNoAllocMaxN)
    return fail(h, RIFT_E_SHAPE, "rift_ile_reduce_noalloc: n = %lld exceeds %lld samples", (long long)n,
                (long long)kNoAllocMaxN);
  if (!h->scratch) return fail(h, RIFT_E_STATE, "no scratch address for device %d", h->device);
  NoAllocScratch *sc = (NoAllocScratch *)h->scratch;  // this device's copy
  const int bps = reduce_bps(n);
  const int64_t seg[2] = {0, n};
  HIPCHK(h, hipMemcpyAsync(sc->seg, seg, sizeof(seg), hipMemcpyHostToDevice, h->stream));
  if (h->precision == RIFT_FP32)
    HIPCHK(h, reduce_partials<float>((const float *)lnL_t, (const float *)ln_ratio, &sc->seg[0], &sc->seg[1], 1, bps,
                                     sc->partials, h->stream));
  else
    HIPCHK(h, reduce_partials<double>((const double *)lnL_t, (const double *)ln_ratio, &sc->seg[0], &sc->seg[1], 1,
                                      bps, sc->partials, h->stream));
  HIPCHK(h, reduce_finish(sc->partials, 1, bps, &sc->merged, nullptr, 0, &sc->result, h->stream));
  HIPCHK(h, hipMemcpyAsync(out, &sc->result, sizeof(rift_ile_result), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return RIFT_OK;
}

rift_status rift_ile_adapt(rift_ile *h, int point, int64_t n, const uint8_t *bins, const void *lnw, unsigned mask,
                           double floor_eps) {
  if (!h) return RIFT_E_INVALID;
  if (point < 0 || point >= h->n_points) return fail(h, RIFT_E_INVALID, "point %d", point);
  if (n < 0 || n > (1 << 23) || (n > 0 && (!bins || !lnw))) return fail(h, RIFT_E_INVALID, "bad adapt arguments");
  if (!(floor_eps > 0.0 && floor_eps <= 1.0)) return fail(h, RIFT_E_INVALID, "floor_eps %g", floor_eps);
  if (mask >> 7) return fail(h, RIFT_E_INVALID, "mask 0x%x", mask);
  std::vector<int64_t> off(1, 0), cnt(1, n);
  std::vector<int> sp(1, point);
  ReduceTuple *round;
  rift_status s;
  int *d_sp;
  void *hist;
  const int bps = hist_blocks(n);
  if ((s = ws_get(h, W_HIST, sizeof(unsigned long long) * 7 * kNB * bps, &hist)) != RIFT_OK) return s;
  if (h->precision == RIFT_FP32) {
    if ((s = reduce_segments<float>(h, (const float *)lnw, nullptr, off, cnt, &round, nullptr, 0, nullptr)) != RIFT_OK)
      return s;
    if ((s = upload(h, W_AUX, sp, &d_sp)) != RIFT_OK) return s;
    int64_t *d_off = (int64_t *)h->ws[W_ITEM_OFF].p, *d_cnt = (int64_t *)h->ws[W_ITEM_CNT].p;
    HIPCHK(h, adapt_launch<float>(bins, n, (const float *)lnw, d_off, d_cnt, d_sp, 1, bps, round,
                                  (unsigned long long *)hist, h->d_props, mask, floor_eps, h->stream));
  } else {
    if ((s = reduce_segments<double>(h, (const double *)lnw, nullptr, off, cnt, &round, nullptr, 0, nullptr)) !=
        RIFT_OK)
      return s;
    if ((s = upload(h, W_AUX, sp, &d_sp)) != RIFT_OK) return s;
    int64_t *d_off = (int64_t *)h->ws[W_ITEM_OFF].p, *d_cnt = (int64_t *)h->ws[W_ITEM_CNT].p;
    HIPCHK(h, adapt_launch<double>(bins, n, (const double *)lnw, d_off, d_cnt, d_sp, 1, bps, round,
                                   (unsigned long long *)hist, h->d_props, mask, floor_eps, h->stream));
  }
  return RIFT_OK;
}

rift_status rift_ile_get_proposal(rift_ile *h, int point, double *cdf, unsigned *mask) {
  if (!h) return RIFT_E_INVALID;
  if (point < 0 || point >= h->n_points || !cdf) return fail(h, RIFT_E_INVALID, "bad get_proposal arguments");
  ProposalDev pr;
  HIPCHK(h, hipMemcpyAsync(&pr, h->d_props + point, sizeof(pr), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  std::memcpy(cdf, pr.cdf, sizeof(pr.cdf));
  if (mask) *mask = pr.mask;
  return RIFT_OK;
}

rift_status rift_ile_set_proposal(rift_ile *h, int point, const double *cdf, unsigned mask) {
  if (!h) return RIFT_E_INVALID;
  if (point < 0 || point >= h->n_points || !cdf || (mask >> 7))
    return fail(h, RIFT_E_INVALID, "bad set_proposal arguments");
  ProposalDev pr;
  std::memset(&pr, 0, sizeof pr);
  for (int d = 0; d < 7; d++) {
    const double *c = cdf + d * (kNB + 1);
    if (c[0] != 0.0 || c[kNB] != 1.0) return fail(h, RIFT_E_INVALID, "cdf[%d] must run from 0 to 1", d);
    for (int b = 0; b < kNB; b++)
      if (!(c[b + 1] > c[b])) return fail(h, RIFT_E_INVALID, "cdf[%d] not strictly increasing at %d", d, b);
    std::memcpy(pr.cdf[d], c, sizeof(double) * (kNB + 1));
  }
  pr.mask = mask;
  // on the handle's stream, after any pending sampling or adaptation that
  // reads or writes the proposals, and complete before the host copy is freed
  HIPCHK(h, hipMemcpyAsync(h->d_props + point, &pr, sizeof(pr), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return RIFT_OK;
}

rift_status rift_ile_get_gmm(rift_ile *h, int point, int *K, unsigned *mask, double *floor_eps, double *n_trained,
                             double *w, double *mu, double *sd) {
  if (!h) return RIFT_E_INVALID;
  if (point < 0 || point >= h->n_points || !K) return fail(h, RIFT_E_INVALID, "bad get_gmm arguments");
  ProposalDev pr;
  HIPCHK(h, hipMemcpyAsync(&pr, h->d_props + point, sizeof(pr), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  *K = pr.gk;
  if (mask) *mask = pr.mask;
  if (floor_eps) *floor_eps = pr.geps;
  if (n_trained) *n_trained = pr.gntr;
  for (int d = 0; d < 7; d++)
    for (int k = 0; k < kMaxG; k++) {
      if (w) w[d * kMaxG + k] = pr.gw[d][k];
      if (mu) mu[d * kMaxG + k] = pr.gmu[d][k];
      if (sd) sd[d * kMaxG + k] = pr.gsd[d][k];
    }
  return RIFT_OK;
}

rift_status rift_ile_set_gmm(rift_ile *h, int point, int K, unsigned mask, double floor_eps, double n_trained,
                             const double *w, const double *mu, const double *sd) {
  if (!h) return RIFT_E_INVALID;
  if (point < 0 || point >= h->n_points || K < 1 || K > kMaxG || (mask >> 7) || !w || !mu || !sd)
    return fail(h, RIFT_E_INVALID, "bad set_gmm arguments");
  if (!(floor_eps >= 0.0 && floor_eps <= 1.0) || !(n_trained >= 0.0))
    return fail(h, RIFT_E_INVALID, "floor_eps %g or n_trained %g", floor_eps, n_trained);
  ProposalDev pr;
  uniform_proposal(pr);
  for (int d = 0; d < 7; d++) {
    double tot = 0.0;
    for (int k = 0; k < kMaxG; k++) {
      const double wk = k < K ? w[d * kMaxG + k] : 0.0, m = k < K ? mu[d * kMaxG + k] : 0.5,
                   s = k < K ? sd[d * kMaxG + k] : 0.5;
      if (!(wk >= 0.0) || !(m >= 0.0 && m <= 1.0) || !(s > 0.0) || !std::isfinite(s))
        return fail(h, RIFT_E_INVALID, "component %d of parameter %d", k, d);
      pr.gw[d][k] = wk;
      pr.gmu[d][k] = m;
      pr.gsd[d][k] = s;
      tot += wk;
    }
    if (((mask >> d) & 1u) && !(std::fabs(tot - 1.0) < 1e-9))
      return fail(h, RIFT_E_INVALID, "weights of parameter %d sum to %g", d, tot);
  }
  gmm_norms(pr);
  h->any_mix = true;
  pr.gk = K;
  pr.mask = mask;
  pr.geps = floor_eps;
  pr.gntr = n_trained;
  // on the handle's stream, after any pending sampling or adaptation that
  // reads or writes the proposals, and complete before the host copy is freed
  HIPCHK(h, hipMemcpyAsync(h->d_props + point, &pr, sizeof(pr), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return RIFT_OK;
}

rift_status rift_ile_adapt_gmm(rift_ile *h, int point, int64_t n, const float *u, const void *lnw, unsigned mask,
                               unsigned pairs, double floor_eps, int K, int n_iter) {
  if (!h) return RIFT_E_INVALID;
  if (point < 0 || point >= h->n_points) return fail(h, RIFT_E_INVALID, "point %d", point);
  if (n < 0 || (n > 0 && (!u || !lnw))) return fail(h, RIFT_E_INVALID, "bad adapt_gmm arguments");
  if (!(floor_eps > 0.0 && floor_eps <= 1.0)) return fail(h, RIFT_E_INVALID, "floor_eps %g", floor_eps);
  if ((mask >> 7) || K < 1 || K > kMaxG || n_iter < 1 || n_iter > 1000)
    return fail(h, RIFT_E_INVALID, "mask 0x%x, K %d (1..%d) or n_iter %d (1..1000)", mask, K, kMaxG, n_iter);
  rift_status s;
  if ((s = check_pairs(h, pairs, mask)) != RIFT_OK) return s;
  std::vector<int64_t> off(1, 0), cnt(1, n);
  std::vector<int> sp(1, point);
  ReduceTuple *round;
  int *d_sp;
  void *part, *part2, *fit, *wt;
  int *d_blk;
  const int bps = em_blocks(n);
  const int wblk = (int)((n + 255) / 256);
  if ((s = ws_get(h, W_EMWT, sizeof(double) * (size_t)std::max<int64_t>(n, 1), &wt)) != RIFT_OK) return s;
  if ((s = upload(h, W_SEG_BLK, std::vector<int>{0, wblk}, &d_blk)) != RIFT_OK) return s;
  if ((s = ws_get(h, W_EMPART, sizeof(double) * 7 * 3 * kMaxG * bps, &part)) != RIFT_OK) return s;
  if ((s = ws_get(h, W_EMPART2, sizeof(double) * kMaxPair * 6 * kMaxG * bps, &part2)) != RIFT_OK) return s;
  if ((s = ws_get(h, W_GMMFIT, 2 * sizeof(GmmDev), &fit)) != RIFT_OK) return s;
  if (h->precision == RIFT_FP32) {
    if ((s = reduce_segments<float>(h, (const float *)lnw, nullptr, off, cnt, &round, nullptr, 0, nullptr)) != RIFT_OK)
      return s;
    if ((s = upload(h, W_AUX, sp, &d_sp)) != RIFT_OK) return s;
    int64_t *d_off = (int64_t *)h->ws[W_ITEM_OFF].p, *d_cnt = (int64_t *)h->ws[W_ITEM_CNT].p;
    HIPCHK(h, gmm_adapt_launch<float>(u, n, (const float *)lnw, d_off, d_cnt, d_sp, 1, bps, round, (double *)part,
                                      (double *)part2, (GmmDev *)fit, h->d_props, mask, pairs, floor_eps, K, n_iter,
                                      d_blk, wblk, (double *)wt, h->stream));
  } else {
    if ((s = reduce_segments<double>(h, (const double *)lnw, nullptr, off, cnt, &round, nullptr, 0, nullptr)) !=
        RIFT_OK)
      return s;
    if ((s = upload(h, W_AUX, sp, &d_sp)) != RIFT_OK) return s;
    int64_t *d_off = (int64_t *)h->ws[W_ITEM_OFF].p, *d_cnt = (int64_t *)h->ws[W_ITEM_CNT].p;
    HIPCHK(h, gmm_adapt_launch<double>(u, n, (const double *)lnw, d_off, d_cnt, d_sp, 1, bps, round, (double *)part,
                                       (double *)part2, (GmmDev *)fit, h->d_props, mask, pairs, floor_eps, K, n_iter,
                                       d_blk, wblk, (double *)wt, h->stream));
  }
  HIPCHK(h, pair_norm_launch(h->d_props, point, 1, h->stream));
  h->any_mix = true;
  return RIFT_OK;
}

rift_status rift_ile_set_gmm_pairs(rift_ile *h, int point, unsigned pairs, const double *w, const double *mu,
                                   const double *cov) {
  if (!h) return RIFT_E_INVALID;
  if (point < 0 || point >= h->n_points || (pairs && (!w || !mu || !cov)))
    return fail(h, RIFT_E_INVALID, "bad set_gmm_pairs arguments");
  ProposalDev pr;
  HIPCHK(h, hipMemcpyAsync(&pr, h->d_props + point, sizeof(pr), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (pr.gk < 1) return fail(h, RIFT_E_INVALID, "point %d holds no mixture (rift_ile_set_gmm first)", point);
  rift_status s = check_pairs(h, pairs, pr.mask);
  if (s != RIFT_OK) return s;
  pr.npair = 0;
  for (int i = 0; i < kMaxPair; i++) {
    const unsigned c = (pairs >> (8 * i)) & 0xFFu;
    if (!c) continue;
    const int p = pr.npair++;
    pr.pa[p] = (int)(c & 15u);
    pr.pb[p] = (int)(c >> 4);
    double tot = 0.0;
    for (int k = 0; k < kMaxG; k++) {
      const double *m = mu + (p * kMaxG + k) * 2, *c3 = cov + (p * kMaxG + k) * 3;
      const double wk = k < pr.gk ? w[p * kMaxG + k] : 0.0;
      const bool on = k < pr.gk;
      const double xx = on ? c3[0] : 0.25, xy = on ? c3[1] : 0.0, yy = on ? c3[2] : 0.25;
      if (!(wk >= 0.0) || (on && !(m[0] >= 0.0 && m[0] <= 1.0 && m[1] >= 0.0 && m[1] <= 1.0)) || !(xx > 0.0) ||
          !(yy > 0.0) || !(std::fabs(xy) < std::sqrt(xx * yy)) || !std::isfinite(xx * yy))
        return fail(h, RIFT_E_INVALID, "component %d of pair %d", k, p);
      pr.pw[p][k] = wk;
      pr.pmu[p][k][0] = on ? m[0] : 0.5;
      pr.pmu[p][k][1] = on ? m[1] : 0.5;
      pr.pcov[p][k][0] = xx;
      pr.pcov[p][k][1] = xy;
      pr.pcov[p][k][2] = yy;
      tot += wk;
    }
    if (!(std::fabs(tot - 1.0) < 1e-9)) return fail(h, RIFT_E_INVALID, "weights of pair %d sum to %g", p, tot);
  }
  HIPCHK(h, hipMemcpyAsync(h->d_props + point, &pr, sizeof(pr), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, pair_norm_launch(h->d_props, point, 1, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return RIFT_OK;
}

rift_status rift_ile_get_gmm_pairs(rift_ile *h, int point, unsigned *pairs, double *w, double *mu, double *cov,
                                   double *box_mass) {
  if (!h) return RIFT_E_INVALID;
  if (point < 0 || point >= h->n_points || !pairs) return fail(h, RIFT_E_INVALID, "bad get_gmm_pairs arguments");
  ProposalDev pr;
  HIPCHK(h, hipMemcpyAsync(&pr, h->d_props + point, sizeof(pr), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  *pairs = 0u;
  const int np = pr.gk > 0 ? pr.npair : 0;
  for (int p = 0; p < np; p++) *pairs |= (unsigned)(pr.pa[p] | (pr.pb[p] << 4)) << (8 * p);
  for (int p = 0; p < kMaxPair; p++) {
    if (box_mass) box_mass[p] = p < np ? pr.pzm[p] : 0.0;
    for (int k = 0; k < kMaxG; k++) {
      if (w) w[p * kMaxG + k] = p < np ? pr.pw[p][k] : 0.0;
      for (int q = 0; q < 2; q++)
        if (mu) mu[(p * kMaxG + k) * 2 + q] = p < np ? pr.pmu[p][k][q] : 0.0;
      for (int q = 0; q < 3; q++)
        if (cov) cov[(p * kMaxG + k) * 3 + q] = p < np ? pr.pcov[p][k][q] : 0.0;
    }
  }
  return RIFT_OK;
}

// checkpoint blob: header, then per point its proposal and its pooled tuple
struct CkptHeader {
  char magic[8];
  int32_t version, n_points;
  int64_t proposal_bytes, tuple_bytes;
  int32_t coords, reserved;  // what the proposals and estimates refer to: bit 0 network frame, bit 1 phase
                             // rotation, bit 2 distance marginalization
};
int32_t coords_of(const rift_ile *h) {
  return (h->net_frame ? 1 : 0) | (h->phase_rot ? 2 : 0) | (h->dmarg ? 4 : 0);
}
constexpr char kCkptMagic[8] = {'R', 'I', 'F', 'T', 'C', 'K', 'P', '1'};

int64_t rift_ile_checkpoint_bytes(const rift_ile *h) {
  if (!h) return -1;
  return (int64_t)sizeof(CkptHeader) + (int64_t)h->n_points * (int64_t)(sizeof(ProposalDev) + sizeof(ReduceTuple));
}

rift_status rift_ile_save_checkpoint(rift_ile *h, void *buf, int64_t bytes) {
  if (!h) return RIFT_E_INVALID;
  if (!buf || bytes < rift_ile_checkpoint_bytes(h)) return fail(h, RIFT_E_INVALID, "checkpoint buffer too small");
  if (!h->have_accum) return fail(h, RIFT_E_STATE, "no pooled estimate to save (run rift_ile_marginalize first)");
  const int np = h->n_points;
  CkptHeader hd;
  std::memcpy(hd.magic, kCkptMagic, 8);
  hd.version = RIFT_ILE_ABI_VERSION;
  hd.n_points = np;
  hd.proposal_bytes = sizeof(ProposalDev);
  hd.tuple_bytes = sizeof(ReduceTuple);
  hd.coords = coords_of(h);
  hd.reserved = 0;
  char *c = (char *)buf;
  std::memcpy(c, &hd, sizeof hd);
  c += sizeof hd;
  HIPCHK(h, hipMemcpyAsync(c, h->d_props, sizeof(ProposalDev) * np, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipMemcpyAsync(c + sizeof(ProposalDev) * np, h->ws[W_ACCUM].p, sizeof(ReduceTuple) * np,
                           hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return RIFT_OK;
}

rift_status rift_ile_load_checkpoint(rift_ile *h, const void *buf, int64_t bytes) {
  if (!h) return RIFT_E_INVALID;
  if (!buf || bytes < (int64_t)sizeof(CkptHeader)) return fail(h, RIFT_E_INVALID, "checkpoint buffer too small");
  CkptHeader hd;
  std::memcpy(&hd, buf, sizeof hd);
  const int np = h->n_points;
  if (std::memcmp(hd.magic, kCkptMagic, 8) != 0 || hd.version != RIFT_ILE_ABI_VERSION || hd.n_points != np ||
      hd.proposal_bytes != (int64_t)sizeof(ProposalDev) || hd.tuple_bytes != (int64_t)sizeof(ReduceTuple) ||
      bytes < rift_ile_checkpoint_bytes(h))
    return fail(h, RIFT_E_INVALID, "checkpoint from another library version or point count");
  // the proposals' tables live in the coordinates the sampler used: a resumed
  // run must draw in the same ones
  if (hd.coords != coords_of(h))
    return fail(h, RIFT_E_INVALID, "checkpoint drawn with network frame %d, phase rotation %d, distance "
                "marginalization %d; the handle has %d, %d, %d", hd.coords & 1, (hd.coords >> 1) & 1,
                (hd.coords >> 2) & 1, h->net_frame ? 1 : 0, h->phase_rot ? 1 : 0, h->dmarg ? 1 : 0);
  const char *c = (const char *)buf + sizeof hd;
  std::vector<ProposalDev> props(np);
  std::memcpy(props.data(), c, sizeof(ProposalDev) * np);
  // every field a kernel uses as an index or divides by is checked before
  // anything reaches the device
  bool mix = false;
  for (const auto &p : props) {
    bool ok = p.gk >= 0 && p.gk <= kMaxG && p.npair >= 0 && p.npair <= kMaxPair && !(p.mask >> 7) &&
              (p.npair == 0 || p.gk > 0);
    for (int d = 0; ok && d < 7; d++) {
      ok = p.cdf[d][0] == 0.0 && p.cdf[d][kNB] == 1.0;
      for (int b = 0; ok && b < kNB; b++) ok = p.cdf[d][b + 1] > p.cdf[d][b];
    }
    for (int d = 0; ok && d < 7; d++)
      for (int k = 0; ok && k < p.gk; k++)
        ok = std::isfinite(p.gw[d][k]) && std::isfinite(p.gmu[d][k]) && p.gsd[d][k] > 0 && std::isfinite(p.gsd[d][k]) &&
             std::isfinite(p.gca[d][k]) && p.gz[d][k] > 0 && std::isfinite(p.gz[d][k]);
    unsigned used = 0u;
    for (int q = 0; ok && q < p.npair; q++) {
      ok = p.pa[q] >= 0 && p.pa[q] < p.pb[q] && p.pb[q] < 7 && ((p.mask >> p.pa[q]) & 1u) &&
           ((p.mask >> p.pb[q]) & 1u) && !((used >> p.pa[q]) & 1u) && !((used >> p.pb[q]) & 1u) && p.pzm[q] > 0 &&
           p.pzm[q] <= 1.0 + 1e-12;
      used |= (1u << p.pa[q]) | (1u << p.pb[q]);
    }
    if (!ok || !(p.geps >= 0 && p.geps <= 1)) return fail(h, RIFT_E_INVALID, "checkpoint: corrupt proposal");
    mix = mix || p.gk > 0;
  }
  if (mix) h->any_mix = true;
  void *accum;
  rift_status s = ws_get(h, W_ACCUM, sizeof(ReduceTuple) * np, &accum);
  if (s != RIFT_OK) return s;
  HIPCHK(h, hipMemcpyAsync(h->d_props, props.data(), sizeof(ProposalDev) * np, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(accum, c + sizeof(ProposalDev) * np, sizeof(ReduceTuple) * np, hipMemcpyHostToDevice,
                           h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->have_accum = true;
  return RIFT_OK;
}

rift_status rift_ile_marginalize(rift_ile *h, const rift_ile_mc *mc, rift_ile_result *out, void *theta_out,
                                 void *lnw_out) {
  if (!h) return RIFT_E_INVALID;
  if (!mc || !out || mc->n_rounds < 1 || (mc->adapt_mask >> 7)) return fail(h, RIFT_E_INVALID, "bad mc arguments");
  if (mc->adapt_mask && !(mc->floor_eps > 0.0 && mc->floor_eps <= 1.0))
    return fail(h, RIFT_E_INVALID, "floor_eps %g", mc->floor_eps);
  if (mc->first_round < 0 || (mc->first_round > 0 && mc->reset_proposal) ||
      (int64_t)mc->first_round + mc->n_rounds > (mc->gmm_pairs ? (1 << 20) : (1 << 30)))
    return fail(h, RIFT_E_INVALID, "first_round %d: >= 0, with reset_proposal = 0 when > 0, rounds below 2^30 (2^20 "
                "with pairs)", mc->first_round);
  if (mc->first_round > 0 && !h->have_accum)
    return fail(h, RIFT_E_STATE, "first_round > 0 needs a pooled estimate (an earlier run or a loaded checkpoint)");
  if (h->precision == RIFT_FP32) return marginalize_impl<float>(h, mc, out, (float *)theta_out, (float *)lnw_out);
  return marginalize_impl<double>(h, mc, out, (double *)theta_out, (double *)lnw_out);
}

rift_status rift_ile_backward(rift_ile *h, int n_items, const rift_ile_item *items, int64_t stride, const void *theta,
                              const void *grad_lnL_t, void *grad_theta, void *lnL_t_out) {
  if (!h) return RIFT_E_INVALID;
  if (h->dmarg) return fail(h, RIFT_E_INVALID, "no adjoint of the distance-marginalized likelihood");
  rift_status s = check_items(h, n_items, items, stride);
  if (s != RIFT_OK) return s;
  if (n_items > 0 && stride > 0 && (!theta || !grad_theta)) return fail(h, RIFT_E_INVALID, "NULL theta or grad");
  Items it = make_items(n_items, items);
  if (h->precision == RIFT_FP32)
    return eval_grad<float>(h, it, stride, (const float *)theta, (float *)lnL_t_out, (const float *)grad_lnL_t,
                            (float *)grad_theta);
  return eval_grad<double>(h, it, stride, (const double *)theta, (double *)lnL_t_out, (const double *)grad_lnL_t,
                           (double *)grad_theta);
}

}  // extern "C"
