// Drives the host side of the C ABI (include/rift_ile.h) for a build of the
// library's host code with AddressSanitizer and UndefinedBehaviorSanitizer:
//   host_driver host    argument and point validation that runs before any
//                       device call (every rejection status of create, calls
//                       on a NULL handle, the precompute's checks)
//   host_driver device  the same plus, on a GPU, item checks, evaluation,
//                       backward, an adaptive run, checkpoint save and load
//                       (good, truncated and corrupted blobs) and the
//                       no-allocation reduction
// Prints "ok <checks>" and exits 0 when every call returned what it should;
// any sanitizer report fails the calling test.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "rift_ile.h"

static int g_checks = 0, g_fail = 0;

static void expect(int got, int want, const char *what) {
  g_checks++;
  if (got != want) {
    std::printf("FAIL %s: status %d, expected %d\n", what, got, want);
    g_fail++;
  }
}

static double urand(unsigned *s) {
  *s = *s * 1664525u + 1013904223u;
  return ((*s >> 8) + 0.5) / 16777216.0;
}

// a small valid point: K = 2 (the LIGO sites), M = 3 modes, n_t = 40
struct PointData {
  int K = 2, M = 3, n_t = 40, pad = 90;
  std::vector<int> ell{2, 2, 3}, em{2, -2, 3};
  std::vector<double> pos{-2.16141492636e06, -3.83469517889e06, 4.60035022664e06,
                          -7.42760447238e04, -5.49628371971e06, 3.22425701744e06};
  std::vector<double> resp, Q, U;
  PointData() {
    unsigned seed = 99u;
    resp.assign(9 * K, 0.0);
    for (int k = 0; k < K; k++) {
      resp[9 * k + 0] = 0.5;
      resp[9 * k + 4] = -0.5;
      resp[9 * k + 1] = resp[9 * k + 3] = 0.1 * (k + 1);
    }
    const int L = n_t + 2 * pad + 3;
    Q.resize((size_t)2 * K * L * M);
    for (auto &q : Q) q = 4.0 * (urand(&seed) - 0.5);
    U.assign((size_t)2 * K * M * M, 0.0);
    for (int k = 0; k < K; k++)  // U = G G^H + I, Hermitian positive definite
      for (int a = 0; a < M; a++)
        for (int b = 0; b < M; b++) {
          double re = a == b ? 1.0 : 0.0, im = 0.0;
          for (int c = 0; c < M; c++) {
            const double ga = 0.3 * (a + 1) * (c + 1) / 9.0, gai = 0.1 * (a - c);
            const double gb = 0.3 * (b + 1) * (c + 1) / 9.0, gbi = 0.1 * (b - c);
            re += ga * gb + gai * gbi;
            im += gai * gb - ga * gbi;
          }
          U[2 * ((size_t)k * M * M + a * M + b)] = re;
          U[2 * ((size_t)k * M * M + a * M + b) + 1] = im;
        }
  }
  rift_ile_point point() const {
    rift_ile_point p;
    std::memset(&p, 0, sizeof p);
    p.n_det = K;
    p.n_modes = M;
    p.n_t = n_t;
    p.pad = pad;
    p.ell = ell.data();
    p.em = em.data();
    p.f_s = 4096.0;
    p.d_ref = 100.0;
    p.gmst = 0.3;
    p.det_pos = pos.data();
    p.det_resp = resp.data();
    p.Q = Q.data();
    p.U = U.data();
    p.V = nullptr;
    return p;
  }
};

static rift_ile_desc desc_of(const rift_ile_point *pts, int n, int precision) {
  rift_ile_desc d;
  std::memset(&d, 0, sizeof d);
  d.n_points = n;
  d.points = pts;
  d.precision = precision;
  d.d_min = 10.0;
  d.d_max = 1000.0;
  d.tau_width = 0.0;
  return d;
}

static void host_checks() {
  rift_ile *h = nullptr;
  expect(rift_ile_create(&h, nullptr, nullptr), RIFT_E_INVALID, "create(NULL desc)");
  expect(rift_ile_create(nullptr, nullptr, nullptr), RIFT_E_INVALID, "create(NULL out)");
  PointData pd;
  rift_ile_point p = pd.point();
  rift_ile_desc d = desc_of(&p, 1, 7);
  expect(rift_ile_create(&h, &d, nullptr), RIFT_E_INVALID, "bad precision");
  d = desc_of(&p, 1, RIFT_FP32);
  d.d_max = 5.0;
  expect(rift_ile_create(&h, &d, nullptr), RIFT_E_INVALID, "distance prior");
  struct Case {
    const char *what;
    int want;
    void (*edit)(rift_ile_point &);
  };
  static std::vector<double> badQ, badU;
  const Case cases[] = {
      {"n_det 0", RIFT_E_SHAPE, [](rift_ile_point &q) { q.n_det = 0; }},
      {"n_modes 40", RIFT_E_SHAPE, [](rift_ile_point &q) { q.n_modes = 40; }},
      {"n_t 0", RIFT_E_SHAPE, [](rift_ile_point &q) { q.n_t = 0; }},
      {"pad 40000", RIFT_E_SHAPE, [](rift_ile_point &q) { q.pad = 40000; }},
      {"pad too small", RIFT_E_WINDOW, [](rift_ile_point &q) { q.pad = 10; }},
      {"NULL Q", RIFT_E_INVALID, [](rift_ile_point &q) { q.Q = nullptr; }},
      {"mode (9, 0)", RIFT_E_INVALID, [](rift_ile_point &q) { static int l[3] = {2, 2, 9}; q.ell = l; }},
      {"f_s NaN", RIFT_E_NONFINITE, [](rift_ile_point &q) { q.f_s = NAN; }},
      {"Q NaN", RIFT_E_NONFINITE,
       [](rift_ile_point &q) {
         const size_t n = (size_t)2 * q.n_det * (q.n_t + 2 * q.pad + 3) * q.n_modes;
         badQ.assign(q.Q, q.Q + n);
         badQ[n - 1] = INFINITY;
         q.Q = badQ.data();
       }},
      {"U not Hermitian", RIFT_E_NOT_HERMITIAN,
       [](rift_ile_point &q) {
         const size_t n = (size_t)2 * q.n_det * q.n_modes * q.n_modes;
         badU.assign(q.U, q.U + n);
         badU[2 * 1 + 1] += 0.5;  // Im U_01 without its partner
         q.U = badU.data();
       }},
  };
  for (const Case &c : cases) {
    rift_ile_point q = pd.point();
    c.edit(q);
    rift_ile_desc dd = desc_of(&q, 1, RIFT_FP32);
    h = reinterpret_cast<rift_ile *>(0x1);
    expect(rift_ile_create(&h, &dd, nullptr), c.want, c.what);
    g_checks++;
    if (h != nullptr) {
      std::printf("FAIL %s: handle not cleared\n", c.what);
      g_fail++;
    }
    g_checks++;
    if (std::strlen(rift_ile_last_error(nullptr)) == 0) {
      std::printf("FAIL %s: no error text\n", c.what);
      g_fail++;
    }
  }
  // calls on a NULL handle
  rift_ile_result r;
  expect(rift_ile_lnL(nullptr, 0, nullptr, 0, nullptr, nullptr), RIFT_E_INVALID, "lnL(NULL)");
  expect(rift_ile_reduce(nullptr, 0, nullptr, nullptr, &r), RIFT_E_INVALID, "reduce(NULL)");
  expect(rift_ile_reduce_noalloc(nullptr, 0, nullptr, nullptr, &r), RIFT_E_INVALID, "reduce_noalloc(NULL)");
  expect(rift_ile_marginalize(nullptr, nullptr, &r, nullptr, nullptr), RIFT_E_INVALID, "marginalize(NULL)");
  expect(rift_ile_backward(nullptr, 0, nullptr, 0, nullptr, nullptr, nullptr, nullptr), RIFT_E_INVALID,
         "backward(NULL)");
  expect(rift_ile_load_checkpoint(nullptr, nullptr, 0), RIFT_E_INVALID, "load_checkpoint(NULL)");
  expect(rift_ile_set_grad_refine(nullptr, 1), RIFT_E_INVALID, "set_grad_refine(NULL)");
  expect((int)rift_ile_checkpoint_bytes(nullptr), -1, "checkpoint_bytes(NULL)");
  for (int s = 1; s >= -9; s--) {
    g_checks++;
    if (!rift_ile_status_string(s)) g_fail++;
  }
  // the precompute's argument checks (before any device work)
  rift_ile_fd_point fd;
  std::memset(&fd, 0, sizeof fd);
  expect(rift_ile_precompute(nullptr, 0, 0, nullptr, nullptr, nullptr), RIFT_E_INVALID, "precompute(NULL)");
  fd.n_det = 1;
  fd.n_modes = 1;
  fd.n_f = 1;
  fd.df = 1.0;
  expect(rift_ile_precompute(&fd, 0, 0, nullptr, nullptr, nullptr), RIFT_E_INVALID, "precompute(NULL arrays)");
}

static void device_checks() {
  PointData pd;
  rift_ile_point pts[2] = {pd.point(), pd.point()};
  for (int prec : {RIFT_FP32, RIFT_FP64}) {
    rift_ile_desc d = desc_of(pts, 2, prec);
    rift_ile *h = nullptr;
    expect(rift_ile_create(&h, &d, nullptr), RIFT_OK, "create");
    if (!h) return;
    const size_t es = prec == RIFT_FP32 ? 4 : 8;
    const int64_t n = 1000;
    // samples: drawn on the device for point 0 and point 1
    void *th = nullptr, *lt = nullptr, *gr = nullptr, *lr = nullptr;
    (void)hipMalloc(&th, 7 * es * 2 * n);
    (void)hipMalloc(&lt, es * 2 * n);
    (void)hipMalloc(&lr, es * 2 * n);
    (void)hipMalloc(&gr, 7 * es * 2 * n);
    // theta [7][2n] from point 0's proposal (the prior, the same for both points)
    expect(rift_ile_sample(h, 0, 7, 0, 0, 2 * n, th, lr, nullptr), RIFT_OK, "sample");
    expect(rift_ile_sample(h, 2, 7, 0, 0, 2 * n, th, lr, nullptr), RIFT_E_INVALID, "sample of a point out of range");
    rift_ile_item it[2] = {{0, 0, n}, {1, n, n}};
    expect(rift_ile_lnL(h, 2, it, 2 * n, th, lt), RIFT_OK, "lnL");
    rift_ile_item bad[3] = {{2, 0, n}, {0, n, n + 1}, {0, -1, 5}};
    expect(rift_ile_lnL(h, 1, &bad[0], 2 * n, th, lt), RIFT_E_INVALID, "item point out of range");
    expect(rift_ile_lnL(h, 1, &bad[1], 2 * n, th, lt), RIFT_E_INVALID, "item past the stride");
    expect(rift_ile_lnL(h, 1, &bad[2], 2 * n, th, lt), RIFT_E_INVALID, "negative offset");
    expect(rift_ile_lnL(h, -1, it, 2 * n, th, lt), RIFT_E_INVALID, "negative item count");
    expect(rift_ile_backward(h, 2, it, 2 * n, th, nullptr, gr, lt), RIFT_OK, "backward");
    rift_ile_result r1, r2;
    expect(rift_ile_reduce(h, 2 * n, lt, nullptr, &r1), RIFT_OK, "reduce");
    expect(rift_ile_reduce_noalloc(h, 2 * n, lt, nullptr, &r2), RIFT_OK, "reduce_noalloc");
    g_checks++;
    if (std::memcmp(&r1, &r2, sizeof r1) != 0) {
      std::printf("FAIL reduce_noalloc differs from reduce\n");
      g_fail++;
    }
    // checkpoints: none before a run, then save / load round trips
    const int64_t cb = rift_ile_checkpoint_bytes(h);
    std::vector<char> blob((size_t)cb);
    expect(rift_ile_save_checkpoint(h, blob.data(), cb), RIFT_E_STATE, "save before a run");
    rift_ile_mc mc;
    std::memset(&mc, 0, sizeof mc);
    mc.seed = 11;
    mc.n_per_round = 3000;
    mc.n_rounds = 2;
    mc.adapt_mask = 0x3F;
    mc.floor_eps = 0.1;
    mc.reset_proposal = 1;
    rift_ile_result res[2];
    expect(rift_ile_marginalize(h, &mc, res, nullptr, nullptr), RIFT_OK, "marginalize");
    expect(rift_ile_save_checkpoint(h, blob.data(), cb - 1), RIFT_E_INVALID, "save into a short buffer");
    expect(rift_ile_save_checkpoint(h, blob.data(), cb), RIFT_OK, "save");
    expect(rift_ile_load_checkpoint(h, blob.data(), cb), RIFT_OK, "load");
    expect(rift_ile_load_checkpoint(h, blob.data(), cb - 8), RIFT_E_INVALID, "load truncated");
    expect(rift_ile_load_checkpoint(h, blob.data(), 4), RIFT_E_INVALID, "load 4 bytes");
    std::vector<char> bad_blob = blob;
    bad_blob[0] ^= 0x5a;  // magic
    expect(rift_ile_load_checkpoint(h, bad_blob.data(), cb), RIFT_E_INVALID, "load with a bad magic");
    // corrupt proposal records: flip bytes throughout the proposal area; every
    // load must either be accepted (a flip in unused space) or refused, and a
    // refused one must leave the handle usable
    int refused = 0;
    for (size_t off = 0; off < blob.size(); off += 97) {
      bad_blob = blob;
      bad_blob[off] = (char)0xff;
      bad_blob[off ^ 1] = (char)0x7f;
      const int st = rift_ile_load_checkpoint(h, bad_blob.data(), cb);
      if (st != RIFT_OK) refused++;
      g_checks++;
      if (st != RIFT_OK && st != RIFT_E_INVALID) {
        std::printf("FAIL corrupt checkpoint at %zu: status %d\n", off, st);
        g_fail++;
      }
    }
    expect(rift_ile_load_checkpoint(h, blob.data(), cb), RIFT_OK, "load after refusals");
    mc.first_round = 2;
    mc.reset_proposal = 0;
    expect(rift_ile_marginalize(h, &mc, res, nullptr, nullptr), RIFT_OK, "resume");
    std::printf("  precision %d: refused %d corrupted checkpoints\n", prec, refused);
    (void)hipFree(th);
    (void)hipFree(lt);
    (void)hipFree(lr);
    (void)hipFree(gr);
    rift_ile_destroy(h);
  }
}

int main(int argc, char **argv) {
  const bool device = argc > 1 && std::strcmp(argv[1], "device") == 0;
  host_checks();
  if (device) device_checks();
  if (g_fail) {
    std::printf("failed %d of %d checks\n", g_fail, g_checks);
    return 1;
  }
  std::printf("ok %d\n", g_checks);
  return 0;
}
