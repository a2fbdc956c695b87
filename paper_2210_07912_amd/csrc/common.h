// Internal definitions shared by the HIP kernels and the host side of the
// library.  Device math here is the per-sample prologue of the ILE likelihood
// (App. D Eq. (def:lnL:Decomposed) of arXiv 2210.07912): source direction,
// antenna pattern, arrival delay, spin-weighted harmonics, coefficients
// a_{k,lm} = (D_ref/D) F_k Y_lm, plus the counter-based generator used by the
// on-device sampler.  The prologue runs in FP64 whatever the bulk precision:
// it costs about one percent of an evaluation, and FP32 trigonometry on the
// sky angles would move the arrival times by ~1e-8 s, which near a loud peak
// shifts ln L by more than the accuracy the estimate is held to.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rift_ile.h"

namespace rift {

// Pointers read from device-resident structs are generic to the compiler,
// and generic (flat) loads are counted by both the vector-memory and the LDS
// counters, so every LDS wait would also wait for them.  Kernels cast such
// pointers to the global address space.
#define RIFT_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const RIFT_GLOBAL T *gp(const T *p) {
  return (const RIFT_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ RIFT_GLOBAL T *gpw(T *p) {
  return (RIFT_GLOBAL T *)p;
}
// A pointer the whole wavefront shares, moved to scalar registers, so that
// loads can use it as their scalar base with a 32-bit per-lane offset.
template <typename T>
__device__ __forceinline__ T *uniform_ptr(T *p) {
  const uint64_t v = (uint64_t)(uintptr_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (T *)(uintptr_t)(((uint64_t)hi << 32) | lo);
}
// Tables that no kernel writes while it reads them (per-point U, V) are read
// through the constant address space: wave-uniform loads from it become
// scalar loads even in kernels that store to global memory.
#define RIFT_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const RIFT_CONST T *cp(const T *p) {
  return (const RIFT_CONST T *)p;
}

constexpr int kMaxDet = RIFT_MAX_DET;
constexpr int kMaxModes = RIFT_MAX_MODES;
constexpr int kMaxYTerms = 8;   // Wigner-d sum terms for l <= 8
constexpr int kMaxHDeg = 8;     // degree of the harmonic polynomial for l <= 8
constexpr int kNB = RIFT_NBINS;
constexpr double kC = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrt2Pi = 2.50662827463100050242;  // sqrt(2 pi)

// Per-point constants, resident in device memory.
struct PointDev {
  int K, M, n_t, pad, L;       // L = n_t + 2 pad + 3 stored rows
  int Lpad;                    // rows allocated per detector (>= L, zero-filled tail)
  int nblk;                    // 16-row blocks covered by the MFMA layout
  int n_bins_key;              // delay-bin count for the tile sort: nq^K
  int nq;                      // bins per detector
  int bin_w;                   // rows per delay bin
  double f_s, d_ref, gmst;
  double rc[kMaxDet][3];       // detector vertex / c  (s)
  double frame[3][3];          // network sky frame: rows x', y', z' (z' along detector 0 -> 1), Earth-fixed
  double D[kMaxDet][9];        // response tensor
  int em[kMaxModes];
  int nterm[kMaxModes];
  double ynorm[kMaxModes];     // sqrt((2l+1)/4pi)
  double ycoef[kMaxModes][kMaxYTerms];
  int ypc[kMaxModes][kMaxYTerms];  // power of cos(iota/2)
  int yps[kMaxModes][kMaxYTerms];  // power of sin(iota/2)
  // The same harmonic as a polynomial: ynorm d(iota) = (sin(iota)/2)^hpar[m]
  // sum_j hpoly[m][j] u^j with u = cos^2(iota/2), degree hdeg[m] = l - hpar[m]
  // (every term of the Wigner-d sum has powers of one parity, that of m)
  double hpoly[kMaxModes][kMaxHDeg + 1];
  int hdeg[kMaxModes];
  int hpar[kMaxModes];
  const double *U;             // [K][M][M][2], values rounded to the bulk precision
  const double *V;             // same or nullptr
  const double *Upk;           // [pairs m<=m'][kMaxDet][2]: U_mm', off-diagonal doubled
  const double *Vpk;           // same packing of V, or nullptr
  const void *Q;               // plain layout: [K][Lpad][M][2] in the bulk precision
  const float *Qm;             // MFMA layout (FP32 handles): [K][Lpad][2 Mp], zero-padded
  int Mp;                      // modes padded to even
};

// --------------------------------------------------------------------------
// Geometry (FP64).  Source direction n = (cos d cos h, cos d sin h, sin d)
// with h = alpha - gmst; polarization basis e1 = (-sin h, cos h, 0),
// e2 = (sin d cos h, sin d sin h, -cos d); X = cos psi e1 + sin psi e2,
// Y = -sin psi e1 + cos psi e2; F_+ = X.D.X - Y.D.Y, F_x = 2 X.D.Y.
// --------------------------------------------------------------------------
struct SkyTrig {
  double ch, sh, cd, sd, cp, sp;
};

__device__ __forceinline__ SkyTrig sky_trig(double alpha, double delta, double psi, double gmst) {
  SkyTrig t;
  sincos(alpha - gmst, &t.sh, &t.ch);
  sincos(delta, &t.sd, &t.cd);
  sincos(psi, &t.sp, &t.cp);
  return t;
}

__device__ __forceinline__ double xDy(const double *D, const double x[3], const double y[3]) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; i++) {
    double r = D[3 * i + 0] * y[0] + D[3 * i + 1] * y[1] + D[3 * i + 2] * y[2];
    s += x[i] * r;
  }
  return s;
}

// Antenna pattern and, optionally, its derivatives in alpha and delta.
__device__ __forceinline__ void antenna(const double *D, const SkyTrig &t, double &Fp, double &Fc,
                                        double *dFa = nullptr, double *dFd = nullptr) {
  double e1[3] = {-t.sh, t.ch, 0.0};
  double e2[3] = {t.sd * t.ch, t.sd * t.sh, -t.cd};
  double X[3], Y[3];
#pragma unroll
  for (int i = 0; i < 3; i++) {
    X[i] = t.cp * e1[i] + t.sp * e2[i];
    Y[i] = -t.sp * e1[i] + t.cp * e2[i];
  }
  Fp = xDy(D, X, X) - xDy(D, Y, Y);
  Fc = 2.0 * xDy(D, X, Y);
  if (dFa) {
    double e1a[3] = {-t.ch, -t.sh, 0.0};
    double e2a[3] = {-t.sd * t.sh, t.sd * t.ch, 0.0};
    double e2d[3] = {t.cd * t.ch, t.cd * t.sh, t.sd};
    double Xa[3], Ya[3], Xd[3], Yd[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
      Xa[i] = t.cp * e1a[i] + t.sp * e2a[i];
      Ya[i] = -t.sp * e1a[i] + t.cp * e2a[i];
      Xd[i] = t.sp * e2d[i];
      Yd[i] = t.cp * e2d[i];
    }
    dFa[0] = 2.0 * (xDy(D, X, Xa) - xDy(D, Y, Ya));
    dFa[1] = 2.0 * (xDy(D, Xa, Y) + xDy(D, X, Ya));
    dFd[0] = 2.0 * (xDy(D, X, Xd) - xDy(D, Y, Yd));
    dFd[1] = 2.0 * (xDy(D, Xd, Y) + xDy(D, X, Yd));
  }
}

// Arrival delay at detector k relative to the geocentre, in seconds.
__device__ __forceinline__ double delay(const double rc[3], const SkyTrig &t) {
  return -(rc[0] * t.cd * t.ch + rc[1] * t.cd * t.sh + rc[2] * t.sd);
}

// --------------------------------------------------------------------------
// Spin-weight -2 harmonics from the Wigner-d sum (coefficients and powers
// tabulated per mode on the host); powers by repeated multiplication.
// --------------------------------------------------------------------------
__device__ __forceinline__ double ipow(double x, int n) {
  double r = 1.0;
  for (int i = 0; i < n; i++) r *= x;
  return r;
}

// Y = ynorm * d(iota) * exp(i m phi); dd = d/diota of the real factor.
__device__ __forceinline__ void harmonic(const PointDev &p, int m, double ci, double si, double cphi_m,
                                         double sphi_m, double &yr, double &yi, double *dyr = nullptr,
                                         double *dyi = nullptr) {
  double d = 0.0, dd = 0.0;
  for (int t = 0; t < p.nterm[m]; t++) {
    int A = p.ypc[m][t], B = p.yps[m][t];
    double c = p.ycoef[m][t];
    d += c * ipow(ci, A) * ipow(si, B);
    if (dyr) {
      double g = 0.0;
      if (A > 0) g -= 0.5 * A * ipow(ci, A - 1) * ipow(si, B + 1);
      if (B > 0) g += 0.5 * B * ipow(ci, A + 1) * ipow(si, B - 1);
      dd += c * g;
    }
  }
  d *= p.ynorm[m];
  yr = d * cphi_m;
  yi = d * sphi_m;
  if (dyr) {
    dd *= p.ynorm[m];
    *dyr = dd * cphi_m;
    *dyi = dd * sphi_m;
  }
}

// Catmull-Rom (Keys a = -1/2) weights for taps at rows b-1, b, b+1, b+2.
template <typename T>
__device__ __forceinline__ void cr_weights(T mu, T w[4]) {
  T m2 = mu * mu, m3 = m2 * mu;
  w[0] = T(0.5) * (-m3 + T(2) * m2 - mu);
  w[1] = T(0.5) * (T(3) * m3 - T(5) * m2 + T(2));
  w[2] = T(0.5) * (T(-3) * m3 + T(4) * m2 + mu);
  w[3] = T(0.5) * (m3 - m2);
}
template <typename T>
__device__ __forceinline__ void cr_dweights(T mu, T w[4]) {
  T m2 = mu * mu;
  w[0] = T(0.5) * (T(-3) * m2 + T(4) * mu - T(1));
  w[1] = T(0.5) * (T(9) * m2 - T(10) * mu);
  w[2] = T(0.5) * (T(-9) * m2 + T(8) * mu + T(1));
  w[3] = T(0.5) * (T(3) * m2 - T(2) * mu);
}

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// --------------------------------------------------------------------------
__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; r++) {
    uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Per-sample shift record: integer row offset n_k and fraction mu_k.
struct Shift {
  int n[kMaxDet];
  double mu[kMaxDet];
  bool ok;
};

// s_k = (tau + dt_k) f_s; n_k = floor(s_k); valid when the 4-tap stencil
// stays inside the stored rows for every window sample: -pad <= n_k <= pad.
__device__ __forceinline__ Shift shifts(const PointDev &p, const SkyTrig &t, double tau) {
  Shift s;
  s.ok = isfinite(tau) && isfinite(t.ch) && isfinite(t.sd);
  for (int k = 0; k < p.K; k++) {
    double sk = (tau + delay(p.rc[k], t)) * p.f_s;
    double fl = floor(sk);
    bool okk = isfinite(sk) && fl >= -p.pad && fl <= p.pad;
    s.ok = s.ok && okk;
    s.n[k] = okk ? (int)fl : 0;
    s.mu[k] = okk ? sk - fl : 0.0;
  }
  return s;
}

// Internal launch interfaces (one per kernel family).
struct TileWork;  // forward

}  // namespace rift
