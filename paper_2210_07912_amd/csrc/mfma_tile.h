// Pieces shared by the matrix-core kernels (forward and adjoint): tile
// geometry, the element order of the MFMA operands, the LDS stage stride and
// wavefront helpers.
#pragma once

#include "common.h"
#include "internal.h"

namespace rift {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTS = 16;          // samples per tile (MFMA columns)
constexpr int kWaves = 4;        // wavefronts per workgroup
constexpr double kLog2e = 1.4426950408889634074;  // the MFMA path works in base-2 logarithms
constexpr float kLn2f = 0.693147180559945309f;

__device__ __forceinline__ int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Element of the (re, im)-interleaved operand vector (length 2 Mp = 4 T) that
// MFMA instruction tt of a detector takes in lane group g.  For the first
// 4 (T / 4) instructions, lane group g holds elements 16 j + 4 g .. 16 j + 4 g + 3
// of quad j = tt / 4, one per instruction, so a lane fetches them with one
// 16-byte load; the other T % 4 instructions take element 16 (T / 4) + 4 r + g.
// The B operands use the same assignment, so the sum over elements is complete.
template <int T>
__device__ __forceinline__ int op_elem(int tt, int g) {
  constexpr int J = T / 4;
  return tt < 4 * J ? 16 * (tt >> 2) + 4 * g + (tt & 3) : 16 * J + 4 * (tt - 4 * J) + g;
}

// B operands of one lane (sample s, element group g) for every detector:
// a_k[e] = (x F_k)(Y_m), e = 2m + part, formed in FP32 from the tile's
// harmonic block (yop: element e of the lane's sample at yop[16 e]) and the
// tile record's x F_k.  The quads hold whole modes (elements 4i..4i+3), so
// their partner element is the lane's own; a tail element's partner is read.
template <int T, int K>
__device__ __forceinline__ void b_operands(const RIFT_GLOBAL float *yop, const RIFT_GLOBAL CoefTile *ct, int s,
                                           int g, bool active, float (&Bop)[K][T]) {
  constexpr int J = T / 4;
  float yv[T], yq[T];
#pragma unroll
  for (int tt = 0; tt < T; tt++) yv[tt] = active ? yop[16 * op_elem<T>(tt, g)] : 0.f;
#pragma unroll
  for (int tt = 0; tt < T; tt++) yq[tt] = tt < 4 * J ? yv[tt ^ 1] : (active ? yop[16 * (op_elem<T>(tt, g) ^ 1)] : 0.f);
#pragma unroll
  for (int k = 0; k < K; k++) {
    const float xr = active ? ct->xf[k][0][s] : 0.f, xi = active ? ct->xf[k][1][s] : 0.f;
#pragma unroll
    for (int tt = 0; tt < T; tt++) {
      const bool im = tt < 4 * J ? (tt & 1) != 0 : (g & 1) != 0;
      // Re a = xr y_re - xi y_im; Im a = xr y_im + xi y_re
      Bop[k][tt] = fmaf(xr, yv[tt], (im ? xi : -xi) * yq[tt]);
    }
  }
}

// Harmonic Y_m = (sin(iota)/2)^par P_m(cos^2(iota/2)) exp(i m phi) of one
// mode from the point's polynomial table (Horner in u = cos^2(iota/2), FP64),
// with exp(i m phi) by repeated products of exp(i phi) = (c1, s1) and
// hs = sin(iota/2) cos(iota/2).
template <typename PT>
__device__ __forceinline__ void harmonic_ym(const PT &p, int m, double u, double hs, double c1, double s1, double &yr,
                                            double &yi) {
  const int deg = p.hdeg[m];
  double d = p.hpoly[m][deg];
  for (int j = deg - 1; j >= 0; j--) d = fma(d, u, p.hpoly[m][j]);
  if (p.hpar[m]) d *= hs;
  const int em = p.em[m], am = em < 0 ? -em : em;
  double cr = d, cim = 0.0;
  for (int q = 0; q < am; q++) {
    double nr = cr * c1 - cim * s1;
    cim = cr * s1 + cim * c1;
    cr = nr;
  }
  yr = cr;
  yi = em < 0 ? -cim : cim;
}

// Row stride (floats) of a staged block of Q in LDS: 4T elements, padded to
// an odd number of 16-byte groups so that the 16-byte reads of 8 consecutive
// rows fall in distinct banks.
template <int T>
constexpr int stage_stride() {
  return 4 * T + ((T % 2 == 0) ? 4 : 0);
}

}  // namespace rift
