// Pieces shared by the matrix-core kernels (forward and adjoint): tile
// geometry, the element order of the MFMA operands, the LDS stage stride and
// wavefront helpers.
#pragma once

#include "common.h"

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

// Row stride (floats) of a staged block of Q in LDS: 4T elements, padded to
// an odd number of 16-byte groups so that the 16-byte reads of 8 consecutive
// rows fall in distinct banks.
template <int T>
constexpr int stage_stride() {
  return 4 * T + ((T % 2 == 0) ? 4 : 0);
}

}  // namespace rift
