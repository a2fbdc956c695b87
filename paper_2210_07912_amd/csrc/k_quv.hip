// Overlaps of Eq. (QUV) (App. D) from frequency-domain inputs: the step that
// prepares Q, U and V for the likelihood.  On a two-sided grid of N samples
// in FFT order (f_i = i df for i < (N+1)/2, (i - N) df otherwise), with the
// weight w_ki = 2 df / S_k(|f_i|) on |f_i| > f_low and 0 elsewhere,
//   Q_k,m(t_n) = sum_i w_ki conj(h_m(f_i)) d_k(f_i) e^{2 pi i f_i t_n}, t_n = n / (N df),
// is an unnormalized inverse DFT of the weighted product (one batched
// complex FFT of length N over every detector and mode), and
//   U_k,mm' = sum_i w_ki conj(h_m(f_i)) h_m'(f_i),
//   V_k,mm' = sum_i w_ki h_m(-f_i) h_m'(f_i)
// are weighted Gram sums over the grid, reduced in a fixed order per entry.
#include <hipfft/hipfft.h>

#include "common.h"
#include "internal.h"

namespace rift {

__device__ __forceinline__ double quv_w(int64_t i, int64_t N, double df, double f_low, double S) {
  const double f = (double)(i < (N + 1) / 2 ? i : i - N) * df;
  return fabs(f) > f_low ? 2.0 * df / S : 0.0;
}

// X[k][m][i] = w_ki conj(h_m(f_i)) d_k(f_i)
__global__ void __launch_bounds__(256) quv_weight_kernel(int M, int64_t N, double df, double f_low,
                                                         const double2 *data, const double *psd,
                                                         const double2 *modes, double2 *X) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int km = blockIdx.y, k = km / M, m = km % M;
  const double w = quv_w(i, N, df, f_low, psd[(size_t)k * N + i]);
  double2 x = {0.0, 0.0};
  if (w != 0.0) {
    const double2 h = modes[(size_t)m * N + i], d = data[(size_t)k * N + i];
    x.x = w * (h.x * d.x + h.y * d.y);
    x.y = w * (h.x * d.y - h.y * d.x);
  }
  X[(size_t)km * N + i] = x;
}

// Q[k][r][m] = X[k][m][(row0 + r) mod N] (after the transform)
__global__ void __launch_bounds__(256) quv_gather_kernel(int M, int64_t N, int64_t row0, int64_t n_rows,
                                                         const double2 *X, double2 *Q) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rows) return;
  const int km = blockIdx.y, k = km / M, m = km % M;
  const int64_t n = ((row0 + r) % N + N) % N;
  Q[((size_t)k * n_rows + r) * M + m] = X[(size_t)km * N + n];
}

// one workgroup per (k, m, m'): U and V entries, each lane a strided part of
// the grid, then a fixed-shape tree over the lanes
__global__ void __launch_bounds__(256) quv_gram_kernel(int M, int64_t N, double df, double f_low, const double *psd,
                                                       const double2 *modes, double2 *U, double2 *V) {
  __shared__ double red[4][256];
  const int e = blockIdx.x, k = e / (M * M), m = (e / M) % M, mp = e % M;
  const double2 *h = modes + (size_t)m * N, *g = modes + (size_t)mp * N;
  double ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += 256) {
    const double w = quv_w(i, N, df, f_low, psd[(size_t)k * N + i]);
    if (w == 0.0) continue;
    const double2 a = h[i], b = g[i], an = h[(N - i) % N];
    ur += w * (a.x * b.x + a.y * b.y);
    ui += w * (a.x * b.y - a.y * b.x);
    vr += w * (an.x * b.x - an.y * b.y);
    vi += w * (an.x * b.y + an.y * b.x);
  }
  red[0][threadIdx.x] = ur;
  red[1][threadIdx.x] = ui;
  red[2][threadIdx.x] = vr;
  red[3][threadIdx.x] = vi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int c = 0; c < 4; c++) red[c][threadIdx.x] += red[c][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    U[e] = double2{red[0][0], red[1][0]};
    V[e] = double2{red[2][0], red[3][0]};
  }
}

hipError_t quv_device(int K, int M, int64_t N, double df, double f_low, const double *data, const double *psd,
                      const double *modes, int64_t row0, int64_t n_rows, double *X, double *Q, double *U, double *V,
                      hipStream_t st) {
  const dim3 gw((unsigned)((N + 255) / 256), (unsigned)(K * M));
  hipLaunchKernelGGL(quv_weight_kernel, gw, dim3(256), 0, st, M, N, df, f_low, (const double2 *)data, psd,
                     (const double2 *)modes, (double2 *)X);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipfftHandle plan;
  int n = (int)N;
  if (hipfftPlanMany(&plan, 1, &n, nullptr, 1, n, nullptr, 1, n, HIPFFT_Z2Z, K * M) != HIPFFT_SUCCESS)
    return hipErrorUnknown;
  hipfftResult r = hipfftSetStream(plan, st);
  if (r == HIPFFT_SUCCESS) r = hipfftExecZ2Z(plan, (hipfftDoubleComplex *)X, (hipfftDoubleComplex *)X, HIPFFT_BACKWARD);
  (void)hipfftDestroy(plan);
  if (r != HIPFFT_SUCCESS) return hipErrorUnknown;
  if (n_rows > 0) {
    const dim3 gg((unsigned)((n_rows + 255) / 256), (unsigned)(K * M));
    hipLaunchKernelGGL(quv_gather_kernel, gg, dim3(256), 0, st, M, N, row0, n_rows, (const double2 *)X,
                       (double2 *)Q);
  }
  hipLaunchKernelGGL(quv_gram_kernel, dim3((unsigned)(K * M * M)), dim3(256), 0, st, M, N, df, f_low, psd,
                     (const double2 *)modes, (double2 *)U, (double2 *)V);
  return hipGetLastError();
}

}  // namespace rift
