/* Drives every routine of the FP64 oracle on a small synthetic point, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (host code
 * only).  Prints a checksum; any sanitizer report fails the calling test. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "rift_oracle.h"

static double urand(unsigned *s) {
  *s = *s * 1664525u + 1013904223u;
  return ((*s >> 8) + 0.5) / 16777216.0;
}

int main(void) {
  enum { K = 2, M = 3, NT = 24, PAD = 100 }; /* PAD covers the largest delay (~21 ms at 4096 Hz) */
  const int L = NT + 2 * PAD + 3;
  int ell[M] = {2, 2, 3}, em[M] = {2, -2, 3};
  double pos[K * 3] = {-2.16e6, -3.83e6, 4.6e6, -7.4e4, -5.5e6, 3.2e6};
  double resp[K * 9];
  unsigned seed = 12345u;
  for (int k = 0; k < K; k++)
    for (int i = 0; i < 9; i++) resp[k * 9 + i] = (i % 4 == 0) ? (i == 0 ? 0.5 : (i == 4 ? -0.5 : 0.0)) : 0.0;
  double *Q = malloc(sizeof(double) * K * L * M * 2), *U = malloc(sizeof(double) * K * M * M * 2);
  for (int i = 0; i < K * L * M * 2; i++) Q[i] = urand(&seed) - 0.5;
  /* U = G G^H, Hermitian positive definite */
  for (int k = 0; k < K; k++) {
    double G[M][M][2];
    for (int a = 0; a < M; a++)
      for (int b = 0; b < M; b++) {
        G[a][b][0] = urand(&seed) - 0.5;
        G[a][b][1] = urand(&seed) - 0.5;
      }
    for (int a = 0; a < M; a++)
      for (int b = 0; b < M; b++) {
        double re = a == b ? 0.1 : 0.0, im = 0.0;
        for (int c = 0; c < M; c++) {
          re += G[a][c][0] * G[b][c][0] + G[a][c][1] * G[b][c][1];
          im += G[a][c][1] * G[b][c][0] - G[a][c][0] * G[b][c][1];
        }
        U[((k * M + a) * M + b) * 2] = re;
        U[((k * M + a) * M + b) * 2 + 1] = im;
      }
  }
  or_point p = {K, M, NT, PAD, ell, em, 4096.0, 100.0, 1.2, pos, resp, Q, U, NULL};
  const int n = 64;
  double th[7 * 64], lr, out[64], g[7 * 64], lt[64];
  uint8_t bins[7 * 64], b7[7];
  uint32_t raw[8];
  for (int i = 0; i < n; i++) {
    double t7[7];
    or_draw(7u, 0u, 0u, (uint64_t)i, 10.0, 1000.0, 1.0 / 4096.0, NULL, 100, 0u, t7, &lr, b7, raw);
    for (int d = 0; d < 7; d++) {
      th[d * n + i] = t7[d];
      bins[d * n + i] = b7[d];
    }
  }
  or_lnL_t_batch(&p, n, n, th, out);
  or_grad_batch(&p, n, n, th, lt, g);
  double cdf[7 * 101];
  or_adapt(n, bins, n, out, 100, 0.1, 0x3Fu, cdf);
  double sum = 0.0;
  for (int i = 0; i < n; i++) {
    double t7[7];
    or_draw_frame(7u, 0u, 1u, (uint64_t)i, 10.0, 1000.0, 0.0, cdf, 100, 0x3Fu, pos, 1.2, t7, &lr, b7, raw);
    sum += lr + t7[0];
  }
  or_result r;
  or_reduce(n, out, &r);
  double ax[9], u0, u1;
  or_network_frame(pos, ax);
  or_frame_u(pos, 1.2, 0.3, -0.2, &u0, &u1);
  /* overlaps on a small grid */
  enum { N = 32 };
  double *data = malloc(sizeof(double) * K * N * 2), *psd = malloc(sizeof(double) * K * N);
  double *modes = malloc(sizeof(double) * M * N * 2), *Qo = malloc(sizeof(double) * K * 5 * M * 2);
  double *Uo = malloc(sizeof(double) * K * M * M * 2), *Vo = malloc(sizeof(double) * K * M * M * 2);
  for (int i = 0; i < K * N * 2; i++) data[i] = urand(&seed) - 0.5;
  for (int i = 0; i < K * N; i++) psd[i] = 1.0 + urand(&seed);
  for (int i = 0; i < M * N * 2; i++) modes[i] = urand(&seed) - 0.5;
  or_quv(K, M, N, 0.5, 1.0, data, psd, modes, 28, 5, Qo, Uo, Vo);
  for (int i = 0; i < n; i++) sum += out[i] + g[i];
  sum += r.lnL_marg + ax[0] + u0 + u1 + Qo[3] + Uo[1] + Vo[2];
  printf("checksum %.17g\n", sum);
  free(Q);
  free(U);
  free(data);
  free(psd);
  free(modes);
  free(Qo);
  free(Uo);
  free(Vo);
  return isfinite(sum) ? 0 : 1;
}
