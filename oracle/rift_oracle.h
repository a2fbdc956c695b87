/*
 * rift_oracle.h -- plain, slow, FP64 CPU reference for the ILE marginalized
 * likelihood (arXiv 2210.07912).  TEST INFRASTRUCTURE ONLY: nothing in the
 * product path may include, link or call this.  It shares no source with the
 * HIP library; only the seeded input generator feeds both.
 *
 * Every routine follows one passage of the paper:
 *   - ln L_full, mode decomposed ........ App. D, Eq. (loglikelihood) /
 *                                         Eq. (def:lnL:Decomposed)
 *   - Q, U, V inner products ............ App. D, Eq. (QUV)
 *   - Monte Carlo estimate of L(lambda) . Sec. II.A, Eq. (lnL:MonteCarlo)
 *   - log-space sums (logsumexp) ........ App. D.2 (finite-precision arithmetic)
 *   - n_eff, n_ESS, n_var ............... App. B, Eqs. (neff), (neff_ESS) and the
 *                                         variance-based sample size
 *   - adaptive-Cartesian histograms ..... Sec. III.B (GPU-accelerated Monte
 *                                         Carlo integration), n_bins = 100
 * Readings where the paper is silent or garbled are listed in the repository's
 * design notes and restated at the routine that uses them.
 */
#ifndef RIFT_ORACLE_H
#define RIFT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* extrinsic parameter order used everywhere */
enum { OR_ALPHA = 0, OR_DELTA = 1, OR_PSI = 2, OR_IOTA = 3, OR_PHI = 4, OR_DIST = 5, OR_TAU = 6, OR_NPAR = 7 };

#define OR_C_SI 299792458.0

typedef struct {
  int K;              /* detectors */
  int M;              /* modes */
  int n_t;            /* window length (marginalization grid) */
  int pad;            /* P: rows before/after the window; L = n_t + 2P + 3 */
  const int *ell, *em;/* [M] */
  double f_s;         /* Hz */
  double d_ref;       /* Mpc at which Q, U, V are computed */
  double gmst;        /* rad */
  const double *det_pos;  /* [K][3] m, Earth-fixed */
  const double *det_resp; /* [K][3][3] response tensor */
  const double *Q;    /* [K][L][M][2] */
  const double *U;    /* [K][M][M][2] */
  const double *V;    /* [K][M][M][2] or NULL */
} or_point;

typedef struct {
  double lnL_marg, sigma_lnL, n_eff, n_ess, n_var, max_lnw;
  int64_t n, n_nonfinite;
} or_result;

int or_rows(const or_point *p);
int or_threads(void); /* OpenMP threads the batch routines use */

/* geometry -------------------------------------------------------------- */
void or_direction(double alpha, double delta, double gmst, double n[3]);
void or_antenna(const double D[9], double alpha, double delta, double psi, double gmst,
                double *fplus, double *fcross);
double or_delay(const double r[3], double alpha, double delta, double gmst);
void or_sylm(int l, int m, double iota, double phi, double *re, double *im);

/* likelihood ------------------------------------------------------------ */
void or_coeffs(const or_point *p, const double *theta, double *a /*[K][M][2]*/, double *B);
void or_catmull_rom(double mu, double w[4], double dw[4]);
void or_ell(const or_point *p, const double *theta, double *ell /*[n_t]*/);
double or_lnL_t(const or_point *p, const double *theta);
/* theta: [7][stride]; out[N]; OpenMP over samples */
void or_lnL_t_batch(const or_point *p, int64_t n, int64_t stride, const double *theta, double *out);
/* Distance-marginalized ln L_tD (theta[OR_DIST] not read): the window values
 * ell_j(D) = x A_j - x^2 B_1 (x = D_ref / D) integrated against the prior
 * p(D) = 3 D^2 / (d_max^3 - d_min^3) by composite 8-point Gauss-Legendre over
 * `panels` equal panels in ln D (<= 0: a count from B_1 that resolves the
 * steepest factor), then averaged over the window. */
double or_lnL_tD(const or_point *p, const double *theta, double d_min, double d_max, int panels);
void or_lnL_tD_batch(const or_point *p, int64_t n, int64_t stride, const double *theta, double d_min,
                     double d_max, int panels, double *out);
void or_gauss_legendre(int n, double *x, double *w);
void or_grad(const or_point *p, const double *theta, double *lnL_t, double grad[7]);
void or_grad_batch(const or_point *p, int64_t n, int64_t stride, const double *theta,
                   double *lnL_t, double *grad /*[7][stride]*/);

/* Monte Carlo reduction ------------------------------------------------- */
void or_reduce(int64_t n, const double *lnw, or_result *out);

/* sampler --------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_u01(uint32_t x);
/* Draw sample i of (point, round) from the product proposal.
 * cdf: [7][nb+1] or NULL (=> the prior for every dimension); adapt_mask selects
 * which dimensions use their histogram.  Writes theta[7] and ln p - ln p_s. */
void or_draw(uint64_t seed, uint32_t point, uint32_t round, uint64_t i,
             double d_min, double d_max, double tau_width,
             const double *cdf, int nb, unsigned adapt_mask,
             double theta[7], double *ln_ratio, uint8_t bins[7], uint32_t raw[8]);
/* The same draw with the sky in the network frame (frame_pos = the Earth-fixed
 * positions of two detectors, [2][3] metres; NULL: the equatorial frame):
 * (u_alpha, u_delta) become (phi'/2pi, (cos theta' + 1)/2) about the
 * baseline, mapped back to (alpha, delta) with gmst. */
void or_draw_frame(uint64_t seed, uint32_t point, uint32_t round, uint64_t i,
                   double d_min, double d_max, double tau_width,
                   const double *cdf, int nb, unsigned adapt_mask,
                   const double *frame_pos, double gmst,
                   double theta[7], double *ln_ratio, uint8_t bins[7], uint32_t raw[8]);
/* The same with the polarization and orbital phase drawn in phase-rotated
 * coordinates when phase != 0: the uniforms of dimensions psi and phi are
 * u_s, u_d and psi = 2 pi (u_s - u_d) mod pi, phi = 2 pi (u_s + u_d) mod 2 pi
 * (or_phase_rot); bins and ln_ratio refer to (u_s, u_d). */
void or_draw_coords(uint64_t seed, uint32_t point, uint32_t round, uint64_t i,
                    double d_min, double d_max, double tau_width,
                    const double *cdf, int nb, unsigned adapt_mask,
                    const double *frame_pos, double gmst, int phase,
                    double theta[7], double *ln_ratio, uint8_t bins[7], uint32_t raw[8]);
void or_phase_rot(double us, double ud, double *psi, double *phi);
/* axes[3][3]: rows x', y', z' of the network frame in Earth-fixed coordinates */
void or_network_frame(const double *frame_pos, double axes[9]);
/* (alpha, delta) -> the frame's prior-CDF coordinates (u_phi', u_cos theta') */
void or_frame_u(const double *frame_pos, double gmst, double alpha, double delta, double *u0, double *u1);
void or_prior_cdf(int dim, const double *theta, double d_min, double d_max, double tau_width, double *u);
/* adapt: histogram of w = exp(lnw - max) over each dimension's prior-CDF
 * coordinate bins, floor-mixed, normalized -> cdf[7][nb+1] */
void or_adapt(int64_t n, const uint8_t *bins /*[7][stride]*/, int64_t stride, const double *lnw,
              int nb, double floor_eps, unsigned adapt_mask, double *cdf);

/* Overlaps of Eq. (QUV) from frequency-domain inputs on a two-sided grid of N
 * samples in FFT order (f_i = i df for i < (N+1)/2, (i - N) df otherwise),
 * bins with |f_i| <= f_low left out, w_ki = 2 df / S_k(|f_i|):
 *   Q[k][r][m] = sum_i w_ki e^{2 pi i f_i t_r} conj(h_m(f_i)) d_k(f_i),
 *                t_r = (row0 + r) / (N df), r < n_rows;
 *   U[k][m][m'] = sum_i w_ki conj(h_m(f_i)) h_m'(f_i);
 *   V[k][m][m'] = sum_i w_ki h_m(-f_i) h_m'(f_i).
 * data [K][N][2], psd [K][N], modes [M][N][2]; outputs complex interleaved:
 * Q [K][n_rows][M][2], U and V [K][M][M][2].  Direct sums, FP64. */
void or_quv(int K, int M, int64_t N, double df, double f_low, const double *data, const double *psd,
            const double *modes, int64_t row0, int64_t n_rows, double *Q, double *U, double *V);

#ifdef __cplusplus
}
#endif
#endif
