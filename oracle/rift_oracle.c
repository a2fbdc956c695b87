/*
 * rift_oracle.c -- FP64 CPU oracle for the ILE marginalized likelihood.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It is written to be
 * read against the paper (arXiv 2210.07912), not to be fast: every sample is
 * evaluated literally, in double precision, with no blocking or fusion.
 *
 * Pins (tests/test_oracle_*.py) tie each function to something other than
 * itself: closed-form antenna patterns, closed-form l=2 harmonics and their
 * orthonormality, the noise-free peak rho^2/2, psi -> psi+pi invariance,
 * brute-force quadrature of the Monte Carlo integral, Philox known-answer
 * vectors, and central finite differences of the gradient.
 */
#include "rift_oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

int or_rows(const or_point *p) { return p->n_t + 2 * p->pad + 3; }

#ifdef _OPENMP
#include <omp.h>
int or_threads(void) { return omp_get_max_threads(); }
#else
int or_threads(void) { return 1; }
#endif

/* ------------------------------------------------------------------------
 * Geometry.  The paper says only that L_full accounts for the detector
 * response and that Q_k is evaluated at the detector's arrival time t_k
 * (Sec. II, Eq. (def:lnL:Decomposed)).  Reading used: the standard tensor
 * antenna pattern F = F_+ + i F_x with F(psi) = F(0) exp(-2 i psi), and
 * t_k = t_geo - r_k . n / c.
 * ---------------------------------------------------------------------- */

/* unit vector towards the source in Earth-fixed axes; Earth-fixed longitude
 * of the source is alpha - gmst. */
void or_direction(double alpha, double delta, double gmst, double n[3]) {
  double h = alpha - gmst;
  n[0] = cos(delta) * cos(h);
  n[1] = cos(delta) * sin(h);
  n[2] = sin(delta);
}

/* polarization basis e1, e2 (both orthogonal to n) and their derivatives
 * with respect to alpha and delta */
static void basis(double alpha, double delta, double gmst, double e1[3], double e2[3],
                  double e1a[3], double e2a[3], double e1d[3], double e2d[3]) {
  double h = alpha - gmst, ch = cos(h), sh = sin(h), cd = cos(delta), sd = sin(delta);
  e1[0] = -sh; e1[1] = ch; e1[2] = 0.0;
  e2[0] = sd * ch; e2[1] = sd * sh; e2[2] = -cd;
  e1a[0] = -ch; e1a[1] = -sh; e1a[2] = 0.0;
  e2a[0] = -sd * sh; e2a[1] = sd * ch; e2a[2] = 0.0;
  e1d[0] = 0.0; e1d[1] = 0.0; e1d[2] = 0.0;
  e2d[0] = cd * ch; e2d[1] = cd * sh; e2d[2] = sd;
}

/* x^T D y for symmetric 3x3 D */
static double quad3(const double D[9], const double x[3], const double y[3]) {
  double s = 0.0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) s += x[i] * D[3 * i + j] * y[j];
  return s;
}

/* F_+ = D : (X X^T - Y Y^T), F_x = D : (X Y^T + Y X^T),
 * X = cos(psi) e1 + sin(psi) e2, Y = -sin(psi) e1 + cos(psi) e2.
 * Optional derivatives with respect to alpha, delta, psi. */
static void antenna_full(const double D[9], double alpha, double delta, double psi, double gmst,
                         double F[2], double Fa[2], double Fd[2], double Fp[2]) {
  double e1[3], e2[3], e1a[3], e2a[3], e1d[3], e2d[3];
  basis(alpha, delta, gmst, e1, e2, e1a, e2a, e1d, e2d);
  double c = cos(psi), s = sin(psi);
  double X[3], Y[3], Xa[3], Ya[3], Xd[3], Yd[3];
  for (int i = 0; i < 3; i++) {
    X[i] = c * e1[i] + s * e2[i];
    Y[i] = -s * e1[i] + c * e2[i];
    Xa[i] = c * e1a[i] + s * e2a[i];
    Ya[i] = -s * e1a[i] + c * e2a[i];
    Xd[i] = c * e1d[i] + s * e2d[i];
    Yd[i] = -s * e1d[i] + c * e2d[i];
  }
  F[0] = quad3(D, X, X) - quad3(D, Y, Y);
  F[1] = 2.0 * quad3(D, X, Y);
  if (Fa) {
    Fa[0] = 2.0 * (quad3(D, X, Xa) - quad3(D, Y, Ya));
    Fa[1] = 2.0 * (quad3(D, Xa, Y) + quad3(D, X, Ya));
  }
  if (Fd) {
    Fd[0] = 2.0 * (quad3(D, X, Xd) - quad3(D, Y, Yd));
    Fd[1] = 2.0 * (quad3(D, Xd, Y) + quad3(D, X, Yd));
  }
  if (Fp) { /* dF/dpsi = -2i F */
    Fp[0] = 2.0 * F[1];
    Fp[1] = -2.0 * F[0];
  }
}

void or_antenna(const double D[9], double alpha, double delta, double psi, double gmst,
                double *fplus, double *fcross) {
  double F[2];
  antenna_full(D, alpha, delta, psi, gmst, F, NULL, NULL, NULL);
  *fplus = F[0];
  *fcross = F[1];
}

double or_delay(const double r[3], double alpha, double delta, double gmst) {
  double n[3];
  or_direction(alpha, delta, gmst, n);
  return -(r[0] * n[0] + r[1] * n[1] + r[2] * n[2]) / OR_C_SI;
}

/* ------------------------------------------------------------------------
 * Spin-weighted spherical harmonics of spin weight -2 (the angular basis of
 * the mode decomposition, Sec. II.A and App. D).  Written from the Wigner-d
 * sum of Goldberg et al., J. Math. Phys. 8, 2155 (1967):
 *   Y^{-2}_{lm}(iota, phi) = sqrt((2l+1)/4pi) d^l_{m,2}(iota) e^{i m phi},
 *   d^l_{m,2} = sum_k (-1)^k sqrt((l+m)!(l-m)!(l+2)!(l-2)!)
 *               / ((l+m-k)!(l-2-k)! k! (k+2-m)!)
 *               cos(iota/2)^(2l+m-2-2k) sin(iota/2)^(2k+2-m).
 * ---------------------------------------------------------------------- */
static double fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; i++) f *= i;
  return f;
}

/* d^l_{m,2}(iota) and its derivative */
static void wigner_d(int l, int m, double iota, double *d, double *dd) {
  double c = cos(0.5 * iota), s = sin(0.5 * iota);
  int kmin = m - 2 > 0 ? m - 2 : 0;
  int kmax = (l + m) < (l - 2) ? (l + m) : (l - 2);
  double norm = sqrt(fact(l + m) * fact(l - m) * fact(l + 2) * fact(l - 2));
  double sum = 0.0, dsum = 0.0;
  for (int k = kmin; k <= kmax; k++) {
    double coef = ((k & 1) ? -1.0 : 1.0) * norm /
                  (fact(l + m - k) * fact(l - 2 - k) * fact(k) * fact(k + 2 - m));
    int A = 2 * l + m - 2 - 2 * k; /* power of cos */
    int Bp = 2 * k + 2 - m;        /* power of sin */
    sum += coef * pow(c, A) * pow(s, Bp);
    /* d/diota [c^A s^B] = -A/2 c^(A-1) s^(B+1) + B/2 c^(A+1) s^(B-1) */
    double t = 0.0;
    if (A > 0) t -= 0.5 * A * pow(c, A - 1) * pow(s, Bp + 1);
    if (Bp > 0) t += 0.5 * Bp * pow(c, A + 1) * pow(s, Bp - 1);
    dsum += coef * t;
  }
  *d = sum;
  *dd = dsum;
}

static void sylm_full(int l, int m, double iota, double phi, double Y[2], double Yi[2]) {
  double d, dd;
  wigner_d(l, m, iota, &d, &dd);
  double nrm = sqrt((2.0 * l + 1.0) / (4.0 * M_PI));
  double cp = cos(m * phi), sp = sin(m * phi);
  Y[0] = nrm * d * cp;
  Y[1] = nrm * d * sp;
  if (Yi) {
    Yi[0] = nrm * dd * cp;
    Yi[1] = nrm * dd * sp;
  }
}

void or_sylm(int l, int m, double iota, double phi, double *re, double *im) {
  double Y[2];
  sylm_full(l, m, iota, phi, Y, NULL);
  *re = Y[0];
  *im = Y[1];
}

/* ------------------------------------------------------------------------
 * Coefficients of the decomposed likelihood, App. D Eq. (def:lnL:Decomposed):
 *   a_{k,lm} = (D_ref / D) F_k Y^{-2}_{lm}(iota, phi)
 *   B = 1/4 sum_k [ a_k^dagger U_k a_k + Re(a_k^T V_k a_k) ]
 * (the (D_ref/D)^2 / 4 prefactor of the printed U/V term is folded into a).
 * Reading: the printed data term omits Re and D_ref/D; ln L is the real
 * log-likelihood ratio Re[(D_ref/D) sum (F Y)^* Q] - B.
 * ---------------------------------------------------------------------- */
static void cmul(const double x[2], const double y[2], double z[2]) {
  double re = x[0] * y[0] - x[1] * y[1];
  double im = x[0] * y[1] + x[1] * y[0];
  z[0] = re;
  z[1] = im;
}

static double quadratic_term(const or_point *p, int k, const double *a /* [M][2] */) {
  int M = p->M;
  const double *U = p->U + (size_t)k * M * M * 2;
  double uterm = 0.0, vterm = 0.0;
  for (int m = 0; m < M; m++)
    for (int mp = 0; mp < M; mp++) {
      const double *u = U + ((size_t)m * M + mp) * 2;
      /* conj(a_m) U_{m m'} a_{m'} */
      double ca[2] = {a[2 * m], -a[2 * m + 1]}, t[2], z[2];
      cmul(ca, u, t);
      cmul(t, a + 2 * mp, z);
      uterm += z[0];
      if (p->V) {
        const double *v = p->V + (size_t)k * M * M * 2 + ((size_t)m * M + mp) * 2;
        cmul(a + 2 * m, v, t);
        cmul(t, a + 2 * mp, z);
        vterm += z[0];
      }
    }
  return 0.25 * (uterm + vterm);
}

void or_coeffs(const or_point *p, const double *theta, double *a, double *B) {
  double x = p->d_ref / theta[OR_DIST];
  double Bsum = 0.0;
  for (int k = 0; k < p->K; k++) {
    double F[2];
    antenna_full(p->det_resp + 9 * k, theta[OR_ALPHA], theta[OR_DELTA], theta[OR_PSI], p->gmst, F,
                 NULL, NULL, NULL);
    for (int m = 0; m < p->M; m++) {
      double Y[2], z[2];
      sylm_full(p->ell[m], p->em[m], theta[OR_IOTA], theta[OR_PHI], Y, NULL);
      cmul(F, Y, z);
      a[(k * p->M + m) * 2 + 0] = x * z[0];
      a[(k * p->M + m) * 2 + 1] = x * z[1];
    }
    Bsum += quadratic_term(p, k, a + (size_t)k * p->M * 2);
  }
  *B = Bsum;
}

/* ------------------------------------------------------------------------
 * Interpolation of Q at a fractional row.  The paper evaluates Q_k at the
 * detector arrival time t_k without saying how off-grid times are handled.
 * Reading: Catmull-Rom (Keys cubic, a = -1/2) over rows b-1..b+2.
 * ---------------------------------------------------------------------- */
void or_catmull_rom(double mu, double w[4], double dw[4]) {
  double m2 = mu * mu, m3 = m2 * mu;
  w[0] = 0.5 * (-m3 + 2.0 * m2 - mu);
  w[1] = 0.5 * (3.0 * m3 - 5.0 * m2 + 2.0);
  w[2] = 0.5 * (-3.0 * m3 + 4.0 * m2 + mu);
  w[3] = 0.5 * (m3 - m2);
  if (dw) {
    dw[0] = 0.5 * (-3.0 * m2 + 4.0 * mu - 1.0);
    dw[1] = 0.5 * (9.0 * m2 - 10.0 * mu);
    dw[2] = 0.5 * (-9.0 * m2 + 8.0 * mu + 1.0);
    dw[3] = 0.5 * (3.0 * m2 - 2.0 * mu);
  }
}

/* fractional row offset of detector k: s = (tau + dt_k) f_s */
static double shift_of(const or_point *p, int k, const double *theta) {
  double dt = or_delay(p->det_pos + 3 * k, theta[OR_ALPHA], theta[OR_DELTA], p->gmst);
  return (theta[OR_TAU] + dt) * p->f_s;
}

/* ln L_full on the window grid t_j = t_q0 + (P + 1 + j)/f_s + tau, j = 0..n_t-1:
 *   ell_j = sum_k Re( sum_m conj(a_km) Qtilde_km(j) ) - B,
 *   Qtilde_k(j) = sum_{q=-1..2} w_q(mu_k) Q_k[P + 1 + j + n_k + q]. */
void or_ell(const or_point *p, const double *theta, double *ell) {
  int K = p->K, M = p->M, L = or_rows(p);
  double *a = (double *)malloc(sizeof(double) * 2 * K * M);
  double B;
  or_coeffs(p, theta, a, &B);
  for (int j = 0; j < p->n_t; j++) ell[j] = -B;
  for (int k = 0; k < K; k++) {
    double s = shift_of(p, k, theta);
    double nf = floor(s);
    int n = (int)nf;
    double w[4];
    or_catmull_rom(s - nf, w, NULL);
    const double *Qk = p->Q + (size_t)k * L * M * 2;
    for (int j = 0; j < p->n_t; j++) {
      int b = p->pad + 1 + j + n;
      double acc = 0.0;
      for (int m = 0; m < M; m++) {
        double qt[2] = {0.0, 0.0};
        for (int q = -1; q <= 2; q++) {
          int r = b + q;
          if (r < 0 || r >= L) { acc = NAN; break; } /* outside the stored rows */
          qt[0] += w[q + 1] * Qk[((size_t)r * M + m) * 2 + 0];
          qt[1] += w[q + 1] * Qk[((size_t)r * M + m) * 2 + 1];
        }
        const double *am = a + (k * M + m) * 2;
        acc += am[0] * qt[0] + am[1] * qt[1]; /* Re(conj(a) qt) */
      }
      ell[j] += acc;
    }
  }
  free(a);
}

/* ------------------------------------------------------------------------
 * Time marginalization: uniform prior over the window grid, rectangle rule,
 * evaluated as a max-shifted logsumexp (App. D.2):
 *   ln L_t = max_j ell_j + ln sum_j exp(ell_j - max) - ln n_t.
 * ---------------------------------------------------------------------- */
static double lse_mean(const double *x, int n) {
  double mx = -INFINITY;
  for (int j = 0; j < n; j++)
    if (x[j] > mx) mx = x[j];
  if (!isfinite(mx)) return mx;
  double s = 0.0;
  for (int j = 0; j < n; j++) s += exp(x[j] - mx);
  return mx + log(s) - log((double)n);
}

double or_lnL_t(const or_point *p, const double *theta) {
  double *ell = (double *)malloc(sizeof(double) * p->n_t);
  or_ell(p, theta, ell);
  double r = lse_mean(ell, p->n_t);
  free(ell);
  return r;
}

void or_lnL_t_batch(const or_point *p, int64_t n, int64_t stride, const double *theta, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    double th[OR_NPAR];
    for (int d = 0; d < OR_NPAR; d++) th[d] = theta[d * stride + i];
    out[i] = or_lnL_t(p, th);
  }
}

/* ------------------------------------------------------------------------
 * Distance marginalization (Sec. III.B, distance marginalization, and the
 * production configuration of Sec. III that pairs it with the adaptive
 * integrator).  The paper cites the technique without its formulas; the
 * definition written out here is this oracle's reading:
 *   L_tD(theta) = int_{d_min}^{d_max} p(D) (1/n_t) sum_j exp(ell_j(D)) dD,
 *   p(D) = 3 D^2 / (d_max^3 - d_min^3)   (the sampler's distance prior),
 * ell_j(D) the window values of Eq. (def:lnL:Decomposed) at distance D and
 * the other six parameters of theta (theta[OR_DIST] is not read).  a_km is
 * proportional to 1/D and B to 1/D^2, so with x = D_ref / D
 *   ell_j(D) = x A_j - x^2 B_1,  A_j = ell_j(D_ref) + B_1,  B_1 = B(D_ref).
 * The integral is a composite Gauss-Legendre rule of 8 nodes per panel over
 * `panels` equal panels in ln D; the double sum over (node, j) is taken in
 * log space with its largest term factored out.  panels <= 0 picks
 * max(2000, 8 B_1 x_min^2 ln(d_max / d_min)) panels, x_min = D_ref / d_max:
 * at least four panels per e-fold of the steepest factor exp(-x^2 B_1) in
 * ln D near d_max, where a loud point's prior samples put their mass.  A
 * node whose bound x A_max - x^2 B_1 + ln(weight) lies more than 60 below
 * the largest is skipped (its n_t terms together are below e^-53 of it).
 * ---------------------------------------------------------------------- */

/* n-point Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on
 * the three-term recurrence of the Legendre polynomials */
static void gauss_legendre(int n, double *x, double *w) {
  for (int i = 0; i < (n + 1) / 2; i++) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; it++) {
      double p0 = 1.0, p1 = 0.0;
      for (int k = 1; k <= n; k++) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
      }
      dp = n * (z * p0 - p1) / (z * z - 1.0);
      double dz = p0 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

void or_gauss_legendre(int n, double *x, double *w) { gauss_legendre(n, x, w); }

double or_lnL_tD(const or_point *p, const double *theta, double d_min, double d_max, int panels) {
  const int NT = p->n_t, NG = 8;
  double th[OR_NPAR];
  for (int d = 0; d < OR_NPAR; d++) th[d] = theta[d];
  th[OR_DIST] = p->d_ref;
  double *A = (double *)malloc(sizeof(double) * NT);
  double *a = (double *)malloc(sizeof(double) * 2 * p->K * p->M);
  double B1;
  or_ell(p, th, A);
  or_coeffs(p, th, a, &B1);
  free(a);
  double amax = -INFINITY;
  for (int j = 0; j < NT; j++) {
    if (isnan(A[j])) { free(A); return NAN; }
    A[j] += B1;
    if (A[j] > amax) amax = A[j];
  }
  if (panels <= 0) {
    const double xm = p->d_ref / d_max, need = 8.0 * B1 * xm * xm * log(d_max / d_min);
    panels = need > 2000.0 ? (int)ceil(need) : 2000;
  }
  double gx[8], gw[8];
  gauss_legendre(NG, gx, gw);
  const double s0 = log(d_min), h = (log(d_max) - s0) / panels;
  const double norm = 3.0 / (d_max * d_max * d_max - d_min * d_min * d_min);
  /* node i: x_i and ln of its weight h/2 w p(D) D (dD = D ds) */
  const int NN = panels * NG;
  double *xs = (double *)malloc(sizeof(double) * NN), *lw = (double *)malloc(sizeof(double) * NN);
  double *top = (double *)malloc(sizeof(double) * NN);
  double mx = -INFINITY;
  for (int q = 0; q < panels; q++)
    for (int g = 0; g < NG; g++) {
      const int i = q * NG + g;
      const double D = exp(s0 + h * (q + 0.5 + 0.5 * gx[g]));
      xs[i] = p->d_ref / D;
      lw[i] = log(0.5 * h * gw[g] * norm * D * D * D);
      top[i] = xs[i] * amax - xs[i] * xs[i] * B1 + lw[i];
      if (top[i] > mx) mx = top[i];
    }
  double sum = 0.0;
  for (int i = 0; i < NN; i++) {
    if (top[i] < mx - 60.0) continue;
    const double c = lw[i] - xs[i] * xs[i] * B1 - mx;
    for (int j = 0; j < NT; j++) sum += exp(xs[i] * A[j] + c);
  }
  free(xs);
  free(lw);
  free(top);
  free(A);
  return mx + log(sum) - log((double)NT);
}

void or_lnL_tD_batch(const or_point *p, int64_t n, int64_t stride, const double *theta, double d_min,
                     double d_max, int panels, double *out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; i++) {
    double th[OR_NPAR];
    for (int d = 0; d < OR_NPAR; d++) th[d] = theta[d * stride + i];
    out[i] = or_lnL_tD(p, th, d_min, d_max, panels);
  }
}

/* ------------------------------------------------------------------------
 * Gradient of ln L_t with respect to the seven extrinsic parameters.
 *   d lnL_t = sum_j p_j d ell_j,  p_j = softmax_j(ell_j)
 *   d ell_j = sum_k Re( sum_m conj(d a_km) Qtilde_km(j) )
 *           + sum_k Re( sum_m conj(a_km) Qtilde'_km(j) ) ds_k
 *           - dB
 * with Qtilde' built from the Catmull-Rom derivative weights (per row) and
 * ds_k = f_s (d tau + d dt_k).
 * ---------------------------------------------------------------------- */
void or_grad(const or_point *p, const double *theta, double *lnL_t, double grad[7]) {
  int K = p->K, M = p->M, L = or_rows(p), NT = p->n_t;
  double alpha = theta[OR_ALPHA], delta = theta[OR_DELTA], psi = theta[OR_PSI];
  double iota = theta[OR_IOTA], phi = theta[OR_PHI], dist = theta[OR_DIST];
  double x = p->d_ref / dist;
  double *ell = (double *)malloc(sizeof(double) * NT);
  double *a = (double *)malloc(sizeof(double) * 2 * K * M);
  double *da = (double *)calloc((size_t)7 * 2 * K * M, sizeof(double)); /* [7][K][M][2] */
  double *Y = (double *)malloc(sizeof(double) * 2 * M);
  double *Yi = (double *)malloc(sizeof(double) * 2 * M);
  double *Fs = (double *)malloc(sizeof(double) * 8 * K); /* F, Fa, Fd, Fp per detector */
  for (int m = 0; m < M; m++) sylm_full(p->ell[m], p->em[m], iota, phi, Y + 2 * m, Yi + 2 * m);
  double B = 0.0;
  for (int k = 0; k < K; k++) {
    double *F = Fs + 8 * k;
    antenna_full(p->det_resp + 9 * k, alpha, delta, psi, p->gmst, F, F + 2, F + 4, F + 6);
    for (int m = 0; m < M; m++) {
      double z[2];
      size_t o = (size_t)(k * M + m) * 2;
      cmul(F, Y + 2 * m, z);
      a[o] = x * z[0];
      a[o + 1] = x * z[1];
      double t[2];
      cmul(F + 2, Y + 2 * m, t); /* alpha */
      da[0 * 2 * K * M + o] = x * t[0]; da[0 * 2 * K * M + o + 1] = x * t[1];
      cmul(F + 4, Y + 2 * m, t); /* delta */
      da[1 * 2 * K * M + o] = x * t[0]; da[1 * 2 * K * M + o + 1] = x * t[1];
      cmul(F + 6, Y + 2 * m, t); /* psi */
      da[2 * 2 * K * M + o] = x * t[0]; da[2 * 2 * K * M + o + 1] = x * t[1];
      cmul(F, Yi + 2 * m, t); /* iota */
      da[3 * 2 * K * M + o] = x * t[0]; da[3 * 2 * K * M + o + 1] = x * t[1];
      /* phi: dY/dphi = i m Y */
      double iy[2] = {-p->em[m] * Y[2 * m + 1], p->em[m] * Y[2 * m]};
      cmul(F, iy, t);
      da[4 * 2 * K * M + o] = x * t[0]; da[4 * 2 * K * M + o + 1] = x * t[1];
      /* distance: da/dD = -a/D */
      da[5 * 2 * K * M + o] = -a[o] / dist; da[5 * 2 * K * M + o + 1] = -a[o + 1] / dist;
    }
    B += quadratic_term(p, k, a + (size_t)k * M * 2);
  }
  /* ell_j and per-detector interpolated windows */
  for (int j = 0; j < NT; j++) ell[j] = -B;
  int *nk = (int *)malloc(sizeof(int) * K);
  double *wk = (double *)malloc(sizeof(double) * 8 * K);
  for (int k = 0; k < K; k++) {
    double s = shift_of(p, k, theta), nf = floor(s);
    nk[k] = (int)nf;
    or_catmull_rom(s - nf, wk + 8 * k, wk + 8 * k + 4);
    const double *Qk = p->Q + (size_t)k * L * M * 2;
    for (int j = 0; j < NT; j++) {
      int b = p->pad + 1 + j + nk[k];
      double acc = 0.0;
      for (int m = 0; m < M; m++) {
        double qt[2] = {0, 0};
        for (int q = -1; q <= 2; q++) {
          qt[0] += wk[8 * k + q + 1] * Qk[((size_t)(b + q) * M + m) * 2];
          qt[1] += wk[8 * k + q + 1] * Qk[((size_t)(b + q) * M + m) * 2 + 1];
        }
        acc += a[(k * M + m) * 2] * qt[0] + a[(k * M + m) * 2 + 1] * qt[1];
      }
      ell[j] += acc;
    }
  }
  double lt = lse_mean(ell, NT);
  *lnL_t = lt;
  double lnN = log((double)NT);
  for (int d = 0; d < 7; d++) grad[d] = 0.0;
  /* direction derivatives for the delays */
  double h = alpha - p->gmst;
  double dn_a[3] = {-cos(delta) * sin(h), cos(delta) * cos(h), 0.0};
  double dn_d[3] = {-sin(delta) * cos(h), -sin(delta) * sin(h), cos(delta)};
  for (int k = 0; k < K; k++) {
    const double *Qk = p->Q + (size_t)k * L * M * 2;
    /* G_k = sum_j p_j Qtilde_k(j), H_k = sum_j p_j Re(a^dag Qtilde'_k(j)) */
    double *G = (double *)calloc((size_t)2 * M, sizeof(double));
    double H = 0.0;
    for (int j = 0; j < NT; j++) {
      double pj = exp(ell[j] - lt - lnN);
      int b = p->pad + 1 + j + nk[k];
      for (int m = 0; m < M; m++) {
        double qt[2] = {0, 0}, qd[2] = {0, 0};
        for (int q = -1; q <= 2; q++) {
          double qr = Qk[((size_t)(b + q) * M + m) * 2], qi = Qk[((size_t)(b + q) * M + m) * 2 + 1];
          qt[0] += wk[8 * k + q + 1] * qr;
          qt[1] += wk[8 * k + q + 1] * qi;
          qd[0] += wk[8 * k + 4 + q + 1] * qr;
          qd[1] += wk[8 * k + 4 + q + 1] * qi;
        }
        G[2 * m] += pj * qt[0];
        G[2 * m + 1] += pj * qt[1];
        H += pj * (a[(k * M + m) * 2] * qd[0] + a[(k * M + m) * 2 + 1] * qd[1]);
      }
    }
    const double *rk = p->det_pos + 3 * k;
    double ddt_a = -(rk[0] * dn_a[0] + rk[1] * dn_a[1] + rk[2] * dn_a[2]) / OR_C_SI;
    double ddt_d = -(rk[0] * dn_d[0] + rk[1] * dn_d[1] + rk[2] * dn_d[2]) / OR_C_SI;
    grad[OR_ALPHA] += H * p->f_s * ddt_a;
    grad[OR_DELTA] += H * p->f_s * ddt_d;
    grad[OR_TAU] += H * p->f_s;
    /* data term through a, minus the quadratic term:
     * dB = 1/2 Re(da^dag U a) + 1/2 Re(da^T V a) */
    const double *U = p->U + (size_t)k * M * M * 2;
    const double *V = p->V ? p->V + (size_t)k * M * M * 2 : NULL;
    const double *ak = a + (size_t)k * M * 2;
    for (int d = 0; d < 6; d++) {
      const double *dak = da + (size_t)d * 2 * K * M + (size_t)k * M * 2;
      double g = 0.0;
      for (int m = 0; m < M; m++) g += dak[2 * m] * G[2 * m] + dak[2 * m + 1] * G[2 * m + 1];
      double dBk = 0.0;
      for (int m = 0; m < M; m++)
        for (int mp = 0; mp < M; mp++) {
          double cda[2] = {dak[2 * m], -dak[2 * m + 1]}, t[2], z[2];
          cmul(cda, U + ((size_t)m * M + mp) * 2, t);
          cmul(t, ak + 2 * mp, z);
          dBk += 0.5 * z[0];
          if (V) {
            cmul(dak + 2 * m, V + ((size_t)m * M + mp) * 2, t);
            cmul(t, ak + 2 * mp, z);
            dBk += 0.5 * z[0];
          }
        }
      grad[d] += g - dBk;
    }
    free(G);
  }
  free(nk); free(wk); free(ell); free(a); free(da); free(Y); free(Yi); free(Fs);
}

void or_grad_batch(const or_point *p, int64_t n, int64_t stride, const double *theta,
                   double *lnL_t, double *grad) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++) {
    double th[OR_NPAR], g[7], l;
    for (int d = 0; d < OR_NPAR; d++) th[d] = theta[d * stride + i];
    or_grad(p, th, &l, g);
    lnL_t[i] = l;
    for (int d = 0; d < 7; d++) grad[d * stride + i] = g[d];
  }
}

/* ------------------------------------------------------------------------
 * Monte Carlo estimate and sample-size measures.
 *   ln L_marg = ln[(1/N) sum_i w_i], Sec. II.A Eq. (lnL:MonteCarlo),
 *   n_eff = sum w / max w  (App. B Eq. (neff)),
 *   n_ESS = (sum w)^2 / sum w^2  (App. B Eq. (neff_ESS)),
 *   n_var = N wbar^2 / s^2 with the unbiased sample variance s^2 (App. B, the
 *           variance-based size; the printed formula is garbled, the words
 *           following it fix this form), sigma_lnL = 1 / sqrt(n_var).
 * Non-finite ln w are counted and excluded.  All sums are taken in log space
 * shifted by max ln w (App. D.2).
 * ---------------------------------------------------------------------- */
void or_reduce(int64_t n, const double *lnw, or_result *out) {
  double mx = -INFINITY;
  int64_t nn = 0, bad = 0;
  for (int64_t i = 0; i < n; i++) {
    if (isnan(lnw[i]) || lnw[i] == INFINITY) { bad++; continue; }
    if (lnw[i] > mx) mx = lnw[i];
  }
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = 0; i < n; i++) {
    if (isnan(lnw[i]) || lnw[i] == INFINITY) continue;
    nn++;
    if (mx == -INFINITY) continue;
    double w = exp(lnw[i] - mx);
    s1 += w;
    s2 += w * w;
  }
  out->n = nn;
  out->n_nonfinite = bad;
  out->max_lnw = mx;
  if (nn == 0 || mx == -INFINITY || s1 <= 0.0) {
    out->lnL_marg = -INFINITY;
    out->n_eff = 0.0;
    out->n_ess = 0.0;
    out->n_var = 0.0;
    out->sigma_lnL = INFINITY;
    return;
  }
  double N = (double)nn;
  out->lnL_marg = mx + log(s1) - log(N);
  out->n_eff = s1; /* sum w / max w with the max weight scaled to 1 */
  out->n_ess = s1 * s1 / s2;
  double wbar = s1 / N;
  double var = nn > 1 ? (s2 - N * wbar * wbar) / (N - 1.0) : 0.0;
  if (var <= 0.0) {
    out->n_var = INFINITY;
    out->sigma_lnL = 0.0;
  } else {
    out->n_var = N * wbar * wbar / var;
    out->sigma_lnL = 1.0 / sqrt(out->n_var);
  }
}

/* ------------------------------------------------------------------------
 * Counter-based random numbers: Philox4x32-10 as defined by Salmon, Moraes,
 * Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11):
 * ten rounds of two 32x32->64 multiplies with multipliers 0xD2511F53 and
 * 0xCD9E8D57, key schedule bumped by the Weyl constants 0x9E3779B9 and
 * 0xBB67AE85 between rounds.
 * ---------------------------------------------------------------------- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    if (r < 9) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* top 24 bits, centred in their cell: (0, 1), exactly representable */
double or_u01(uint32_t x) { return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0); }

/* prior inverse CDFs, u -> theta (priors of the workloads: alpha uniform on
 * [0, 2pi), sin(delta) and cos(iota) uniform on [-1, 1], psi uniform on
 * [0, pi), phi uniform on [0, 2pi), p(D) ~ D^2 on [d_min, d_max], tau uniform
 * on [-w/2, w/2)). */
static double prior_inv(int d, double u, double d_min, double d_max, double tau_width) {
  switch (d) {
  case OR_ALPHA: return 2.0 * M_PI * u;
  case OR_DELTA: return asin(2.0 * u - 1.0);
  case OR_PSI: return M_PI * u;
  case OR_IOTA: return acos(2.0 * u - 1.0);
  case OR_PHI: return 2.0 * M_PI * u;
  case OR_DIST: {
    double a3 = d_min * d_min * d_min, b3 = d_max * d_max * d_max;
    return cbrt(a3 + u * (b3 - a3));
  }
  default: return (u - 0.5) * tau_width;
  }
}

void or_prior_cdf(int d, const double *theta, double d_min, double d_max, double tau_width, double *u) {
  double t = theta[d];
  switch (d) {
  case OR_ALPHA: *u = t / (2.0 * M_PI); break;
  case OR_DELTA: *u = 0.5 * (sin(t) + 1.0); break;
  case OR_PSI: *u = t / M_PI; break;
  case OR_IOTA: *u = 0.5 * (1.0 + cos(t)); break;
  case OR_PHI: *u = t / (2.0 * M_PI); break;
  case OR_DIST: {
    double a3 = d_min * d_min * d_min, b3 = d_max * d_max * d_max;
    *u = (t * t * t - a3) / (b3 - a3);
    break;
  }
  default: *u = tau_width > 0 ? t / tau_width + 0.5 : 0.5;
  }
}

/* Sample i of (point, round).  Counter (i_lo, i_hi, 2 round + half, point),
 * key (seed_lo, seed_hi); dimension d uses output word d of the two blocks.
 * An adapted dimension draws its prior-CDF coordinate from the piecewise-
 * constant histogram density by inverse CDF (Sec. III.B: separable sampling
 * prior, 100-bin histograms in adaptive dimensions), so that
 * ln p - ln p_s = -sum_d ln h_d(u_d).  bins[d] receives the histogram bin of
 * the sample's prior-CDF coordinate in every dimension. */
/* Rotated detector-network-frame sky coordinates (Sec. II.A, added
 * coordinate systems; Sec. II.C: usable with the GPU integrator): the north
 * pole of the sampled sky is the unit vector from detector 0 to detector 1,
 * so the arrival-time difference of that pair depends on the polar angle
 * alone.  Axes: z' along the baseline, x' = normalize(e_z x z') (e_x x z' if
 * the baseline lies along e_z), y' = z' x x'.  The sky prior is isotropic,
 * so phi' uniform on [0, 2pi) and cos theta' uniform on [-1, 1] is the same
 * prior; only the coordinates the histograms adapt in change. */
static void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

static void unit3(double a[3]) {
  double n = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  for (int i = 0; i < 3; i++) a[i] /= n;
}

void or_network_frame(const double *pos, double axes[9]) {
  double z[3] = {pos[3] - pos[0], pos[4] - pos[1], pos[5] - pos[2]}, x[3], y[3];
  unit3(z);
  const double ez[3] = {0.0, 0.0, 1.0}, ex[3] = {1.0, 0.0, 0.0};
  cross3(ez, z, x);
  if (sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) < 1e-6) cross3(ex, z, x);
  unit3(x);
  cross3(z, x, y);
  for (int i = 0; i < 3; i++) {
    axes[i] = x[i];
    axes[3 + i] = y[i];
    axes[6 + i] = z[i];
  }
}

void or_frame_u(const double *pos, double gmst, double alpha, double delta, double *u0, double *u1) {
  double ax[9];
  or_network_frame(pos, ax);
  const double h = alpha - gmst;
  const double n[3] = {cos(delta) * cos(h), cos(delta) * sin(h), sin(delta)};
  double np[3];
  for (int i = 0; i < 3; i++) np[i] = ax[3 * i] * n[0] + ax[3 * i + 1] * n[1] + ax[3 * i + 2] * n[2];
  double ph = atan2(np[1], np[0]);
  if (ph < 0.0) ph += 2.0 * M_PI;
  *u0 = ph / (2.0 * M_PI);
  *u1 = 0.5 * (np[2] + 1.0);
}

/* (u0, u1) in the frame -> (alpha, delta) */
static void frame_sky(const double *pos, double gmst, double u0, double u1, double *alpha, double *delta) {
  double ax[9];
  or_network_frame(pos, ax);
  const double ph = 2.0 * M_PI * u0, ct = 2.0 * u1 - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct));
  const double np[3] = {st * cos(ph), st * sin(ph), ct};
  double n[3];
  for (int i = 0; i < 3; i++) n[i] = np[0] * ax[i] + np[1] * ax[3 + i] + np[2] * ax[6 + i];
  *delta = asin(fmax(-1.0, fmin(1.0, n[2])));
  double a = atan2(n[1], n[0]) + gmst;
  a = fmod(a, 2.0 * M_PI);
  if (a < 0.0) a += 2.0 * M_PI;
  *alpha = a;
}

/* Phase-rotated coordinates for the polarization and the orbital phase
 * (App. D, more flexible sampling models: sky- and phase-rotated coordinates
 * for the loudest signals; App. E, better ILE integration: coordinates that
 * simplify the phase posterior).  The polarization rotates every detector's F_k by exp(-2 i psi) and
 * Y_lm carries exp(i m phi), so a (2, 2) mode depends on (psi, phi) only
 * through d = phi - psi and a (2, -2) mode only through s = phi + psi: a loud
 * source dominated by one of them has its likelihood flat along one of the
 * two and peaked along the other.  The two uniforms of the psi and phi
 * dimensions become u_s = s / 4 pi and u_d = d / 4 pi in [0, 1):
 *   psi = 2 pi (u_s - u_d) mod pi,   phi = 2 pi (u_s + u_d) mod 2 pi.
 * The map from [0, 1)^2 onto the (psi, phi) torus [0, pi) x [0, 2 pi) is
 * four to one with constant Jacobian, so it carries the uniform measure to
 * the uniform one: the prior stays uniform in (u_s, u_d) and the importance
 * ratio of a draw is 1 / p_s(u_s, u_d) in those coordinates. */
static void phase_rot(double us, double ud, double *psi, double *phi) {
  const double x = 2.0 * M_PI * (us - ud), y = 2.0 * M_PI * (us + ud);
  *psi = x - M_PI * floor(x / M_PI);
  *phi = y - 2.0 * M_PI * floor(y / (2.0 * M_PI));
}

void or_phase_rot(double us, double ud, double *psi, double *phi) { phase_rot(us, ud, psi, phi); }

void or_draw_coords(uint64_t seed, uint32_t point, uint32_t round, uint64_t i, double d_min, double d_max,
                    double tau_width, const double *cdf, int nb, unsigned adapt_mask, const double *frame_pos,
                    double gmst, int phase, double theta[7], double *ln_ratio, uint8_t bins[7], uint32_t raw[8]) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t r[8];
  for (int half = 0; half < 2; half++) {
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), 2u * round + (uint32_t)half, point};
    or_philox4x32_10(ctr, key, r + 4 * half);
  }
  if (raw) memcpy(raw, r, sizeof(r));
  double lr = 0.0, us[7];
  for (int d = 0; d < 7; d++) {
    double v = or_u01(r[d]);
    double u = v;
    int bin = (int)floor(v * nb); /* exact: v has 25 significant bits */
    if (cdf && (adapt_mask >> d) & 1u) {
      const double *c = cdf + (size_t)d * (nb + 1);
      /* largest b with c[b] <= v */
      int lo = 0, hi = nb; /* invariant c[lo] <= v < c[hi] */
      while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (c[mid] <= v) lo = mid; else hi = mid;
      }
      double mass = c[lo + 1] - c[lo];
      u = ((double)lo + (v - c[lo]) / mass) / nb;
      lr -= log(mass * nb);
      bin = lo;
    }
    if (bins) bins[d] = (uint8_t)bin;
    us[d] = u;
    theta[d] = prior_inv(d, u, d_min, d_max, tau_width);
  }
  if (frame_pos) frame_sky(frame_pos, gmst, us[OR_ALPHA], us[OR_DELTA], &theta[OR_ALPHA], &theta[OR_DELTA]);
  if (phase) phase_rot(us[OR_PSI], us[OR_PHI], &theta[OR_PSI], &theta[OR_PHI]);
  *ln_ratio = lr;
}

void or_draw_frame(uint64_t seed, uint32_t point, uint32_t round, uint64_t i, double d_min, double d_max,
                   double tau_width, const double *cdf, int nb, unsigned adapt_mask, const double *frame_pos,
                   double gmst, double theta[7], double *ln_ratio, uint8_t bins[7], uint32_t raw[8]) {
  or_draw_coords(seed, point, round, i, d_min, d_max, tau_width, cdf, nb, adapt_mask, frame_pos, gmst, 0, theta,
                 ln_ratio, bins, raw);
}

void or_draw(uint64_t seed, uint32_t point, uint32_t round, uint64_t i, double d_min, double d_max,
             double tau_width, const double *cdf, int nb, unsigned adapt_mask, double theta[7],
             double *ln_ratio, uint8_t bins[7], uint32_t raw[8]) {
  or_draw_frame(seed, point, round, i, d_min, d_max, tau_width, cdf, nb, adapt_mask, NULL, 0.0, theta, ln_ratio,
                bins, raw);
}

/* Adaptation between rounds (Sec. III.B).  Reading of the garbled histogram
 * formula: nb equal bins in each dimension's prior-CDF coordinate, bin mass
 * proportional to the summed importance weight w = exp(lnw - max lnw) of the
 * round's samples in the bin, mixed with a uniform floor eps and normalized:
 *   h_b = (1 - eps) nb m_b / sum m + eps,   cdf[b+1] = cdf[b] + h_b / nb.
 * bins[d][i] is the bin of sample i in dimension d (as returned by or_draw).
 * A dimension outside adapt_mask, or a round without a finite weight, gets
 * the uniform table. */
void or_adapt(int64_t n, const uint8_t *bins, int64_t stride, const double *lnw, int nb,
              double floor_eps, unsigned adapt_mask, double *cdf) {
  double mx = -INFINITY;
  for (int64_t i = 0; i < n; i++)
    if (isfinite(lnw[i]) && lnw[i] > mx) mx = lnw[i];
  double *mass = (double *)calloc(nb, sizeof(double));
  for (int d = 0; d < 7; d++) {
    double *c = cdf + (size_t)d * (nb + 1);
    memset(mass, 0, sizeof(double) * nb);
    double tot = 0.0;
    if (((adapt_mask >> d) & 1u) && isfinite(mx)) {
      for (int64_t i = 0; i < n; i++) {
        if (!isfinite(lnw[i])) continue;
        double w = exp(lnw[i] - mx);
        mass[bins[d * stride + i]] += w;
        tot += w;
      }
    }
    c[0] = 0.0;
    for (int b = 0; b < nb; b++) {
      double h = tot > 0.0 ? (1.0 - floor_eps) * nb * mass[b] / tot + floor_eps : 1.0;
      c[b + 1] = c[b] + h / nb;
    }
    /* the running sum may drift by rounding: pin the last edge to 1 */
    for (int b = 1; b <= nb; b++) c[b] /= c[nb];
  }
  free(mass);
}

/* ------------------------------------------------------------------------
 * Q, U, V of Eq. (QUV) (App. D), written as the sums they are on a discrete
 * two-sided frequency grid: the inner product <a|b>_k = 2 int df conj(a~) b~ /
 * S_k(|f|) over |f| > f_low, with Q_k,lm(t) = <h_lm(. + t)|d>_k (the mode
 * shifted to time t gives the factor e^{2 pi i f t}), U = <h_lm|h_l'm'>_k and
 * V = <h*_lm|h_l'm'>_k, where the transform of h*_lm at f is conj(h~_lm(-f)).
 * ---------------------------------------------------------------------- */
static double grid_f(int64_t i, int64_t N, double df) { return (double)(i < (N + 1) / 2 ? i : i - N) * df; }

void or_quv(int K, int M, int64_t N, double df, double f_low, const double *data, const double *psd,
            const double *modes, int64_t row0, int64_t n_rows, double *Q, double *U, double *V) {
  double *w = (double *)malloc(sizeof(double) * (size_t)N);
  for (int k = 0; k < K; k++) {
    for (int64_t i = 0; i < N; i++) w[i] = fabs(grid_f(i, N, df)) > f_low ? 2.0 * df / psd[(size_t)k * N + i] : 0.0;
    const double *d = data + (size_t)k * N * 2;
    for (int m = 0; m < M; m++) {
      const double *h = modes + (size_t)m * N * 2;
      for (int64_t r = 0; r < n_rows; r++) {
        const int64_t n = ((row0 + r) % N + N) % N;
        double sr = 0.0, si = 0.0;
        for (int64_t i = 0; i < N; i++) {
          if (w[i] == 0.0) continue;
          /* conj(h) d */
          const double xr = h[2 * i] * d[2 * i] + h[2 * i + 1] * d[2 * i + 1];
          const double xi = h[2 * i] * d[2 * i + 1] - h[2 * i + 1] * d[2 * i];
          /* e^{2 pi i f_i t_r} = e^{2 pi i (i n mod N) / N} */
          const int64_t ph = (int64_t)(((__int128)i * n) % N);
          const double a = 2.0 * M_PI * (double)ph / (double)N;
          const double c = cos(a), s = sin(a);
          sr += w[i] * (xr * c - xi * s);
          si += w[i] * (xr * s + xi * c);
        }
        Q[(((size_t)k * n_rows + r) * M + m) * 2] = sr;
        Q[(((size_t)k * n_rows + r) * M + m) * 2 + 1] = si;
      }
      for (int mp = 0; mp < M; mp++) {
        const double *g = modes + (size_t)mp * N * 2;
        double ur = 0.0, ui = 0.0, vr = 0.0, vi = 0.0;
        for (int64_t i = 0; i < N; i++) {
          if (w[i] == 0.0) continue;
          const int64_t j = (N - i) % N; /* -f_i */
          ur += w[i] * (h[2 * i] * g[2 * i] + h[2 * i + 1] * g[2 * i + 1]);
          ui += w[i] * (h[2 * i] * g[2 * i + 1] - h[2 * i + 1] * g[2 * i]);
          vr += w[i] * (h[2 * j] * g[2 * i] - h[2 * j + 1] * g[2 * i + 1]);
          vi += w[i] * (h[2 * j] * g[2 * i + 1] + h[2 * j + 1] * g[2 * i]);
        }
        const size_t o = (((size_t)k * M + m) * M + mp) * 2;
        U[o] = ur;
        U[o + 1] = ui;
        V[o] = vr;
        V[o + 1] = vi;
      }
    }
  }
  free(w);
}
