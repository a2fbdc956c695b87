/*
 * rift_ile.h -- C ABI of the MI355X (gfx950) ILE marginalized-likelihood
 * library: for each intrinsic point, draw extrinsic samples, evaluate the
 * mode-decomposed log-likelihood from the overlaps Q and U, marginalize it
 * over a reference-time window with a log-sum-exp, and importance-weight the
 * results into ln L_marg with FP64 sample-size diagnostics.
 *
 * Paper: "Expanding RIFT: Improving performance for GW parameter inference"
 * (arXiv 2210.07912).  The likelihood is App. D Eq. (loglikelihood) /
 * Eq. (def:lnL:Decomposed) with the overlaps of Eq. (QUV); the Monte Carlo
 * estimate is Sec. II.A Eq. (lnL:MonteCarlo); the sample-size measures are
 * App. B Eqs. (neff), (neff_ESS) and the variance-based size; the adaptive
 * histogram proposal is Sec. III.B (GPU-accelerated Monte Carlo integration);
 * the Gaussian-mixture proposal, separable and with correlated pairs, is
 * Sec. III.B (adaptive sampling with Gaussian mixture models) with App. A.
 * Beyond those: the adjoint gradient, the Q/U/V precompute of Eq. (QUV),
 * network-frame sky coordinates (Sec. II.A), and checkpoints of a run.
 *
 * Conventions common to every call
 *   - No C++ exception crosses this boundary.  Every call returns a
 *     rift_status; rift_ile_last_error() gives the text of the last failure
 *     on a handle.
 *   - "host" pointers are read during the call only.  "device" pointers are
 *     HIP device allocations owned by the caller; they must stay valid until
 *     the work enqueued on the handle's stream has completed.
 *   - Extrinsic parameters are structure-of-arrays theta[7][stride] in the
 *     order of rift_param below; angles in radians, distance in Mpc, tau in
 *     seconds.  A RIFT_FP32 handle takes float theta and returns float
 *     ln L_t; a RIFT_FP64 handle takes and returns double.
 *   - Complex arrays are interleaved (re, im) doubles, row-major.
 *   - Calls on one handle are serialized on its stream; a handle must not be
 *     used from two threads at once.  Distinct handles are independent.
 *   - Per-sample results that are not finite (a sample whose arrival time
 *     falls outside the stored rows, a non-finite theta) never fail a call:
 *     they are returned as NaN and counted in rift_ile_result.n_nonfinite,
 *     and excluded from every sum.
 */
#ifndef RIFT_ILE_H
#define RIFT_ILE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RIFT_ILE_ABI_VERSION 3

typedef enum {
  RIFT_OK = 0,
  RIFT_E_INVALID = -1,       /* bad argument (NULL, negative count, unknown enum) */
  RIFT_E_SHAPE = -2,         /* inconsistent or unsupported sizes */
  RIFT_E_NOT_HERMITIAN = -3, /* U_k not Hermitian (relative 1e-6) or V_k not symmetric */
  RIFT_E_WINDOW = -4,        /* pad too small for the detectors' light travel time */
  RIFT_E_NONFINITE = -5,     /* NaN/Inf in Q, U, V or the point constants */
  RIFT_E_OOM = -6,           /* device allocation failed */
  RIFT_E_DEVICE = -7,        /* HIP runtime error (launch, copy, fault) */
  RIFT_E_STATE = -8          /* call not valid in the handle's current state */
} rift_status;

typedef enum { RIFT_FP32 = 0, RIFT_FP64 = 1 } rift_precision;

typedef enum {
  RIFT_ALPHA = 0, /* right ascension */
  RIFT_DELTA = 1, /* declination */
  RIFT_PSI = 2,   /* polarization angle */
  RIFT_IOTA = 3,  /* inclination */
  RIFT_PHI = 4,   /* orbital phase */
  RIFT_DIST = 5,  /* luminosity distance, Mpc */
  RIFT_TAU = 6,   /* offset of the time window, s */
  RIFT_NPAR = 7
} rift_param;

#define RIFT_MAX_DET 3
#define RIFT_MAX_MODES 32
#define RIFT_NBINS 100

typedef struct rift_ile rift_ile;

/* One intrinsic point: the overlaps of App. D Eq. (QUV) at reference
 * distance d_ref.  Q_k holds L = n_t + 2*pad + 3 rows sampled at f_s; row r
 * is time t_q0 + r / f_s.  Window sample j (j = 0..n_t-1) is the geocentric
 * time t_q0 + (pad + 1 + j) / f_s + tau; detector k sees it at that time plus
 * its delay dt_k = -r_k . n / c, so the 4-tap interpolation stencil stays
 * inside the stored rows whenever |tau + dt_k| f_s <= pad. */
typedef struct {
  int n_det;              /* K, 1..RIFT_MAX_DET */
  int n_modes;            /* M, 1..RIFT_MAX_MODES */
  int n_t;                /* window samples, >= 1 */
  int pad;                /* rows before and after the window, ceil(f_s max|r_k|/c) .. 32767 */
  const int *ell, *em;    /* host [M]: mode (l, m), 2 <= l <= 8, |m| <= l */
  double f_s;             /* sample rate, Hz */
  double d_ref;           /* distance at which Q, U, V were computed, Mpc */
  double gmst;            /* Greenwich sidereal angle, rad */
  const double *det_pos;  /* host [K][3]: detector vertex, Earth-fixed, m */
  const double *det_resp; /* host [K][3][3]: symmetric response tensor D_k */
  const double *Q;        /* host [K][L][M] complex: Q_{k,lm}(t_r) */
  const double *U;        /* host [K][M][M] complex Hermitian: U_{k,lm,l'm'} */
  const double *V;        /* host [K][M][M] complex symmetric, or NULL (V = 0) */
} rift_ile_point;

typedef struct {
  int n_points;
  const rift_ile_point *points; /* host [n_points] */
  int precision;                /* rift_precision */
  double d_min, d_max;          /* distance prior p(D) ~ D^2 on [d_min, d_max], Mpc */
  double tau_width;             /* tau prior: uniform on [-w/2, w/2) s; 0 fixes tau = 0 */
} rift_ile_desc;

/* A segment of a sample array evaluated against one point. */
typedef struct {
  int point;       /* index into the handle's points */
  int64_t offset;  /* first column of theta / ln L_t */
  int64_t count;   /* number of samples */
} rift_ile_item;

typedef struct {
  double lnL_marg;   /* ln[(1/N) sum_i w_i], Sec. II.A Eq. (lnL:MonteCarlo) */
  double sigma_lnL;  /* 1 / sqrt(n_var): relative error of the estimate */
  double n_eff;      /* sum w / max w, App. B Eq. (neff) */
  double n_ess;      /* (sum w)^2 / sum w^2, App. B Eq. (neff_ESS) */
  double n_var;      /* N wbar^2 / s^2 (unbiased s^2), App. B variance-based size */
  double max_lnw;    /* largest finite ln w */
  int64_t n;         /* finite samples counted */
  int64_t n_nonfinite;
} rift_ile_result;

typedef struct {
  uint64_t seed;              /* Philox key */
  int64_t n_per_round;        /* samples per point per round; ignored if n_per_point */
  const int64_t *n_per_point; /* host [n_points] or NULL */
  int n_rounds;               /* >= 1 */
  unsigned adapt_mask;        /* bit d: adapt parameter d after each round (0: prior only) */
  double floor_eps;           /* uniform floor mixed into each adapted histogram, (0, 1] */
  int reset_proposal;         /* 1: start from the prior (else from the current tables) */
  /* Gradient-informed refinement (flags & RIFT_MC_GRADIENT, adapt_mask != 0):
   * between rounds, the n_ascent samples of largest ln w of each point climb
   * ln L_t for ascent_steps steps along the adjoint gradient (normalized
   * steps in the prior-CDF coordinates of the adapted parameters, each step
   * kept only if ln L_t rises), and the next proposal places a fraction
   * ascent_mix of each adapted histogram around the points reached.  Every
   * round's proposal is fixed before the round is drawn, so the pooled
   * estimate stays unbiased. */
  unsigned flags;
  int n_ascent;               /* 1..256 (0: 64) */
  int ascent_steps;           /* >= 1 (0: 12) */
  double ascent_mix;          /* [0, 1 - floor_eps) (0: 0.3) */
  /* Gaussian-mixture proposal (Sec. III.B, adaptive sampling with Gaussian
   * mixture models; App. A) in place of the histograms: gmm_components
   * (1..4) normals per adapted parameter, each truncated to the parameter's
   * prior-CDF coordinate [0, 1], plus the uniform floor floor_eps; between
   * rounds gmm_iters weighted EM iterations (0: 10) from the current mixture,
   * then the online update that combines it with the new fit by sample
   * counts.  0: histograms.  Not combined with RIFT_MC_GRADIENT. */
  int gmm_components;
  int gmm_iters;
  /* Correlated pairs of the mixture proposal (needs gmm_components > 0 and
   * n_rounds <= 2^20): byte i (i < 3) = a | b << 4 names a pair a < b < 7 of
   * adapted parameters (0: none; pairs disjoint); such a pair gets
   * gmm_components bivariate components in its two prior-CDF coordinates
   * (App. A, finite domains): draws from the untruncated mixture rejected
   * outside the unit square (64 tries, Philox counter word 2 =
   * 3 2^30 | round << 10 | pair << 8 | try).  A draw none of whose tries
   * lands in the square (probability f = (1 - Z)^64, Z = sum_k pi_k Z_k,
   * Z_k the component's mass in the square) is given up: the sample keeps
   * its raw uniforms and ln ratio -inf (zero weight; it stays in the count).
   * Kept draws are weighted with p_s = floor_eps + (1 - floor_eps) (1 - f)
   * sum_k pi_k N_k / Z, their density among all draws. */
  unsigned gmm_pairs;
  /* Resume: the Philox round index of the first round (counter word 2 uses
   * first_round + r).  0: a fresh pooled estimate.  > 0 (with
   * reset_proposal = 0): the rounds continue the handle's pooled estimate and
   * proposals, as left by an earlier run or rift_ile_load_checkpoint, so a
   * run split at any round gives bit-identical results to an unsplit one;
   * RIFT_E_STATE when the handle holds no pooled estimate. */
  int first_round;
} rift_ile_mc;

#define RIFT_MC_GRADIENT 1u

/* Create a handle for desc->n_points points on the current HIP device.
 * Validates every point (shapes, finiteness, Hermitian U, symmetric V, pad
 * large enough), then deep-copies Q/U/V into library-owned device memory in
 * the kernels' layouts; the caller may free its inputs once this returns.
 * stream: a hipStream_t (NULL = the null stream) used by every later call.
 * Errors: RIFT_E_INVALID, RIFT_E_SHAPE, RIFT_E_NOT_HERMITIAN, RIFT_E_WINDOW,
 * RIFT_E_NONFINITE, RIFT_E_OOM, RIFT_E_DEVICE.  On error *out is NULL. */
rift_status rift_ile_create(rift_ile **out, const rift_ile_desc *desc, void *stream);

/* Release the handle and its device memory (synchronizes its stream). */
void rift_ile_destroy(rift_ile *h);

/* Text of the last error on h (or of the last failed create when h is NULL). */
const char *rift_ile_last_error(const rift_ile *h);
/* Text of a status (an int, so that any value a caller holds is valid;
 * values that are no rift_status give "unknown status"). */
const char *rift_ile_status_string(int s);
int rift_ile_abi_version(void);

/* Diagnostics: time the dominant evaluation kernel (the persistent matrix-
 * core kernel, or the plain kernel) with HIP events on the handle's stream.
 * Returns, in *ms_total and *launches, the summed duration and the count of
 * the launches timed since the previous call (synchronizing if there were
 * any), then enables (enable != 0) or disables timing.  Either output may be
 * NULL. */
rift_status rift_ile_profile(rift_ile *h, int enable, double *ms_total, int64_t *launches);

/* Rebind the handle to another stream. */
rift_status rift_ile_set_stream(rift_ile *h, void *stream);

/* Graph replay of the FP32 evaluation (batching: the evaluation of many
 * points launched as one unit).  With enable != 0, each evaluation run of
 * rift_ile_lnL / rift_ile_marginalize on an FP32 handle (the delay-bin sort,
 * the coefficient pass and the persistent matrix-core launches of all (T, K)
 * classes, fanned out over the handle's side streams) is captured once into a
 * hipGraph on the handle's stream and replayed whenever a later run has the
 * same shape and buffers (later rounds of marginalize, repeated calls on the
 * same workspace).  Results are bit-identical to the direct launches.  Not
 * used while rift_ile_profile timing is on, for FP64 handles or for the
 * adjoint.  The handle owns the graphs until destroy or until disabled.
 * Returns RIFT_E_INVALID for a NULL handle. */
rift_status rift_ile_set_graph(rift_ile *h, int enable);

/* Diagnostics of the graph replay: graphs captured and replays launched since
 * the handle was created (either output may be NULL). */
rift_status rift_ile_graph_stats(const rift_ile *h, int64_t *captures, int64_t *replays);

/* Frequency-domain inputs of one intrinsic point for rift_ile_precompute:
 * a two-sided grid of N samples in FFT order, f_i = i df for i < (N + 1) / 2
 * and (i - N) df otherwise (the time series it transforms to has N samples
 * at f_s = N df). */
typedef struct {
  int n_det;            /* K, 1..RIFT_MAX_DET */
  int n_modes;          /* M, 1..RIFT_MAX_MODES */
  int64_t n_f;          /* N, 2..2^30 */
  double df;            /* grid spacing, Hz, > 0 */
  double f_low;         /* bins with |f_i| <= f_low are left out of every sum (Hz, >= 0) */
  const double *data;   /* host [K][N][2]: d~_k(f_i), complex interleaved */
  const double *psd;    /* host [K][N]: S_n,k(|f_i|), finite and > 0 where |f_i| > f_low */
  const double *modes;  /* host [M][N][2]: h~_lm(f_i) at the reference distance */
} rift_ile_fd_point;

/* The overlaps of App. D Eq. (QUV) from frequency-domain inputs, the step
 * that prepares Q, U and V for rift_ile_create.  With the inner product
 * <a|b>_k = 2 sum_i df conj(a~(f_i)) b~(f_i) / S_n,k(|f_i|) over |f_i| > f_low:
 *   Q[k][r][m] = <h_m(. + t_r)|d>_k = 2 sum_i df/S e^{2 pi i f_i t_r} conj(h~_m) d~_k,
 *                t_r = (row0 + r) / f_s for r < n_rows (rows wrap modulo N),
 *   U[k][m][m'] = <h_m|h_m'>_k,   V[k][m][m'] = <h*_m|h_m'>_k = 2 sum_i df/S h~_m(-f_i) h~_m'(f_i).
 * Q is an unnormalized inverse DFT of the weighted product (one batched
 * complex FFT over detectors and modes, hipFFT), U and V fixed-order FP64
 * sums per entry.  Outputs are caller-owned host arrays, complex
 * interleaved FP64: Q [K][n_rows][M][2] (the row layout of
 * rift_ile_point.Q; NULL allowed when n_rows == 0), U and V [K][M][M][2].
 * Runs on the current device and blocks; it allocates and frees its own
 * device buffers (inputs, a K M N scratch, outputs) and FFT plan.  Errors:
 * RIFT_E_INVALID (NULL array, df or f_low invalid), RIFT_E_SHAPE (K, M, N or
 * n_rows out of range), RIFT_E_NONFINITE (non-finite input, or a PSD value
 * <= 0 in band), RIFT_E_OOM, RIFT_E_DEVICE (HIP or FFT failure). */
rift_status rift_ile_precompute(const rift_ile_fd_point *in, int64_t row0, int64_t n_rows, double *Q, double *U,
                                double *V);

/* Sky coordinates of the sampler (Sec. II.A, rotated detector-network-frame
 * sky coordinates; Sec. II.C: usable with the GPU integrator).  With
 * enable != 0, rift_ile_sample and rift_ile_marginalize draw the sky of each
 * point in its network frame: the north pole is the unit vector from the
 * point's detector 0 to its detector 1 (Earth-fixed), the x axis is
 * normalize(e_z x pole) (e_x x pole for a pole along e_z), y = pole x x.  The
 * sky's two uniform coordinates become the frame azimuth / 2 pi and
 * (cos(polar angle) + 1) / 2, so the adaptive histograms of dimensions 0 and
 * 1 (and the bins written by rift_ile_sample) refer to those; the prior is
 * isotropic either way, so ln p - ln p_s keeps its form, and the returned
 * theta is still (alpha, delta).  A point with one detector keeps the
 * equatorial axes.  Default off.  Returns RIFT_E_INVALID for a NULL handle. */
rift_status rift_ile_set_network_frame(rift_ile *h, int enable);

/* Polarization and orbital phase of the sampler in phase-rotated coordinates
 * (App. D, more flexible sampling models: sky- and phase-rotated coordinates
 * for the loudest signals; App. E, better ILE integration: polarization and
 * phase coordinates that simplify the phase posterior).
 * With enable != 0, rift_ile_sample and rift_ile_marginalize draw the two
 * uniforms of dimensions psi and phi as u_s = (phi + psi) / 4 pi and
 * u_d = (phi - psi) / 4 pi and return
 *   psi = 2 pi (u_s - u_d) mod pi,   phi = 2 pi (u_s + u_d) mod 2 pi.
 * A (2, 2) mode depends on (psi, phi) only through phi - psi and a (2, -2)
 * mode only through phi + psi, so for a source dominated by either the
 * likelihood varies along one of u_s, u_d and is flat along the other, which
 * a product proposal captures.  The map is four to one with a constant
 * Jacobian: the prior is uniform in (u_s, u_d), ln p - ln p_s keeps its form,
 * and the adaptive histograms and mixtures of dimensions psi and phi (and the
 * bins rift_ile_sample writes) refer to u_s and u_d.  Combines with the
 * network frame.  rift_ile_marginalize returns RIFT_E_INVALID when this is on
 * together with RIFT_MC_GRADIENT.  A checkpoint records the coordinate
 * switches (and distance marginalization) and loads only into a handle with
 * the same ones.  Default off.
 * Returns RIFT_E_INVALID for a NULL handle. */
rift_status rift_ile_set_phase_rotation(rift_ile *h, int enable);

/* Distance marginalization (Sec. III.B, distance marginalization; Sec. III's
 * production configuration pairs it with the adaptive integrator).  With
 * enable != 0, rift_ile_lnL and rift_ile_marginalize return, in place of
 * ln L_t, the distance-marginalized
 *   ln L_tD = ln int p(D) (1/n_t) sum_j exp(ell_j(D)) dD,
 *   p(D) = 3 D^2 / (d_max^3 - d_min^3) on the handle's [d_min, d_max],
 * and theta's distance row is not read (any value, NaN included).  With
 * x = D_ref / D every window value is x A_j - x^2 B (A_j the data term, B the
 * quadratic term at D_ref), so each sample is evaluated once at D_ref and
 * integrated over D by a Gauss-Legendre rule in ln x placed on the part of
 * the prior range where the integrand's envelope is within T of its peak:
 * 24 nodes and T = 30 nats on FP32 handles (rule error below 1e-5), 3 x 24
 * nodes and T = 50 on FP64 handles (below 1e-10).  FP32 handles take two
 * passes over the window (its largest data term, then the sums per node).
 * rift_ile_marginalize then draws the six other parameters (the distance row
 * of theta_out is a prior draw that enters no weight) and returns
 * RIFT_E_INVALID if adapt_mask or a proposal it continues from adapts the
 * distance, or with RIFT_MC_GRADIENT; rift_ile_backward returns
 * RIFT_E_INVALID.  A checkpoint records the switch.  Default off.  Returns
 * RIFT_E_INVALID for a NULL handle. */
rift_status rift_ile_set_distance_marginalization(rift_ile *h, int enable);

/* Precision of the FP32 adjoint (rift_ile_backward on an RIFT_FP32 handle).
 * The gradient of ln L_t is an average of d ell_j / d theta under the window
 * softmax p_j (App. D Eq. (def:lnL:Decomposed) differentiated).  For a loud
 * sample the data term and the quadratic term nearly cancel in each component,
 * and FP32 rounding of the contraction is then a visible part of the result.
 * With enable != 0 (the default), every sample whose softmax mass lies in at
 * most 3 window blocks of 16 samples (the blocks whose maximum came within
 * 40 of the sample's running maximum ell) is re-evaluated in FP64 over those
 * blocks: coefficients, quadratic term, contraction, ell_j, p_j and the chain
 * rule; its gradient and ln L_t output are replaced by the FP64 values (mass
 * outside the blocks is below n_t e^-40 of the total).  Other samples keep
 * the FP32 values.  enable == 0: FP32 throughout.  Returns RIFT_E_INVALID for
 * a NULL handle. */
rift_status rift_ile_set_grad_refine(rift_ile *h, int enable);

/* Per-class launch configuration of the FP32 evaluation (batching: every
 * (T, K) class of points, T = ceil(M / 2) MFMA steps and K detectors, is one
 * persistent launch).  Two forms of the same kernel exist: "staged" (each
 * workgroup copies the rows of Q its unit needs into LDS, one barrier per two
 * 16-row blocks) and "direct" (each wavefront loads its own operands from
 * global memory one block ahead, no barrier, less LDS and more resident
 * workgroups); each runs with as many workgroups as the device keeps resident
 * or with half as many per compute unit; the direct form also comes compiled
 * with its registers capped so that three or four wavefronts fit on a SIMD,
 * the staged form capped for three (more resident workgroups where LDS allows
 * them).  The seven configurations are numbered 1 staged, 2 direct, 3 staged
 * at half residency, 4 direct at half residency, 5 direct capped for three
 * wavefronts per SIMD, 6 direct capped for four, 7 staged capped for three;
 * their results are bit-identical.  mode 1 (the default): the first
 * evaluation of a class on the handle, for each n_t bucket (floor(log2) of
 * the class's longest window), runs all seven twice on that call's data,
 * timed with events (that call waits for them), and later calls use the
 * fastest by the better of its two runs (configuration 1 unless another is
 * at least 3 % faster).  mode 0: every
 * class runs staged; mode 2: every class runs direct; modes 3, 4 and 5: every
 * class runs configuration 5, 6 or 7 (measurements made so far are kept for a
 * later mode 1).  Runs with a class not yet measured are not
 * captured by the graph replay.  Returns RIFT_E_INVALID for a NULL handle or
 * another mode. */
rift_status rift_ile_set_autotune(rift_ile *h, int mode);

/* The configuration each (T, K) class ran with last: modes[(T - 1) * 3 +
 * (K - 1)] for T = 1..16 and K = 1..3 (48 ints, caller-owned) is 0 (not run
 * yet) or 1..7 as numbered above.  Returns RIFT_E_INVALID for a NULL handle
 * or array. */
rift_status rift_ile_autotune_table(const rift_ile *h, int *modes);

/* Persisted autotuning.  path: a text file of lines
 * "<arch> <T> <K> <n_t bucket> <configuration>" (arch: the device's gfx
 * name).  The lines for this device's arch are read now (later lines win;
 * malformed lines are skipped; a missing file is not an error) and every
 * configuration the handle measures from now on is appended, so another
 * handle or process that loads the file starts with those classes measured.
 * NULL: stop appending.  Errors: RIFT_E_INVALID for a NULL handle or a file
 * that exists but cannot be read; a failed append is skipped silently. */
rift_status rift_ile_set_autotune_cache(rift_ile *h, const char *path);

/* Extrinsic sample draw (Sec. II.A; Sec. III.B: random numbers generated on
 * the GPU).  Writes samples first..first+n-1 of (point, round): Philox4x32-10
 * with key = seed and counter = (i_lo, i_hi, 2 round + half, point); each
 * parameter takes one 32-bit word, mapped through the prior's inverse CDF or,
 * for a parameter adapted in the point's proposal, through its 100-bin
 * histogram or its Gaussian mixture (see rift_ile_set_gmm; a correlated pair
 * none of whose tries lands in the unit square gives ln_ratio -inf).
 * theta: device [7][n]; ln_ratio: device [n] (handle precision)
 * receives ln p - ln p_s (or NULL); bins: device uint8 [7][n] receives each
 * sample's histogram bin per parameter (floor(100 u) under a mixture) (or
 * NULL).  Asynchronous. */
rift_status rift_ile_sample(rift_ile *h, int point, uint64_t seed, uint32_t round, int64_t first,
                            int64_t n, void *theta, void *ln_ratio, uint8_t *bins);

/* Time-marginalized log-likelihood (App. D Eq. (def:lnL:Decomposed), window
 * log-sum-exp of App. D.2): for every item, columns offset..offset+count-1 of
 * theta are evaluated against the item's point and
 *   ln L_t = ln[(1/n_t) sum_j exp(ell_j)]
 * is written to the same columns of lnL_t.  theta: device [7][stride];
 * lnL_t: device [stride].  items: host [n_items].  Asynchronous.  Errors:
 * RIFT_E_INVALID (NULL handle or arrays, items outside stride); RIFT_E_SHAPE
 * on the plain (VALU) form when the handle's longest window does not fit four
 * samples' rows in LDS (FP64: n_t above about 2300). */
rift_status rift_ile_lnL(rift_ile *h, int n_items, const rift_ile_item *items, int64_t stride,
                         const void *theta, void *lnL_t);

/* FP64 Monte Carlo reduction (Sec. II.A Eq. (lnL:MonteCarlo), App. B) of
 * ln w_i = ln L_t,i + ln_ratio_i over n samples.  lnL_t and ln_ratio:
 * device [n] in the handle's precision (ln_ratio may be NULL: 0).
 * Synchronizes and writes *out on the host. */
rift_status rift_ile_reduce(rift_ile *h, int64_t n, const void *lnL_t, const void *ln_ratio,
                            rift_ile_result *out);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the reduction of
 * rift_ile_reduce, same arguments and identical results, that allocates
 * nothing.  Its partial sums, segment bounds and result live in a
 * file-scope device array of the library (about 50 KB, one copy per device,
 * held until the process ends), whose address rift_ile_create takes once per
 * device.  Every call on a device shares that array and leaves it as the last
 * call wrote it; calls that overlap on one device (other threads, other
 * handles on other streams) race and must be serialized by the caller.  Any
 * n in 0..2^40 (RIFT_E_SHAPE above that); nothing in the array needs to start
 * at zero.  Synchronizes the handle's stream and writes *out on the host. */
rift_status rift_ile_reduce_noalloc(rift_ile *h, int64_t n, const void *lnL_t, const void *ln_ratio,
                                    rift_ile_result *out);

/* Adapt the point's proposal (Sec. III.B): FP64 weighted 100-bin histograms of
 * w = exp(ln w - max ln w) over each masked parameter's prior-CDF coordinate,
 * mixed with a uniform floor:  h_b = (1 - eps) 100 m_b / sum m + eps.
 * bins: device uint8 [7][n] (as written by rift_ile_sample); lnw: device
 * [n] in the handle's precision, n <= 2^23.  Weights are accumulated
 * deterministically (50-bit fixed point within blocks of 8192 samples, FP64
 * across blocks in block order).  Parameters outside mask revert to the
 * prior.  Asynchronous. */
rift_status rift_ile_adapt(rift_ile *h, int point, int64_t n, const uint8_t *bins, const void *lnw,
                           unsigned mask, double floor_eps);

/* Read / replace a point's proposal: cdf host [7][101] bin edges of the
 * prior-CDF coordinate (cdf[d][0] = 0, cdf[d][100] = 1, nondecreasing with
 * positive steps), mask as in rift_ile_adapt.  get synchronizes. */
rift_status rift_ile_get_proposal(rift_ile *h, int point, double *cdf, unsigned *mask);
rift_status rift_ile_set_proposal(rift_ile *h, int point, const double *cdf, unsigned mask);

/* Gaussian-mixture proposal of a point (Sec. III.B, adaptive sampling with
 * Gaussian mixture models; App. A): for each parameter d in mask,
 * p_s(u) = floor_eps + (1 - floor_eps) sum_k w[d][k] N_t(u; mu[d][k], sd[d][k])
 * in the prior-CDF coordinate u in [0, 1), N_t the normal truncated to
 * [0, 1].  w, mu, sd: host [7][4] row-major (components k >= K ignored).
 * The sampler draws v from the parameter's usual Philox word and the
 * component from a second Philox block (counter word 2 = 2^31 | (2 round +
 * half)); then u = mu + sd Phi^-1(Phi(a) + v (Phi(b) - Phi(a))).
 * set: K in 1..4, weights of each masked parameter >= 0 summing to 1
 * (within 1e-9), 0 <= mu <= 1, sd > 0, floor_eps in [0, 1], n_trained >= 0
 * (the sample count the online update weights the mixture with); returns
 * RIFT_E_INVALID otherwise.  get: *K = 0 when the point holds a histogram
 * proposal; any output pointer but K may be NULL; synchronizes.  A later
 * rift_ile_set_proposal or histogram adaptation replaces the mixture. */
rift_status rift_ile_get_gmm(rift_ile *h, int point, int *K, unsigned *mask, double *floor_eps, double *n_trained,
                             double *w, double *mu, double *sd);
rift_status rift_ile_set_gmm(rift_ile *h, int point, int K, unsigned mask, double floor_eps, double n_trained,
                             const double *w, const double *mu, const double *sd);

/* One round's update of a point's Gaussian-mixture proposal (App. A) from n
 * samples: u device float [7][n] prior-CDF coordinates (as the sampler drew
 * them), lnw device [n] in the handle's precision.  Weights
 * w = exp(ln w - max ln w) (0 for non-finite ln w); n_iter (1..1000)
 * weighted EM iterations over the masked parameters, starting from the
 * point's mixture when it has K components (else from equal weights, means
 * (k + 1/2) / K, sd 1 / (2 K)), untruncated normals, sd >= 1e-4; then the
 * online update: components matched by the smallest summed symmetric
 * Mahalanobis distance over all permutations and combined with weights
 * N = n_trained and M = the number of samples whose ln w is neither NaN nor
 * +inf.  pairs (coded as in rift_ile_mc, parameters in mask): those
 * parameters are fitted jointly by bivariate components (sd >= 1e-4 per
 * axis, |correlation| <= 0.99); starting from the point's mixture needs the
 * same K and pairs.  Sums are FP64 in a fixed order.  Asynchronous. */
rift_status rift_ile_adapt_gmm(rift_ile *h, int point, int64_t n, const float *u, const void *lnw, unsigned mask,
                               unsigned pairs, double floor_eps, int K, int n_iter);

/* Correlated pairs of a point's mixture (pairs coded as in rift_ile_mc):
 * w host [3][4], mu [3][4][2], cov [3][4][3] (xx, xy, yy), pair slot p the
 * p-th nonzero byte of pairs, components k >= K ignored.  set: the point must
 * hold a mixture (rift_ile_set_gmm), both parameters of each pair in its
 * mask; weights >= 0 summing to 1 (within 1e-9), means in [0, 1]^2,
 * covariances positive definite; computes each component's mass in the
 * unit square; synchronizes.  get: box_mass [3] (or NULL) receives
 * sum_k pi_k Z_k per pair; outputs other than pairs may be NULL;
 * synchronizes.  Errors: RIFT_E_INVALID. */
rift_status rift_ile_set_gmm_pairs(rift_ile *h, int point, unsigned pairs, const double *w, const double *mu,
                                   const double *cov);
rift_status rift_ile_get_gmm_pairs(rift_ile *h, int point, unsigned *pairs, double *w, double *mu, double *cov,
                                   double *box_mass);

/* The whole step for every point (Sec. II.A Eq. (lnL:MonteCarlo) estimated
 * with adaptive importance sampling as in Sec. III.B, GPU-accelerated Monte
 * Carlo integration; sample sizes of App. B): for each round, draw samples
 * from the current proposal, evaluate ln L_t, form ln w, fold them into a pooled FP64
 * estimate over all rounds (each sample weighted with its own round's p_s),
 * and after every round (the last included, so the proposals left behind
 * are the next round's) adapt the masked parameters' histograms from that
 * round's weights.  All points run together in each launch.  out: host
 * [n_points].  theta_out (device [7][total]) and lnw_out (device [total]),
 * both in the handle's precision, if not NULL, receive every sample in
 * (round, point, sample) order, total = n_rounds * sum of per-point counts.
 * Per-point counts per round are limited to 2^23 when adapting.
 * Synchronizes. */
rift_status rift_ile_marginalize(rift_ile *h, const rift_ile_mc *mc, rift_ile_result *out,
                                 void *theta_out, void *lnw_out);

/* Checkpoint of a Monte Carlo run: every point's proposal (histograms or
 * mixture, pairs and sample counts included) and its pooled FP64 estimate
 * (max, sums of e^{ln w - max} and their squares, counts), as raw bytes with a
 * header (magic, ABI version, point count, record sizes).  bytes: host
 * buffer size; rift_ile_checkpoint_bytes gives the size needed (-1 for a
 * NULL handle).  save needs a completed rift_ile_marginalize (RIFT_E_STATE
 * otherwise); load checks the header against this handle (RIFT_E_INVALID on a
 * mismatch).  Both synchronize.  With the same points, a load followed by
 * rift_ile_marginalize with first_round = the rounds done so far continues
 * the run exactly. */
int64_t rift_ile_checkpoint_bytes(const rift_ile *h);
rift_status rift_ile_save_checkpoint(rift_ile *h, void *buf, int64_t bytes);
rift_status rift_ile_load_checkpoint(rift_ile *h, const void *buf, int64_t bytes);

/* Gradient of ln L_t (App. D Eq. (def:lnL:Decomposed) with the window
 * log-sum-exp, differentiated; the paper gives no passage on the gradient
 * itself) with respect to the seven parameters, through the
 * antenna patterns F_k(alpha, delta, psi), the delays dt_k(alpha, delta) and
 * tau (via the Catmull-Rom derivative of Q), the harmonics Y_lm(iota, phi) and
 * the distance.  grad_theta[d][i] = g_i d ln L_t,i / d theta_d with
 * g = grad_lnL_t (device [stride], or NULL for 1).  lnL_t_out (device
 * [stride] or NULL) receives ln L_t.  Same items/stride/layout as
 * rift_ile_lnL.  On an RIFT_FP32 handle the samples whose softmax mass lies
 * in at most three window blocks are re-evaluated in FP64 (see
 * rift_ile_set_grad_refine).  Asynchronous. */
rift_status rift_ile_backward(rift_ile *h, int n_items, const rift_ile_item *items, int64_t stride,
                              const void *theta, const void *grad_lnL_t, void *grad_theta,
                              void *lnL_t_out);

#ifdef __cplusplus
}
#endif
#endif
