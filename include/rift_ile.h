/*
 * rift_ile.h -- C ABI of the MI355X (gfx950) factored extrinsic likelihood.
 *
 * The library evaluates, for every extrinsic sample
 *   theta = (ra, dec, psi, incl, phiref, tref, dist)
 * of one intrinsic point, the factored log-likelihood of the paper's
 * Eq. (def:lnL:Decomposed) (matrix form Eq. (lnL:MatrixForm)):
 *
 *   lnL = x Re sum_k sum_lm conj(F_k Y_lm) Q_{k,lm}(t_k)
 *       - x^2/4 sum_k [ |F_k|^2 Y^H U_k Y + Re(F_k^2 Y^T V_k Y) ],   x = D_ref / dist,
 *
 * with the static complex antenna factor F_k = F+_k + i Fx_k of detector k, the
 * arrival time t_k = tref - r_k . N (N the unit vector towards the source), the
 * spin-weighted harmonics Y_lm = -2Y_lm(incl, phiref) of Eq. (strain_mode), and
 * Q read between its stored samples by the four-point cubic of
 * Eq. (q-time-pregrid) (4-point Lagrange on nodes j-1..j+2; nodes outside the
 * stored window read zero).  It then reduces the weighted samples into the
 * Monte-Carlo marginal likelihood of Eq. (lnL:MonteCarlo),
 *
 *   ln Z = ln[ (1/N) sum_i exp(lnL_i + lnw_i) ],   lnw_i = ln(p/p_s) of sample i,
 *
 * and the effective sample size of Eq. (neff), n_eff = sum_i p_i / max_i p_i.
 * The gradient entry points return d lnL / d(ra, dec, psi, incl or cos incl,
 * phiref, tref, dist or ln dist), in the coordinates the caller gives theta in
 * (Sec. "The differentiable likelihood").
 *
 * Conventions (where the paper is silent or inconsistent):
 *   - Earth-fixed frame: x towards the Greenwich meridian on the equator, z
 *     north.  Greenwich hour angle gha = gmst_rad - ra.  N = (cos dec cos gha,
 *     -cos dec sin gha, sin dec).  Polarisation axes X = -cos psi e_a + sin psi
 *     e_d, Y = sin psi e_a + cos psi e_d with e_a = (sin gha, cos gha, 0),
 *     e_d = (-sin dec cos gha, sin dec sin gha, cos dec).
 *     F+ = D:(X X^T - Y Y^T), Fx = D:(X Y^T + Y X^T).
 *   - All times are seconds relative to one geocentric reference epoch: Q is
 *     sampled at t_j = t0 + j dt, tref is on the same axis.
 *
 * Memory: bulk arrays are DEVICE pointers owned by the caller.  Small metadata
 * (mode list, detector geometry, per-point sample counts) are HOST pointers.
 * Complex numbers are interleaved (re, im) doubles.  The library keeps no
 * pointer to caller memory after a call returns, except a plan, which keeps
 * copies of what it needs.
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  Evaluation
 * calls on a plan only enqueue work and return; outputs are valid once the
 * stream has reached them, and such calls can be captured into a HIP graph.
 * Plan creation and destruction synchronise the stream (they allocate and
 * free device memory and stage small host tables).  The one-shot entry points
 * (rift_ile_lnL, rift_ile_lnZ, rift_ile_grad) create and destroy a plan
 * internally, so they return only after their work has finished: their
 * outputs are valid on return, and they are not capturable.
 *
 * Errors: a negative status means nothing was enqueued and nothing written
 * (invalid arguments are detected on the host before any launch), except
 * RIFT_EDEVICE, which reports a failed HIP call (e.g. a launch).  Faults that
 * happen asynchronously on the device surface at the next synchronisation.
 * Non-finite sample values are not errors: that sample's lnL is NaN, and so is
 * the ln Z of its point.  lnw = -inf excludes a sample from ln Z.
 */
#ifndef RIFT_ILE_H
#define RIFT_ILE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RIFT_ILE_VERSION 2
#define RIFT_ILE_MAX_DET 8   /* detectors per point */
#define RIFT_ILE_MAX_MODES 25 /* modes per point */
#define RIFT_ILE_MAX_NT (1 << 26) /* Q samples per mode and detector */
#define RIFT_ILE_MAX_L 8     /* largest l of a mode; |m| <= l */

typedef enum {
  RIFT_OK = 0,
  RIFT_EINVAL = -1,      /* bad argument (null pointer, size or mode out of range) */
  RIFT_EDEVICE = -2,     /* a HIP runtime call failed */
  RIFT_ENOMEM = -3,      /* device or host allocation failed */
  RIFT_EUNSUPPORTED = -4, /* valid request this library does not implement */
  RIFT_ESCRATCH = -5      /* rift_ile_lnZ_noalloc: the request needs more device memory than
                             its fixed scratch (RIFT_ILE_NOALLOC_SCRATCH_BYTES) */
} rift_status;

typedef enum {
  RIFT_FP64 = 0,  /* every step in IEEE double */
  RIFT_MIXED = 1, /* FP32 pass with an a-priori error bound b_i per sample
                     (angles reduced and sky frame, arrival times and the sum
                     over detectors kept in FP64), then an FP64 recompute of
                     every sample whose bound exceeds 1e-4 nats and that can
                     matter: for ln Z, every one that can weigh more than
                     e^-(ln N + 12) of the best; for rift_ile_lnL, every one
                     that can lie within 20 nats of the best.  FP64 log-sum-exp */
  RIFT_FP32 = 2   /* rift_ile_lnL only: the FP32 pass alone, every value within
                     its returned bound b_i of the FP64 result */
} rift_precision;

/* Coordinates of rows 3 and 6 of theta in the gradient entry points (a
 * bitwise or; the gradient is taken in the same coordinates). */
#define RIFT_COORD_COS_INCL 1 /* row 3 holds cos(incl) instead of incl */
#define RIFT_COORD_LN_DIST 2  /* row 6 holds ln(dist) instead of dist */

/* One intrinsic point lambda: the precomputed arrays of Eq. (QUV) and the
 * detector network. */
typedef struct {
  int32_t n_det;            /* K, 1..RIFT_ILE_MAX_DET */
  int32_t n_modes;          /* M, 1..RIFT_ILE_MAX_MODES */
  int32_t n_t;              /* samples of Q per mode and detector, 4 .. RIFT_ILE_MAX_NT */
  const int32_t *lm;        /* HOST [M][2]: (l, m), 2 <= l <= RIFT_ILE_MAX_L, |m| <= l, no repeats */
  double t0;                /* time of Q sample 0 (s) */
  double dt;                /* Q sample spacing (s), > 0 */
  const double *Q;          /* DEVICE [K][M][n_t] complex: Q_{k,lm}(t_j), paper index order */
  const double *U;          /* DEVICE [K][M][M] complex, U_{k,lm,l'm'}, Hermitian (not checked) */
  const double *V;          /* DEVICE [K][M][M] complex, V_{k,lm,l'm'}, symmetric (not checked) */
  const double *det_tensor; /* HOST [K][3][3] response tensor D_k, symmetric */
  const double *det_pos;    /* HOST [K][3] detector position / c (light-seconds) */
  double gmst_rad;          /* sidereal angle of the static response (rad) */
  double d_ref;             /* D_ref of Eq. (strain_mode), same unit as dist */
} rift_ile_point;

/* theta layout used by every entry point: DEVICE, structure of arrays
 * [7][n] doubles: ra, dec, psi, incl, phiref, tref (s), dist (the gradient
 * entry points take rows 3 and 6 in the coordinates their `coords` names). */

/* lnL of n samples of one point, Eq. (def:lnL:Decomposed).
 * lnL: DEVICE [n] output.  lnL_bnd: DEVICE [n] output or NULL: an upper bound
 * on |lnL_i - lnL_i(FP64)| per sample (0 for RIFT_FP64 and for every value
 * recomputed in FP64).  precision: RIFT_FP64; RIFT_MIXED (every sample that
 * can lie within 20 nats of the largest lnL is within 1e-4 of its FP64 value,
 * every other one within its bound); RIFT_FP32 (no recompute).
 * n == 0 is a no-op. */
int rift_ile_lnL(const rift_ile_point *pt, int64_t n, const double *theta, double *lnL,
                 double *lnL_bnd, int precision, void *stream);

/* ln Z and n_eff of n_points intrinsic points, Eqs. (lnL:MonteCarlo), (neff).
 * n_per_point: HOST [n_points], each >= 1; the samples of point p are the
 * n_per_point[p] consecutive columns of theta after those of points < p.
 * theta: DEVICE [7][N] with N = sum(n_per_point).  lnw: DEVICE [N] or NULL
 * (all zero).  lnZ, neff: DEVICE [n_points] outputs (neff may be NULL).
 * lnL: DEVICE [N] output of every sample's lnL, or NULL.
 * precision: RIFT_FP64 or RIFT_MIXED.  All points are evaluated by one launch
 * of the likelihood kernel (tiles of (point, sample block)). */
int rift_ile_lnZ(const rift_ile_point *pts, int32_t n_points, const int64_t *n_per_point,
                 const double *theta, const double *lnw, double *lnZ, double *neff, double *lnL,
                 int precision, void *stream);

/* lnL and its gradient for n samples of one point (Sec. "The differentiable
 * likelihood").  theta: DEVICE [7][n], rows 3 and 6 in the coordinates
 * `coords` (0: incl, dist; RIFT_COORD_COS_INCL: cos(incl); RIFT_COORD_LN_DIST:
 * ln(dist)).  grad: DEVICE [7][n] output, d lnL / d(ra, dec, psi, row 3,
 * phiref, tref, row 6) in those same coordinates; lnL: DEVICE [n] or NULL.
 * A cos(incl) outside [-1, 1] gives NaN lnL and gradient for that sample; at
 * cos(incl) = +-1 the cos(incl) derivative is infinite (or NaN) wherever the
 * incl derivative is not zero.  precision: RIFT_FP64 (RIFT_MIXED and
 * RIFT_FP32 return RIFT_EUNSUPPORTED: the gradient is FP64 only).  A batch
 * that cannot give every CU 256 samples is evaluated 16 lanes per sample, a
 * larger one a lane per sample (the two differ only in rounding order). */
int rift_ile_grad(const rift_ile_point *pt, int64_t n, const double *theta, int coords, double *lnL,
                  double *grad, int precision, void *stream);

/* ------------------------------------------------------------------------ */
/* Plans: points prepared once (repacked tables, harmonic-basis coefficients,
 * launch configuration), then evaluated many times without any allocation,
 * host synchronisation or host-to-device copy, so that the evaluation calls
 * can be captured into a HIP graph.                                          */
typedef struct rift_ile_plan_s *rift_ile_plan;

/* Prepare n_points points for batches whose point p has n_per_point[p]
 * samples (HOST array, each >= 1).  Enqueues the preparation on `stream`
 * (device memory for the plan is allocated synchronously).  *out receives the
 * plan.  The initial launch shape is {256, 4, 0, 0}, or for a batch too small
 * to give every CU two 1024-sample tiles, one-block tiles of 64 to 256 samples
 * (rift_ile_plan_get_config reports it). */
int rift_ile_plan_create(const rift_ile_point *pts, int32_t n_points, const int64_t *n_per_point,
                         int precision, void *stream, rift_ile_plan *out);

/* ln Z / n_eff of every point of the plan for one batch laid out as in
 * rift_ile_lnZ.  lnL, lnL_bnd: DEVICE [N] or NULL: every sample's lnL and its
 * a-priori bound on |lnL_i - lnL_i(FP64)| (0 for FP64 values: RIFT_FP64, and
 * the samples RIFT_MIXED recomputed).  lnZ_err: DEVICE [n_points] or NULL,
 * receives an upper bound on |ln Z - ln Z_FP64| (RIFT_MIXED) or 0 (RIFT_FP64). */
int rift_ile_plan_lnZ(rift_ile_plan plan, const double *theta, const double *lnw, double *lnZ,
                      double *neff, double *lnL, double *lnL_bnd, double *lnZ_err, void *stream);

/* lnL (may be NULL) and gradient of n samples of point `point` of the plan;
 * theta, coords and grad as in rift_ile_grad (FP64 whatever the plan's
 * precision). */
int rift_ile_plan_grad(rift_ile_plan plan, int32_t point, int64_t n, const double *theta, int coords,
                       double *lnL, double *grad, void *stream);

/* Autotuner: time the candidate launch shapes on this batch and keep the
 * fastest (synchronises `stream`; not capturable). Returns the chosen index. */
int rift_ile_plan_tune(rift_ile_plan plan, const double *theta, const double *lnw, void *stream);

/* Launch shape of the plan: threads per block, samples per tile, persistent
 * blocks per CU (0: one block per tile, the initial shape; a positive value
 * runs a work queue over the tiles, one of the tuner's candidates).  Setting
 * validates on the host: RIFT_EINVAL for values out of
 * range, RIFT_EUNSUPPORTED for a block whose likelihood kernel would need more
 * LDS than one block may hold (16 KiB per wavefront for the data term's read
 * staging, plus a per-lane column for the l <= 8 class). */
typedef struct {
  int32_t block;         /* 64, 128, 256, 512 */
  int32_t tile_blocks;   /* samples per tile = block * tile_blocks */
  int32_t blocks_per_cu; /* persistent grid = blocks_per_cu * CUs; 0 = one block per tile */
  int32_t sort;          /* 1: bin the batch by detector arrival times first so that a
                            wavefront's Q reads share cache lines; 0: evaluate in input order */
} rift_ile_config;
int rift_ile_plan_get_config(rift_ile_plan plan, rift_ile_config *cfg);
int rift_ile_plan_set_config(rift_ile_plan plan, const rift_ile_config *cfg);

/* Statistics of the last rift_ile_plan_lnZ call on the plan (synchronises the
 * stream it ran on): samples recomputed in FP64 by the mixed path, summed over
 * points. */
int rift_ile_plan_refined(rift_ile_plan plan, int64_t *n_refined);

/* Timing of the plan's main evaluation kernel (the per-sample likelihood
 * kernel of rift_ile_plan_lnZ, or the gradient kernel of rift_ile_plan_grad):
 * enable != 0 clears the record and starts bracketing every such launch with
 * HIP events on its stream; enable == 0 stops.  _read synchronises on the
 * recorded events and returns the summed kernel time (ms) and the number of
 * launches.  Not for use under graph capture. */
int rift_ile_plan_profile(rift_ile_plan plan, int enable);
int rift_ile_plan_profile_read(rift_ile_plan plan, double *total_ms, int64_t *launches);

int rift_ile_plan_destroy(rift_ile_plan plan);

/* ------------------------------------------------------------------------ */
/* Generalised detector response (Sec. "A generalized detector response"): the
 * mode index widens to the composite index A = (a, lm) and the static antenna
 * factor F_k to a coefficient C~^k_a per composite term, Eq.
 * (slowrot:lnL:Decomposed) / (slowrot:lnL:MatrixForm):
 *   lnL = x Re sum_k sum_a sum_lm conj(C~^k_a Y_lm) Q_{k,a lm}(t_k)
 *       - x^2/4 sum_k [ c_k^H U_k c_k + Re(c_k^T V_k c_k) ],  c_{k,(a,lm)} = C~^k_a Y_lm.
 * RIFT_RESP_ROTATION (Earth rotation, Path A): n_terms = 5, a <-> sidereal
 *   harmonic n = a - 2; C~_n = A_n(dec, psi) e^{i n g(tref)} e^{i n omega (t_k - tref)}
 *   with F_k(g) = sum_n A_n e^{i n g} over the Greenwich hour angle
 *   g(t) = gmst_rad + omega t - ra (Eqs. (slowrot:Fharm), (slowrot:postphase));
 *   the bank's modulation e^{i n omega t} is referenced to the template's own
 *   time, and the delay is held at the arrival time of the sky frame at tref.
 *   omega = 0 with every term's template equal to its mode is the static
 *   likelihood.
 * RIFT_RESP_ARMS (finite arms, Path D): n_terms = p_max + 1 <= 8, a <-> order p;
 *   C~_p = b_p = 1/2 [(x.N)^p e:xx - (y.N)^p e:yy] with the arm unit vectors
 *   x, y of each detector and e = e+ + i ex (Eq. (fsize:bp)); static sky frame;
 *   p_max = 0 is the static likelihood (with det_tensor = (x x^T - y y^T)/2).
 * RIFT_RESP_ROTATION_DELAY (Earth rotation with the delay drift, Path B):
 *   n_terms = 5 (order 0, Path A), 12 (order 1) or 21 (order 2); a <-> (p, n),
 *   p = 0: a = n + 2 (n = -2..2), p = 1: a = 5 + n + 3 (n = -3..3), p = 2:
 *   a = 12 + n + 4 (n = -4..4); the delay tau = -r_k . N over
 *   the hour angle carries the harmonics 0, +-1, so the drift -dt since t_ref
 *   has, in the modulation phase, the three terms -cos(dec) Re(rho e^{i g(tref)})
 *   (m = 0) and cos(dec)/2 (rho e^{i g(tref)})^(+-1 conjugated for m = -1),
 *   rho = r_x + i r_y; C_(p, n) = (1/p!) sum_{n' + m = n} A_n' e^{i n' g(tref)}
 *   [(-dt)^{*p}]_m (Eqs. (slowrot:delay), (slowrot:master)), then the post-phase
 *   e^{i n omega (t_k - tref)}.  The bank's term (p, n) is the p-th time
 *   derivative of the modes, modulated. */
#define RIFT_RESP_ROTATION 1
#define RIFT_RESP_ARMS 2
#define RIFT_RESP_ROTATION_DELAY 3
typedef struct {
  int32_t n_det;            /* K, 1..RIFT_ILE_MAX_DET */
  int32_t n_modes;          /* M, 1..RIFT_ILE_MAX_MODES */
  int32_t n_t;              /* samples per series, 4 .. RIFT_ILE_MAX_NT */
  const int32_t *lm;        /* HOST [M][2] (l, m) as in rift_ile_point */
  double t0, dt;            /* Q grid t_j = t0 + j dt (s) */
  int32_t response;         /* RIFT_RESP_ROTATION, RIFT_RESP_ARMS or RIFT_RESP_ROTATION_DELAY */
  int32_t n_terms;          /* composite terms per detector (5; p_max + 1 <= 8; 5, 12 or 21) */
  const double *Q;          /* DEVICE [K][n_terms][M][n_t] complex: Q_{k,(a,lm)}(t_j) */
  const double *U;          /* DEVICE [K][n_terms M][n_terms M] complex, index a M + i; Hermitian */
  const double *V;          /* DEVICE, same layout; symmetric */
  const double *det_tensor; /* HOST [K][3][3] */
  const double *det_pos;    /* HOST [K][3] light-seconds */
  const double *det_arms;   /* HOST [K][2][3] arm unit vectors x, y (RIFT_RESP_ARMS), else unused */
  double gmst_rad;          /* sidereal angle at t = 0 (rad) */
  double omega;             /* sidereal rate (rad/s), the rotation responses; |omega| |det_pos[k]| <= 1
                               for every detector (the turn over the light-travel time, at most
                               one radian: 1e4 times the Earth's), else RIFT_EINVAL */
  double d_ref;
} rift_ile_point_wide;

/* lnL of n samples (theta DEVICE [7][n] as for rift_ile_lnL) in FP64; lnL:
 * DEVICE [n].  Same errors and non-finite semantics as rift_ile_lnL.  Both
 * calls enqueue on `stream` and return: the host arrays of *pt are read
 * before return; Q, U, V, theta and lnw must stay valid until the stream has
 * run the work.  Per call the library takes stream-ordered scratch
 * (hipMallocAsync / hipFreeAsync on `stream`) for U and V packed in the
 * order of the contraction, 32 K n_terms (n_terms + 1) / 2 C^2 bytes with
 * C = 5, 12 or 25 the mode capacity at or above M, and 16 bytes per 256
 * samples for ln Z; RIFT_ENOMEM when that fails. */
int rift_ile_wide_lnL(const rift_ile_point_wide *pt, int64_t n, const double *theta, double *lnL,
                      void *stream);
/* ln Z and n_eff (DEVICE [1] each, neff may be NULL) of n >= 1 samples with
 * weights lnw (DEVICE [n] or NULL), Eqs. (lnL:MonteCarlo), (neff); lnL:
 * DEVICE [n] or NULL. */
int rift_ile_wide_lnZ(const rift_ile_point_wide *pt, int64_t n, const double *theta, const double *lnw,
                      double *lnZ, double *neff, double *lnL, void *stream);

/* ------------------------------------------------------------------------ */
/* Direct marginalisation over distance (Sec. "Distance: locating a moving
 * peak"): lnL is exactly K x - R x^2 / 2 in x = d_ref / D (Eq. (ap:dexp)), so
 * the likelihood marginalised over the distance prior,
 *   L_d = int dD p(D) e^{lnL(D)},
 * is taken per sample by an adaptive Gauss-Hermite rule centred on the peak
 * x* = K / R and scaled by sigma_x = R^{-1/2} (Eqs. (ap:dpeak), (ap:dgh)):
 *   ln L_d = K^2 / 2R + ln sigma_x + ln sum_i W_i p_x(x* + xi_i sigma_x),
 * with (xi_i, W_i) the n_nodes-point rule of the weight e^{-xi^2/2} and
 * p_x the prior p(D) = 3 D^2 / (d_max^3 - d_min^3) on [d_min, d_max] (uniform
 * in Euclidean volume) written in x.  No node inside the prior gives -inf
 * (the rule's answer for a peak far outside it); R <= 0, which only rounding
 * produces where the model has no power (and K = 0 with it), gives 0 (lnL = 0
 * at every distance); non-finite samples give NaN.  The rule resolves the
 * integral where sigma_x is small against the prior's extent in x; a sample
 * with almost no model power (sigma_x far wider than the prior) may get -inf. */
typedef struct {
  double d_min, d_max; /* prior support (Mpc, the unit of d_ref): 0 < d_min < d_max <= 1e60 */
  int32_t n_nodes;     /* Gauss-Hermite nodes, 1 .. 64 */
} rift_ile_dist_prior;

/* ln L_d per sample (lnLd: DEVICE [N] or NULL) and, per point, ln Z_d =
 * ln[(1/n) sum_i e^{ln L_d,i + lnw_i}] with n_eff (Eqs. (lnL:MonteCarlo),
 * (neff)) over the plan's batch.  theta as for rift_ile_plan_lnZ; its distance
 * row is not read.  FP64 whatever the plan's precision; the plan's launch
 * shape and binning apply.  Enqueues and returns (capturable); the rule is
 * computed on the host when n_nodes changes.  RIFT_EINVAL for a bad prior. */
int rift_ile_plan_lnZ_dmarg(rift_ile_plan plan, const double *theta, const double *lnw,
                            const rift_ile_dist_prior *prior, double *lnZ, double *neff, double *lnLd,
                            void *stream);

/* The gradient of the likelihood marginalised over distance, for samplers
 * that move in the six other coordinates (Sec. "Sampler menu": a chain with
 * distance marginalised).  lnL is exactly K x - R x^2 / 2 in x = d_ref / D
 * (Eq. (ap:dexp)), so d ln L_d = <x> grad K - <x^2> grad R / 2 under the
 * distance posterior; one pass of the gradient's adjoint forms K, R and their
 * gradients, and its last step takes the moments from the same adaptive
 * Gauss-Hermite rule as rift_ile_plan_lnZ_dmarg (node weights
 * W_i p_x(x_i)).  This is the derivative of the integral; it differs from
 * the rule's own derivative by the rule's error (small where the distance
 * posterior is narrow against the prior's variation).  Where the model has
 * no power (R <= 0) the moments are the prior's; a sample with no node
 * inside the prior gets ln L_d = -inf and derivative 0; a non-finite sample
 * NaN.  theta: DEVICE [7][n] in the samplers' coordinates (ra, dec, psi,
 * cos incl, phiref, tref, -; row 6 not read); lnLd: DEVICE [n] or NULL;
 * grad: DEVICE [7][n] output, d ln L_d / d(ra, dec, psi, cos incl, phiref,
 * tref) and 0 in row 6.  `point` is a point of the plan.  RIFT_EINVAL: as
 * rift_ile_plan_lnZ_dmarg's prior, n < 0, a bad point, null or misaligned
 * pointers.  Enqueues and returns; no scratch. */
int rift_ile_plan_grad_dmarg(rift_ile_plan plan, int32_t point, int64_t n, const double *theta,
                             const rift_ile_dist_prior *prior, double *lnLd, double *grad, void *stream);

/* Direct marginalisation over geocentric time by the fixed-spacing rule
 * (Sec. "Time: representing the correlations and placing the integration
 * nodes", Eq. (ap:tfixed)) under a prior uniform on the window
 * [t_start, t_start + (n_t - 1) h]:
 *   ln L_t = ln[(h / T) sum_k w_k e^{lnL(t_start + k h)}],  T = (n_t - 1) h,
 * with composite Simpson weights w = (1, 4, 2, 4, ..., 2, 4, 1) / 3 (n_t odd).
 * The model-norm term is evaluated once per sample, the data term at each
 * time.  The rule resolves the peak only where h is below its width,
 * 1 / (2 pi rho sigma_f) (Eq. (ap:sigmat)); choosing h is the caller's. */
typedef struct {
  double t_start, h; /* first time (s, the axis of t_ref) and spacing (s), h > 0 */
  int32_t n_t;       /* odd, 3 .. 1000001 */
} rift_ile_time_rule;

/* ln L_t per sample (lnLt: DEVICE [N] or NULL) and, per point, ln Z_t and
 * n_eff over the plan's batch, as rift_ile_plan_lnZ_dmarg; theta's t_ref row
 * is not read.  FP64; enqueues and returns (capturable); RIFT_EINVAL for a
 * bad rule.  Cost per sample: one model-norm term and n_t data terms. */
int rift_ile_plan_lnZ_tmarg(rift_ile_plan plan, const double *theta, const double *lnw,
                            const rift_ile_time_rule *rule, double *lnZ, double *neff, double *lnLt,
                            void *stream);

/* Marginalisation over geocentric time by the band-limited full-window rule
 * (Eq. (ap:tband)) under a prior uniform on the node window
 * [t_start, t_start + (n_t - 1) h].  At fixed other parameters the exponent is
 * x kappa(t) - x^2 quad with kappa the data term, which is band limited: it
 * is taken at the n_t nodes t_start + j h (the data term's only evaluations),
 * reconstructed at n_fine points per node interval by the sinc series
 *   kappa(t) ~ sum_j kappa_j sinc((t - t_j) / h),
 * and the exponentials at the (n_t - 1) n_fine + 1 fine points are summed by
 * the trapezoid rule (ends 1/2):
 *   ln L_t = ln[(1 / ((n_t - 1) n_fine)) sum_k w_k e^{l_k}].
 * The series is truncated to the window, so h must sample kappa's band
 * (h below 1 / (2 f_max)) and the window should hold the correlation's
 * support; n_fine resolves the exponential's peak (n_fine >~ h / sigma_t). */
typedef struct {
  double t_start, h; /* first node (s, the axis of t_ref) and node spacing (s), h > 0 */
  int32_t n_t;       /* nodes, 2 .. 64 */
  int32_t n_fine;    /* fine intervals per node interval, 1 .. 64 */
} rift_ile_band_rule;

/* ln L_t per sample (lnLt: DEVICE [N] or NULL) and, per point, ln Z_t and
 * n_eff over the plan's batch, as rift_ile_plan_lnZ_tmarg; theta's t_ref row is
 * not read.  FP64; enqueues and returns, with stream-ordered scratch of at
 * most 8 (n_t N + 127 n_fine + N) bytes; RIFT_EINVAL for a bad rule.  Cost per
 * sample: one model-norm term, n_t data terms, then ((n_t - 1) n_fine + 1)
 * sums of at most 64 products and one exp each. */
int rift_ile_plan_lnZ_tband(rift_ile_plan plan, const double *theta, const double *lnw,
                            const rift_ile_band_rule *rule, double *lnZ, double *neff, double *lnLt,
                            void *stream);

/* Direct marginalisation over polarisation (Sec. "Angles: finite harmonic
 * content"): at fixed other parameters the complex antenna factor carries
 * e^{-2 i psi}, so lnL is exactly q(u) = a + Re(c1 e^{iu}) + Re(c2 e^{2iu})
 * in u = 2 psi (Eq. (ap:psiexp)), with c1 from the data term and a, c2 from the
 * model norm, all from one gather and one contraction per sample.  With psi
 * uniform on [0, pi):
 *   RIFT_PSI_TRAPEZOID: L_psi = (1/n) sum_j e^{q(2 pi j / n)}, the periodic
 *     trapezoid rule on n points (the product grid; exact as n grows);
 *   RIFT_PSI_LAPLACE:   L_psi = e^{q(u*)} sqrt(2 pi / A) / (2 pi) at the dominant
 *     maximum u* with A = -q''(u*) (Eq. (ap:psilaplace); relative error O(1/A)),
 *     where A >= 100; a q without such a maximum (weak signal, or two maxima
 *     merging) is integrated by the trapezoid rule on 256 points instead;
 *   RIFT_PSI_CELLS:     the stationary-point cells of Eq. (ap:psicells): the
 *     unit-circle roots of the quartic 2 c2 z^4 + c1 z^3 - conj(c1) z
 *     - 2 conj(c2) (z = e^{iu}, from q' = 0) cut the circle into cells on
 *     which q is monotone, each integrated by 8-point Gauss-Legendre on
 *     sub-intervals sized by its own curvature (2 sigma steps to 8 sigma
 *     from its top, then doubling; sigma = min(A^{-1/2}, width / 8)):
 *     accurate at any amplitude and for several peaks. */
#define RIFT_PSI_TRAPEZOID 0
#define RIFT_PSI_LAPLACE 1
#define RIFT_PSI_CELLS 2
typedef struct {
  int32_t method;   /* RIFT_PSI_TRAPEZOID, RIFT_PSI_LAPLACE or RIFT_PSI_CELLS */
  int32_t n_points; /* trapezoid: 1 .. 65536 points on the circle; ignored otherwise */
} rift_ile_psi_rule;

/* ln L_psi per sample (lnLp: DEVICE [N] or NULL) and, per point, ln Z_psi and
 * n_eff over the plan's batch, as rift_ile_plan_lnZ_dmarg; theta's psi row
 * only sets where the rule's points start (the integral covers the whole
 * period).  FP64; enqueues and returns (capturable); RIFT_EINVAL for a bad
 * rule. */
int rift_ile_plan_lnZ_pmarg(rift_ile_plan plan, const double *theta, const double *lnw,
                            const rift_ile_psi_rule *rule, double *lnZ, double *neff, double *lnLp, void *stream);

/* Joint marginalisation over the reference phase and polarisation by
 * exact-reconstruction adaptive integration (ERAI; Sec. "Angles: finite
 * harmonic content", Eqs. (ap:angleharm), (ap:nyquist)), with phiref uniform
 * on [0, 2 pi) and psi on [0, pi).  At fixed sky, inclination, time and
 * distance, lnL is a finite trigonometric polynomial in (phiref, 2 psi): of
 * degree 2 in 2 psi and 2 m_max in phiref (m_max the largest |m| of the
 * plan's modes).  Its coefficients are fixed exactly by the data term at
 * 2 m_max + 1 and the model norm at 4 m_max + 1 phases (one gather of the
 * correlation tables per data-term phase, the psi dependence analytic); the
 * exponential of the reconstructed model is then averaged over the periodic
 * grid of n_phi x n_psi offsets from the sample's (phiref, psi):
 *   ln L = ln[(1 / (n_phi n_psi)) sum_{a, b} e^{lnL(phi + 2 pi a / n_phi,
 *                                                 psi + pi b / n_psi)}].
 * The grid is the caller's to size from the signal's amplitude (its peak
 * narrows as 1 / rho). */
typedef struct {
  int32_t n_phi, n_psi; /* fine grid, 1 .. 4096 each */
} rift_ile_angle_rule;

/* ln L per sample (lnLa: DEVICE [N] or NULL) and, per point, ln Z and n_eff
 * over the plan's batch; theta's phiref and psi rows set where the grid
 * starts.  FP64; enqueues and returns, with stream-ordered scratch of
 * 8 ((4 m_max + 2 + 3 (4 m_max + 1)) N + 26 n_phi + 4 n_psi + N) bytes at
 * most; RIFT_EINVAL for a bad rule, RIFT_EUNSUPPORTED for modes with
 * |m| > 4.  Cost per sample: 2 m_max + 1 data terms, 4 m_max + 1 model-norm
 * contractions, then n_phi n_psi exponentials. */
int rift_ile_plan_lnZ_erai(rift_ile_plan plan, const double *theta, const double *lnw,
                           const rift_ile_angle_rule *rule, double *lnZ, double *neff, double *lnLa, void *stream);

/* The n-point Gauss-Hermite rule of the weight e^{-x^2/2} (1 <= n <= 64) that
 * the distance marginal uses: HOST nodes[n] ascending and weights[n]. */
int rift_ile_gauss_hermite(int n, double *nodes, double *weights);

/* ------------------------------------------------------------------------ */
/* Fourier refinement of sampled series, Eq. (q-time-pregrid): each series of
 * n native samples (spacing h) is extended by its reversed copy to a
 * continuous period of 2n samples, its spectrum zero-padded by r (the Nyquist
 * bin split in halves) and transformed back, keeping the (n - 1) r + 1 samples
 * at spacing h / r that span the original window; the nodes are reproduced.
 * Computed as the equivalent real interpolation operator (a periodic sinc of
 * period 2n in closed form) applied to every series.
 * q: DEVICE [n_series][n] complex; fine: DEVICE [n_series][(n - 1) r + 1]
 * complex (not overlapping q).  2 <= n, 1 <= r <= 64, (n - 1) r + 1 <= 2^28.
 * Enqueues and returns; stream-ordered scratch of 8 r (3n - 1) bytes
 * (hipMallocAsync / hipFreeAsync on `stream`). */
int rift_ile_pregrid(const double *q, int64_t n_series, int32_t n, int32_t r, double *fine, void *stream);

/* ------------------------------------------------------------------------ */
/* Leapfrog drift for gradient-based samplers in the coordinates of
 * RIFT_COORD_COS_INCL | RIFT_COORD_LN_DIST (Sec. "Sampling the
 * differentiable extrinsic likelihood"): theta[a][i] += step[a] p[a][i] for
 * the seven rows, then cos incl (row 3) folded back into [-1, 1] by
 * reflection, p[3][i] changing sign after an odd number of folds (the
 * reversible, volume-preserving treatment of the bounded coordinate).
 * theta, p: DEVICE [7][n] (updated in place); step: HOST [7].  Enqueues and
 * returns; capturable.  Non-finite values pass through unchanged. */
int rift_ile_leapfrog_drift(int64_t n, double *theta, double *p, const double *step, void *stream);

/* One Metropolis-adjusted Hamiltonian Monte Carlo transition per chain on the
 * likelihood's gradient (Sec. "Sampling the differentiable extrinsic
 * likelihood"), in the sampler coordinates (ra, dec, psi, cos incl, phiref,
 * tref, ln dist), with the random numbers supplied by the caller:
 *   p = z / sigma (mass diag(sigma^-2)); n_leapfrog leapfrog steps of size
 *   eps on U = -lnL - ln prior (half kick, rift_ile_leapfrog_drift with
 *   step eps sigma^2, gradient by rift_ile_plan_grad, half kick); accepted
 *   when ln u < H0 - H1, H = U + sum_a sigma_a^2 p_a^2 / 2.
 * The prior is the isotropic, uniform-in-volume one of the samples: in these
 * coordinates ln cos dec + 3 ln D on the box |dec| < pi/2, |cos incl| <= 1,
 * t_min <= tref <= t_max, d_min <= D <= d_max (ra, psi, phiref periodic), so
 * a proposal outside the box is rejected.
 * theta: DEVICE [7][n], the chains' states (updated: the proposal where
 * accepted, else unchanged); z: DEVICE [7][n] standard normals; u: DEVICE [n]
 * uniforms in (0, 1); sigma: HOST [7] > 0; lnL: DEVICE [n] or NULL (lnL at the
 * returned states); accepted: DEVICE [n] or NULL (1 / 0).  `point` is a point
 * of the plan (its tables give the likelihood).  Host arguments are checked
 * before any device work (RIFT_EINVAL: n < 0, eps not finite and > 0,
 * n_leapfrog outside [1, 10000], sigma not finite and > 0, an empty box,
 * d_min <= 0, null or misaligned pointers); n = 0 is a no-op.  Enqueues and
 * returns; stream-ordered scratch of 192 n bytes. */
typedef struct {
  double t_min, t_max; /* the tref box (s) */
  double d_min, d_max; /* the distance box (Mpc), 0 < d_min < d_max */
} rift_ile_hmc_prior;
int rift_ile_plan_hmc(rift_ile_plan plan, int32_t point, int64_t n, double *theta, const double *z, const double *u,
                      const double *sigma, double eps, int32_t n_leapfrog, const rift_ile_hmc_prior *prior,
                      double *lnL, int32_t *accepted, void *stream);

/* The same transition on the tempered target L^beta p of Eq.
 * (sampler-menu:tempered-target), 0 <= beta <= 1 (the moves of an SMC
 * ladder): U = -beta lnL - ln prior; lnL (the output) stays the untempered
 * likelihood.  beta = 1 is rift_ile_plan_hmc bit for bit.  RIFT_EINVAL for
 * beta outside [0, 1], otherwise as rift_ile_plan_hmc. */
int rift_ile_plan_hmc_tempered(rift_ile_plan plan, int32_t point, int64_t n, double *theta, const double *z,
                               const double *u, const double *sigma, double eps, int32_t n_leapfrog,
                               const rift_ile_hmc_prior *prior, double beta, double *lnL, int32_t *accepted,
                               void *stream);

/* One No-U-Turn transition per chain (Sec. "Sampler menu": multinomial NUTS
 * with the generalised criterion) on the tempered target L^beta p, in the
 * coordinates and with the prior box of rift_ile_plan_hmc, the random numbers
 * the caller's: momenta p = z / sigma; at depth j the trajectory doubles in
 * direction -1 if dirs[j] < 1/2 else +1 by a subtree of 2^j leapfrog steps
 * (size eps) from that edge.  Within a subtree the leaves are built outward;
 * leaf k (weight e^{-H}) becomes the subtree's candidate when the next of
 * `leaves` is below its share of the subtree's weight so far, and every
 * completed aligned block of 2, 4, .. leaves is checked for a U-turn
 * (sigma^2 p_edge . rho > 0 at both edges, rho the block's momentum sum).  A
 * U-turn inside the subtree, or a leaf whose energy exceeds the start's by
 * 1000, discards it and ends the transition; otherwise its candidate
 * replaces the transition's with probability min(1, W_subtree / W) against
 * merges[j], and a U-turn of the whole trajectory ends it.  At most
 * max_depth (1 .. 10) doublings.
 * theta: DEVICE [7][n] (replaced by the transitions' draws); z: DEVICE [7][n];
 * dirs, merges: DEVICE [max_depth][n]; leaves: DEVICE [2^max_depth - 1][n]
 * (uniforms); sigma: HOST [7]; lnL: DEVICE [n] or NULL (lnL at the draws);
 * info: DEVICE int32 [3][n] or NULL (doublings completed, leapfrog steps,
 * divergent).  The chains step in lockstep, one gradient launch per step for
 * the batch; the call synchronises `stream` every fourth step to stop once no
 * chain is active.  Stream-ordered scratch of 8 (112 + 14 max_depth) n bytes
 * and a little more.  A start whose energy is not finite is returned
 * unchanged.  RIFT_EINVAL as rift_ile_plan_hmc_tempered, and for max_depth
 * outside 1 .. 10. */
int rift_ile_plan_nuts(rift_ile_plan plan, int32_t point, int64_t n, double *theta, const double *z,
                       const double *dirs, const double *merges, const double *leaves, const double *sigma,
                       double eps, int32_t max_depth, const rift_ile_hmc_prior *prior, double beta, double *lnL,
                       int32_t *info, void *stream);

/* HMC and NUTS transitions on the likelihood marginalised over distance
 * (Sec. "Sampler menu": a chain with distance marginalised): as
 * rift_ile_plan_hmc_tempered and rift_ile_plan_nuts, with the target
 * L_d^beta p, L_d the marginal of rift_ile_plan_lnZ_dmarg under the distance
 * prior `dprior` and its gradient from rift_ile_plan_grad_dmarg.  The
 * distance row is not part of the target: it carries no momentum (it is
 * returned unchanged), and the prior drops its ln D term and distance box.
 * lnLd: DEVICE [n] or NULL, ln L_d at the returned states.  RIFT_EINVAL as
 * the untempered entries, and for a null or invalid dprior. */
int rift_ile_plan_hmc_dmarg(rift_ile_plan plan, int32_t point, int64_t n, double *theta, const double *z,
                            const double *u, const double *sigma, double eps, int32_t n_leapfrog,
                            const rift_ile_hmc_prior *prior, const rift_ile_dist_prior *dprior, double beta,
                            double *lnLd, int32_t *accepted, void *stream);
int rift_ile_plan_nuts_dmarg(rift_ile_plan plan, int32_t point, int64_t n, double *theta, const double *z,
                             const double *dirs, const double *merges, const double *leaves, const double *sigma,
                             double eps, int32_t max_depth, const rift_ile_hmc_prior *prior,
                             const rift_ile_dist_prior *dprior, double beta, double *lnLd, int32_t *info,
                             void *stream);

/* One update of an SMC tempering ladder (Sec. "Sampler menu",
 * Eq. (sampler-menu:smc-update)) over n weighted particles: with W the
 * normalised weights from lnW (DEVICE [n], any normalisation; -inf excludes a
 * particle) and lnL (DEVICE [n]) their log-likelihoods, the next rung is the
 * largest beta' in (beta, 1] whose incremental weights r = L^(beta' - beta)
 * keep the conditional effective-size fraction (sum W r)^2 / sum W r^2 at or
 * above `target` (0 < target <= 1), or 1 if the whole remaining step does;
 * then ln(Z_beta' / Z_beta) = ln sum W r and lnW is replaced by the normalised
 * ln(W r) (in place).  out: DEVICE [2] = (beta', dlnZ).  The search is a
 * safeguarded Newton iteration on the log fraction (non-increasing in the
 * step), a fixed 40 passes at most, all on the device: enqueues and returns,
 * with stream-ordered scratch of about 50 KB.  A NaN input gives NaN
 * outputs.  RIFT_EINVAL: n < 1, beta outside [0, 1], target outside (0, 1],
 * null or misaligned pointers. */
int rift_ile_smc_reweight(int64_t n, const double *lnL, double *lnW, double beta, double target, double *out,
                          void *stream);

/* Systematic resampling of n particles with one uniform u in [0, 1): draw i
 * takes the first particle whose normalised cumulative weight exceeds
 * (i + u) / n.  lnW: DEVICE [n]; theta_in, theta_out: DEVICE [7][n], distinct,
 * both NULL or both given (theta_out[:, i] = theta_in[:, a_i]); ancestors:
 * DEVICE int64 [n] (a_i) or NULL, not both outputs NULL.  The caller resets
 * the weights to equal afterwards.  Enqueues and returns, with
 * stream-ordered scratch of about 8 n bytes. */
int rift_ile_smc_resample(int64_t n, const double *lnW, double u, const double *theta_in, double *theta_out,
                          int64_t *ancestors, void *stream);

/* The adaptive cloud's random-walk Metropolis move after resampling (Sec.
 * "Mode coverage, adaptive clouds, and evidence": a proposal covariance
 * estimated from the current cloud), one per chain, on the tempered target
 * L^beta p of Eq. (sampler-menu:tempered-target) in the sampler coordinates
 * (ra, dec, psi, cos incl, phiref, tref, ln dist): the proposal
 * c' = c + L z with L L^T = scale cov (Cholesky on the device), accepted when
 * ln u < beta (lnL(c') - lnL(c)) + ln p(c') - ln p(c) with L^0 = 1 and p the
 * prior of rift_ile_plan_hmc (a proposal outside its box, or a NaN, is
 * rejected).  lnL(c') comes from the plan's point `point`.
 * theta: DEVICE [7][n] chain states (updated where accepted); z: DEVICE
 * [7][n] standard normals; u: DEVICE [n] uniforms in (0, 1); cov: DEVICE
 * [7][7] symmetric (the lower triangle is read; e.g. rift_ile_moments of the
 * cloud); lnL: DEVICE [n], lnL at the states on entry and at the returned
 * states on exit; accepted: DEVICE int32 [n] or NULL; status: DEVICE int32
 * [1] or NULL, 0, or 1 when scale cov is not positive definite (then no
 * chain moves).  RIFT_EINVAL: n < 0, beta outside [0, 1], scale not finite
 * and > 0, an empty box or d_min <= 0, null or misaligned pointers.  Enqueues
 * and returns; stream-ordered scratch of 120 n + 256 bytes. */
int rift_ile_plan_rwm(rift_ile_plan plan, int32_t point, int64_t n, double *theta, const double *z, const double *u,
                      const double *cov, double scale, const rift_ile_hmc_prior *prior, double beta, double *lnL,
                      int32_t *accepted, int32_t *status, void *stream);

/* Weighted mean and covariance of a cloud of states (the moments that fit one
 * component of the proposal below; Sec. "Mode coverage, adaptive clouds, and
 * evidence"): with W_i the weights e^{lnw_i} normalised over the cloud (equal
 * when lnw is NULL), mean = sum_i W_i c_i and cov = sum_i W_i (c_i - mean)
 * (c_i - mean)^T, the population form, over the samples of non-zero weight
 * (a sample with lnw = -inf is not read).  c: DEVICE [7][n] in any
 * coordinates (no periodic reduction: pass chain states unwrapped); lnw:
 * DEVICE [n] or NULL; mean: DEVICE [7], cov: DEVICE [7][7] (symmetric)
 * outputs, NaN when no sample has weight (n = 0 included) or a weight is NaN.
 * RIFT_EINVAL: n < 0, null or misaligned pointers.  Enqueues and returns;
 * deterministic; stream-ordered scratch of about 300 bytes per 256 samples
 * (at most 300 KB). */
int rift_ile_moments(int64_t n, const double *c, const double *lnw, double *mean, double *cov, void *stream);

/* Independent draws from a defensive Gaussian-mixture proposal and their
 * importance weights, Eq. (sampler-menu:is): q = alpha p + (1 - alpha)
 * sum_m a_m N_m, with p the samples' prior and N_m the Gaussian of mean
 * mean[m] and covariance scale cov[m] (one component per recovered mode,
 * Sec. "Mode coverage, adaptive clouds, and evidence"), in the sampler
 * coordinates (ra, dec, psi, cos incl, phiref, tref, ln D).
 * The prior is the isotropic, uniform-in-volume one, normalised on the box
 * ra, phiref in [0, 2 pi), psi in [0, pi), |dec| < pi/2, |cos incl| <= 1,
 * tref in [t_min, t_max], D in [d_min, d_max]: ln p = ln cos dec + 3 ln D +
 * const.  ra, psi and phiref are periodic, so N_m is the density of its
 * Gaussian draw taken modulo the periods (the sum over periodic images,
 * truncated where the images left out carry under 2e-19 of the mass per row).
 * Per draw i: u[i] < alpha draws from the prior by its inverse distribution
 * functions of v[:, i] (ra = 2 pi v0, dec = asin(2 v1 - 1), psi = pi v2,
 * cos incl = 2 v3 - 1, phiref = 2 pi v4, tref = t_min + (t_max - t_min) v5,
 * ln D = ln(d_min^3 + v6 (d_max^3 - d_min^3)) / 3); otherwise component m,
 * the first with u[i] < alpha + (1 - alpha)(a_0 + .. + a_m), draws
 * mean[m] + L z[:, i] with L L^T = scale cov[m] (Cholesky), reduced into the
 * box's periods.  lnw[i] = ln p - ln q with q's full density (every
 * component), so that rift_ile_lnZ(theta, lnw) is ln Z_IS = ln (1/N) sum_i
 * L_i p_i / q_i.  A draw outside the box has lnw = -inf and is returned
 * clamped onto it (dec, cos incl, tref, ln D), so its likelihood is finite.
 * theta: DEVICE [7][n] output in the likelihood's coordinates (incl = acos,
 * dist = exp); lnw: DEVICE [n] output; comp: DEVICE int32 [n] or NULL (-1
 * for the prior, else m); z: DEVICE [7][n] standard normals; v: DEVICE
 * [7][n] and u: DEVICE [n] uniforms in [0, 1); status: DEVICE int32 [1] or
 * NULL, set to 0, or to 1 + m for the first refused component.
 * mix->a: HOST [n_comp], each > 0, summing to 1 within 1e-12; mean: DEVICE
 * [n_comp][7]; cov: DEVICE [n_comp][7][7] symmetric (the lower triangle is
 * read).  A component is refused on the device when scale cov[m] is not
 * positive definite or a mean is not finite, or when its marginal width in a
 * periodic row exceeds half the period (|sigma| <= pi for ra and phiref,
 * pi/2 for psi): every lnw and theta is then NaN.  RIFT_EINVAL: n < 0;
 * n_comp outside [0, RIFT_IS_MAX_COMP]; alpha outside [0, 1] (alpha = 1 when
 * n_comp = 0); scale not finite and > 0; an empty box or d_min <= 0; a bad
 * a; rows outside 1 .. 0x7f; null or misaligned pointers.  Enqueues and
 * returns; stream-ordered scratch of 784 bytes per component.
 * A likelihood marginalised over some rows (distance, phiref, psi in the
 * kernel) is normalised over the others: with mix->rows naming the sampled
 * rows S, the components are the Gaussians of those rows (mean and
 * covariance restricted to S, drawn from z at the rows of S), every other
 * row is drawn from the prior by v as a prior draw is, and p and q in the
 * weight are the densities of the rows of S alone (the marginal prior of S;
 * the box and the periodic images of S). */
#define RIFT_IS_MAX_COMP 32
typedef struct {
  int32_t n_comp;     /* components, 0 .. RIFT_IS_MAX_COMP */
  double alpha;       /* the prior's share, 0 <= alpha <= 1 */
  double scale;       /* s > 0, the covariance widening */
  const double *a;    /* HOST [n_comp] component weights */
  const double *mean; /* DEVICE [n_comp][7] */
  const double *cov;  /* DEVICE [n_comp][7][7] */
  int32_t rows;       /* bit j set when row j is sampled by the components, 1 .. 0x7f (0x7f: all) */
} rift_ile_mixture;
int rift_ile_mixture_is(int64_t n, const rift_ile_mixture *mix, const rift_ile_hmc_prior *prior, const double *z,
                        const double *v, const double *u, double *theta, double *lnw, int32_t *comp,
                        int32_t *status, void *stream);

/* ------------------------------------------------------------------------ */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): rift_ile_lnZ with
 * the same arguments, semantics and results (the same kernels and launch
 * shape), whose working memory -- repacked tables, basis coefficients, tiles,
 * partial sums and, in mixed precision, the per-sample scratch of the
 * recompute -- lives in a fixed device array of RIFT_ILE_NOALLOC_SCRATCH_BYTES
 * that the library holds on each GPU it runs on until the process ends.  It
 * calls no hipMalloc or hipFree (the host bookkeeping uses the host heap).
 * A request whose working memory does not fit returns RIFT_ESCRATCH before
 * anything is enqueued; about 7 MB serve a 3-detector, 21-mode point of 6554
 * samples per series in FP64 (16 more bytes per sample in mixed precision).
 * Every call on one GPU uses that GPU's one array: calls that overlap on a
 * GPU (other threads, other streams) race and must be serialised by the
 * caller.  Synchronises `stream` before returning, like rift_ile_lnZ. */
#define RIFT_ILE_NOALLOC_SCRATCH_BYTES (64u << 20)
int rift_ile_lnZ_noalloc(const rift_ile_point *pts, int32_t n_points, const int64_t *n_per_point,
                         const double *theta, const double *lnw, double *lnZ, double *neff, double *lnL,
                         int precision, void *stream);

const char *rift_ile_strerror(int status);
int rift_ile_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RIFT_ILE_H */
