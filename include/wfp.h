/*
 * wfp.h -- C ABI of the MI355X (gfx950) FP64 implementation of the
 * windowed Fourier projection (WFP) march for point scatterers on a string
 * (Al Hassanieh, Barnett, Greengard, "A fast algorithm for the wave equation
 * using time-windowed Fourier projection").
 *
 * Problem (Section 1, eqs. (WE)-(kink), (gj); periodic box: Section 2,
 * eq. (peri)): M springs at x_j in [-pi, pi) with stiffness beta_j > 0 are
 * hit by the incident field u_inc(x, t) = f(x - t).  The scattered field is
 * the single-layer potential of densities sigma_j(t) (eqs. (singleLayerSol),
 * (SLPp)), which solve the Volterra system (IEfree)/(periodicIE)
 *     -sigma_j(t) - beta_j u(x_j, t) = g_j(t) = beta_j f(x_j - t).
 *
 * Method (Sections 2-4): u = u_L + u_H with the Kaiser-Bessel blending
 * window phi of timescale delta = W dt (eqs. (phi), (b)); u_H is the
 * truncated Fourier series sum_{|k|<=K} alpha_k e^{-ikx} (eq. (historySol1))
 * advanced by the exact propagator of the Lemma with the trapezoid driving
 * terms of eq. (hkcompdisc); the densities' spectra S_k (eq. (densco)) come
 * from a type-1 NUFFT and u_H at the scatterers from a type-2 NUFFT; u_L is
 * the N_L-node Gauss-Legendre rule with p-point interpolation of Section 4.1;
 * each step solves the sparse system (linearSystem).  Free space adds the
 * radiation-boundary projection of Section 4.4.
 *
 * Conventions
 *   - Time levels t_L = L dt, L = 0, 1, 2, ...  A "step" computes one new
 *     level sigma^L from the levels before it (zero history before L = 0,
 *     so the first step solves (I + S) sigma^0 = -g^0).
 *   - All problem data passed to wfp_plan_create are HOST pointers and are
 *     copied; the caller may free them after the call returns.
 *   - All arrays passed to wfp_run / wfp_get_state / wfp_set_state are
 *     DEVICE pointers (caller-owned, on the plan's device); these calls are
 *     asynchronous and ordered on the plan's stream.
 *   - Per-scatterer arrays are in the caller's original order.
 *   - Complex arrays are interleaved (re, im) doubles.
 *   - No C++ exception crosses this boundary; every call returns a status.
 *     On error, wfp_last_error() returns a thread-local message.
 */
#ifndef WFP_H
#define WFP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t wfp_status;

#define WFP_OK 0
#define WFP_EINVAL (-1)     /* bad argument: M <= 0, dt <= 0, odd p, NaN input, NULL pointer */
#define WFP_EDOMAIN (-2)    /* K dt > pi, delta = W dt >= pi, free-space point outside Omega,
                               unsupported size (e.g. transform too long for one workgroup) */
#define WFP_ENOMEM (-3)     /* device or host allocation failed */
#define WFP_EHIP (-4)       /* a HIP runtime call failed */
#define WFP_ESTATE (-5)     /* call not valid in the plan's current state */
#define WFP_ENONFINITE (-6) /* check_finite: the newest densities or the mode state hold NaN or Inf */

#define WFP_PERIODIC 0      /* periodic box [-pi, pi) (Section 2) */
#define WFP_FREE_SPACE 1    /* free space via outgoing windowing (Section 4.4) */

#define WFP_ABI_VERSION 7

typedef struct wfp_plan wfp_plan;

/* Problem statement (Section 1).  Host pointers, copied by wfp_plan_create. */
typedef struct {
  int64_t M;               /* number of springs, >= 1 */
  const double* x;         /* [M] positions in [-pi, pi); free space: inside Omega */
  const double* beta;      /* [M] stiffnesses > 0 */
  int32_t boundary;        /* WFP_PERIODIC or WFP_FREE_SPACE */
  int32_t n_packets;       /* 1..64 */
  const double* packets;   /* [n_packets][5] = (amp, centre, width, omega, phase):
                              f(s) = sum amp exp(-(s-centre)^2/(2 width^2)) cos(omega (s-centre) + phase);
                              periodised over 2 pi in the periodic box */
  int64_t R;               /* number of receivers (extra targets, Section 3.1), >= 0 */
  const double* x_recv;    /* [R] receiver positions (may be NULL when R == 0) */
} wfp_problem;

/* Discretisation parameters.  A zero field selects the default shown. */
typedef struct {
  double dt;               /* time step, > 0 (required) */
  double eps_window;       /* window tolerance eps; b = ln(1/eps)           [1e-12] */
  double gamma;            /* Nyquist fraction lost to windowing (Remark r:gamma)  [0.5] */
  int32_t W;               /* window length in steps, delta = W dt          [round(2b/(pi gamma))] */
  int32_t p;               /* interpolation order (even)                     [8] */
  int64_t K;               /* highest Fourier mode: periodic floor(pi/dt); free space the largest
                              K <= pi/dt with 2K = 2^a 5^b                     [rule] */
  int32_t n_gl_local;      /* Gauss-Legendre nodes of the local rule N_L     [W] */
  int32_t n_gl_pq;         /* Gauss-Legendre nodes for p_k, q_k  N_g         [32] */
  int32_t rbc_period;      /* free space: levels between RBC projections     [ceil(W h/dt), h = pi/K] */
  int32_t nufft_width;     /* spreading-kernel width in fine-grid points     [16] */
  int32_t solve_iters;     /* Jacobi sweeps of the per-step solve            [from a contraction bound] */
  int32_t checkpoint_every;/* > 0: wfp_run stores the march state every this many levels (for
                              wfp_adjoint, which replays each segment from its checkpoint);
                              -C < 0: wfp_run records every level's densities and forward
                              derivative term (16 M bytes a level, in blocks of C levels, C
                              <= 2^20; periodic plans with R >= 1 only) and wfp_adjoint needs
                              no replay; 0: neither                           [0] */
  int32_t overlap_cus;     /* > 0: wfp_run puts the history chain (spread, FFTs, modes) and the
                              solve on a stream restricted to the first overlap_cus compute
                              units and the local sum on the others, the next level's local
                              sum (lags >= 2) overlapping the current level's chain and solve
                              (results are the same bit for bit); < 0: one stream; 0: the
                              library's choice, which is one XCD's compute units when the local
                              sum reads at least 64 MB per level, else one stream   [0] */
  int32_t local_mode;      /* 1: local weights stored per pair (read every level); 2: evaluated on the
                              fly every level (memory O(M), arithmetic O(pairs N_L p)); 3: stored once
                              per unordered pair (Q_m depends on the distance alone) and applied to
                              both rows, about half the bytes of 1 (the gradient pass's
                              derivative weights likewise); 0: 3 when half of
                              the per-pair set-up fits in 60% of the free device memory and
                              either the springs have 96 or more neighbours on average or the
                              per-pair weights would not fit, else 1 when they fit, else on
                              the fly                                         [0] */
  int32_t check_finite;    /* nonzero: every wfp_run ends by checking the newest density level and the
                              mode state alpha, alpha' for NaN or Inf (one small kernel), waits for the
                              plan's stream and returns WFP_ENONFINITE if any is found (the levels stay
                              marched: an unstable march, e.g. with very stiff springs, is caught
                              here); 0: no check, wfp_run stays asynchronous      [0] */
} wfp_params;

/* Derived sizes of a plan (read-only report). */
typedef struct {
  int64_t M, R, K, n_fine, n_pairs, n_pairs_recv, level;
  int32_t W, p, m_max, n_gl_local, rbc_period, nufft_width, solve_iters, boundary;
  double dt, delta, b, solve_contraction;
  int64_t device_bytes;
  int64_t n_weights_nonzero;   /* nonzero stored local weights of lag >= 1 (scatterer rows) */
  int64_t n_weights_stored;    /* stored local weights of lag >= 1 (scatterer rows) */
  int32_t solve_mode;          /* 0: dense inverses of small nearby-runs and LDS tiles,
                                  1: global Jacobi sweeps (dense nearby coupling) */
  int32_t overlap_cus;         /* compute units of the concurrent history chain, -1: one stream */
  int32_t local_mode;          /* 1: stored local weights, 2: evaluated on the fly, 3: stored once per
                                  unordered pair */
  int32_t reserved;
  int64_t n_weights_lag1;      /* nonzero stored local weights of lag 1 (part of n_weights_nonzero) */
  int32_t n_solve_tiles;       /* solve_mode 0: LDS tiles of the Jacobi solve (long nearby runs) */
  int32_t n_direct_tiles;      /* solve_mode 0: groups of small nearby runs solved by stored inverses */
  int32_t sweep_wave;          /* solve_mode 1: 1 when a wavefront sweeps each row (long rows), else 0 */
  int32_t reserved2;
} wfp_info;

/* Stages of one level, for wfp_get_profile. */
#define WFP_STAGE_SPREAD 0     /* type-1 spreading onto the fine grid */
#define WFP_STAGE_FFT_FWD 1    /* real-to-complex FFT of the fine grid */
#define WFP_STAGE_MODES 2      /* deconvolution, spectra ring, FIR, propagator */
#define WFP_STAGE_RBC 3        /* free-space RBC projection (two kernels) */
#define WFP_STAGE_FFT_INV 4    /* complex-to-real FFT for the type-2 transform */
#define WFP_STAGE_LOCAL 5      /* local sum (stored weights: its lags >= 2 part) */
#define WFP_STAGE_SOLVE 6      /* per-step solve (stored weights: with the local sum's lag-1 part) */
#define WFP_STAGE_RECV 7       /* receivers */
#define WFP_N_STAGES 8

/* Create a plan: validates the problem, sorts the springs, precomputes the
 * window, the one-step kernels p_k, q_k, the NUFFT deconvolution factors,
 * neighbour ranges and the local weights Q_m(d) of every pair closer than
 * delta (stored on the device), and zeroes the state (level 0).
 * `stream` is a hipStream_t (NULL = default stream).  Synchronous.
 * Errors: WFP_EINVAL, WFP_EDOMAIN, WFP_ENOMEM, WFP_EHIP; *out is NULL then. */
wfp_status wfp_plan_create(const wfp_problem* prob, const wfp_params* par, void* stream,
                           wfp_plan** out);

/* Release every device and host resource of the plan (NULL is a no-op). */
void wfp_plan_destroy(wfp_plan* plan);

/* Fill *info with the plan's derived sizes. */
wfp_status wfp_plan_info(const wfp_plan* plan, wfp_info* info);

/* March n_steps levels (Section 4.2, eq. (periodicIE_disc)).
 *   sigma_out  device [ceil(n_steps / save_every)][M] or NULL: row i holds the
 *              densities of the (i*save_every)-th level computed by this call.
 *   save_every >= 1 (ignored when sigma_out is NULL).
 *   u_recv_out device [n_steps][R] or NULL: u(x_r, t_L) at every level computed
 *              (u_L + u_H, eqs. (localSol2) and (historySol1)).
 * Asynchronous on the plan's stream, unless the plan checks for non-finite
 * values (check_finite), which waits for the stream at the end.  The first
 * call allocates the plan's block of driving-data levels (device memory held
 * until wfp_plan_destroy); checkpointing and recording runs allocate each
 * checkpoint or recorded block the first time they reach it (held until
 * wfp_plan_destroy, reused after wfp_reset); nothing else is allocated.
 * Errors: WFP_EINVAL, WFP_EHIP, WFP_ENONFINITE, WFP_ENOMEM. */
wfp_status wfp_run(wfp_plan* plan, int64_t n_steps, double* sigma_out, int64_t save_every,
                   double* u_recv_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): wfp_run that never
 * allocates.  The block of driving-data levels that wfp_run allocates on its
 * first call (and the finite-check flag) lives instead in the library's
 * static scratch array, 8 MiB per GPU, held by each GPU the library runs on
 * until the process ends.  Same arguments, outputs and stream ordering as
 * wfp_run.  Limits: M <= 1048544 springs (one level of driving data must fit);
 * plans with checkpoint_every != 0 (their checkpoints or recorded levels are allocated) and plans
 * with stage timing on (it creates events) are refused with WFP_EINVAL.  The
 * scratch array is shared by every call on one GPU and keeps the last call's
 * contents; each call recomputes what it reads, but calls that overlap on one
 * GPU (other threads, or other streams not ordered with this one) race.
 * Errors: WFP_EINVAL, WFP_EHIP, WFP_ENONFINITE. */
wfp_status wfp_run_noalloc(wfp_plan* plan, int64_t n_steps, double* sigma_out, int64_t save_every,
                           double* u_recv_out);

/* March n_steps levels like wfp_run, with the driving data supplied by the
 * caller instead of computed from the plan's incident packets: any incident
 * wave, or data read off a manufactured solution (Section 6.1).
 *   g  device [n_steps][M], caller's spring order: row i holds g_j at the
 *      plan's level + i, the right side of the spring condition
 *      -sigma_j - beta_j u(x_j, t) = g_j (eq. (gj): beta_j f(x_j - t) for an
 *      incident wave f(x - t)).  Read during the call's stream work; the
 *      caller keeps it alive until the stream has passed it.
 *   sigma_out, save_every, u_recv_out as for wfp_run.
 * One stream (no concurrent chain).  After it, wfp_adjoint refuses with
 * WFP_ESTATE until wfp_reset: its forward replay computes the packets' data.
 * Errors: WFP_EINVAL (g NULL with n_steps > 0), WFP_EHIP, WFP_ENONFINITE. */
wfp_status wfp_run_driven(wfp_plan* plan, int64_t n_steps, const double* g, double* sigma_out,
                          int64_t save_every, double* u_recv_out);

/* The explicit local part at the springs for the next level L (the plan's
 * level), eqs. (localSol1)/(localSol2) without the implicit lag 0:
 *   out[j] = sum_{m>=1} sum_{l: d_jl < delta} (1/2) Q_m(d_jl) sigma_l^{L-m}
 * from the current density history.  out: device [M], caller order.  Useful
 * to check the local sum on its own (e.g. after wfp_set_state).
 * Asynchronous on the plan's stream.  Errors: WFP_EINVAL, WFP_EHIP. */
wfp_status wfp_local_part(wfp_plan* plan, double* out);

/* Gradient of a receiver loss J(u) through the march (not in the paper: the
 * transpose of every step of Section 4.2, run backwards in time).
 * Requires a periodic plan with R >= 1 (any local_mode) and
 * checkpoint_every != 0 whose levels 0 .. n_levels-1 were computed by
 * wfp_run since plan creation or wfp_reset (no wfp_set_state in between); the
 * plan's own state is not changed.  The adjoint level applies the same local
 * sum as the forward one: Q_m depends on the distance alone, so the sum over
 * pairs is its own transpose.
 *   dJdu       device [n_levels][R]: dJ/du(x_r, t_L) for the levels 0..n_levels-1
 *   grad_beta  device [M] (caller order): dJ/dbeta_j
 *   grad_x     device [M] (caller order) or NULL: dJ/dx_j (the local weights are
 *              differentiated in the distance; where a pair sits exactly at the
 *              nearby/intermediate switch d = dt the one-sided derivative of
 *              its class is used)
 * Device memory: the first call allocates an adjoint march state and, with
 * checkpoints, a replay state, a segment of checkpoint_every + m_max - 1
 * density levels and one of checkpoint_every derivative terms; with grad_x,
 * derivative weights as large as the local weights (stored per ordered pair
 * or once per pair, as the weights are; with weights on the fly their
 * derivatives are evaluated on the fly too, each pair once, in the pass
 * that also forms the next adjoint level's local sum, and only three column
 * buffers of the size of the forward one are added).  With recorded levels
 * (checkpoint_every < 0) the recorded blocks take the place of the replay.
 * Asynchronous on the plan's stream.
 * Errors: WFP_EINVAL, WFP_EDOMAIN (free space; grad_x with the weights on
 * the fly and m_max = W + p/2 > 46, more lags than its LDS stage holds),
 * WFP_ESTATE, WFP_ENOMEM, WFP_EHIP. */
wfp_status wfp_adjoint(wfp_plan* plan, int64_t n_levels, const double* dJdu, double* grad_beta,
                       double* grad_x);

/* Checkpoint / resume.  With L the next level to be computed:
 *   hist   device [m_max][M]:      hist[m][j] = sigma_j^{L-1-m}
 *   ring   device [W][K+1][2]:     ring[m][k] = S_k^{L-2-m}  (spectra of past levels)
 *   alpha  device [K+1][2], dalpha device [K+1][2]: alpha_k^{L-1}, alpha'_k^{L-1}
 * Any pointer may be NULL on get (that part is skipped).  set_state requires all.
 * Asynchronous on the plan's stream. */
wfp_status wfp_get_state(wfp_plan* plan, int64_t* level, double* hist, double* ring,
                         double* alpha, double* dalpha);
wfp_status wfp_set_state(wfp_plan* plan, int64_t level, const double* hist, const double* ring,
                         const double* alpha, const double* dalpha);

/* Per-stage timing with HIP events recorded around every kernel of later
 * wfp_run calls on the plan's stream (enable != 0 clears the accumulators;
 * timing adds event overhead to the march, and while it is on every stage runs
 * on the plan's stream, without the concurrent history chain, so that each
 * stage is timed alone).  wfp_get_profile synchronises the
 * stream and returns, per stage, the summed kernel milliseconds and launch
 * counts (arrays of WFP_N_STAGES; either may be NULL). */
wfp_status wfp_set_profiling(wfp_plan* plan, int32_t enable);
wfp_status wfp_get_profile(wfp_plan* plan, double* ms, int64_t* launches);

/* Return the plan to level 0 with zero history (stream-ordered). */
wfp_status wfp_reset(wfp_plan* plan);

/* Schedule choice by measurement (not in the paper): from level 0, marches
 * 2 + trial_levels levels with the history chain and solve on one stream, and
 * with them on 1, 2, 3 and 4 XCDs' worth of compute units beside the local
 * sum (the overlap_cus parameter), keeps the fastest, reports it in
 * *overlap_cus (may be NULL; -1 = one stream) and returns the plan to level 0
 * with zero history.  Synchronous.  Which split wins depends on the sizes:
 * the chain gains from running beside the local sum while its kernels are
 * latency-bound (K of a few thousand) and loses once they are bandwidth-bound
 * (K of 1e5 and more).  Plans with checkpoints (checkpoint_every > 0) march
 * on one stream and keep it.  Errors: WFP_EINVAL (trial_levels < 1),
 * WFP_ESTATE (plan not at level 0). */
wfp_status wfp_plan_autotune(wfp_plan* plan, int32_t trial_levels, int32_t* overlap_cus);

/* Batched form (not in the paper): n independent periodic problems, each
 * with its own x, beta, incident field, receivers, dt and level count,
 * marched in lockstep.  Each stage of a level is one launch over an (instance, block) work
 * list and the whole level is one HIP graph replayed per level; every instance
 * computes what its own plan would, to rounding (the same kernel bodies; a plan
 * marched on its own adds the lag-1 part of its local sum separately).
 *   wfp_batch_create  host problem data as for wfp_plan_create (probs[n],
 *                     pars[n]); builds one plan per instance (one stream each;
 *                     local weights stored per pair, stored once per pair or on
 *                     the fly per pars[i].local_mode, on the fly with p = 8 only;
 *                     local_mode 0 here: stored for the instances with the fewest
 *                     neighbour pairs while their weights fit in 45 % of the free
 *                     device memory, once per pair where the springs have 96 or
 *                     more neighbours or only half fits, else on the fly).
 *                     Synchronous.
 *                     Errors: WFP_EDOMAIN (free space, or an instance whose
 *                     stages exceed the LDS), WFP_EINVAL (checkpoint_every != 0:
 *                     no gradient pass in batches), as for plans.
 *   wfp_batch_run     march n_steps levels of every instance; sigma_final is a
 *                     HOST array of n DEVICE pointers (entries may be NULL, the
 *                     array may be NULL): instance i's densities of its last
 *                     level, [M_i] in caller order.  u_recv_out likewise: the
 *                     field at instance i's R_i receivers at every level of the
 *                     call, [n_steps][R_i] (eqs. (localSol2), (historySol1)).
 *                     Ordered after prior work on `stream`; later work on
 *                     `stream` waits for it.  A call that passes receiver
 *                     outputs (or follows one that did) first waits for the
 *                     batch's earlier work.
 *   wfp_batch_set_levels  per-instance level counts (each problem's own N_t):
 *                     instance i computes levels 0 .. n_levels[i] - 1 and then
 *                     leaves every launch of the level (its blocks return at
 *                     once; its state stays at its last level) while the
 *                     others go on.  n_levels is a HOST array of n entries;
 *                     an entry <= 0, or n_levels NULL, means no limit.  Stays
 *                     in force across runs and resets.  sigma_final then holds
 *                     each instance's own last level; receiver rows of levels
 *                     at or beyond an instance's end are not written.  Waits
 *                     for the batch's earlier work.
 *   wfp_batch_reset   all instances back to level 0.
 *   wfp_batch_autotune  from level 0: times trial_levels levels for each
 *                     launch shape: the local sum's (4 or 8 rows per block,
 *                     with or without the XCD-aware block order) times the
 *                     spread tile (0: one fine-grid row per workgroup, the
 *                     type-1 spread fused into the transform's row pass; 1: a
 *                     separate pass over tiles of 256 consecutive cells, the
 *                     row pass reading the spread grid; the sources are
 *                     binned per fine-grid cell either way), keeps the
 *                     fastest, reports it and leaves the batch at level 0.
 *                     Every shape computes the same bits.
 *   wfp_batch_set_shape  sets that launch shape directly (rows_per_block 4 or
 *                     8, xcd_remap 0 or 1, spread_pass 0 or 1); waits for the
 *                     batch's earlier work.  Errors: WFP_EINVAL.
 *   wfp_batch_size    number of instances and the current level.
 *   wfp_batch_plan    instance i's plan (owned by the batch: never destroy it;
 *                     wfp_get_state / wfp_plan_info on it are valid between runs).
 *   wfp_batch_destroy releases everything (NULL is a no-op). */
typedef struct wfp_batch wfp_batch;
wfp_status wfp_batch_create(int32_t n, const wfp_problem* probs, const wfp_params* pars, void* stream,
                            wfp_batch** out);
wfp_status wfp_batch_run(wfp_batch* batch, int64_t n_steps, double* const* u_recv_out,
                         double* const* sigma_final);
wfp_status wfp_batch_set_levels(wfp_batch* batch, const int64_t* n_levels);
wfp_status wfp_batch_reset(wfp_batch* batch);
wfp_status wfp_batch_autotune(wfp_batch* batch, int32_t trial_levels, int32_t* rows_per_block,
                              int32_t* xcd_remap, int32_t* spread_pass);
wfp_status wfp_batch_set_shape(wfp_batch* batch, int32_t rows_per_block, int32_t xcd_remap,
                               int32_t spread_pass);
wfp_status wfp_batch_size(const wfp_batch* batch, int32_t* n, int64_t* level);
wfp_plan* wfp_batch_plan(wfp_batch* batch, int32_t i);
void wfp_batch_destroy(wfp_batch* batch);

const char* wfp_status_string(wfp_status s);
const char* wfp_last_error(void);
int32_t wfp_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* WFP_H */
