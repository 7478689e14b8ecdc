/*
 * brmppi.h -- C ABI of the MI355X (gfx950) BR-MPPI control-update library.
 *
 * One call computes one control update of Barrier-Rate guided MPPI for a
 * kinematic tractor-trailer (arXiv 2508.05773): S perturbed input sequences
 * over a horizon T are rolled out through eq. (6) while every step is
 * projected onto the barrier-rate equalities of eq. (9) with the soft-bound
 * closed form of eqs. (11)-(12); the contouring cost of eqs. (13)-(15) is
 * accumulated; the new nominal sequence is the exponentially weighted average
 * of the applied sequences (Sec. III-B, eq. (5)).
 *
 * All device work runs in the library's HIP kernels.  The caller provides the
 * device memory (an arena, e.g. a torch uint8 tensor) and the HIP streams; the
 * library sub-allocates from the arena and never calls hipMalloc.
 *
 * Conventions
 *  - All pointers in the problem / outputs structs are HOST pointers unless
 *    the field says otherwise.  The caller owns every host buffer; inputs are
 *    copied before the call returns.  Output buffers are written only when the
 *    call returns BRMPPI_OK (or BRMPPI_ENONFINITE, see below).
 *  - Return codes: 0 = success, >0 = pending, <0 = error.  No C++ exception
 *    crosses the ABI.  An invalid argument leaves the library state unchanged.
 *    brmppi_last_error() returns a thread-local message for the last error.
 *  - Layouts are row-major float32: a sequence is [T][3] with columns
 *    (jerk, steer rate, progress rate); a path is [n][4] with columns
 *    (x, y, theta1_ref, theta2_ref) sampled every ds metres of arc length.
 *  - Threading: one context may be used from one application thread; the
 *    served form (submit/poll) adds one internal request thread per context.
 */
#ifndef BRMPPI_H
#define BRMPPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define BRMPPI_OK 0
#define BRMPPI_PENDING 1          /* poll: the ticket is still in flight */
#define BRMPPI_EINVAL (-1)        /* invalid argument; nothing changed */
#define BRMPPI_ENOMEM (-2)        /* does not fit in the arena */
#define BRMPPI_EAGAIN (-3)        /* served form: request queue full, retry */
#define BRMPPI_ENONFINITE (-4)    /* every rollout cost was NaN/Inf: the nominal
                                     sequence is returned, warm start untouched */
#define BRMPPI_ENOTICKET (-5)     /* unknown or already consumed ticket */
#define BRMPPI_EDEVICE (-6)       /* a HIP call failed */
#define BRMPPI_ETIMEDOUT (-7)     /* brmppi_wait deadline passed */
#define BRMPPI_ESTATE (-8)        /* missing state (no path / no warm start) */
#define BRMPPI_ECANCELED (-9)     /* served form: the context was destroyed before the
                                     request was admitted */

/* ---- limits ------------------------------------------------------------- */
#define BRMPPI_MAX_OBS 32         /* obstacle rows per solve: obstacles x footprint discs */
#define BRMPPI_MAX_DISCS 4        /* footprint discs per body (tractor, trailer) */
#define BRMPPI_MAX_T 512          /* horizon */
#define BRMPPI_MAX_S (1u << 22)   /* samples per solve */
#define BRMPPI_MAX_PATH (1u << 20)/* waypoints per path */
#define BRMPPI_MAX_BATCH 1024     /* instances per brmppi_solve_batch */
#define BRMPPI_NOALLOC_MAX_BYTES (64u << 20) /* static scratch of brmppi_solve_noalloc */

/* ---- problem flags ------------------------------------------------------ */
#define BRMPPI_GUIDANCE_OFF 1u    /* plain MPPI: sampled inputs applied unprojected */
#define BRMPPI_HITCH_OFF 2u       /* no hitch-angle rows (N_c = n_obs) */
#define BRMPPI_X0_RESIDENT 4u     /* start from the controller's device-resident plant
                                     state (brmppi_set_state / brmppi_closed_loop) */
#define BRMPPI_ADVANCE_PLANT 8u   /* after the update, advance the resident plant state by
                                     the first averaged input (jerk and steer rate clamped
                                     to [j_lo, j_hi], [w_lo, w_hi]) with eq. (6) in FP64 */
#define BRMPPI_COLLISION_PENALTY 16u /* the paper's second baseline (Sec. V), whose form it
                                     does not give: w_col * sum_o max(0, -h_o(x, t))^2,
                                     h_o the obstacle function of eq. (16) at the
                                     current state, added to every stage cost and to the
                                     terminal cost; usually with BRMPPI_GUIDANCE_OFF */
#define BRMPPI_HITCH_QP 32u       /* hitch-angle stabiliser (Sec. IV-D, eq. (19)) before the
                                     plant step (needs BRMPPI_ADVANCE_PLANT): the applied
                                     (j, omega) minimise ||u - U_new[0]||^2 over the input box
                                     with Q_h = diag(qh_j, qh_w), subject to the discrete CBF
                                     condition Lf + g u >= -alpha_h hhat of both hitch rows
                                     (the first-order expanded barrier of the rollouts);
                                     solved exactly in FP64 on the device; when no input
                                     satisfies it, the box-clipped U_new[0] is applied */

/* ---- context flags ------------------------------------------------------ */
#define BRMPPI_CTX_PROFILE 1u     /* time every kernel of the blocking calls with HIP events */
#define BRMPPI_CTX_PROFILE_ROLLOUT 2u /* time only the rollout and noise kernels (lower overhead) */

typedef struct brmppi_ctx brmppi_ctx;

typedef struct {
  void* arena;                /* DEVICE memory, >= 256-byte aligned, owned by the caller,
                                 must outlive the context */
  size_t arena_bytes;
  void* streams[4];           /* hipStream_t handles (default priority); streams[0] runs the
                                 blocking calls, all of them serve submit/poll batches */
  uint32_t n_streams;         /* 1..4 */
  uint32_t max_controllers;   /* controller slots (resident path + warm start each) */
  uint32_t max_inflight;      /* served form: queued + running requests (0 = 4096) */
  const char* autotune_cache; /* JSON launch-shape cache path, or NULL */
  uint32_t flags;             /* BRMPPI_CTX_* */
  int32_t device;             /* HIP device ordinal of the arena and streams */
} brmppi_config;

/* Tuning parameters (all SI units).  Groups:
 *  vehicle, eq. (6) / (18):   Ts, l1 (wheelbase), lh (hitch offset), l2 (trailer
 *                              length), dtheta_max, kappa (hitch limit dtheta_max -
 *                              kappa v), r_disc (footprint disc radius, eq. (16))
 *  contouring, eq. (13):      Qc, Ql, Qth1, Qth2, R_j, R_w, mu, nu_bar
 *  projection, eq. (11):      W_j, W_w, W_a (diagonal weight W), rho,
 *                              input bounds [j_lo, j_hi], [w_lo, w_hi]
 *  barrier rates, eq. (9):    alpha0 (initial rate of every row), soft bounds
 *                              [alpha_lo, alpha_hi] on the next rate
 *  sampling (Sec. III-B):     sigma_j, sigma_w, sigma_nu (input noise),
 *                              sigma_a (auxiliary-input noise)
 *  guard:                     h_eps (|hhat| floor in each row)
 *  baseline (Sec. V):         w_col, weight of the collision penalty added to the
 *                              stage and terminal costs under BRMPPI_COLLISION_PENALTY
 *  stabiliser, eq. (19):      qh_j, qh_w (diagonal Q_h), alpha_h (class-K rate of the
 *                              hitch rows) of the CBF-QP under BRMPPI_HITCH_QP
 *  footprint, Sec. IV-C:      discs of radius r_disc covering the vehicle: disc_tractor[k]
 *                              (k < n_disc_tractor) metres ahead of the tractor's rear
 *                              axle along its heading, disc_trailer[k] (k < n_disc_trailer)
 *                              metres behind the hitch along the trailer's heading (the
 *                              hitch sits lh behind the rear axle).  Every (disc, obstacle)
 *                              pair is one barrier row, disc by disc (tractor discs first),
 *                              obstacles in order; eq. (17) expands each around its disc
 *                              centre along the drift (inputs zero).  1..4 discs per body
 *                              counted together at least 1; n_obs times the disc count at
 *                              most BRMPPI_MAX_OBS.  The defaults are one disc at the rear
 *                              axle, the point eq. (16) uses. */
typedef struct {
  float Ts, l1, lh, l2, dtheta_max, kappa, r_disc;
  float Qc, Ql, Qth1, Qth2, R_j, R_w, mu, nu_bar;
  float W_j, W_w, W_a, rho, j_lo, j_hi, w_lo, w_hi;
  float alpha0, alpha_lo, alpha_hi, sigma_j, sigma_w, sigma_nu, sigma_a;
  float h_eps;
  float w_col;   /* weight of the collision-penalty baseline (BRMPPI_COLLISION_PENALTY) */
  float qh_j, qh_w, alpha_h;  /* hitch-angle stabiliser (BRMPPI_HITCH_QP): Q_h, class-K rate */
  float disc_tractor[BRMPPI_MAX_DISCS], disc_trailer[BRMPPI_MAX_DISCS];
  uint32_t n_disc_tractor, n_disc_trailer;
} brmppi_params;

/* Obstacle (Sec. IV-C, eq. (16)): centre (cx, cy) at t = 0, semi-axes (mx, my),
 * orientation heading, super-ellipse exponent e (2 or 4; other values are
 * EINVAL), constant velocity (vx, vy) for the prediction of Assumption 2.  The
 * semi-axes are inflated by params->r_disc. */
typedef struct { float cx, cy, mx, my, heading, e, vx, vy; } brmppi_obstacle;

/* One control update (the finite-horizon problem of eq. (8) plus MPPI inputs). */
typedef struct {
  uint32_t controller;        /* slot owning the resident path and warm start */
  uint32_t S, T;              /* samples (1..BRMPPI_MAX_S), horizon (1..BRMPPI_MAX_T) */
  float x0[8];                /* px, py, v, a, theta1, theta2, delta, psi (ignored with
                                 BRMPPI_X0_RESIDENT) */
  const float* u_nom;         /* T*3 nominal sequence, or NULL = the controller's resident
                                 warm start (the shifted result of its last update) */
  const brmppi_obstacle* obs; /* n_obs records */
  uint32_t n_obs;             /* 0..BRMPPI_MAX_OBS, and n_obs x footprint discs <= BRMPPI_MAX_OBS */
  float t0;                   /* time of x0 for moving obstacles */
  float lambda;               /* temperature of the weights, > 0 */
  uint64_t seed;              /* Philox key */
  uint32_t instance;          /* Philox counter word 3 */
  uint32_t flags;             /* BRMPPI_GUIDANCE_OFF | BRMPPI_HITCH_OFF | BRMPPI_X0_RESIDENT |
                                 BRMPPI_ADVANCE_PLANT | BRMPPI_COLLISION_PENALTY |
                                 BRMPPI_HITCH_QP */
  const brmppi_params* params;/* NULL = the controller's parameters (brmppi_set_params;
                                 brmppi_default_params until set) */
} brmppi_problem;

/* Statistics of one update.  (Every barrier row takes part in the projection
 * at every step -- no row is switched off by a buffer zone -- so a fraction of
 * active rows would be 1 by construction and is not reported.) */
typedef struct {
  float J_min;                /* min_s J_s */
  float Z;                    /* sum_s exp(-(J_s - J_min)/lambda) */
  float ess;                  /* effective sample size 1/sum wbar^2 */
  int32_t status;             /* BRMPPI_OK or BRMPPI_ENONFINITE */
  double latency_us;          /* submit/solve entry to result ready (host clock) */
} brmppi_stats;

/* Optional extra outputs of brmppi_solve_ex (host buffers; NULL = skip). */
typedef struct {
  float* u_out;               /* T*3 new nominal sequence (eq. (5)) -- required */
  float* J_out;               /* S rollout costs, +inf where non-finite */
  float* useq_out;            /* 3*T*S applied inputs, layout [t][k][s] */
} brmppi_outputs;

/* ---- lifecycle ---------------------------------------------------------- */
/* Create a context over a caller-owned device arena.  Errors: EINVAL (NULL
 * or misaligned arena, n_streams outside 1..4, max_controllers 0), EDEVICE. */
int brmppi_create(const brmppi_config* cfg, brmppi_ctx** out);
/* Drain in-flight work, stop the request thread, free host resources.  The
 * arena is the caller's and is not touched afterwards. */
int brmppi_destroy(brmppi_ctx* ctx);
const char* brmppi_last_error(void);

/* Counters of a context (host bookkeeping; no device work). */
typedef struct {
  uint64_t scratch_grows;     /* times a call had to re-allocate the solve scratch in the arena */
  uint64_t pinned_grows;      /* times a call had to re-allocate a pinned staging buffer
                                 (hipHostFree + hipHostMalloc); staging of 1 MiB per stream is
                                 allocated at create */
  uint64_t arena_bytes;       /* size of the caller's arena */
  uint64_t arena_used;        /* bytes of it sub-allocated now */
  uint64_t served_done;       /* served requests completed by the device */
  uint64_t served_failed;     /* served requests that failed before or at launch */
} brmppi_info;
int brmppi_get_info(brmppi_ctx* ctx, brmppi_info* out);

/* ---- parameters ---------------------------------------------------------- */
/* The library's defaults (the paper's tuned values are unpublished): the
 * Sec. V input bounds j in [-2, 2] m/s^3, omega in [-0.9, 0.9] rad/s; a
 * 4 m / 0.5 m / 10 m tractor-trailer, hitch limit 0.7 - 0.05 v rad, footprint
 * disc 1 m; Ts 0.05 s; sampling noise (1.0, 0.3, 0.5) and 0.2 for the
 * auxiliary inputs; W the inverse sampling covariance, rho 0.1; barrier rates
 * 0.5 within [-1, 1]; Qc = Ql = 2, Qth = 1, R = 0.05, mu 0.5, nu_bar 2 m/s;
 * w_col 1000; Q_h = W's input block, alpha_h 0.5.  Errors: EINVAL (NULL). */
int brmppi_default_params(brmppi_params* out);
/* Parameters a controller's problems use when their params pointer is NULL
 * (NULL here restores the defaults).  Errors: EINVAL (out of range, non-finite
 * or inconsistent values; nothing changed). */
int brmppi_set_params(brmppi_ctx* ctx, uint32_t controller, const brmppi_params* params);

/* ---- controller state --------------------------------------------------- */
/* Copy a reference path zeta(psi) (Sec. IV-B) into the controller's device
 * slot; it stays resident for every later solve of that controller.
 * path: n*4 host floats, n in 2..BRMPPI_MAX_PATH, ds > 0. */
int brmppi_set_path(brmppi_ctx* ctx, uint32_t controller, const float* path, uint32_t n, float ds);
/* Read / replace the resident warm start (the receding-horizon shift of
 * Sec. III-B).  T*3 host floats. */
int brmppi_get_nominal(brmppi_ctx* ctx, uint32_t controller, float* u, uint32_t T);
int brmppi_set_nominal(brmppi_ctx* ctx, uint32_t controller, const float* u, uint32_t T);
/* Resident FP64 plant state used by BRMPPI_X0_RESIDENT and brmppi_closed_loop. */
int brmppi_set_state(brmppi_ctx* ctx, uint32_t controller, const double x[8]);
int brmppi_get_state(brmppi_ctx* ctx, uint32_t controller, double x[8]);

/* ---- plain solve (blocking) --------------------------------------------- */
/* One control update on streams[0]; returns when u_out holds the new nominal
 * sequence (T*3).  The controller's warm start becomes the shifted result.
 * Errors: EINVAL, ESTATE (no path; u_nom NULL without a warm start of length
 * T), ENOMEM, EDEVICE; ENONFINITE (u_out = nominal sequence). */
int brmppi_solve(brmppi_ctx* ctx, const brmppi_problem* p, float* u_out, brmppi_stats* st);
int brmppi_solve_ex(brmppi_ctx* ctx, const brmppi_problem* p, const brmppi_outputs* out,
                    brmppi_stats* st);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): brmppi_solve with its
 * scratch in a static device array of BRMPPI_NOALLOC_MAX_BYTES (64 MiB) per
 * GPU, held until the process ends, instead of a block of the arena.  The call
 * allocates nothing: no arena block, no pinned staging (the 1 MiB buffer made
 * at create must hold the inputs), no HIP events (profiling flags are ignored).
 * The controller's path, warm start and plant state stay where brmppi_set_path
 * put them; results and the warm-start shift equal brmppi_solve's, bitwise.
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents (the counters a call needs at zero are uploaded with its inputs);
 * calls of one process on one GPU are serialised, and a call returns only
 * after its device work is done.  Errors: as brmppi_solve; ENOMEM when the
 * update needs more scratch than the array holds (about S*T*(3 + 5 + n_obs)*4
 * bytes) or its inputs more than the staging buffer; ESTATE when the array's
 * address could not be taken at create. */
int brmppi_solve_noalloc(brmppi_ctx* ctx, const brmppi_problem* p, float* u_out, brmppi_stats* st);

/* ---- batched solve (blocking) ------------------------------------------- */
/* n independent updates (distinct controllers) together: persistent rollout
 * launches over a tile list (one per constraint bucket present; a bucket too
 * small to fill the device joins the next heavier one), then one persistent
 * reduce over every instance, captured in a HIP graph and replayed while the
 * batch keeps its shape.  u_outs[i] receives T_i*3 floats; st may be NULL or
 * an array of n.  Each instance's result equals its plain solve, bitwise. */
int brmppi_solve_batch(brmppi_ctx* ctx, const brmppi_problem* p, uint32_t n, float* const* u_outs,
                       brmppi_stats* st);

/* ---- served form (asynchronous, continuous batching) -------------------- */
/* Queue one update; returns at once with a ticket.  The request thread admits
 * queued requests as controller slots and arena memory free up and launches
 * them together with whatever else is pending, overlapping on the device.
 * Requests of one controller run in submission order; with
 * BRMPPI_X0_RESIDENT | BRMPPI_ADVANCE_PLANT a controller runs its closed loop
 * on the device (each request starts where the previous one left the plant).
 * Errors: EINVAL, ESTATE, EAGAIN (max_inflight reached), ENOMEM (can never fit). */
int brmppi_submit(brmppi_ctx* ctx, const brmppi_problem* p, uint64_t* ticket);
/* Non-blocking: BRMPPI_PENDING while in flight; otherwise copies the result
 * (T*3) and stats, releases the ticket and returns its status. */
int brmppi_poll(brmppi_ctx* ctx, uint64_t ticket, float* u_out, brmppi_stats* st);
/* Blocking variant of poll with a deadline (ETIMEDOUT). */
int brmppi_wait(brmppi_ctx* ctx, uint64_t ticket, float* u_out, brmppi_stats* st, uint32_t timeout_ms);

/* ---- closed loop on the device ------------------------------------------ */
/* n_updates receding-horizon updates of one controller without host round
 * trips: update k solves from the resident plant state with seed p->seed + k,
 * then advances the plant by the first averaged input (jerk and steer rate
 * clamped to [j_lo, j_hi], [w_lo, w_hi]) with eq. (6) in FP64.  x_out
 * ((n_updates+1)*8 doubles) and u_applied ((n_updates)*3 floats) are optional
 * host buffers filled at the end.  p->u_nom seeds the first update (NULL =
 * resident warm start); BRMPPI_X0_RESIDENT is implied. */
int brmppi_closed_loop(brmppi_ctx* ctx, const brmppi_problem* p, uint32_t n_updates, double* x_out,
                       float* u_applied);

/* ---- launch shapes / profiling ------------------------------------------ */
/* Time each candidate launch shape (block size and variant: lanes per
 * sample, noise drawn in the kernel or by a separate parallel kernel) on
 * synthetic problems with a 48-step horizon, rollout plus reduction as a plain
 * solve runs them, and keep the fastest per constraint bucket (0, <=2, <=8,
 * <=16, <=32 obstacles) and sample-count class (<=2048, <=8192, <=32768,
 * more), plus the block size of the batched persistent kernel; a shape whose
 * tiles reduce themselves wins ties within 2 %.  Writes the JSON cache named
 * in the config (if any), with every candidate's time.  Shapes never change a
 * result bit. */
int brmppi_autotune(brmppi_ctx* ctx);
/* Force a rollout launch shape for every plain and batched launch: block size
 * 64..256 (multiple of 64) and variant 0 = one lane per sample, noise drawn in
 * the kernel; 1 = one lane, noise from the parallel kernel; 2 / 3 / 4 = two /
 * four / eight lanes per sample, noise from the parallel kernel (batched
 * launches always use variant 0; an instance without guidance runs variant
 * 0 or 1; a plain solve whose normals would take more than 2 GiB or half the
 * arena runs variant 0).  block 0 restores the tuned/default choice.  EINVAL for a block
 * outside 64..256 or not a multiple of 64, or a variant above 4. */
int brmppi_set_launch(brmppi_ctx* ctx, uint32_t block, uint32_t variant);
/* Kernel timings accumulated under BRMPPI_CTX_PROFILE (every kernel of the
 * blocking calls) or BRMPPI_CTX_PROFILE_ROLLOUT (rollout and noise only), from
 * HIP events on the launching stream (ms totals and launch counts):
 * out[0..1] rollout, out[2..3] reduce (weights + average + shift + plant),
 * out[4..5] noise.  A profiling context launches batches directly instead of
 * replaying their graph. */
int brmppi_profile_read(brmppi_ctx* ctx, double out[6]);
int brmppi_profile_reset(brmppi_ctx* ctx);

/* ---- debug entry points (parity tests) ---------------------------------- */
/* Philox4x32-10 on the device: n counters (host, n*4) under one key -> n*4
 * outputs (host). */
int brmppi_debug_philox(brmppi_ctx* ctx, const uint32_t* ctr, const uint32_t key[2], uint32_t n,
                        uint32_t* out);
/* The normals the rollout kernel draws: for each of n (sample, step) pairs
 * (host, n*2) the first K normals -> out (host, n*K). */
int brmppi_debug_normals(brmppi_ctx* ctx, uint64_t seed, uint32_t instance, const uint32_t* s_tau,
                         uint32_t n, uint32_t K, float* out);
/* The two factors of the kernels' Box-Muller transform (Sec. III-B sampling)
 * for n raw Philox words r (host): out[3i] = sqrt(-2 ln u), out[3i + 1] =
 * cos(2 pi u), out[3i + 2] = sin(2 pi u), with u = ((r >> 9) + 1/2) / 2^23
 * (host, n*3 floats).  n <= 2^24. */
int brmppi_debug_box_muller(brmppi_ctx* ctx, const uint32_t* r, uint32_t n, float* out);

#ifdef __cplusplus
}
#endif
#endif /* BRMPPI_H */
