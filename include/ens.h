/*
 * ens.h -- C ABI of libens, an MI355X (gfx950) library that integrates very
 * many independent, low-dimensional, non-stiff ODE systems in FP64, one
 * system per GPU lane with its state held in registers.
 *
 * The operations follow the problem statement of Nagy, Plavecz and Hegedus,
 * "Solving large number of non-stiff, low-dimensional ordinary differential
 * equation systems on GPUs and CPUs" (arXiv:2011.01740):
 *   - an ensemble is N independent instances of one model, each with its own
 *     parameters and initial conditions, solved by one thread each (Sec. 1,
 *     Sec. 3.2.1, per-thread approach);
 *   - models: dx/dt = x^2 - p (Sec. 3), Lorenz (Sec. 4.1), the dimensionless
 *     Keller--Miksis bubble equation with coefficients C0..C12 computed from
 *     the physical parameters (Sec. 4.2), the pressure-relief valve with the
 *     Newtonian impact law (Sec. 4.3);
 *   - solvers: classic RK4 with a fixed step (Sec. 3, Sec. 4.1) and the
 *     Runge--Kutta--Cash--Karp 5(4) scheme with embedded error control and
 *     equal relative and absolute tolerances (Sec. 4.2.1, Sec. 4.3.1);
 *   - integration phases (a forcing period for Keller--Miksis; local maximum
 *     to local maximum of the displacement for the valve), per-step
 *     accessories (phase maximum / minimum of y1 over the step points, no
 *     dense output), and event location with a tolerance (Sec. 4.2.1,
 *     Sec. 4.3, Sec. 4.3.1);
 *   - shared parameters common to an ensemble, kept in on-chip shared memory
 *     (Sec. 3.2.1).
 * Step-size controller, error norm, phase-end truncation and event location
 * are not printed in the paper; the library uses fixed readings:
 *   err_i = h sum_j (b5_j - b4_j) k_ji;  E = max_i |err_i| /
 *   (atol + rtol max(|y_i|, |y5_i|));  accept iff E <= 1 or h <= dt_min;
 *   fac = 0.9 E^(-1/5) (5 if E = 0); h *= clamp(fac, 0.2, 5) after an accepted
 *   step, clamp(fac, 0.2, 1) after a rejected one, then h is clamped to
 *   [dt_min, dt_max]; a phase's last step is truncated to land on its end and
 *   the next phase restarts from the untruncated proposal; an event
 *   overshoot (g > 0 before, g < -event_tol after) is retried from the same
 *   point with the secant step h g_old / (g_old - g_new).
 *
 * Conventions
 *   - Every function returns ENS_OK (0) or a negative ens_status.  Argument
 *     errors return ENS_E_INVAL and leave the handle unchanged; the message
 *     is available from ens_last_error.  HIP runtime failures return
 *     ENS_E_HIP.  Problems of single systems (a step-size floor, a non-finite
 *     state, a step cap) never fail a call: they set that system's status
 *     word (ENS_SYS_*), read through ENS_STATUS.
 *   - Per-system arrays are component-major ("structure of arrays"): element
 *     (c, i) of a [C][n] array is at c * n + i.  Doubles are IEEE binary64.
 *   - Pointers tagged with `where` are host memory (ENS_HOST) or device
 *     memory on the handle's device (ENS_DEVICE).  The library copies inputs
 *     and never keeps a caller pointer past the call.  It owns all its
 *     device buffers, allocated at ens_create / the first ens_solve that
 *     needs them and released by ens_destroy.
 *   - Work is enqueued on the handle's HIP stream.  ens_solve returns once
 *     the work is enqueued.  ens_read with ENS_HOST waits for the stream;
 *     with ENS_DEVICE it is stream-ordered and does not wait.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef LIBENS_ENS_H_
#define LIBENS_ENS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ens_ctx *ens_t;

enum ens_status {
  ENS_OK = 0,
  ENS_E_INVAL = -1,   /* bad argument (message in ens_last_error)            */
  ENS_E_NOMEM = -2,   /* device allocation failed                            */
  ENS_E_HIP = -3,     /* HIP runtime error                                   */
  ENS_E_ORDER = -4,   /* call out of order (e.g. solve before set_params)    */
  ENS_E_UNSUPPORTED = -5 /* combination the library does not implement     */
};

/* Models (dimension D / per-system parameters P / shared parameters S). */
enum ens_model {
  ENS_QUAD = 0,   /* dx/dt = x^2 - p.          D=1  P=1 (p)           S=0   */
  ENS_LORENZ = 1, /* Lorenz.                   D=3  P=1 (rho)         S=2:
                     (sigma, beta)                                           */
  ENS_KM = 2,     /* Keller--Miksis.           D=2  P=2 (P_A1 [Pa], f1 [Hz])
                     S=11: (rho_L, c_L, p_V, sigma, mu_L, gamma, P_inf, R_E,
                     P_A2, f2, theta), SI units.  With P_A2 != 0 (dual-
                     frequency drive, Sec. 4.2) the second drive runs on
                     the absolute time: its phase is carried across the
                     integration phases (ENS_DRIVE_PHASE)                  */
  ENS_PRV = 3,    /* relief valve + impacts.   D=3  P=1 (q)           S=4:
                     (kappa, delta, beta, r)                                 */
  /* The division and transcendental variants of the introductory example
   * (Sec. 3.3), built for RK4 only (measurement of what a division or a
   * sine costs per step against the FMA-only dx/dt = x^2 - p): */
  ENS_DIV = 4,    /* dx/dt = 1/x - p x.        D=1  P=1 (p)           S=0   */
  ENS_SIN = 5,    /* dx/dt = p sin(x).         D=1  P=1 (p)           S=0   */
  ENS_KM6 = 6     /* Keller--Miksis with the six control parameters of
                     Sec. 4.2 per system, for sweeps over any of them.
                                              D=2  P=6 (P_A1 [Pa], f1 [Hz],
                     P_A2 [Pa], f2 [Hz], theta, R_E [m])  S=7: (rho_L, c_L,
                     p_V, sigma, mu_L, gamma, P_inf).  Adaptive solvers
                     only; the same equation, phases, records and second-
                     drive phase as ENS_KM                                 */
};

/* Solvers: classic RK4 with a fixed step; Runge--Kutta--Cash--Karp 5(4)
 * (six stages per attempt, the paper's GPU and ODEINT scheme); Runge--Kutta--
 * Dormand--Prince 5(4) (the paper's Julia scheme, Sec. 4.2.1: seven stages,
 * the last being f at the new point, so an accepted step's last stage is the
 * next step's first -- 6 evaluations per attempt, plus one where a phase
 * starts or after an impact or lift-off).  Both adaptive schemes use the same
 * controller, phases, accessories and events. */
enum ens_solver { ENS_RK4 = 0, ENS_RKCK45 = 1, ENS_RKDP45 = 2 };
enum ens_where { ENS_HOST = 0, ENS_DEVICE = 1 };

/* Per-system status bits (ENS_STATUS). */
enum ens_sys_status {
  ENS_SYS_OK = 0,
  ENS_SYS_DT_MIN = 1,      /* a step was accepted only because h <= dt_min   */
  ENS_SYS_MAX_STEPS = 2,   /* stopped at max_steps attempted steps           */
  ENS_SYS_NONFINITE = 4,   /* stopped: state or error estimate not finite    */
  ENS_SYS_SETTLED = 8,     /* valve: no local maximum within t_cap; stopped  */
  ENS_SYS_EVENT_ITER = 16, /* an event was accepted after the retry cap      */
  ENS_SYS_SEATED = 32      /* valve: an impact slower than v_stick seated it */
};

/* Rows of the ENS_STATS int64 [ENS_NSTAT][n] array. */
enum ens_stat_row {
  ENS_ST_ACCEPTED = 0, ENS_ST_REJECTED = 1, ENS_ST_NRHS = 2,
  ENS_ST_IMPACTS = 3, ENS_ST_PHASES = 4, ENS_ST_EVRETRY = 5, ENS_NSTAT = 6
};

/* Rows of the ENS_CARRY double [ENS_NCARRY][n] array (adaptive solvers):
 * what a system's current integration phase has gathered so far.  A solve
 * that stops inside a phase (step cap, the valve's impact budget) leaves it
 * here, and the next solve on the handle continues that phase from it: the
 * running y1 maximum and minimum over the phase's step points (the
 * accessories of Sec. 4.2.1, per-system values updated after every
 * successful step), the time at which the phase began (the valve's settled
 * guard counts from it) and whether the valve rests on its seat (1) or not
 * (0).  ens_set_state resets every system to a fresh phase (-inf, +inf, its
 * t0, 0). */
enum ens_carry_row {
  ENS_CARRY_YMAX = 0, ENS_CARRY_YMIN = 1, ENS_CARRY_TPS = 2, ENS_CARRY_SEATED = 3,
  ENS_NCARRY = 4
};

#define ENS_MAX_ENSEMBLES 16
#define ENS_MAX_SHARED 16

/* Caller-supplied device allocator (ens_desc.alloc / free): alloc returns
 * `bytes` of device memory on the handle's device, at least 256-byte
 * aligned, or NULL on failure; free releases what alloc returned.  ctx is
 * ens_desc.alloc_ctx, passed through untouched.  Both run on the calling
 * thread, inside ens_create and the first calls that need a buffer (never
 * inside ens_solve or ens_order_by_work once the handle's buffers exist). */
typedef void *(*ens_alloc_fn)(size_t bytes, void *ctx);
typedef void (*ens_free_fn)(void *ptr, void *ctx);

/* Handle description.  The n systems may be split into n_ensembles
 * sub-ensembles (contiguous index ranges, each with its own shared
 * parameters and budgets) that are solved together in one launch. */
typedef struct {
  int32_t model;          /* enum ens_model                                  */
  int32_t solver;         /* enum ens_solver                                 */
  int64_t n;              /* number of systems, >= 0                         */
  int32_t n_ensembles;    /* 1..ENS_MAX_ENSEMBLES                            */
  int32_t device;         /* HIP device ordinal                              */
  const int64_t *ens_offsets; /* host, n_ensembles + 1 ascending offsets from
                             0 to n; NULL means one ensemble [0, n)          */
  void *hip_stream;       /* hipStream_t to enqueue on; NULL = null stream   */
  int32_t tangent;        /* adaptive solvers, fixed-length-phase models
                             (QUAD, LORENZ, KM, KM6): K = tangent vectors
                             (0 .. D) of the variational equation
                             d(v)/dt = J(t, y) v integrated along with each
                             system, for its K largest Lyapunov exponents.
                             The state becomes [D (1 + K)][n] (y, then
                             v_1 .. v_K; the caller sets the initial
                             tangents), all under error control; at every
                             phase end the tangents are orthonormalised in
                             order (Gram--Schmidt) and the record gains K
                             fields, the log length of each before its
                             scaling (F = 1 + K).  Exponent j over recorded
                             phases k: sum_k record[k][j] / (their number x
                             t_phase).  This is the per-phase trajectory
                             manipulation (renormalisation) of the paper's
                             introduction, done inside the solve.  0 = off */
  int32_t reserved_;      /* must be 0                                       */
  ens_alloc_fn alloc;     /* device allocator for every buffer the handle
                             owns, or NULL for hipMalloc / hipFree; alloc and
                             free are given together or not at all          */
  ens_free_fn free;
  void *alloc_ctx;        /* passed to alloc and free                        */
} ens_desc;

/* Creates a handle, allocates every buffer a solve on it needs on `device`
 * (parameters, state, outputs, and for the adaptive solvers the queue, the
 * queue order and the scratch of ens_order_by_work, and for Keller--Miksis
 * the coefficients of each system's right-hand side, 16 doubles per system,
 * which every solve derives first and its kernel then loads; records are allocated by
 * the first solve that keeps more of them than before; ens_set_order,
 * ens_set_params_gather and ens_tune allocate their scratch on first use and
 * keep it)
 * and sets every sub-ensemble's shared parameters to the model defaults
 * (Lorenz sigma = 10, beta = 8/3; Keller--Miksis water at 25 C with R_E =
 * 10 um; valve kappa = 1.25, delta = 10, beta = 20, r = 0.8).
 * Errors: ENS_E_INVAL (bad model/solver/n/offsets, out == NULL),
 * ENS_E_NOMEM, ENS_E_HIP.  *out is NULL on failure. */
int ens_create(const ens_desc *desc, ens_t *out);

/* Releases the handle and all its device memory after waiting for its
 * stream.  NULL is accepted.  Returns ENS_OK or ENS_E_HIP. */
int ens_destroy(ens_t h);

/* Message of the last failed call on h; with h NULL, of the calling thread's
 * last failed call on any handle (or one that had no handle yet, such as a
 * failed ens_create).  The string stays valid until the next call on that
 * handle (NULL: the thread's next failing call). */
const char *ens_last_error(ens_t h);

/* Per-system parameters p: [P][n] doubles (see ens_model), copied in.
 * Keller--Miksis: the lane derives C0..C12 from (P_A1, f1) and the shared
 * constants when it picks the system up.  Errors: ENS_E_INVAL, ENS_E_HIP. */
int ens_set_params(ens_t h, const double *p, int32_t where);

/* Per-system parameters gathered from a larger sweep: system i takes column
 * idx[i] of p_full [P][n_full] (device arrays; idx has the handle's n
 * entries, each in [0, n_full)).  Used to re-solve a subset of a sweep.
 * Errors: ENS_E_INVAL, ENS_E_HIP. */
int ens_set_params_gather(ens_t h, const double *p_full, int64_t n_full, const int64_t *idx);

/* Order in which the RKCK45 work queue hands systems to lanes: the k-th
 * system taken is order[k], a permutation of 0..n-1 (n entries, host or
 * device per `where`; copied in and checked).  Every system's arithmetic is
 * its own, so results do not depend on the order; the launch time does: a
 * longest-first order (for instance by the attempted steps of a previous
 * solve, ENS_STATS) keeps the longest systems from starting last and groups
 * systems of similar length in a wavefront (the paper's advice on limiting
 * divergence, Sec. 3.2.1).  NULL restores the index order.  RK4 ignores it.
 * Errors: ENS_E_INVAL (not a permutation; the previous order is dropped),
 * ENS_E_NOMEM, ENS_E_HIP. */
int ens_set_order(ens_t h, const int64_t *order, int32_t where);

/* Longest-first queue order from the last RKCK45 solve on this handle: the
 * systems sorted by attempted steps (accepted + rejected, ENS_STATS of that
 * solve) in decreasing order, ties in index order, become the order of
 * ens_set_order.  Typical use: solve a few phases, call this, solve the rest
 * (the step counts of the first phases predict those of the later ones).
 * Errors: ENS_E_ORDER (no previous RKCK45 solve), ENS_E_NOMEM, ENS_E_HIP. */
int ens_order_by_work(ens_t h);

/* Shared parameters of sub-ensemble `ensemble` (host array of n_shared
 * doubles, n_shared == S of the model). */
int ens_set_shared(ens_t h, int32_t ensemble, const double *shared, int32_t n_shared);

/* Budgets of sub-ensemble `ensemble` for the adaptive solver: phases to
 * integrate (>= 0; -1 = use ens_solve_opts.n_phases) and impact budget
 * (valve only: stop after this many impacts, 0 = none). */
int ens_set_budget(ens_t h, int32_t ensemble, int64_t n_phases, int64_t max_impacts);

/* Initial state y0: [D][n]; t0 and h0: [n] or NULL (t = 0, h = dt0).  Time
 * is phase-local for fixed-length phases (Keller--Miksis: tau in [0, 1)) and
 * absolute for the valve.  Keller--Miksis adaptive handles: the second
 * drive's phase (ENS_DRIVE_PHASE) is set to 0.  Passing the ENS_STATE /
 * ENS_TIME / ENS_H outputs of a solve (and, for a dual-frequency Keller--
 * Miksis drive, ENS_DRIVE_PHASE through ens_set_drive_phase) resumes it;
 * so does a further ens_solve without ens_set_state, which also continues a
 * phase that the previous solve stopped inside (ENS_CARRY).  Adaptive
 * handles: every system starts a fresh phase (ENS_CARRY reset). */
int ens_set_state(ens_t h, const double *y0, const double *t0, const double *h0,
                  int32_t where);

/* Adaptive solvers: sets the carried phase accessories, [ENS_NCARRY][n]
 * doubles in the ENS_CARRY layout (for instance read from another handle
 * after its solve), after ens_set_state.  Together with ens_set_state's
 * y0 / t0 / h0 (and ENS_DRIVE_PHASE) a solve stopped inside a phase resumes
 * exactly.  ENS_HOST copies and waits; ENS_DEVICE is stream-ordered.
 * Errors: ENS_E_UNSUPPORTED (RK4), ENS_E_ORDER (no state yet), ENS_E_INVAL,
 * ENS_E_HIP. */
int ens_set_carry(ens_t h, const double *carry, int32_t where);

/* Keller--Miksis, adaptive solvers (Sec. 4.2, dual-frequency forcing): sets
 * the second drive's phase per system, [n] doubles in cycles (the
 * ENS_DRIVE_PHASE layout), after ens_set_state.  ENS_HOST copies and waits;
 * ENS_DEVICE is stream-ordered.  Errors: ENS_E_UNSUPPORTED (other models or
 * RK4), ENS_E_ORDER (no state yet), ENS_E_INVAL, ENS_E_HIP. */
int ens_set_drive_phase(ens_t h, const double *phi, int32_t where);

/* Solve options.  Fields not used by the chosen solver are ignored. */
typedef struct {
  /* RK4 */
  double dt;          /* fixed step (> 0)                                    */
  int64_t n_steps;    /* steps (>= 0)                                        */
  /* RKCK45 */
  double t_phase;     /* length of a fixed-length phase (not the valve)      */
  double dt0, dt_min, dt_max, rtol, atol;
  double event_tol;   /* valve event tolerance on the event function         */
  double t_cap;       /* valve: longest phase before the system is settled   */
  double v_stick;     /* valve: impact speed below which it seats            */
  int64_t n_phases;   /* default phases per system                           */
  int64_t n_record;   /* record ring length R (>= 0): phase k -> slot k % R  */
  int64_t max_steps;  /* attempted-step cap per system, 0 = none             */
  int32_t max_event_iter; /* secant retries per event                        */
  /* launch (0 = tuned/default choice) */
  int32_t block;      /* threads per block: multiple of 64, <= 1024          */
  int32_t spl;        /* RK4: systems per lane, 1, 2 or 4                    */
  int32_t refill;     /* RKCK45: idle lanes a wave waits for before it takes
                         new systems from the queue (1..64)                  */
  int32_t grid;       /* RKCK45: persistent blocks (0 = resident capacity)   */
  int32_t use_graph;  /* RKCK45: capture the launch sequence in a hipGraph
                         and replay it                                       */
  /* accessory */
  int32_t locate_max; /* Keller--Miksis, adaptive solvers: besides the step
                         points, a phase's y1max also takes y1 where y2 = y1'
                         falls through 0 inside a step, located on the
                         step's cubic Hermite interpolant (f at both ends:
                         free with RKDP45, two evaluations with RKCK45) by
                         bisection; other models: ENS_E_UNSUPPORTED        */
  int32_t reserved_;  /* must be 0                                           */
  int64_t spread;     /* RKCK45/RKDP45 launch: the first `spread` positions
                         of the queue order (the longest systems, e.g. the
                         largest-budget sub-ensemble first in index order,
                         or after ens_order_by_work) are handed to the
                         first wave slot of each SIMD and the rest to the
                         others, so that long systems start one per SIMD
                         instead of sharing one; either group takes from the
                         other once its own is empty.  Waves that carry head
                         systems raise their issue priority (models without
                         their own remaining-work priority).  Results do not
                         depend on it.  0 = one queue; 0 <= spread <= n    */
} ens_solve_opts;

/* Fills opts with the defaults: dt 0.01, n_steps 1000, t_phase 1, dt0 1e-2,
 * dt_min 1e-14, dt_max 0.1, rtol = atol = 1e-10, event_tol 1e-6, t_cap 50,
 * v_stick 1e-9, n_phases 1, n_record 1, max_steps 0, max_event_iter 20, and
 * zero (automatic) launch fields. */
void ens_default_opts(ens_solve_opts *opts);

/* Enqueues the integration of all n systems from the current state.  RK4:
 * n_steps steps of dt; ENS_ACC receives the maximum of y1 over the initial
 * point and every step end point.  RKCK45: each system runs its phases (or
 * until its impact budget, step cap, or a terminating status), recording
 * per phase y1max (valve: y1 at the located local maximum, and y1min) into
 * the record ring, then the library-owned state holds the final y, t, h.
 * RKCK45 Keller--Miksis waves raise their hardware issue priority by their
 * estimated remaining work (last phase's attempts x phases left), so that
 * the longest systems are not slowed by short ones sharing a SIMD; results
 * do not depend on it, and the environment variable ENS_NO_PRIORITY (set,
 * any value) switches it off for the solves that follow.
 * Errors: ENS_E_INVAL (bad options), ENS_E_ORDER (no params or state yet),
 * ENS_E_UNSUPPORTED, ENS_E_NOMEM, ENS_E_HIP. */
int ens_solve(ens_t h, const ens_solve_opts *opts);

enum ens_field {
  ENS_STATE = 0,   /* double [D][n]                                          */
  ENS_TIME = 1,    /* double [n]                                             */
  ENS_H = 2,       /* double [n]: step the next solve would try              */
  ENS_ACC = 3,     /* double [n]: RK4 running max of y1                      */
  ENS_RECORDS = 4, /* double [R][F][n]; F = 2 for the valve (y1max, y1min),
                      1 otherwise; slots never written hold NaN             */
  ENS_STATS = 5,   /* int64 [ENS_NSTAT][n]                                   */
  ENS_STATUS = 6,  /* int32 [n]                                              */
  ENS_DRIVE_PHASE = 7, /* double [n], Keller--Miksis (ENS_KM, ENS_KM6)
                      adaptive handles: phase of the second drive in
                      cycles of omega2, in [0, 1), at
                      the start of the system's current integration phase;
                      its forcing angle is 2 pi (phase + C11 tau) + theta,
                      C11 = f2 / f1 (Sec. 4.2).  Zeroed by ens_set_state,
                      advanced by C11 t_phase (modulo 1) at every phase end */
  ENS_CARRY = 8    /* double [ENS_NCARRY][n], adaptive handles: the running
                      phase's accessories (enum ens_carry_row)              */
};

/* Copies a result field into dst (bytes must equal the field size).
 * ENS_HOST waits for the stream; ENS_DEVICE is stream-ordered.  Errors:
 * ENS_E_INVAL (size, field), ENS_E_ORDER (field not produced yet), ENS_E_HIP. */
int ens_read(ens_t h, int32_t field, void *dst, size_t bytes, int32_t where);

/* Size in bytes of a field as ens_read expects it (0 if not produced yet). */
size_t ens_field_bytes(ens_t h, int32_t field);

/* Autotuner.  Runs short trial solves of the handle's current problem for
 * each launch candidate -- RK4: block {1024, 512, 256, 128, 64} x systems per
 * lane {4, 2, 1} (in that order) on min(n_steps, trial_len) steps; RKCK45: block {64, 128,
 * 256} x refill threshold {1, 8, 32, 64} with every system capped at
 * min(phases, trial_len) phases and impacts -- timing each with HIP events
 * (best of three), restores the state it started from (state, clock, step,
 * drive phase, carried accessories), and stores the fastest choice (a
 * candidate displaces an earlier one only when faster by more than 2%, so
 * that near-ties resolve to the same choice from run to run) in a
 * process-wide cache keyed by (model, solver, device
 * architecture, floor(log2 n)).  Later ens_solve calls whose launch fields
 * are 0 use the cached choice.  If the environment variable ENS_TUNE_CACHE
 * names a file, the cache is read from it on first use and rewritten after
 * each tuning.  best (may be NULL) receives opts with the chosen launch
 * fields, best_ms (may be NULL) the trial time.  trial_len <= 0 means 256
 * (RK4) or 2 (RKCK45).  Errors: ENS_E_ORDER (no params/state), ENS_E_INVAL,
 * ENS_E_HIP. */
int ens_tune(ens_t h, const ens_solve_opts *opts, int64_t trial_len, ens_solve_opts *best,
             float *best_ms);

/* Launch actually used by the last ens_solve: block size, systems per lane,
 * grid, refill threshold.  Any pointer may be NULL. */
int ens_last_launch(ens_t h, int32_t *block, int32_t *spl, int32_t *grid, int32_t *refill);

/* Milliseconds between HIP events recorded on the handle's stream right
 * before and after the integration kernel of the last ens_solve (waits for
 * the stream). */
int ens_last_kernel_ms(ens_t h, float *ms);

/* Measurement helper (not part of the method): the FP64 FMA rate the device
 * sustains, from 8 independent FMA chains per lane, 8 waves per SIMD on every
 * compute unit, `iters` rounds per chain (one untimed warm-up launch, then one
 * launch timed with HIP events on the null stream).  *tflops receives
 * 2 x chains x iters x lanes / time in TFLOP/s, *ms (may be NULL) the time.
 * This is the peak the clock under dense FP64 load allows, beside the
 * published one that assumes the 2.4 GHz peak engine clock.
 * Errors: ENS_E_INVAL (iters <= 0, tflops NULL, bad device), ENS_E_HIP. */
int ens_micro_fma(int32_t device, int64_t iters, double *tflops, float *ms);

#ifdef __cplusplus
}
#endif
#endif /* LIBENS_ENS_H_ */
