/*
 * CPU reference ("oracle") for ensemble integration of many independent,
 * low-dimensional ODE systems, after Nagy, Plavecz and Hegedus,
 * "Solving large number of non-stiff, low-dimensional ordinary differential
 * equation systems on GPUs and CPUs" (arXiv:2011.01740).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is plain, serial, double-precision
 * C compiled without floating-point contraction.  It exists to check the GPU
 * library; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header or constant table
 * with the GPU library.
 *
 * Layouts: every per-system array is component-major ("structure of arrays"):
 * element (c, i) of a [C][n] array is at index c * n + i.
 *
 * Models and their parameters
 *   ORC_QUAD    dx/dt = x^2 - p                  (Sec. 3, introductory example)
 *               D = 1, per-system p = (p), shared = none
 *   ORC_LORENZ  Lorenz system                    (Sec. 4.1)
 *               D = 3, per-system p = (rho), shared = (sigma, beta)
 *   ORC_KM      dimensionless Keller--Miksis     (Sec. 4.2)
 *               D = 2, per-system p = (P_A1 [Pa], f1 [Hz]),
 *               shared = (rho_L, c_L, p_V, sigma, mu_L, gamma, P_inf, R_E,
 *                         P_A2, f2, theta)
 *   ORC_PRV     pressure-relief valve + impacts  (Sec. 4.3)
 *               D = 3, per-system p = (q), shared = (kappa, delta, beta, r)
 *   ORC_DIV     dx/dt = 1/x - p x                (Sec. 3.3, the division
 *               variant of the introductory example) D = 1, p = (p)
 *   ORC_SIN     dx/dt = p sin(x)                 (Sec. 3.3, the
 *               transcendental variant)          D = 1, p = (p)
 *   ORC_KM6     Keller--Miksis with the six control parameters of Sec. 4.2
 *               per system: p = (P_A1, f1, P_A2, f2, theta, R_E),
 *               shared = (rho_L, c_L, p_V, sigma, mu_L, gamma, P_inf)
 */
#ifndef ENS_ORACLE_H
#define ENS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_QUAD = 0, ORC_LORENZ = 1, ORC_KM = 2, ORC_PRV = 3, ORC_DIV = 4, ORC_SIN = 5,
       ORC_KM6 = 6 };

/* Per-system status bits. */
enum {
  ORC_SYS_OK = 0,
  ORC_SYS_DT_MIN = 1,      /* a step was accepted only because h <= dt_min   */
  ORC_SYS_MAX_STEPS = 2,   /* stopped at the attempted-step cap              */
  ORC_SYS_NONFINITE = 4,   /* stopped: state or error estimate not finite    */
  ORC_SYS_SETTLED = 8,     /* PRV: no local maximum within t_cap; stopped    */
  ORC_SYS_EVENT_ITER = 16, /* an event was accepted after the retry cap      */
  ORC_SYS_SEATED = 32      /* PRV: the valve came to rest on its seat once   */
};

/* Statistics rows of the [ORC_NSTAT][n] int64 output. */
enum { ORC_ST_ACCEPTED = 0, ORC_ST_REJECTED = 1, ORC_ST_NRHS = 2,
       ORC_ST_IMPACTS = 3, ORC_ST_PHASES = 4, ORC_ST_EVRETRY = 5, ORC_NSTAT = 6 };

int orc_dim(int model);       /* state dimension D, or -1 */
int orc_nparam(int model);    /* per-system parameter count P, or -1 */
int orc_nshared(int model);   /* shared parameter count, or -1 */

/* Right-hand side of one system at time t.  Returns 0, or -1 for a bad model. */
int orc_rhs(int model, double t, const double *y, const double *p,
            const double *shared, double *dydt);

/* Keller--Miksis coefficients C0..C12 of one system (Sec. 4.2). */
void orc_km_coeffs(const double *p, const double *shared, double *C);

/* Classic RK4 with a fixed step (Sec. 3 and Sec. 4.1).  Runs nsteps steps of
 * size dt from t0 = 0.  y_out: [D][n] final state; y1max: [n] maximum of the
 * first component over the initial point and every step end point. */
int orc_rk4(int model, int64_t n, const double *params, const double *shared,
            const double *y0, double dt, int64_t nsteps, double *y_out,
            double *y1max, int nthreads);

/* Options of the adaptive Cash--Karp solver. */
typedef struct {
  double t_phase;    /* length of a fixed-length phase (QUAD, LORENZ, KM) */
  double dt0;        /* first step if h0 == NULL                           */
  double dt_min, dt_max;
  double rtol, atol;
  double event_tol;  /* PRV event tolerance                                */
  double t_cap;      /* PRV: longest Poincare phase before "settled"       */
  double v_stick;    /* PRV: impact speed below which the valve seats      */
  int64_t n_phases;  /* phases to integrate                                */
  int64_t n_record;  /* records kept: the last n_record phases             */
  int64_t max_impacts; /* PRV: stop after this many impacts (0: no limit)  */
  int64_t max_steps;   /* cap on attempted steps per system                */
  int32_t max_event_iter; /* secant retries per event                      */
  int32_t scheme;    /* ORC_CASH_KARP or ORC_DORMAND_PRINCE                  */
  int32_t locate_max; /* KM: also take y1 where y2 falls through 0 inside a
                         step, on the step's cubic Hermite interpolant       */
  int32_t lyapunov;  /* fixed-length phases: k = lyapunov tangents (0 .. D)
                        of the variational equation d(dv)/dt = J(t, y) dv
                        ride along (error control on everything); the
                        state is [y; v_1; ...; v_k] (D (1 + k) components);
                        at every phase end the tangents are orthonormalised
                        in order (Gram--Schmidt) and record fields 1 .. k
                        hold the log lengths before the scaling          */
} orc_opts;

/* Adaptive schemes: Cash--Karp 5(4) (six stages) and Dormand--Prince 5(4)
 * (seven stages, first-same-as-last). */
enum { ORC_CASH_KARP = 0, ORC_DORMAND_PRINCE = 1 };

/* Number of record fields per phase: PRV records (y1max, y1min), other models
 * record y1max. */
int orc_nrec_fields(int model);

/* Adaptive Runge--Kutta 5(4) (Cash--Karp or Dormand--Prince, opt->scheme)
 * with error control, integration phases, per-step accessories, and (PRV)
 * event location with the impact law.
 *
 *  params [P][n], shared [S], y0 [D][n];  t0, h0: [n] or NULL (0 and dt0).
 *  phi0 [n] or NULL (0): Keller--Miksis, the second drive's phase in cycles
 *    of omega2 at the start of the current phase (its forcing angle is
 *    2 pi (phi0 + C11 tau) + C12 within the phase); ignored otherwise.
 *  y_out [D][n], t_out [n], h_out [n], phi_out [n]: state, phase-local
 *    (QUAD/LORENZ/KM) or absolute (PRV) time, the step size the next call
 *    would try, and the second drive's phase (KM; passing all four back
 *    resumes the solve).
 *  records [n_record][F][n]: a ring, phase k of this call in slot
 *    k % n_record; F = 1 + k with k = opt->lyapunov tangents (y1max, then
 *    their log growths).
 *  With k tangents, y0 and y_out are [D (1 + k)][n]: the state, then the
 *    tangent vectors.  stats [ORC_NSTAT][n], status [n].  Any output pointer may
 *    be NULL.
 */
/* Jacobian d f_i / d y_j of a model's right-hand side at (t, y), row-major
 * [D][D] (Keller--Miksis: with the second drive's phase 0). */
int orc_jacobian(int model, double t, const double *y, const double *p,
                 const double *shared, double *J);

int orc_rkck45(int model, int64_t n, const double *params, const double *shared,
               const double *y0, const double *t0, const double *h0, const double *phi0,
               const orc_opts *opt, double *y_out, double *t_out, double *h_out,
               double *phi_out, double *records, int64_t *stats, int32_t *status,
               int nthreads);

/* What a system carries from one call to the next besides (y, t, h, phi):
 * the running phase's y1max and y1min, the start time of the current phase
 * (the valve's settled guard measures from it) and the valve's seated state
 * (1 or 0).  Rows of the [ORC_NCARRY][n] carry arrays. */
enum { ORC_CARRY_YMAX = 0, ORC_CARRY_YMIN = 1, ORC_CARRY_TPS = 2, ORC_CARRY_SEATED = 3,
       ORC_NCARRY = 4 };

/* orc_rkck45 with three optional arrays (NULL: not used):
 *  carry_in [ORC_NCARRY][n]: the carried values from a previous call's
 *    carry_out; NULL starts every system fresh (no running maximum or
 *    minimum, phase start at t0, not seated).  Passing carry_out back with
 *    y_out, t_out, h_out and phi_out resumes a solve exactly, also one that
 *    stopped inside a phase (step cap, impact budget).
 *  carry_out [ORC_NCARRY][n].
 *  hx [2][n]: the smallest and the largest accepted step of the call (steps
 *    cut short to land on a phase end are not counted); +inf / -inf when no
 *    step was accepted. */
int orc_rkck45_ext(int model, int64_t n, const double *params, const double *shared,
                   const double *y0, const double *t0, const double *h0, const double *phi0,
                   const orc_opts *opt, double *y_out, double *t_out, double *h_out,
                   double *phi_out, double *records, int64_t *stats, int32_t *status,
                   const double *carry_in, double *carry_out, double *hx, int nthreads);

/* One Cash--Karp step without error control, for order and stability tests:
 * y5 = fifth-order result, y4 = embedded fourth-order result. */
int orc_rkck_step(int model, double t, const double *y, const double *p,
                  const double *shared, double h, double *y5, double *y4);

/* The Cash--Karp coefficients the oracle uses: a[6][6] (row-major, lower
 * triangle), b5[6], b4[6], c[6]. */
void orc_rkck_tableau(double *a, double *b5, double *b4, double *c);

/* The Dormand--Prince 5(4) tableau: a [7][7] row-major, b5, b4, c [7]. */
void orc_rkdp_tableau(double *a, double *b5, double *b4, double *c);

/* One Dormand--Prince attempt from (t, y) with step h (k1 evaluated): the
 * fifth-order y5 and the embedded fourth-order y4. */
int orc_rkdp_step(int model, double t, const double *y, const double *p,
                  const double *shared, double h, double *y5, double *y4);

#ifdef __cplusplus
}
#endif
#endif
