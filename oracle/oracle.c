/*
 * CPU reference ("oracle") for the ensemble integrators.
 *
 * TEST INFRASTRUCTURE ONLY: plain serial FP64 C, built with
 * -O2 -ffp-contract=off and libm, one system at a time.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg use it.  The optional
 * OpenMP loop over systems only runs independent systems side by side; each
 * system is integrated by the same serial code.
 *
 * What it follows (arXiv:2011.01740, Nagy, Plavecz, Hegedus):
 *   - models: the introductory example dx/dt = x^2 - p (Sec. 3); the Lorenz
 *     system (Sec. 4.1); the dimensionless Keller--Miksis equation with its
 *     pre-computed coefficients C0..C12 (Sec. 4.2); the pressure-relief valve
 *     with the Newtonian impact law (Sec. 4.3);
 *   - solvers: classic fourth-order Runge--Kutta with a fixed step (Sec. 3,
 *     Sec. 4.1) and the Runge--Kutta--Cash--Karp 5(4) scheme with embedded
 *     error control, rtol = atol (Sec. 4.2.1, Sec. 4.3.1);
 *   - integration phases: the Keller--Miksis phase is one forcing period
 *     tau in [0, 1] of the first drive; the valve phase runs from one local
 *     maximum of the displacement to the next (Sec. 4.3);
 *   - the second drive of the Keller--Miksis forcing is a function of the
 *     absolute time (Sec. 4.2, the far-field pressure), so it does not
 *     restart with the phase: its angle is 2 pi (phi2 + C11 tau) + C12, with
 *     phi2 the drive's phase in cycles at the start of the phase, advanced by
 *     C11 t_phase (modulo 1) at every phase end;
 *   - accessories: the phase maximum of y1 taken over the natural step end
 *     points, updated after every successful step, without dense output
 *     (Sec. 4.2.1); for the valve the recorded maximum is y1 at the located
 *     local maximum (the Poincare point) and the phase minimum is taken over
 *     the step end points, impacts contributing 0 (Sec. 4.3);
 *   - events: impact (y1 reaches 0 moving down) and local maximum (y2 goes
 *     from positive to negative), located to an absolute tolerance on the
 *     event function, then the impact law y1 = 0, y2 -> -r y2 (Sec. 4.3,
 *     Sec. 4.3.1).
 *
 * The paper does not print the step-size controller, the error norm, the way
 * an event is located, or what happens after a truncated last step of a
 * phase.  The readings implemented here, binding for the GPU library too:
 *   - error:  err_i = h * sum_j (b5_j - b4_j) k_j,i ;
 *             E = max_i |err_i| / (atol + rtol * max(|y_i|, |y5_i|)) ;
 *   - the fifth-order solution is propagated;
 *   - accept iff E <= 1 or h <= dt_min (the latter sets ORC_SYS_DT_MIN);
 *   - fac = 0.9 E^(-1/5) (5 if E == 0); accepted: h *= clamp(fac, 0.2, 5);
 *     rejected: h *= clamp(fac, 0.2, 1); then h is clamped to [dt_min, dt_max];
 *   - a fixed-length phase truncates the step that would pass its end; if
 *     that step is accepted the phase ends exactly at t_phase, the clock is
 *     reset to 0 and the next phase starts with the untruncated proposal;
 *   - an event overshoot (g > 0 before the step, g < -tol after it) discards
 *     the step and retries from the same point with the secant step
 *     h * g_old / (g_old - g_new); the smallest such step wins; at most
 *     max_event_iter retries, after which the step is taken as located;
 *   - records are a ring: phase k (0-based, counted within one call) is
 *     stored in slot k mod n_record;
 *   - a call may stop inside a phase (step cap, impact budget); what the
 *     phase has gathered so far -- its running y1 maximum and minimum (the
 *     accessories of Sec. 4.2.1, per-system values updated after every
 *     successful step), its start time, and whether the valve rests on its
 *     seat -- is carried out of the call with (y, t, h) and, passed back,
 *     continues the phase exactly (orc_rkck45_ext).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXD 12  /* state dimension, the tangents included (Lorenz: 3 + 3 x 3) */
#define MAXDB 3  /* a model's own dimension */

int orc_dim(int model) {
  switch (model) {
    case ORC_QUAD: return 1;
    case ORC_LORENZ: return 3;
    case ORC_KM: return 2;
    case ORC_KM6: return 2;
    case ORC_PRV: return 3;
    case ORC_DIV: return 1;
    case ORC_SIN: return 1;
  }
  return -1;
}

int orc_nparam(int model) {
  switch (model) {
    case ORC_QUAD: return 1;
    case ORC_LORENZ: return 1;
    case ORC_KM: return 2;
    case ORC_KM6: return 6;
    case ORC_PRV: return 1;
    case ORC_DIV: return 1;
    case ORC_SIN: return 1;
  }
  return -1;
}

int orc_nshared(int model) {
  switch (model) {
    case ORC_QUAD: return 0;
    case ORC_LORENZ: return 2;
    case ORC_KM: return 11;
    case ORC_KM6: return 7;
    case ORC_PRV: return 4;
    case ORC_DIV: return 0;
    case ORC_SIN: return 0;
  }
  return -1;
}

int orc_nrec_fields(int model) { return model == ORC_PRV ? 2 : 1; }

/* ------------------------------------------------------------------ models */

/* Keller--Miksis coefficients, Sec. 4.2 (the list C0..C12 after the
 * dimensionless numerator and denominator).  p = (P_A1, f1); shared =
 * (rho_L, c_L, p_V, sigma, mu_L, gamma, P_inf, R_E, P_A2, f2, theta).
 * C8 carries the second drive's angular frequency omega2: the time derivative
 * of P_A2 sin(omega2 t + theta) brings omega2 into that term (the printed
 * formula shows omega1; with P_A2 = 0 both readings give C8 = 0). */
void orc_km_coeffs(const double *p, const double *sh, double *C) {
  const double PA1 = p[0], f1 = p[1];
  const double rhoL = sh[0], cL = sh[1], pV = sh[2], sigma = sh[3], muL = sh[4];
  const double gam = sh[5], Pinf = sh[6], RE = sh[7], PA2 = sh[8], f2 = sh[9];
  const double theta = sh[10];
  const double pi = 3.14159265358979323846;
  const double w1 = 2.0 * pi * f1;
  const double w2 = 2.0 * pi * f2;
  const double s = 2.0 * pi / (RE * w1); /* 2 pi / (R_E omega1) */
  const double pg0 = Pinf - pV + 2.0 * sigma / RE;
  C[0] = (1.0 / rhoL) * pg0 * s * s;
  C[1] = (1.0 - 3.0 * gam) / (rhoL * cL) * pg0 * s;
  C[2] = (Pinf - pV) / rhoL * s * s;
  C[3] = 2.0 * sigma / (rhoL * RE) * s * s;
  C[4] = 4.0 * muL / (rhoL * RE * RE) * (2.0 * pi / w1);
  C[5] = PA1 / rhoL * s * s;
  C[6] = PA2 / rhoL * s * s;
  C[7] = RE * w1 * PA1 / (rhoL * cL) * s * s;
  C[8] = RE * w2 * PA2 / (rhoL * cL) * s * s;
  C[9] = RE * w1 / (2.0 * pi * cL);
  C[10] = 3.0 * gam;
  C[11] = w2 / w1;
  C[12] = theta;
}

typedef struct {
  int model;
  int D;           /* integrated dimension: Db (1 + tangent)                  */
  int Db;          /* the model's own dimension                            */
  int tangent;     /* tangent vectors of the variational equation riding
                      along (Lyapunov exponents), 0 .. Db                  */
  double p[6];     /* per-system parameters                                */
  const double *sh;/* shared parameters                                    */
  double C[13];    /* Keller--Miksis coefficients                          */
  double phi2;     /* Keller--Miksis: phase of the second drive (cycles of
                      omega2) when the current phase began                 */
  int seated;      /* valve resting on its seat (sticking guard)           */
} sysctx;

/* dx/dt = x^2 - p (Sec. 3). */
static void rhs_quad(const sysctx *s, const double *y, double *f) {
  f[0] = y[0] * y[0] - s->p[0];
}

/* dx/dt = 1/x - p x: the introductory example with a division (Sec. 3.3). */
static void rhs_div(const sysctx *s, const double *y, double *f) {
  f[0] = 1.0 / y[0] - s->p[0] * y[0];
}

/* dx/dt = p sin(x): the introductory example with a transcendental function
 * (Sec. 3.3). */
static void rhs_sin(const sysctx *s, const double *y, double *f) {
  f[0] = s->p[0] * sin(y[0]);
}

/* Lorenz system (Sec. 4.1): sigma (y - x), p x - y - x z, x y - beta z. */
static void rhs_lorenz(const sysctx *s, const double *y, double *f) {
  const double sigma = s->sh[0], beta = s->sh[1], rho = s->p[0];
  f[0] = sigma * (y[1] - y[0]);
  f[1] = rho * y[0] - y[1] - y[0] * y[2];
  f[2] = y[0] * y[1] - beta * y[2];
}

/* Dimensionless Keller--Miksis equation (Sec. 4.2): dy1 = y2,
 * dy2 = N_KM / D_KM, with tau the dimensionless time. */
static void rhs_km(const sysctx *s, double tau, const double *y, double *f) {
  const double *C = s->C;
  const double pi = 3.14159265358979323846;
  const double y1 = y[0], y2 = y[1];
  const double rx = 1.0 / y1;
  const double a1 = 2.0 * pi * tau;
  /* tau is local to the phase (it restarts at 0 every forcing period of the
   * first drive); the second drive keeps running across phases, so its angle
   * is 2 pi C11 tau_abs + C12 with tau_abs = (phase start) + tau, written as
   * 2 pi (phi2 + C11 tau) + C12, phi2 being C11 x (phase start) reduced
   * modulo 1 */
  const double a2 = 2.0 * pi * (s->phi2 + C[11] * tau) + C[12];
  const double N = (C[0] + C[1] * y2) * pow(rx, C[10])
                   - C[2] * (1.0 + C[9] * y2)
                   - C[3] * rx
                   - C[4] * y2 * rx
                   - (1.0 - C[9] * y2 / 3.0) * 1.5 * y2 * y2
                   - (C[5] * sin(a1) + C[6] * sin(a2)) * (1.0 + C[9] * y2)
                   - y1 * (C[7] * cos(a1) + C[8] * cos(a2));
  const double Dn = y1 - C[9] * y1 * y2 + C[4] * C[9];
  f[0] = y2;
  f[1] = N / Dn;
}

/* Pressure-relief valve (Sec. 4.3): y1' = y2, y2' = -kappa y2 - (y1 + delta)
 * + y3, y3' = beta (q - y1 sqrt(y3)).  While the valve rests on its seat the
 * body does not move and the chamber fills: y1' = y2' = 0, y3' = beta q. */
static void rhs_prv(const sysctx *s, const double *y, double *f) {
  const double kappa = s->sh[0], delta = s->sh[1], beta = s->sh[2], q = s->p[0];
  if (s->seated) {
    f[0] = 0.0;
    f[1] = 0.0;
    f[2] = beta * q;
    return;
  }
  f[0] = y[1];
  f[1] = -kappa * y[1] - (y[0] + delta) + y[2];
  f[2] = beta * (q - y[0] * sqrt(y[2]));
}

static void rhs_base(const sysctx *s, double t, const double *y, double *f) {
  switch (s->model) {
    case ORC_QUAD: rhs_quad(s, y, f); break;
    case ORC_LORENZ: rhs_lorenz(s, y, f); break;
    case ORC_KM:
    case ORC_KM6: rhs_km(s, t, y, f); break;
    case ORC_PRV: rhs_prv(s, y, f); break;
    case ORC_DIV: rhs_div(s, y, f); break;
    case ORC_SIN: rhs_sin(s, y, f); break;
  }
}

/* Jacobian J[i][j] = d f_i / d y_j of the model's right-hand side, row-major
 * [Db][Db], for the variational equation d(dy)/dt = J(t, y) dy. */
static void jacobian(const sysctx *s, double t, const double *y, double *J) {
  switch (s->model) {
    case ORC_QUAD: J[0] = 2.0 * y[0]; break;
    case ORC_DIV: J[0] = -1.0 / (y[0] * y[0]) - s->p[0]; break;
    case ORC_SIN: J[0] = s->p[0] * cos(y[0]); break;
    case ORC_LORENZ: {
      const double sigma = s->sh[0], beta = s->sh[1], rho = s->p[0];
      J[0] = -sigma;       J[1] = sigma; J[2] = 0.0;
      J[3] = rho - y[2];   J[4] = -1.0;  J[5] = -y[0];
      J[6] = y[1];         J[7] = y[0];  J[8] = -beta;
      break;
    }
    case ORC_KM:
    case ORC_KM6: {
      /* f2 = N / D with N, D of the Keller--Miksis right-hand side:
       * d f2 / d y_j = (dN/dy_j - f2 dD/dy_j) / D */
      const double *C = s->C;
      const double pi = 3.14159265358979323846;
      const double y1 = y[0], y2 = y[1];
      const double rx = 1.0 / y1;
      const double a1 = 2.0 * pi * t;
      const double a2 = 2.0 * pi * (s->phi2 + C[11] * t) + C[12];
      const double fs = C[5] * sin(a1) + C[6] * sin(a2);
      const double fc = C[7] * cos(a1) + C[8] * cos(a2);
      const double gas = pow(rx, C[10]);
      double f[2];
      rhs_km(s, t, y, f);
      const double Dn = y1 - C[9] * y1 * y2 + C[4] * C[9];
      const double dN1 = -C[10] * (C[0] + C[1] * y2) * gas * rx + C[3] * rx * rx
                         + C[4] * y2 * rx * rx - fc;
      const double dN2 = C[1] * gas - C[2] * C[9] - C[4] * rx - 3.0 * y2
                         + 1.5 * C[9] * y2 * y2 - C[9] * fs;
      const double dD1 = 1.0 - C[9] * y2, dD2 = -C[9] * y1;
      J[0] = 0.0;
      J[1] = 1.0;
      J[2] = (dN1 - f[1] * dD1) / Dn;
      J[3] = (dN2 - f[1] * dD2) / Dn;
      break;
    }
    case ORC_PRV: {
      const double kappa = s->sh[0], beta = s->sh[2], q = s->p[0];
      const double r = sqrt(y[2]);
      J[0] = 0.0;          J[1] = 1.0;    J[2] = 0.0;
      J[3] = -1.0;         J[4] = -kappa; J[5] = 1.0;
      J[6] = -beta * r;    J[7] = 0.0;    J[8] = -beta * y[0] / (2.0 * r);
      (void)q;
      break;
    }
  }
}

/* The integrated right-hand side: the model's, and with the tangent the
 * variational equation on the second half of the state. */
static void rhs(const sysctx *s, double t, const double *y, double *f) {
  rhs_base(s, t, y, f);
  if (s->tangent) {
    const int Db = s->Db;
    double J[MAXDB * MAXDB];
    jacobian(s, t, y, J);
    for (int v = 1; v <= s->tangent; ++v)
      for (int i = 0; i < Db; ++i) {
        double acc = 0.0;
        for (int j = 0; j < Db; ++j) acc += J[i * Db + j] * y[v * Db + j];
        f[v * Db + i] = acc;
      }
  }
}

static int ctx_init(sysctx *s, int model, const double *p, const double *sh) {
  if (orc_dim(model) < 0) return -1;
  memset(s, 0, sizeof(*s));
  s->model = model;
  s->D = orc_dim(model);
  s->Db = s->D;
  for (int j = 0; j < orc_nparam(model); ++j) s->p[j] = p[j];
  s->sh = sh;
  if (model == ORC_KM) orc_km_coeffs(p, sh, s->C);
  if (model == ORC_KM6) {
    /* the same equation with (P_A2, f2, theta, R_E) taken per system */
    const double p2[2] = {p[0], p[1]};
    const double sh11[11] = {sh[0], sh[1], sh[2], sh[3], sh[4], sh[5], sh[6],
                             p[5], p[2], p[3], p[4]};
    orc_km_coeffs(p2, sh11, s->C);
  }
  return 0;
}

int orc_jacobian(int model, double t, const double *y, const double *p,
                 const double *shared, double *J) {
  sysctx s;
  if (ctx_init(&s, model, p, shared)) return -1;
  jacobian(&s, t, y, J);
  return 0;
}

int orc_rhs(int model, double t, const double *y, const double *p,
            const double *shared, double *dydt) {
  sysctx s;
  if (ctx_init(&s, model, p, shared)) return -1;
  rhs(&s, t, y, dydt);
  return 0;
}

/* ------------------------------------------------------------------ RK4 */

/* Classic fourth-order Runge--Kutta step (Sec. 3):
 * k1 = f(t, y), k2 = f(t + h/2, y + h/2 k1), k3 = f(t + h/2, y + h/2 k2),
 * k4 = f(t + h, y + h k3), y <- y + h/6 (k1 + 2 k2 + 2 k3 + k4). */
static void rk4_step(const sysctx *s, double t, double *y, double h) {
  const int D = s->D;
  double k1[MAXD], k2[MAXD], k3[MAXD], k4[MAXD], yt[MAXD];
  rhs(s, t, y, k1);
  for (int i = 0; i < D; ++i) yt[i] = y[i] + (h / 2.0) * k1[i];
  rhs(s, t + h / 2.0, yt, k2);
  for (int i = 0; i < D; ++i) yt[i] = y[i] + (h / 2.0) * k2[i];
  rhs(s, t + h / 2.0, yt, k3);
  for (int i = 0; i < D; ++i) yt[i] = y[i] + h * k3[i];
  rhs(s, t + h, yt, k4);
  for (int i = 0; i < D; ++i)
    y[i] = y[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

int orc_rk4(int model, int64_t n, const double *params, const double *shared,
            const double *y0, double dt, int64_t nsteps, double *y_out,
            double *y1max, int nthreads) {
  const int D = orc_dim(model), P = orc_nparam(model);
  if (D < 0 || n < 0 || nsteps < 0) return -1;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
  for (int64_t i = 0; i < n; ++i) {
    double p[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, y[MAXD];
    for (int j = 0; j < P; ++j) p[j] = params[j * n + i];
    sysctx s;
    ctx_init(&s, model, p, shared);
    for (int c = 0; c < D; ++c) y[c] = y0[c * n + i];
    double ymax = y[0];
    for (int64_t j = 0; j < nsteps; ++j) {
      rk4_step(&s, (double)j * dt, y, dt);
      if (y[0] > ymax) ymax = y[0];
    }
    if (y_out)
      for (int c = 0; c < D; ++c) y_out[c * n + i] = y[c];
    if (y1max) y1max[i] = ymax;
  }
  return 0;
}

/* ------------------------------------------------------------------ Cash--Karp */

/* Runge--Kutta--Cash--Karp 5(4) coefficients (J. R. Cash and A. H. Karp,
 * ACM TOMS 16 (1990) 201), the scheme the paper's GPU package uses. */
static const double CK_C[6] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0};
static const double CK_A[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0, 0, 0},
    {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0, 0},
    {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0,
     253.0 / 4096.0, 0}};
static const double CK_B5[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0,
                                0.0, 512.0 / 1771.0};
static const double CK_B4[6] = {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0,
                                13525.0 / 55296.0, 277.0 / 14336.0, 1.0 / 4.0};

void orc_rkck_tableau(double *a, double *b5, double *b4, double *c) {
  for (int i = 0; i < 6; ++i) {
    for (int j = 0; j < 6; ++j) a[i * 6 + j] = CK_A[i][j];
    b5[i] = CK_B5[i];
    b4[i] = CK_B4[i];
    c[i] = CK_C[i];
  }
}

/* One attempted step: the six stages, the fifth-order result y5 and the
 * embedded error estimate err = h * sum_j (b5_j - b4_j) k_j. */
static void rkck_attempt(const sysctx *s, double t, const double *y, double h,
                         double *y5, double *err) {
  const int D = s->D;
  double k[6][MAXD], yt[MAXD];
  rhs(s, t, y, k[0]);
  for (int st = 1; st < 6; ++st) {
    for (int i = 0; i < D; ++i) {
      double acc = 0.0;
      for (int l = 0; l < st; ++l) acc += CK_A[st][l] * k[l][i];
      yt[i] = y[i] + h * acc;
    }
    rhs(s, t + CK_C[st] * h, yt, k[st]);
  }
  for (int i = 0; i < D; ++i) {
    double a5 = 0.0, ae = 0.0;
    for (int l = 0; l < 6; ++l) {
      a5 += CK_B5[l] * k[l][i];
      ae += (CK_B5[l] - CK_B4[l]) * k[l][i];
    }
    y5[i] = y[i] + h * a5;
    err[i] = h * ae;
  }
}

int orc_rkck_step(int model, double t, const double *y, const double *p,
                  const double *shared, double h, double *y5, double *y4) {
  sysctx s;
  double err[MAXD];
  if (ctx_init(&s, model, p, shared)) return -1;
  rkck_attempt(&s, t, y, h, y5, err);
  for (int i = 0; i < s.D; ++i) y4[i] = y5[i] - err[i];
  return 0;
}

/* ------------------------------------------------------------------ Dormand--Prince */

/* Runge--Kutta--Dormand--Prince 5(4) coefficients (J. R. Dormand and P. J.
 * Prince, J. Comput. Appl. Math. 6 (1980) 19), the scheme of the paper's
 * Julia runs (Sec. 4.2.1).  The last row of A equals the fifth-order weights:
 * the seventh stage is the derivative at the new point, so an accepted step's
 * k7 is the next step's k1 (first same as last). */
static const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
static const double DP_A[7][7] = {
    {0, 0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0}};
static const double DP_B5[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                                -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
static const double DP_B4[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                                -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};

void orc_rkdp_tableau(double *a, double *b5, double *b4, double *c) {
  for (int i = 0; i < 7; ++i) {
    for (int j = 0; j < 7; ++j) a[i * 7 + j] = DP_A[i][j];
    b5[i] = DP_B5[i];
    b4[i] = DP_B4[i];
    c[i] = DP_C[i];
  }
}

/* One attempted step.  k1 holds f(t, y) on entry if have_k1, else it is
 * evaluated (and returned in k1); k7 receives f(t + h, y5).  Returns the
 * number of RHS evaluations (6 or 7). */
static int rkdp_attempt(const sysctx *s, double t, const double *y, double h, double *k1,
                        int have_k1, double *y5, double *err, double *k7) {
  const int D = s->D;
  double k[7][MAXD], yt[MAXD];
  int nf = 6;
  if (!have_k1) {
    rhs(s, t, y, k1);
    nf = 7;
  }
  for (int i = 0; i < D; ++i) k[0][i] = k1[i];
  for (int st = 1; st < 7; ++st) {
    for (int i = 0; i < D; ++i) {
      double acc = 0.0;
      for (int l = 0; l < st; ++l) acc += DP_A[st][l] * k[l][i];
      yt[i] = y[i] + h * acc;
    }
    if (st == 6)
      for (int i = 0; i < D; ++i) y5[i] = yt[i];     /* row 7 of A = b5 */
    rhs(s, t + DP_C[st] * h, yt, k[st]);
  }
  for (int i = 0; i < D; ++i) {
    double ae = 0.0;
    for (int l = 0; l < 7; ++l) ae += (DP_B5[l] - DP_B4[l]) * k[l][i];
    err[i] = h * ae;
    k7[i] = k[6][i];
  }
  return nf;
}

int orc_rkdp_step(int model, double t, const double *y, const double *p,
                  const double *shared, double h, double *y5, double *y4) {
  sysctx s;
  double err[MAXD], k1[MAXD], k7[MAXD];
  if (ctx_init(&s, model, p, shared)) return -1;
  rkdp_attempt(&s, t, y, h, k1, 0, y5, err, k7);
  for (int i = 0; i < s.D; ++i) y4[i] = y5[i] - err[i];
  return 0;
}

static double clampd(double x, double lo, double hi) {
  return x < lo ? lo : (x > hi ? hi : x);
}

static void put_record(double *records, int64_t n, int F, int64_t R, int64_t phase,
                       int64_t i, double ymax, double ymin) {
  if (!records || R <= 0) return;
  const int64_t slot = phase % R;
  records[(slot * F + 0) * n + i] = ymax;
  if (F > 1) records[(slot * F + 1) * n + i] = ymin;
}

/* The record fields after the first with the tangents: the phase's log
 * growth of each tangent after Gram--Schmidt. */
static void put_growth(double *records, int64_t n, int F, int64_t R, int64_t phase, int64_t i,
                       const double *g, int k) {
  if (!records || R <= 0) return;
  const int64_t slot = phase % R;
  for (int v = 0; v < k; ++v) records[(slot * F + 1 + v) * n + i] = g[v];
}

/* Dense output of a step from (t, y0) to (t + h, y1) with derivatives f0,
 * f1 at its ends: the cubic Hermite interpolant, component c at theta in
 * [0, 1]. */
static double hermite(const double *y0, const double *y1, const double *f0, const double *f1,
                      double h, int c, double th) {
  const double t2 = th * th, t3 = t2 * th;
  return (2.0 * t3 - 3.0 * t2 + 1.0) * y0[c] + (t3 - 2.0 * t2 + th) * h * f0[c] +
         (-2.0 * t3 + 3.0 * t2) * y1[c] + (t3 - t2) * h * f1[c];
}

/* A local maximum of y1 inside a step in which y2 = y1' falls from > 0 to
 * <= 0: the zero of the interpolant's y2 by bisection on theta (60 halvings
 * reach adjacent doubles), and the interpolant's y1 there. */
static double located_max(const double *y0, const double *y1, const double *f0,
                          const double *f1, double h) {
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (hermite(y0, y1, f0, f1, h, 1, mid) > 0.0)
      lo = mid;
    else
      hi = mid;
  }
  return hermite(y0, y1, f0, f1, h, 0, 0.5 * (lo + hi));
}

/* Smallest and largest accepted step (hx may be NULL).  Steps cut short to
 * land on a phase end are not counted: their length is set by the phase
 * end, not by the error control. */
static void note_step(double hx[2], double h) {
  if (!hx) return;
  if (h < hx[0]) hx[0] = h;
  if (h > hx[1]) hx[1] = h;
}

/* Integrate one system through its phases.  y, t, h are updated in place. */
static void solve_one(sysctx *s, const orc_opts *o, double *y, double *tp, double *hp,
                      double *records, int64_t n, int64_t i, int64_t st[ORC_NSTAT],
                      int32_t *status, double carry[ORC_NCARRY], double hx[2]) {
  const int D = s->D;
  /* with k tangents the record fields 1 .. k are the phase's log growths */
  const int F = s->tangent ? 1 + s->tangent : orc_nrec_fields(s->model);
  const int Db = s->Db;            /* the model's own components      */
  const int fixed_len = (s->model != ORC_PRV);
  const double tol_ev = o->event_tol;
  double t = *tp, h = *hp;
  /* the running phase's accessories and the seated state, carried over
   * from the previous call (a solve that stopped inside a phase resumes
   * it) */
  double t_ps = carry[ORC_CARRY_TPS];     /* start time of the current phase */
  double ymax = carry[ORC_CARRY_YMAX], ymin = carry[ORC_CARRY_YMIN];
  s->seated = carry[ORC_CARRY_SEATED] != 0.0;
  int64_t phase = 0, attempts = 0;
  int ev_iter = 0;
  double y5[MAXD], err[MAXD];
  /* Dormand--Prince: k1 = f(t, y) of the next attempt when have_k1 */
  const int dp = o->scheme == ORC_DORMAND_PRINCE;
  double k1[MAXD], k7[MAXD];
  int have_k1 = 0;

  while (phase < o->n_phases) {
    if (o->max_steps > 0 && attempts >= o->max_steps) {
      *status |= ORC_SYS_MAX_STEPS;
      break;
    }
    double h_try = h;
    int trunc = 0;
    if (fixed_len && t + h_try >= o->t_phase) {
      h_try = o->t_phase - t;
      trunc = 1;
    }
    if (dp) {
      st[ORC_ST_NRHS] += rkdp_attempt(s, t, y, h_try, k1, have_k1, y5, err, k7);
      have_k1 = 1;  /* k1 = f(t, y) stays valid while the step is retried */
    } else {
      rkck_attempt(s, t, y, h_try, y5, err);
      st[ORC_ST_NRHS] += 6;
    }
    attempts++;

    /* error norm */
    double E = 0.0;
    int finite = 1;
    /* with the tangent every component is under error control: near a
     * stable fixed point the model's own components would let the step
     * grow past the tangent's stability limit */
    for (int c = 0; c < D; ++c) {
      const double sc = o->atol + o->rtol * fmax(fabs(y[c]), fabs(y5[c]));
      const double r = fabs(err[c]) / sc;
      if (!isfinite(y5[c]) || !isfinite(r)) finite = 0;
      if (r > E) E = r;
    }
    if (!finite) {
      *status |= ORC_SYS_NONFINITE;
      break;
    }
    const double fac = (E == 0.0) ? 5.0 : 0.9 * pow(E, -0.2);
    if (E > 1.0 && h_try > o->dt_min) {
      st[ORC_ST_REJECTED]++;
      h = clampd(h_try * clampd(fac, 0.2, 1.0), o->dt_min, o->dt_max);
      continue;
    }
    if (E > 1.0) *status |= ORC_SYS_DT_MIN;
    const double h_next = clampd(h_try * clampd(fac, 0.2, 5.0), o->dt_min, o->dt_max);

    if (s->model == ORC_PRV) {
      /* event detection on the step (t, y) -> (t + h_try, y5) */
      double hs = INFINITY;
      int over = 0;
      if (!s->seated) {
        const double g1o = y[0], g1n = y5[0];   /* impact: y1 decreasing  */
        const double g2o = y[1], g2n = y5[1];   /* local max: y2 decreasing */
        if (g1o > 0.0 && g1n < -tol_ev) {
          hs = fmin(hs, h_try * g1o / (g1o - g1n));
          over = 1;
        }
        if (g1o == 0.0 && g1n < -tol_ev) {
          /* a rebound swallowed inside one step: no secant is defined from
           * g = 0, so the step is halved */
          hs = fmin(hs, 0.5 * h_try);
          over = 1;
        }
        if (g2o > 0.0 && g2n < -tol_ev) {
          hs = fmin(hs, h_try * g2o / (g2o - g2n));
          over = 1;
        }
      } else {
        const double delta = s->sh[1];
        const double g3o = y[2] - delta, g3n = y5[2] - delta; /* increasing */
        if (g3o < 0.0 && g3n > tol_ev) {
          hs = fmin(hs, h_try * (-g3o) / (g3n - g3o));
          over = 1;
        }
      }
      if (over && ev_iter < o->max_event_iter) {
        ev_iter++;
        st[ORC_ST_EVRETRY]++;
        h = hs;
        continue;
      }
      if (over) *status |= ORC_SYS_EVENT_ITER;
      ev_iter = 0;

      /* accept */
      const double y1o = y[0], y2o = y[1];
      (void)y1o;
      const int was_seated = s->seated;
      for (int c = 0; c < D; ++c) y[c] = y5[c];
      t = t + h_try;
      st[ORC_ST_ACCEPTED]++;
      note_step(hx, h_try);
      h = h_next;
      for (int c = 0; c < D; ++c) k1[c] = k7[c];   /* first same as last */
      int phase_end = 0, stop = 0;
      if (was_seated) {
        if (y[2] - s->sh[1] >= 0.0) {
          s->seated = 0; /* lift-off */
          have_k1 = 0;
        }
      } else if (y[0] <= 0.0 && y[1] < 0.0) {
        have_k1 = 0;   /* the impact law changes the state */
        /* located impact: Newtonian restitution, Sec. 4.3 */
        const double v_in = y[1];
        const double r = s->sh[3], delta = s->sh[1];
        y[0] = 0.0;
        y[1] = -r * v_in;
        st[ORC_ST_IMPACTS]++;
        if (fabs(v_in) < o->v_stick && y[2] < delta) {
          s->seated = 1;
          y[1] = 0.0;
          *status |= ORC_SYS_SEATED;
        }
        if (o->max_impacts > 0 && st[ORC_ST_IMPACTS] >= o->max_impacts) stop = 1;
      } else if (y2o > 0.0 && y[1] <= 0.0) {
        phase_end = 1; /* located local maximum of y1 */
      }
      if (y[0] > ymax) ymax = y[0];
      if (y[0] < ymin) ymin = y[0];
      if (phase_end) {
        /* the Poincare point: y1 at the located local maximum */
        have_k1 = 0;   /* every phase starts with k1 evaluated */
        put_record(records, n, F, o->n_record, phase, i, y[0], ymin);
        phase++;
        st[ORC_ST_PHASES] = phase;
        ymax = -INFINITY;
        ymin = INFINITY;
        t_ps = t;
      } else if (t - t_ps >= o->t_cap) {
        /* settled guard: no local maximum for t_cap time units */
        put_record(records, n, F, o->n_record, phase, i, ymax, ymin);
        phase++;
        st[ORC_ST_PHASES] = phase;
        *status |= ORC_SYS_SETTLED;
        stop = 1;
      }
      if (stop) break;
      continue;
    }

    /* fixed-length phases (QUAD, LORENZ, KM) */
    if (o->locate_max && (s->model == ORC_KM || s->model == ORC_KM6) && y[1] > 0.0 &&
        y5[1] <= 0.0) {
      /* the maximum of y1 between the step points: Dormand--Prince has f at
       * both ends (k1, k7); Cash--Karp evaluates them */
      double f0[MAXD], f1[MAXD];
      if (dp) {
        for (int c = 0; c < D; ++c) {
          f0[c] = k1[c];
          f1[c] = k7[c];
        }
      } else {
        rhs(s, t, y, f0);
        rhs(s, t + h_try, y5, f1);
        st[ORC_ST_NRHS] += 2;
      }
      const double ym = located_max(y, y5, f0, f1, h_try);
      if (ym > ymax) ymax = ym;
    }
    for (int c = 0; c < D; ++c) y[c] = y5[c];
    for (int c = 0; c < D; ++c) k1[c] = k7[c];   /* first same as last */
    st[ORC_ST_ACCEPTED]++;
    if (y[0] > ymax) ymax = y[0];
    if (trunc) {
      have_k1 = 0;   /* every phase starts with k1 evaluated (the clock resets) */
      /* the phase ends exactly at t_phase; next phase from 0 with the
       * untruncated proposal h */
      double growth[MAXDB];
      if (s->tangent) {
        /* Lyapunov renormalisation (Benettin et al.): Gram--Schmidt on the
         * tangents in order, each first made orthogonal to the ones before
         * it and then scaled to unit length; its log length before the
         * scaling is the phase's growth along that direction */
        for (int v = 1; v <= s->tangent; ++v) {
          double *w = y + v * Db;
          for (int u = 1; u < v; ++u) {
            const double *q = y + u * Db;
            double dot = 0.0;
            for (int c = 0; c < Db; ++c) dot += q[c] * w[c];
            for (int c = 0; c < Db; ++c) w[c] = w[c] - dot * q[c];
          }
          double nrm2 = 0.0;
          for (int c = 0; c < Db; ++c) nrm2 += w[c] * w[c];
          const double nrm = sqrt(nrm2);
          growth[v - 1] = log(nrm);
          for (int c = 0; c < Db; ++c) w[c] = w[c] / nrm;
        }
        put_record(records, n, F, o->n_record, phase, i, ymax, 0.0);
        put_growth(records, n, F, o->n_record, phase, i, growth, s->tangent);
      } else {
        put_record(records, n, F, o->n_record, phase, i, ymax, ymin);
      }
      phase++;
      st[ORC_ST_PHASES] = phase;
      ymax = -INFINITY;
      t = 0.0;
      t_ps = 0.0;
      if (s->model == ORC_KM || s->model == ORC_KM6) {
        /* the second drive went through C11 x t_phase cycles in the phase */
        const double v = s->phi2 + s->C[11] * o->t_phase;
        s->phi2 = v - floor(v);
      }
    } else {
      note_step(hx, h_try);
      t = t + h_try;
      h = h_next;
    }
  }
  *tp = t;
  *hp = h;
  carry[ORC_CARRY_YMAX] = ymax;
  carry[ORC_CARRY_YMIN] = ymin;
  carry[ORC_CARRY_TPS] = t_ps;
  carry[ORC_CARRY_SEATED] = s->seated ? 1.0 : 0.0;
}

int orc_rkck45(int model, int64_t n, const double *params, const double *shared,
               const double *y0, const double *t0, const double *h0, const double *phi0,
               const orc_opts *opt, double *y_out, double *t_out, double *h_out,
               double *phi_out, double *records, int64_t *stats, int32_t *status,
               int nthreads) {
  return orc_rkck45_ext(model, n, params, shared, y0, t0, h0, phi0, opt, y_out, t_out, h_out,
                        phi_out, records, stats, status, NULL, NULL, NULL, nthreads);
}

int orc_rkck45_ext(int model, int64_t n, const double *params, const double *shared,
                   const double *y0, const double *t0, const double *h0, const double *phi0,
                   const orc_opts *opt, double *y_out, double *t_out, double *h_out,
                   double *phi_out, double *records, int64_t *stats, int32_t *status,
                   const double *carry_in, double *carry_out, double *hx, int nthreads) {
  const int D = orc_dim(model), P = orc_nparam(model);
  if (D < 0 || n < 0 || !opt) return -1;
  if (opt->n_record < 0 || opt->n_phases < 0) return -1;
  if (!(opt->rtol >= 0.0) || !(opt->atol > 0.0) || !(opt->dt_min > 0.0) ||
      !(opt->dt_max >= opt->dt_min))
    return -1;
  if (model != ORC_PRV && !(opt->t_phase > 0.0)) return -1;
  if (opt->locate_max && model != ORC_KM && model != ORC_KM6) return -1;
  if (opt->lyapunov && (model == ORC_PRV || opt->locate_max)) return -1;
  if (opt->lyapunov < 0 || opt->lyapunov > D || (D > MAXDB && opt->lyapunov)) return -1;
  const int Dint = D * (1 + opt->lyapunov);   /* integrated dimension */
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t i = 0; i < n; ++i) {
    double p[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, y[MAXD];
    for (int j = 0; j < P; ++j) p[j] = params[j * n + i];
    sysctx s;
    ctx_init(&s, model, p, shared);
    if (opt->lyapunov) {
      s.tangent = opt->lyapunov;
      s.D = Dint;
    }
    s.phi2 = phi0 ? phi0[i] : 0.0;
    for (int c = 0; c < Dint; ++c) y[c] = y0[c * n + i];
    double t = t0 ? t0[i] : 0.0;
    double h = h0 ? h0[i] : opt->dt0;
    int64_t st[ORC_NSTAT] = {0, 0, 0, 0, 0, 0};
    int32_t stat = ORC_SYS_OK;
    double hxi[2] = {INFINITY, -INFINITY};
    double cy[ORC_NCARRY] = {-INFINITY, INFINITY, t, 0.0};   /* a fresh start */
    if (carry_in)
      for (int k = 0; k < ORC_NCARRY; ++k) cy[k] = carry_in[k * n + i];
    solve_one(&s, opt, y, &t, &h, records, n, i, st, &stat, cy, hx ? hxi : NULL);
    if (carry_out)
      for (int k = 0; k < ORC_NCARRY; ++k) carry_out[k * n + i] = cy[k];
    if (hx) {
      hx[i] = hxi[0];
      hx[n + i] = hxi[1];
    }
    if (y_out)
      for (int c = 0; c < Dint; ++c) y_out[c * n + i] = y[c];
    if (t_out) t_out[i] = t;
    if (h_out) h_out[i] = h;
    if (phi_out) phi_out[i] = s.phi2;
    if (stats)
      for (int k = 0; k < ORC_NSTAT; ++k) stats[k * n + i] = st[k];
    if (status) status[i] = stat;
  }
  return 0;
}
