/*
 * Vectorised, unrolled CPU code for the Lorenz RK4 ensemble: a measurement
 * baseline, not part of the GPU library and not the oracle.
 *
 * It applies the CPU techniques of Sec. 3.1 of arXiv:2011.01740 to the same
 * workload the GPU kernel runs, so that the GPU can be compared with a CPU
 * code written to the paper's advice and not only with the plain serial
 * oracle: explicit SIMD over systems (8 doubles per vector, one system per
 * element), U independent vectors per iteration for instruction-level
 * parallelism (the paper's unrolling over systems), FMAs, the state held in
 * registers for all steps, and OpenMP threads over blocks of systems.  The
 * arithmetic is the GPU kernel's accumulated stage form: the RK4 combination
 * is summed stage by stage, sigma is folded into the stage coefficients, and
 * the third variable is carried as w = rho - z, in which the right-hand side
 * is all multiply-adds (y' = x w - y, w' = beta rho - beta w - x y; RK4
 * commutes with the change of variable, so only rounding differs).
 * Function multiversioning picks AVX-512, AVX2 or plain SSE2 code at load
 * time for the machine it runs on.
 *
 * Layout: P [n] (rho), Y [3][n] (x, y, z; in/out), M [n] (out: running max of
 * x over the initial point and every step end point).
 */
#include <stdint.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double v8 __attribute__((vector_size(64)));
#define W 8   /* systems per vector      */
#define U 4   /* vectors per iteration   */

typedef struct {
  double dt, h2, h3, h6, sh, sh2, sh3, sh6, beta;
} coef;

typedef long long v8i __attribute__((vector_size(64)));
/* unaligned load / store, broadcast, and max as a compare-and-select (macros,
 * so that each function-multiversioning clone compiles them for its target) */
#define LD(p) ({ v8 v_; memcpy(&v_, (p), sizeof v_); v_; })
#define ST(p, v) do { v8 v_ = (v); memcpy((p), &v_, sizeof v_); } while (0)
#define BC(s) ((v8){(s), (s), (s), (s), (s), (s), (s), (s)})
#define VMAX(a, b) ({ v8 a_ = (a), b_ = (b); v8i k_ = a_ > b_; \
                      (v8)(((v8i)a_ & k_) | ((v8i)b_ & ~k_)); })

/* U x W systems starting at i0, all n_steps steps. */
__attribute__((target_clones("avx512f", "arch=haswell", "default")))
static void block8(const double *P, double *Y, double *M, int64_t n, int64_t i0,
                   int64_t nsteps, coef c) {
  v8 x[U], y[U], w[U], r[U], br[U], m[U];
  const v8 be = BC(c.beta);
  for (int u = 0; u < U; ++u) {
    const int64_t i = i0 + (int64_t)u * W;
    r[u] = LD(P + i);
    br[u] = be * r[u];
    x[u] = LD(Y + i);
    y[u] = LD(Y + n + i);
    w[u] = r[u] - LD(Y + 2 * n + i);
    m[u] = x[u];
  }
  const v8 dt = BC(c.dt), h2 = BC(c.h2), h3 = BC(c.h3), h6 = BC(c.h6);
  const v8 sh = BC(c.sh), sh2 = BC(c.sh2), sh3 = BC(c.sh3), sh6 = BC(c.sh6);
  for (int64_t s = 0; s < nsteps; ++s) {
    for (int u = 0; u < U; ++u) {
      const v8 x0 = x[u], y0 = y[u], w0 = w[u], b = br[u];
      v8 d, ky, kw, ax, ay, aw, xs, ys, ws;
      d = y0 - x0;
      ky = x0 * w0 - y0;
      kw = b - be * w0 - x0 * y0;
      ax = x0 + sh6 * d;
      ay = y0 + h6 * ky;
      aw = w0 + h6 * kw;
      xs = x0 + sh2 * d;
      ys = y0 + h2 * ky;
      ws = w0 + h2 * kw;
      d = ys - xs;
      ky = xs * ws - ys;
      kw = b - be * ws - xs * ys;
      ax += sh3 * d;
      ay += h3 * ky;
      aw += h3 * kw;
      xs = x0 + sh2 * d;
      ys = y0 + h2 * ky;
      ws = w0 + h2 * kw;
      d = ys - xs;
      ky = xs * ws - ys;
      kw = b - be * ws - xs * ys;
      ax += sh3 * d;
      ay += h3 * ky;
      aw += h3 * kw;
      xs = x0 + sh * d;
      ys = y0 + dt * ky;
      ws = w0 + dt * kw;
      d = ys - xs;
      ky = xs * ws - ys;
      kw = b - be * ws - xs * ys;
      x[u] = ax + sh6 * d;
      y[u] = ay + h6 * ky;
      w[u] = aw + h6 * kw;
      m[u] = VMAX(x[u], m[u]);
    }
  }
  for (int u = 0; u < U; ++u) {
    const int64_t i = i0 + (int64_t)u * W;
    ST(Y + i, x[u]);
    ST(Y + n + i, y[u]);
    if (nsteps > 0) ST(Y + 2 * n + i, r[u] - w[u]);
    ST(M + i, m[u]);
  }
}

/* One system at a time, for the tail of n that does not fill a block. */
static void one(const double *P, double *Y, double *M, int64_t n, int64_t i, int64_t nsteps,
                coef c) {
  const double r = P[i], b = c.beta * r;
  double x = Y[i], y = Y[n + i], w = r - Y[2 * n + i], m = x;
  for (int64_t s = 0; s < nsteps; ++s) {
    double d, ky, kw, ax, ay, aw, xs, ys, ws;
    d = y - x;
    ky = x * w - y;
    kw = b - c.beta * w - x * y;
    ax = x + c.sh6 * d;
    ay = y + c.h6 * ky;
    aw = w + c.h6 * kw;
    xs = x + c.sh2 * d;
    ys = y + c.h2 * ky;
    ws = w + c.h2 * kw;
    d = ys - xs;
    ky = xs * ws - ys;
    kw = b - c.beta * ws - xs * ys;
    ax += c.sh3 * d;
    ay += c.h3 * ky;
    aw += c.h3 * kw;
    xs = x + c.sh2 * d;
    ys = y + c.h2 * ky;
    ws = w + c.h2 * kw;
    d = ys - xs;
    ky = xs * ws - ys;
    kw = b - c.beta * ws - xs * ys;
    ax += c.sh3 * d;
    ay += c.h3 * ky;
    aw += c.h3 * kw;
    xs = x + c.sh * d;
    ys = y + c.dt * ky;
    ws = w + c.dt * kw;
    d = ys - xs;
    ky = xs * ws - ys;
    kw = b - c.beta * ws - xs * ys;
    x = ax + c.sh6 * d;
    y = ay + c.h6 * ky;
    w = aw + c.h6 * kw;
    m = x > m ? x : m;
  }
  Y[i] = x;
  Y[n + i] = y;
  if (nsteps > 0) Y[2 * n + i] = r - w;
  M[i] = m;
}

/* Returns 0, or -1 for bad arguments.  nthreads < 1 means 1. */
int cpu_lorenz_rk4(const double *P, double *Y, double *M, int64_t n, double dt, int64_t nsteps,
                   double sigma, double beta, int nthreads) {
  if (n < 0 || nsteps < 0 || !(dt > 0.0) || (n > 0 && (!P || !Y || !M))) return -1;
  coef c;
  c.dt = dt;
  c.h2 = 0.5 * dt;
  c.h3 = dt / 3.0;
  c.h6 = dt / 6.0;
  c.sh = sigma * dt;
  c.sh2 = sigma * c.h2;
  c.sh3 = sigma * c.h3;
  c.sh6 = sigma * c.h6;
  c.beta = beta;
  const int64_t per = (int64_t)U * W;
  const int64_t nb = n / per;
  if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t b = 0; b < nb; ++b) block8(P, Y, M, n, b * per, nsteps, c);
  for (int64_t i = nb * per; i < n; ++i) one(P, Y, M, n, i, nsteps, c);
  return 0;
}
