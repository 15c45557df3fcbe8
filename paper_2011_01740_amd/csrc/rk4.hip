// Fixed-step classic RK4 over an ensemble, one system per lane (Sec. 3,
// Sec. 4.1 of arXiv:2011.01740).  The state of each system lives in VGPRs for
// all n steps; HBM is touched once to load (parameters, state) and once to
// store (state, running maximum of y1).
//
// Each lane may carry SPL independent systems ("systems per lane"): the
// stage arithmetic of the SPL systems is interleaved, which gives the
// scheduler independent FP64 instructions to issue while one chain waits
// (the paper's stage-level unrolling, Sec. 3.1.4, applied to a GPU lane).
// System k of lane t of block b is  b * (block * SPL) + k * block + t,  so
// every load and store of a wave is a contiguous 512-byte segment.
//
// The RK4 combination y + h/6 (k1 + 2 k2 + 2 k3 + k4) is accumulated stage by
// stage (acc = y + h/6 k1, acc += h/3 k2, acc += h/3 k3, acc += h/6 k4), so
// no stage derivative outlives its stage.  For the Lorenz system the stage
// derivative of x, sigma (y - x), is never formed: sigma is folded into the
// stage coefficients and the difference y - x feeds both FMAs directly.  The
// kernel carries w = rho - z instead of z: RK4 commutes with an affine change
// of variable (its iterates for w are rho minus those for z, up to rounding),
// and in w the right-hand side is all FMAs, y' = x w - y and
// w' = beta rho - beta w - x y, with beta rho held per system.  A step is
// then 33 FMAs and 4 subtractions.
#include "ens_internal.h"

namespace ens {
namespace {

// One RK4 step of one Lorenz system in the accumulated, sigma-folded form,
// in the variables (x, y, w = rho - z); brho = beta rho.
struct LorenzCoef {
  double dt, h2, h3, h6, sh, sh2, sh3, sh6, beta;
};

// Running maximum with one v_max_f64.  The same as a compare-and-select here
// (a NaN state stays NaN, and both keep the last number).  Written out
// because the compiler, unable to prove the loop-carried maximum canonical,
// adds a second v_max (x, x) per iteration to quiet it: one VALU slot in 23
// of the two-step loop of the one-dimensional models, one in 16 per
// system of the Lorenz loop.
__device__ __forceinline__ double vmax(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

__device__ __forceinline__ void lorenz_step(double &x, double &y, double &w, double &m,
                                            double brho, const LorenzCoef &c) {
  const double x0 = x, y0 = y, w0 = w;
  double d, ky, kw, ax, ay, aw, xs, ys, ws;
  // stage 1 at (x0, y0, w0)
  d = y0 - x0;
  ky = fma(x0, w0, -y0);
  kw = fma(-x0, y0, fma(-c.beta, w0, brho));
  ax = fma(c.sh6, d, x0);
  ay = fma(c.h6, ky, y0);
  aw = fma(c.h6, kw, w0);
  xs = fma(c.sh2, d, x0);
  ys = fma(c.h2, ky, y0);
  ws = fma(c.h2, kw, w0);
  // stage 2
  d = ys - xs;
  ky = fma(xs, ws, -ys);
  kw = fma(-xs, ys, fma(-c.beta, ws, brho));
  ax = fma(c.sh3, d, ax);
  ay = fma(c.h3, ky, ay);
  aw = fma(c.h3, kw, aw);
  xs = fma(c.sh2, d, x0);
  ys = fma(c.h2, ky, y0);
  ws = fma(c.h2, kw, w0);
  // stage 3
  d = ys - xs;
  ky = fma(xs, ws, -ys);
  kw = fma(-xs, ys, fma(-c.beta, ws, brho));
  ax = fma(c.sh3, d, ax);
  ay = fma(c.h3, ky, ay);
  aw = fma(c.h3, kw, aw);
  xs = fma(c.sh, d, x0);
  ys = fma(c.dt, ky, y0);
  ws = fma(c.dt, kw, w0);
  // stage 4
  d = ys - xs;
  ky = fma(xs, ws, -ys);
  kw = fma(-xs, ys, fma(-c.beta, ws, brho));
  x = fma(c.sh6, d, ax);
  y = fma(c.h6, ky, ay);
  w = fma(c.h6, kw, aw);
  m = vmax(m, x);
}

__global__ void k_fill_u32(unsigned *p, unsigned v, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    p[i] = v;
}

template <int SPL>
__global__ __launch_bounds__(1024) void k_rk4_lorenz(const double *__restrict__ P,
                                                     double *__restrict__ Y,
                                                     double *__restrict__ ACC, int64_t n,
                                                     double dt, int64_t nsteps,
                                                     double sigma, double beta) {
  const int64_t base = (int64_t)blockIdx.x * ((int64_t)blockDim.x * SPL) + threadIdx.x;
  double x[SPL], y[SPL], w[SPL], r[SPL], br[SPL], m[SPL];
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    const bool ok = i < n;
    r[k] = ok ? P[i] : 0.0;
    br[k] = beta * r[k];
    x[k] = ok ? Y[i] : 0.0;
    y[k] = ok ? Y[n + i] : 0.0;
    w[k] = r[k] - (ok ? Y[2 * n + i] : 0.0);
    m[k] = x[k];
  }
  // uniform stage coefficients (scalar registers)
  LorenzCoef c;
  c.dt = dt;
  c.h2 = 0.5 * dt;
  c.h3 = dt / 3.0;
  c.h6 = dt / 6.0;
  c.sh = sigma * dt;
  c.sh2 = sigma * c.h2;
  c.sh3 = sigma * c.h3;
  c.sh6 = sigma * c.h6;
  c.beta = beta;
  // four steps per iteration: the loop-carried state needs no copies and the
  // loop control is one issue slot in ~600
  int64_t s = 0;
  for (; s + 3 < nsteps; s += 4) {
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
      lorenz_step(x[k], y[k], w[k], m[k], br[k], c);
      lorenz_step(x[k], y[k], w[k], m[k], br[k], c);
      lorenz_step(x[k], y[k], w[k], m[k], br[k], c);
      lorenz_step(x[k], y[k], w[k], m[k], br[k], c);
    }
  }
  for (; s < nsteps; ++s) {
#pragma unroll
    for (int k = 0; k < SPL; ++k) lorenz_step(x[k], y[k], w[k], m[k], br[k], c);
  }
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i < n) {
      Y[i] = x[k];
      Y[n + i] = y[k];
      if (nsteps > 0) Y[2 * n + i] = r[k] - w[k];  // else z stays as given, bit for bit
      ACC[i] = m[k];
    }
  }
}

// The one-dimensional introductory example (Sec. 3) and its division and
// transcendental variants (Sec. 3.3).  The quadratic right-hand side is one
// FMA; the others are written as a user would: an IEEE division, and the
// device library's sine.
struct FQuad {
  __device__ static double f(double x, double p) { return fma(x, x, -p); }
};
struct FDiv {
  __device__ static double f(double x, double p) { return fma(-p, x, 1.0 / x); }
};
struct FSin {
  __device__ static double f(double x, double p) { return p * sin(x); }
};

// One RK4 step of a one-dimensional model in the accumulated stage form; m
// is the running maximum.
template <class F>
__device__ __forceinline__ void scalar_step(double &x, double &m, double p, double dt,
                                            double h2, double h3, double h6) {
  const double x0 = x;
  double f, a, xs;
  f = F::f(x0, p);
  a = fma(h6, f, x0);
  xs = fma(h2, f, x0);
  f = F::f(xs, p);
  a = fma(h3, f, a);
  xs = fma(h2, f, x0);
  f = F::f(xs, p);
  a = fma(h3, f, a);
  xs = fma(dt, f, x0);
  f = F::f(xs, p);
  x = fma(h6, f, a);
  m = vmax(m, x);
}

// One-dimensional models, SPL systems per lane.
template <class F, int SPL>
__global__ __launch_bounds__(1024) void k_rk4_scalar(const double *__restrict__ P,
                                                     double *__restrict__ Y,
                                                     double *__restrict__ ACC, int64_t n,
                                                     double dt, int64_t nsteps) {
  const int64_t base = (int64_t)blockIdx.x * ((int64_t)blockDim.x * SPL) + threadIdx.x;
  double x[SPL], p[SPL], m[SPL];
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    const bool ok = i < n;
    // idle lanes (past n) sit at x = p = 1, where every variant is finite
    p[k] = ok ? P[i] : 1.0;
    x[k] = ok ? Y[i] : 1.0;
    m[k] = x[k];
  }
  const double h2 = 0.5 * dt, h3 = dt / 3.0, h6 = dt / 6.0;
  // 11 FMAs and one v_max per step; two steps per iteration, so that the
  // loop-carried state needs no register copy
  for (int64_t s = nsteps >> 1; s != 0; --s) {
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
      scalar_step<F>(x[k], m[k], p[k], dt, h2, h3, h6);
      scalar_step<F>(x[k], m[k], p[k], dt, h2, h3, h6);
    }
  }
  if (nsteps & 1) {
#pragma unroll
    for (int k = 0; k < SPL; ++k) scalar_step<F>(x[k], m[k], p[k], dt, h2, h3, h6);
  }
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i < n) {
      Y[i] = x[k];
      ACC[i] = m[k];
    }
  }
}

__global__ void k_fill_f64(double *p, double v, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    p[i] = v;
}

template <int SPL>
hipError_t rk4_spl(int model, int block, const double *p, double *y, double *acc,
                   int64_t n, double dt, int64_t nsteps, const double *shared,
                   hipStream_t s) {
  const int64_t per_block = (int64_t)block * SPL;
  const int64_t blocks = (n + per_block - 1) / per_block;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  const dim3 g((unsigned)blocks), b(block);
  switch (model) {
    case ENS_LORENZ:
      hipLaunchKernelGGL(k_rk4_lorenz<SPL>, g, b, 0, s, p, y, acc, n, dt, nsteps, shared[0],
                         shared[1]);
      break;
    case ENS_QUAD:
      hipLaunchKernelGGL((k_rk4_scalar<FQuad, SPL>), g, b, 0, s, p, y, acc, n, dt, nsteps);
      break;
    case ENS_DIV:
      hipLaunchKernelGGL((k_rk4_scalar<FDiv, SPL>), g, b, 0, s, p, y, acc, n, dt, nsteps);
      break;
    case ENS_SIN:
      hipLaunchKernelGGL((k_rk4_scalar<FSin, SPL>), g, b, 0, s, p, y, acc, n, dt, nsteps);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rk4(int model, int block, int spl, const double *p, double *y,
                      double *acc, int64_t n, double dt, int64_t nsteps,
                      const double *shared, hipStream_t s) {
  switch (spl) {
    case 1: return rk4_spl<1>(model, block, p, y, acc, n, dt, nsteps, shared, s);
    case 2: return rk4_spl<2>(model, block, p, y, acc, n, dt, nsteps, shared, s);
    case 4: return rk4_spl<4>(model, block, p, y, acc, n, dt, nsteps, shared, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fill_f64(double *p, double v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t count,
                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned *p, unsigned v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

}  // namespace ens
