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
// stage coefficients and the difference y - x feeds both FMAs directly.
#include "ens_internal.h"

namespace ens {
namespace {

// One RK4 step of one Lorenz system in the accumulated, sigma-folded form.
struct LorenzCoef {
  double dt, h2, h3, h6, sh, sh2, sh3, sh6, beta;
};

__device__ __forceinline__ void lorenz_step(double &x, double &y, double &z, double &m,
                                            double rho, const LorenzCoef &c) {
  const double x0 = x, y0 = y, z0 = z;
  double d, ky, kz, ax, ay, az, xs, ys, zs;
  // stage 1 at (x0, y0, z0)
  d = y0 - x0;
  ky = fma(-x0, z0, fma(rho, x0, -y0));
  kz = fma(x0, y0, -c.beta * z0);
  ax = fma(c.sh6, d, x0);
  ay = fma(c.h6, ky, y0);
  az = fma(c.h6, kz, z0);
  xs = fma(c.sh2, d, x0);
  ys = fma(c.h2, ky, y0);
  zs = fma(c.h2, kz, z0);
  // stage 2
  d = ys - xs;
  ky = fma(-xs, zs, fma(rho, xs, -ys));
  kz = fma(xs, ys, -c.beta * zs);
  ax = fma(c.sh3, d, ax);
  ay = fma(c.h3, ky, ay);
  az = fma(c.h3, kz, az);
  xs = fma(c.sh2, d, x0);
  ys = fma(c.h2, ky, y0);
  zs = fma(c.h2, kz, z0);
  // stage 3
  d = ys - xs;
  ky = fma(-xs, zs, fma(rho, xs, -ys));
  kz = fma(xs, ys, -c.beta * zs);
  ax = fma(c.sh3, d, ax);
  ay = fma(c.h3, ky, ay);
  az = fma(c.h3, kz, az);
  xs = fma(c.sh, d, x0);
  ys = fma(c.dt, ky, y0);
  zs = fma(c.dt, kz, z0);
  // stage 4
  d = ys - xs;
  ky = fma(-xs, zs, fma(rho, xs, -ys));
  kz = fma(xs, ys, -c.beta * zs);
  x = fma(c.sh6, d, ax);
  y = fma(c.h6, ky, ay);
  z = fma(c.h6, kz, az);
  m = fmax(m, x);
}

template <int SPL>
__global__ __launch_bounds__(1024) void k_rk4_lorenz(const double *__restrict__ P,
                                                     double *__restrict__ Y,
                                                     double *__restrict__ ACC, int64_t n,
                                                     double dt, int64_t nsteps,
                                                     double sigma, double beta) {
  const int64_t base = (int64_t)blockIdx.x * ((int64_t)blockDim.x * SPL) + threadIdx.x;
  double x[SPL], y[SPL], z[SPL], r[SPL], m[SPL];
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    const bool ok = i < n;
    r[k] = ok ? P[i] : 0.0;
    x[k] = ok ? Y[i] : 0.0;
    y[k] = ok ? Y[n + i] : 0.0;
    z[k] = ok ? Y[2 * n + i] : 0.0;
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
  // two steps per iteration: the loop-carried state then needs no copies
  for (int64_t s = 0; s + 1 < nsteps; s += 2) {
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
      lorenz_step(x[k], y[k], z[k], m[k], r[k], c);
      lorenz_step(x[k], y[k], z[k], m[k], r[k], c);
    }
  }
  if (nsteps & 1) {
#pragma unroll
    for (int k = 0; k < SPL; ++k) lorenz_step(x[k], y[k], z[k], m[k], r[k], c);
  }
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i < n) {
      Y[i] = x[k];
      Y[n + i] = y[k];
      Y[2 * n + i] = z[k];
      ACC[i] = m[k];
    }
  }
}

// dx/dt = x^2 - p (Sec. 3): the same accumulated stage form.
template <int SPL>
__global__ __launch_bounds__(1024) void k_rk4_quad(const double *__restrict__ P,
                                                   double *__restrict__ Y,
                                                   double *__restrict__ ACC, int64_t n,
                                                   double dt, int64_t nsteps) {
  const int64_t base = (int64_t)blockIdx.x * ((int64_t)blockDim.x * SPL) + threadIdx.x;
  double x[SPL], p[SPL], m[SPL];
#pragma unroll
  for (int k = 0; k < SPL; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    const bool ok = i < n;
    p[k] = ok ? P[i] : 0.0;
    x[k] = ok ? Y[i] : 0.0;
    m[k] = x[k];
  }
  const double h2 = 0.5 * dt, h3 = dt / 3.0, h6 = dt / 6.0;
  for (int64_t s = 0; s < nsteps; ++s) {
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
      const double x0 = x[k], pk = p[k];
      double f, a, xs;
      f = fma(x0, x0, -pk);
      a = fma(h6, f, x0);
      xs = fma(h2, f, x0);
      f = fma(xs, xs, -pk);
      a = fma(h3, f, a);
      xs = fma(h2, f, x0);
      f = fma(xs, xs, -pk);
      a = fma(h3, f, a);
      xs = fma(dt, f, x0);
      f = fma(xs, xs, -pk);
      x[k] = fma(h6, f, a);
      m[k] = x[k] > m[k] ? x[k] : m[k];
    }
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
  if (model == ENS_LORENZ) {
    hipLaunchKernelGGL(k_rk4_lorenz<SPL>, dim3((unsigned)blocks), dim3(block), 0, s, p, y,
                       acc, n, dt, nsteps, shared[0], shared[1]);
  } else {
    hipLaunchKernelGGL(k_rk4_quad<SPL>, dim3((unsigned)blocks), dim3(block), 0, s, p, y,
                       acc, n, dt, nsteps);
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

}  // namespace ens
