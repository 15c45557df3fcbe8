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
  const double h2 = 0.5 * dt, h3 = dt / 3.0, h6 = dt / 6.0;
  const double sh = sigma * dt, sh2 = sigma * h2, sh3 = sigma * h3, sh6 = sigma * h6;
  for (int64_t s = 0; s < nsteps; ++s) {
#pragma unroll
    for (int k = 0; k < SPL; ++k) {
      const double x0 = x[k], y0 = y[k], z0 = z[k], rho = r[k];
      double d, ky, kz, ax, ay, az, xs, ys, zs;
      // stage 1 at (x0, y0, z0)
      d = y0 - x0;
      ky = fma(-x0, z0, fma(rho, x0, -y0));
      kz = fma(x0, y0, -beta * z0);
      ax = fma(sh6, d, x0);
      ay = fma(h6, ky, y0);
      az = fma(h6, kz, z0);
      xs = fma(sh2, d, x0);
      ys = fma(h2, ky, y0);
      zs = fma(h2, kz, z0);
      // stage 2
      d = ys - xs;
      ky = fma(-xs, zs, fma(rho, xs, -ys));
      kz = fma(xs, ys, -beta * zs);
      ax = fma(sh3, d, ax);
      ay = fma(h3, ky, ay);
      az = fma(h3, kz, az);
      xs = fma(sh2, d, x0);
      ys = fma(h2, ky, y0);
      zs = fma(h2, kz, z0);
      // stage 3
      d = ys - xs;
      ky = fma(-xs, zs, fma(rho, xs, -ys));
      kz = fma(xs, ys, -beta * zs);
      ax = fma(sh3, d, ax);
      ay = fma(h3, ky, ay);
      az = fma(h3, kz, az);
      xs = fma(sh, d, x0);
      ys = fma(dt, ky, y0);
      zs = fma(dt, kz, z0);
      // stage 4
      d = ys - xs;
      ky = fma(-xs, zs, fma(rho, xs, -ys));
      kz = fma(xs, ys, -beta * zs);
      x[k] = fma(sh6, d, ax);
      y[k] = fma(h6, ky, ay);
      z[k] = fma(h6, kz, az);
      m[k] = x[k] > m[k] ? x[k] : m[k];
    }
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
