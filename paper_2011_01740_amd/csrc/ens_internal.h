// Internal declarations of libens (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ens.h"

namespace ens {

// Model sizes: state dimension, per-system parameters, shared parameters,
// record fields.
struct ModelInfo {
  int D, P, S, F;
};
ModelInfo model_info(int model);

// Per-sub-ensemble descriptor, copied into LDS by the persistent kernel.
struct alignas(16) EnsDesc {
  double shared[ENS_MAX_SHARED];
  int64_t first, last;      // index range [first, last)
  int64_t n_phases;         // phases per system
  int64_t max_impacts;      // valve impact budget (0 = none)
};

// Everything the persistent adaptive kernel needs, passed by value.
// The per-system arrays and the queue: the persistent kernel touches them
// only when a lane takes up or puts down a system or ends a phase, so it
// reads these pointers from device memory at those points instead of holding
// them in scalar registers through the step loop.
struct RkckCold {
  const double *p;          // [P][n]
  double *y;                // [D][n] in/out
  double *phi2;             // [n] in/out: Keller--Miksis second drive's phase, or null
  double *t;                // [n] in/out
  double *h;                // [n] in/out
  double *rec;              // [R][F][n] or null
  int64_t *stats;           // [ENS_NSTAT][n]
  int32_t *status;          // [n]
  unsigned long long *queue;// [2]: positions taken from the rest, from the head
  const int64_t *order;     // [n] system taken at each queue position, or null
  double *carry;            // [ENS_NCARRY][n] in/out: the running phase's
                            // y1max, y1min, start time, valve seated (1/0)
  double *coef;             // [ENS_MAX_COEF][n]: each system's model coefficients,
                            // filled at the start of a solve (Keller--Miksis), or null
};

struct RkckArgs {
  const RkckCold *cold;     // device copy of the pointers above
  int64_t spread;           // head [0, spread) of the queue order: one wave per SIMD
  const EnsDesc *desc;      // [n_ens]
  int64_t n;
  int64_t R;
  int32_t n_ens;
  int32_t refill;           // idle lanes a wave waits for before refilling
  double t_phase, dt_min, dt_max, rtol, atol, event_tol, t_cap, v_stick;
  int64_t max_steps;
  int32_t max_event_iter;
  int32_t prioritize;       // waves raise their issue priority by remaining work
  int32_t locate_max;       // Keller--Miksis: maxima located on the step interpolant
};

// Kernel variants of the Keller--Miksis model (ENS_KM itself is the fast
// single-drive kernel): for a polytropic exponent with 3 gamma != 21/5 or
// dt_max > 1/8 (general power through exp/log, sincospi at every stage); and
// both with the second drive (its phase carried across phases).
constexpr int ENS_KM_GENERAL = 100;
constexpr int ENS_KM_DUAL = 101;       // general arithmetic + second drive
constexpr int ENS_KM_DUAL_FAST = 102;  // fast arithmetic + second drive
constexpr int ENS_KM6_GENERAL = 103;   // ENS_KM6 on the general arithmetic
// K x kTangentModel added to any of the above: the same model with K
// tangents of its variational equation.
constexpr int kTangentModel = 1000;

// Validation of the adaptive solve options for a model (ENS_OK, or an
// ens_status with the reason in *msg).
int check_adaptive_opts(int model, int tangent, int64_t n, const ens_solve_opts *o,
                        std::string *msg);
// The kernel variant that integrates `model` with these sub-ensembles'
// shared parameters and step cap (fast or general Keller--Miksis arithmetic,
// second drive, tangents).
int kernel_model(int model, int tangent, const double (*shared)[ENS_MAX_SHARED], int n_ens,
                 double dt_max);
// A model's default shared parameters (ENS_MAX_SHARED doubles).
void default_shared(int model, double *sh);
// The calling thread's last error message (ens_last_error(NULL)).
void set_thread_error(const char *msg);

// Kernel launchers (stream-ordered; return hipSuccess or the launch error).
// Fresh phase accessories [ENS_NCARRY][n] from the clock t [n].
hipError_t launch_fresh_carry(double *carry, const double *t, int64_t n, hipStream_t s);
hipError_t launch_set_cold(RkckCold *dst, const RkckCold &c, hipStream_t s);
// Most model coefficients per system that a solve precomputes (Keller--Miksis:
// the coefficients of its right-hand side, derived from the system's
// parameters and the shared constants), and the kernel that fills them
// (nothing to do for a model without such coefficients).
constexpr int ENS_MAX_COEF = 16;
hipError_t launch_rkck_coef(int model, const RkckArgs &a, hipStream_t s);
hipError_t launch_rk4(int model, int block, int spl, const double *p, double *y,
                      double *acc, int64_t n, double dt, int64_t nsteps,
                      const double *shared, hipStream_t s);
// solver: ENS_RKCK45 or ENS_RKDP45.
hipError_t launch_rkck(int model, int solver, int block, int grid, const RkckArgs &a,
                       hipStream_t s);
// Resident-wave capacity of the persistent kernel for this model, solver and block.
int rkck_max_blocks(int model, int solver, bool locate_max, int block);
hipError_t launch_fill_f64(double *p, double v, int64_t count, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, int64_t count,
                           hipStream_t s);
hipError_t launch_fill_u32(unsigned *p, unsigned v, int64_t count, hipStream_t s);

}  // namespace ens
