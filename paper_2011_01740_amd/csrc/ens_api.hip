// Host implementation of the C ABI declared in include/ens.h.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>

#include "ens_internal.h"

namespace ens {

ModelInfo model_info(int model) {
  switch (model) {
    case ENS_QUAD: return {1, 1, 0, 1};
    case ENS_LORENZ: return {3, 1, 2, 1};
    case ENS_KM: return {2, 2, 11, 1};
    case ENS_KM6: return {2, 6, 7, 1};
    case ENS_PRV: return {3, 1, 4, 2};
    case ENS_DIV: return {1, 1, 0, 1};
    case ENS_SIN: return {1, 1, 0, 1};
  }
  return {0, 0, 0, 0};
}

int check_adaptive_opts(int model, int tangent, int64_t n, const ens_solve_opts *o,
                        std::string *msg) {
  auto pos = [](double v) { return v > 0.0 && std::isfinite(v); };
  auto bad = [&](int code, const char *m) {
    *msg = m;
    return code;
  };
  if (!pos(o->dt0) || !pos(o->dt_min) || !pos(o->dt_max) || o->dt_max < o->dt_min)
    return bad(ENS_E_INVAL, "need 0 < dt_min <= dt_max and dt0 > 0");
  if (!(o->rtol >= 0.0) || !pos(o->atol)) return bad(ENS_E_INVAL, "need rtol >= 0 and atol > 0");
  if (model != ENS_PRV && !pos(o->t_phase)) return bad(ENS_E_INVAL, "t_phase must be > 0");
  if (model == ENS_PRV && (!pos(o->event_tol) || !pos(o->t_cap) || !(o->v_stick >= 0.0)))
    return bad(ENS_E_INVAL, "bad event_tol, t_cap or v_stick");
  if (o->n_phases < 0 || o->n_phases > (int64_t)UINT32_MAX || o->n_record < 0 ||
      o->max_steps < 0 || o->max_event_iter < 0)
    return bad(ENS_E_INVAL, "bad phase, record or step counts");
  if (o->max_steps > (int64_t)UINT32_MAX) return bad(ENS_E_INVAL, "max_steps above 2^32");
  if (o->spread < 0 || o->spread > n || o->reserved_ != 0)
    return bad(ENS_E_INVAL, "spread must be in [0, n], reserved_ 0");
  if (o->locate_max && tangent)
    return bad(ENS_E_UNSUPPORTED, "locate_max is not built with the tangent");
  if (o->locate_max && model != ENS_KM && model != ENS_KM6)
    return bad(ENS_E_UNSUPPORTED, "locate_max is built for Keller--Miksis");
  return ENS_OK;
}

// Keller--Miksis: the fast kernel (Newton fifth root, angle-addition forcing
// phase) needs 3 gamma = 21/5 in every sub-ensemble and dt_max <= 1/8;
// otherwise the general variant runs, and a second drive (P_A2 != 0) in any
// sub-ensemble selects the variant that carries it.
int kernel_model(int model, int tangent, const double (*shared)[ENS_MAX_SHARED], int n_ens,
                 double dt_max) {
  int kmodel = model;
  if (model == ENS_KM) {
    bool dual = false;
    if (dt_max > 0.125) kmodel = ENS_KM_GENERAL;
    for (int e = 0; e < n_ens; ++e) {
      if (std::fabs(3.0 * shared[e][5] - 4.2) >= 1e-12) kmodel = ENS_KM_GENERAL;
      if (shared[e][8] != 0.0) dual = true;
    }
    if (dual) kmodel = kmodel == ENS_KM ? ENS_KM_DUAL_FAST : ENS_KM_DUAL;
  }
  if (model == ENS_KM6) {
    if (dt_max > 0.125) kmodel = ENS_KM6_GENERAL;
    for (int e = 0; e < n_ens; ++e)
      if (std::fabs(3.0 * shared[e][5] - 4.2) >= 1e-12) kmodel = ENS_KM6_GENERAL;
  }
  if (tangent) kmodel += tangent * kTangentModel;
  return kmodel;
}

void default_shared(int model, double *sh) {
  switch (model) {
    case ENS_LORENZ:
      sh[0] = 10.0;
      sh[1] = 8.0 / 3.0;
      break;
    case ENS_KM:
    case ENS_KM6: {
      // ENS_KM6 takes the first 7 (the fluid), the rest are per system
      const double w[11] = {997.0, 1497.0, 3166.0, 0.0728, 8.9e-4, 1.4,
                            1.0e5, 10.0e-6, 0.0,    0.0,    0.0};
      for (int i = 0; i < (model == ENS_KM ? 11 : 7); ++i) sh[i] = w[i];
      break;
    }
    case ENS_PRV:
      sh[0] = 1.25;
      sh[1] = 10.0;
      sh[2] = 20.0;
      sh[3] = 0.8;
      break;
    default: break;
  }
}


}  // namespace ens

using ens::EnsDesc;

struct ens_ctx {
  int model = 0, solver = 0;
  int tangent = 0;  // tangents of the variational equation (mi.D, mi.F include them)
  ens::ModelInfo mi{};
  int64_t n = 0;
  int n_ens = 1;
  std::vector<int64_t> off;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream for graph capture
  int device = 0;
  std::string err;
  // per-sub-ensemble settings
  double shared[ENS_MAX_ENSEMBLES][ENS_MAX_SHARED] = {};
  int64_t ens_phases[ENS_MAX_ENSEMBLES];
  int64_t ens_impacts[ENS_MAX_ENSEMBLES];
  std::vector<EnsDesc> desc_dev_copy;  // what d_desc currently holds
  // device buffers
  double *d_p = nullptr, *d_y = nullptr, *d_t = nullptr, *d_h = nullptr;
  double *d_acc = nullptr, *d_rec = nullptr;
  double *d_phi = nullptr;  // Keller--Miksis adaptive: second drive's phase [n]
  int64_t *d_stats = nullptr;
  int32_t *d_status = nullptr;
  unsigned long long *d_queue = nullptr;
  ens::RkckCold *d_cold = nullptr;   // the kernel's cold pointers, in device memory
  int64_t *d_order = nullptr;  // queue order (ens_set_order), valid if use_order
  bool use_order = false;
  double *d_carry = nullptr;   // adaptive: [ENS_NCARRY][n] carried phase accessories
  double *d_coef = nullptr;    // Keller--Miksis adaptive: [ENS_MAX_COEF][n] coefficients
  // scratch kept for the handle's lifetime (allocated at create or first use)
  char *d_sort = nullptr;      // ens_order_by_work: keys, indices, sort temporaries
  size_t sort_tmp = 0;         // bytes of rocPRIM temporaries inside d_sort
  unsigned *d_seen = nullptr;  // ens_set_order: permutation check [n] + flag
  int *d_flag = nullptr;       // ens_set_params_gather: index check flag
  double *d_snap = nullptr;    // ens_tune: snapshot of y, t, h, phi, carry
  // caller's allocator (ens_desc.alloc / free), or null for hipMalloc / hipFree
  ens_alloc_fn ualloc = nullptr;
  ens_free_fn ufree = nullptr;
  void *uctx = nullptr;
  EnsDesc *d_desc = nullptr;
  size_t rec_cap = 0;   // doubles allocated in d_rec
  int64_t R = 0;        // record ring length of the last adaptive solve
  bool have_p = false, have_y = false, h_init = false;
  bool have_acc = false, have_adaptive = false, timed = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int last_block = 0, last_spl = 0, last_grid = 0, last_refill = 0;
  // cached graph of the adaptive launch sequence
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  ens::RkckArgs g_args{};
  int g_block = 0, g_grid = 0, g_model = -1;
  bool g_fill_h = false;
  double g_dt0 = 0.0;
  int64_t trial_cap = 0;  // > 0 while tuning: cap on phases and impacts
};

namespace {

thread_local std::string g_err;

int fail(ens_ctx *h, int code, const std::string &msg) {
  g_err = msg;
  if (h) h->err = msg;
  return code;
}

int hip_fail(ens_ctx *h, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(h, e == hipErrorOutOfMemory ? ENS_E_NOMEM : ENS_E_HIP, m);
}

#define ENS_HIP(ctx, call)                                  \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #call); \
  } while (0)

// Selects the handle's device for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};


// Every device buffer of a handle comes from here: the caller's allocator
// when the handle has one, else hipMalloc.
hipError_t h_alloc_bytes(ens_ctx *h, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  if (h->ualloc) {
    *p = h->ualloc(bytes, h->uctx);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

template <class T>
hipError_t dalloc(ens_ctx *h, T **p, size_t count) {
  return h_alloc_bytes(h, (void **)p, count * sizeof(T));
}

template <class T>
void dfree(ens_ctx *h, T *&p) {
  if (p) {
    if (h->ufree)
      h->ufree((void *)p, h->uctx);
    else
      (void)hipFree((void *)p);
  }
  p = nullptr;
}

// Bytes of the ens_order_by_work scratch for n systems: two key arrays and
// one index array (256-byte aligned each), then the sort's temporaries.
size_t sort_key_bytes(int64_t n) { return ((size_t)n * 8 + 255) & ~(size_t)255; }

hipMemcpyKind kind_in(int where) {
  return where == ENS_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
}

void free_graph(ens_ctx *h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
}

// p[j][i] = p_full[j][idx[i]]
__global__ void k_gather_params(const double *__restrict__ pf, int64_t n_full,
                                const int64_t *__restrict__ idx, int64_t n, int P, double *p,
                                int *bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t src = idx[i];
  if (src < 0 || src >= n_full) {
    *bad = 1;
    return;
  }
  for (int j = 0; j < P; ++j) p[j * n + i] = pf[j * n_full + src];
}

// Permutation check: every entry in range and every system taken once.
__global__ void k_check_order(const int64_t *__restrict__ order, int64_t n,
                              unsigned *__restrict__ seen, int *bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t v = order[i];
  if (v < 0 || v >= n || atomicAdd(&seen[v], 1u) != 0u) *bad = 1;
}

// A fresh phase for every system: no running maximum or minimum, the phase
// starting at the system's clock, not seated.
__global__ void k_fresh_carry(double *__restrict__ carry, const double *__restrict__ t,
                              int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  carry[ENS_CARRY_YMAX * n + i] = -INFINITY;
  carry[ENS_CARRY_YMIN * n + i] = INFINITY;
  carry[ENS_CARRY_TPS * n + i] = t[i];
  carry[ENS_CARRY_SEATED * n + i] = 0.0;
}

// Sort keys for a longest-first queue: attempted steps of the last solve.
__global__ void k_work_keys(const int64_t *__restrict__ stats, int64_t n,
                            unsigned long long *__restrict__ key, int64_t *__restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = (unsigned long long)(stats[ENS_ST_ACCEPTED * n + i] + stats[ENS_ST_REJECTED * n + i]);
  idx[i] = i;
}

// ---------------------------------------------------------------- tuning cache
struct TuneVal {
  int block = 0, spl = 0, refill = 0;
  float ms = 0.f;
};
using TuneKey = std::tuple<int, int, std::string, int>;
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;
bool g_tune_loaded = false;

std::string arch_of(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

int n_bucket(int64_t n) {
  int b = 0;
  while (n > 1) {
    n >>= 1;
    ++b;
  }
  return b;
}

// File format: one "model solver arch bucket block spl refill ms" line per entry.
void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *path = std::getenv("ENS_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  char arch[64];
  int m, so, b, bl, sp, rf;
  float ms;
  while (std::fscanf(f, "%d %d %63s %d %d %d %d %f", &m, &so, arch, &b, &bl, &sp, &rf, &ms) == 8)
    g_tune[TuneKey(m, so, std::string(arch), b)] = TuneVal{bl, sp, rf, ms};
  std::fclose(f);
}

void tune_save_locked() {
  const char *path = std::getenv("ENS_TUNE_CACHE");
  if (!path || !*path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  for (const auto &kv : g_tune)
    std::fprintf(f, "%d %d %s %d %d %d %d %.6f\n", std::get<0>(kv.first), std::get<1>(kv.first),
                 std::get<2>(kv.first).c_str(), std::get<3>(kv.first), kv.second.block,
                 kv.second.spl, kv.second.refill, kv.second.ms);
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}

bool tune_lookup(int model, int solver, int device, int64_t n, TuneVal *v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  auto it = g_tune.find(TuneKey(model, solver, arch_of(device), n_bucket(n)));
  if (it == g_tune.end()) return false;
  *v = it->second;
  return true;
}

void tune_store(int model, int solver, int device, int64_t n, const TuneVal &v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tune[TuneKey(model, solver, arch_of(device), n_bucket(n))] = v;
  tune_save_locked();
}

}  // namespace

namespace ens {
hipError_t launch_fresh_carry(double *carry, const double *t, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fresh_carry, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, carry, t,
                     n);
  return hipGetLastError();
}

void set_thread_error(const char *msg) { g_err = msg; }
}  // namespace ens

extern "C" {

int ens_set_order(ens_t h, const int64_t *order, int32_t where) {
  if (!h) return fail(nullptr, ENS_E_INVAL, "ens_set_order: NULL handle");
  if (where != ENS_HOST && where != ENS_DEVICE)
    return fail(h, ENS_E_INVAL, "ens_set_order: bad where");
  if (!order || h->n == 0) {
    h->use_order = false;
    return ENS_OK;
  }
  DeviceGuard g(h->device);
  const size_t bytes = (size_t)h->n * sizeof(int64_t);
  if (h->solver == ENS_RK4) return ENS_OK;  // no work queue
  if (!h->d_seen) {
    hipError_t e = dalloc(h, &h->d_seen, (size_t)h->n + 16);
    if (e != hipSuccess) return fail(h, ENS_E_NOMEM, "ens_set_order: device allocation failed");
  }
  h->use_order = false;
  unsigned *seen = h->d_seen;
  int *bad = (int *)(seen + h->n);
  int hb = 0;
  hipError_t e = hipMemcpyAsync(h->d_order, order, bytes,
                                where == ENS_HOST ? hipMemcpyHostToDevice
                                                  : hipMemcpyDeviceToDevice, h->stream);
  if (e == hipSuccess) e = ens::launch_fill_u32(seen, 0u, h->n + 16, h->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_check_order, dim3((unsigned)((h->n + 255) / 256)), dim3(256), 0,
                       h->stream, h->d_order, h->n, seen, bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "ens_set_order");
  if (hb) return fail(h, ENS_E_INVAL, "ens_set_order: not a permutation of 0..n-1");
  h->use_order = true;
  return ENS_OK;
}

int ens_order_by_work(ens_t h) {
  if (!h) return fail(nullptr, ENS_E_INVAL, "ens_order_by_work: NULL handle");
  if (h->solver == ENS_RK4 || !h->have_adaptive)
    return fail(h, ENS_E_ORDER, "ens_order_by_work: needs a previous adaptive solve");
  if (h->n == 0) return ENS_OK;
  DeviceGuard g(h->device);
  const int64_t n = h->n;
  // the order and the sort's scratch were allocated with the handle: no
  // allocation and no wait between a pilot solve and the solve it orders
  h->use_order = false;
  size_t tmp_bytes = h->sort_tmp;
  const size_t kb = sort_key_bytes(n);
  char *buf = h->d_sort;
  auto *key_in = (unsigned long long *)buf;
  auto *key_out = (unsigned long long *)(buf + kb);
  auto *idx_in = (int64_t *)(buf + 2 * kb);
  hipLaunchKernelGGL(k_work_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream,
                     h->d_stats, n, key_in, idx_in);
  // radix sort is stable: systems of equal work keep their index order
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = rocprim::radix_sort_pairs_desc(buf + 3 * kb, tmp_bytes, key_in, key_out, idx_in,
                                       h->d_order, (size_t)n, 0u, 48u, h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "ens_order_by_work");
  h->use_order = true;
  return ENS_OK;
}

int ens_set_params_gather(ens_t h, const double *p_full, int64_t n_full, const int64_t *idx) {
  if (!h) return fail(nullptr, ENS_E_INVAL, "ens_set_params_gather: NULL handle");
  if (h->n > 0 && (!p_full || !idx || n_full <= 0))
    return fail(h, ENS_E_INVAL, "ens_set_params_gather: bad arguments");
  DeviceGuard g(h->device);
  if (h->n > 0) {
    if (!h->d_flag && dalloc(h, &h->d_flag, 64) != hipSuccess)
      return fail(h, ENS_E_NOMEM, "ens_set_params_gather: device allocation failed");
    int *bad = h->d_flag;
    int hb = 0;
    hipError_t e = ens::launch_fill_u32((unsigned *)bad, 0u, 1, h->stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_gather_params, dim3((unsigned)((h->n + 255) / 256)), dim3(256), 0,
                         h->stream, p_full, n_full, idx, h->n, h->mi.P, h->d_p, bad);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "ens_set_params_gather");
    if (hb) return fail(h, ENS_E_INVAL, "ens_set_params_gather: index out of range");
  }
  h->have_p = true;
  return ENS_OK;
}


const char *ens_last_error(ens_t h) { return h ? h->err.c_str() : g_err.c_str(); }

void ens_default_opts(ens_solve_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->dt = 0.01;
  o->n_steps = 1000;
  o->t_phase = 1.0;
  o->dt0 = 1e-2;
  o->dt_min = 1e-14;
  o->dt_max = 0.1;
  o->rtol = 1e-10;
  o->atol = 1e-10;
  o->event_tol = 1e-6;
  o->t_cap = 50.0;
  o->v_stick = 1e-9;
  o->n_phases = 1;
  o->n_record = 1;
  o->max_steps = 0;
  o->max_event_iter = 20;
}

int ens_create(const ens_desc *d, ens_t *out) {
  if (!out) return fail(nullptr, ENS_E_INVAL, "ens_create: out is NULL");
  *out = nullptr;
  if (!d) return fail(nullptr, ENS_E_INVAL, "ens_create: desc is NULL");
  if (d->model < ENS_QUAD || d->model > ENS_KM6)
    return fail(nullptr, ENS_E_INVAL, "ens_create: unknown model");
  if (d->solver != ENS_RK4 && d->solver != ENS_RKCK45 && d->solver != ENS_RKDP45)
    return fail(nullptr, ENS_E_INVAL, "ens_create: unknown solver");
  if (d->n < 0 || d->n > (int64_t)INT32_MAX)
    return fail(nullptr, ENS_E_INVAL, "ens_create: n must be in [0, 2^31)");
  if (d->n_ensembles < 1 || d->n_ensembles > ENS_MAX_ENSEMBLES)
    return fail(nullptr, ENS_E_INVAL, "ens_create: n_ensembles out of range");
  if (d->solver == ENS_RK4 && (d->model == ENS_KM || d->model == ENS_KM6 || d->model == ENS_PRV))
    return fail(nullptr, ENS_E_UNSUPPORTED, "ens_create: RK4 is built for QUAD, LORENZ, DIV, SIN");
  if (d->solver != ENS_RK4 && (d->model == ENS_DIV || d->model == ENS_SIN))
    return fail(nullptr, ENS_E_UNSUPPORTED, "ens_create: DIV and SIN are built for RK4");
  std::vector<int64_t> off;
  if (d->ens_offsets) {
    off.assign(d->ens_offsets, d->ens_offsets + d->n_ensembles + 1);
    if (off.front() != 0 || off.back() != d->n)
      return fail(nullptr, ENS_E_INVAL, "ens_create: offsets must run from 0 to n");
    for (int e = 0; e < d->n_ensembles; ++e)
      if (off[e + 1] < off[e])
        return fail(nullptr, ENS_E_INVAL, "ens_create: offsets must be ascending");
  } else {
    if (d->n_ensembles != 1)
      return fail(nullptr, ENS_E_INVAL, "ens_create: offsets required for n_ensembles > 1");
    off = {0, d->n};
  }
  if ((d->alloc == nullptr) != (d->free == nullptr))
    return fail(nullptr, ENS_E_INVAL, "ens_create: alloc and free go together");
  if (d->reserved_ != 0) return fail(nullptr, ENS_E_INVAL, "ens_create: reserved_ must be 0");
  if (d->tangent < 0 || d->tangent > 3)
    return fail(nullptr, ENS_E_INVAL, "ens_create: tangent must be in [0, D]");
  if (d->tangent && (d->solver == ENS_RK4 || d->model == ENS_PRV))
    return fail(nullptr, ENS_E_UNSUPPORTED,
                "ens_create: tangent is built for the adaptive solvers with fixed-length phases");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(nullptr, ENS_E_HIP, "ens_create: no HIP device");
  if (d->device < 0 || d->device >= ndev)
    return fail(nullptr, ENS_E_INVAL, "ens_create: bad device ordinal");

  ens_ctx *h = new (std::nothrow) ens_ctx();
  if (!h) return fail(nullptr, ENS_E_NOMEM, "ens_create: out of host memory");
  h->model = d->model;
  h->solver = d->solver;
  h->mi = ens::model_info(d->model);
  h->tangent = d->tangent;
  if (h->tangent > h->mi.D) {
    delete h;
    return fail(nullptr, ENS_E_INVAL, "ens_create: more tangents than the model's dimension");
  }
  if (h->tangent) {  // state [y; v_1 .. v_K], records (y1max, K log growths)
    h->mi.D *= 1 + h->tangent;
    h->mi.F = 1 + h->tangent;
  }
  h->n = d->n;
  h->n_ens = d->n_ensembles;
  h->off = off;
  h->stream = (hipStream_t)d->hip_stream;
  h->device = d->device;
  h->ualloc = d->alloc;
  h->ufree = d->free;
  h->uctx = d->alloc_ctx;
  for (int e = 0; e < ENS_MAX_ENSEMBLES; ++e) {
    ens::default_shared(h->model, h->shared[e]);
    h->ens_phases[e] = -1;
    h->ens_impacts[e] = 0;
  }
  DeviceGuard g(h->device);
  if (!g.ok) {
    delete h;
    return fail(nullptr, ENS_E_HIP, "ens_create: hipSetDevice failed");
  }
  const size_t n = (size_t)h->n;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = dalloc(h, &h->d_p, (size_t)h->mi.P * n);
  if (e == hipSuccess) e = dalloc(h, &h->d_y, (size_t)h->mi.D * n);
  if (e == hipSuccess) e = dalloc(h, &h->d_t, n);
  if (e == hipSuccess) e = dalloc(h, &h->d_h, n);
  if (e == hipSuccess && h->solver == ENS_RK4) e = dalloc(h, &h->d_acc, n);
  if (e == hipSuccess && h->solver != ENS_RK4) {
    e = dalloc(h, &h->d_stats, (size_t)ENS_NSTAT * n);
    if (e == hipSuccess) e = dalloc(h, &h->d_status, n);
    if (e == hipSuccess) e = dalloc(h, &h->d_queue, 2);
    if (e == hipSuccess) e = dalloc(h, &h->d_cold, 1);
    if (e == hipSuccess) e = dalloc(h, &h->d_desc, ENS_MAX_ENSEMBLES);
    if (e == hipSuccess && (h->model == ENS_KM || h->model == ENS_KM6)) e = dalloc(h, &h->d_phi, n);
    if (e == hipSuccess && (h->model == ENS_KM || h->model == ENS_KM6))
      e = dalloc(h, &h->d_coef, (size_t)ens::ENS_MAX_COEF * n);
    if (e == hipSuccess) e = dalloc(h, &h->d_carry, (size_t)ENS_NCARRY * n);
    if (e == hipSuccess) e = dalloc(h, &h->d_order, n);
    // ens_order_by_work's scratch: sort keys in and out, indices, rocPRIM
    // temporaries (sized by a query that allocates nothing)
    if (e == hipSuccess)
      e = rocprim::radix_sort_pairs_desc(nullptr, h->sort_tmp, (const unsigned long long *)nullptr,
                                         (unsigned long long *)nullptr, (const int64_t *)nullptr,
                                         (int64_t *)nullptr, n, 0u, 48u, h->stream);
    if (e == hipSuccess) e = dalloc(h, &h->d_sort, 3 * sort_key_bytes(h->n) + h->sort_tmp);
  }
  if (e == hipSuccess) e = hipEventCreate(&h->ev0);
  if (e == hipSuccess) e = hipEventCreate(&h->ev1);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    int code = hip_fail(nullptr, e, "ens_create: device allocation");
    ens_destroy(h);
    return code;
  }
  *out = h;
  return ENS_OK;
}

int ens_destroy(ens_t h) {
  if (!h) return ENS_OK;
  DeviceGuard g(h->device);
  hipError_t e = hipSuccess;
  if (g.ok) e = hipStreamSynchronize(h->stream);
  free_graph(h);
  dfree(h, h->d_p);
  dfree(h, h->d_y);
  dfree(h, h->d_t);
  dfree(h, h->d_h);
  dfree(h, h->d_acc);
  dfree(h, h->d_rec);
  dfree(h, h->d_phi);
  dfree(h, h->d_stats);
  dfree(h, h->d_status);
  dfree(h, h->d_queue);
  dfree(h, h->d_cold);
  dfree(h, h->d_order);
  dfree(h, h->d_desc);
  dfree(h, h->d_carry);
  dfree(h, h->d_coef);
  dfree(h, h->d_sort);
  dfree(h, h->d_seen);
  dfree(h, h->d_flag);
  dfree(h, h->d_snap);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  delete h;
  return e == hipSuccess ? ENS_OK : ENS_E_HIP;
}

int ens_set_params(ens_t h, const double *p, int32_t where) {
  if (!h) return fail(nullptr, ENS_E_INVAL, "ens_set_params: NULL handle");
  if (!p && h->n > 0) return fail(h, ENS_E_INVAL, "ens_set_params: p is NULL");
  if (where != ENS_HOST && where != ENS_DEVICE)
    return fail(h, ENS_E_INVAL, "ens_set_params: bad where");
  DeviceGuard g(h->device);
  const size_t bytes = (size_t)h->mi.P * h->n * sizeof(double);
  if (bytes) ENS_HIP(h, hipMemcpyAsync(h->d_p, p, bytes, kind_in(where), h->stream));
  if (where == ENS_HOST && bytes) ENS_HIP(h, hipStreamSynchronize(h->stream));
  h->have_p = true;
  return ENS_OK;
}

int ens_set_shared(ens_t h, int32_t ensemble, const double *shared, int32_t n_shared) {
  if (!h) return fail(nullptr, ENS_E_INVAL, "ens_set_shared: NULL handle");
  if (ensemble < 0 || ensemble >= h->n_ens)
    return fail(h, ENS_E_INVAL, "ens_set_shared: ensemble out of range");
  if (n_shared != h->mi.S)
    return fail(h, ENS_E_INVAL, "ens_set_shared: wrong number of shared parameters");
  if (n_shared > 0 && !shared) return fail(h, ENS_E_INVAL, "ens_set_shared: NULL array");
  for (int i = 0; i < n_shared; ++i)
    if (!std::isfinite(shared[i]))
      return fail(h, ENS_E_INVAL, "ens_set_shared: non-finite value");
  for (int i = 0; i < n_shared; ++i) h->shared[ensemble][i] = shared[i];
  return ENS_OK;
}

int ens_set_budget(ens_t h, int32_t ensemble, int64_t n_phases, int64_t max_impacts) {
  if (!h) return fail(nullptr, ENS_E_INVAL, "ens_set_budget: NULL handle");
  if (ensemble < 0 || ensemble >= h->n_ens)
    return fail(h, ENS_E_INVAL, "ens_set_budget: ensemble out of range");
  if (n_phases < -1 || n_phases > (int64_t)UINT32_MAX || max_impacts < 0)
    return fail(h, ENS_E_INVAL, "ens_set_budget: bad budget");
  h->ens_phases[ensemble] = n_phases;
  h->ens_impacts[ensemble] = max_impacts;
  return ENS_OK;
}

int ens_set_state(ens_t h, const double *y0, const double *t0, const double *h0,
                  int32_t where) {
  if (!h) return fail(nullptr, ENS_E_INVAL, "ens_set_state: NULL handle");
  if (!y0 && h->n > 0) return fail(h, ENS_E_INVAL, "ens_set_state: y0 is NULL");
  if (where != ENS_HOST && where != ENS_DEVICE)
    return fail(h, ENS_E_INVAL, "ens_set_state: bad where");
  DeviceGuard g(h->device);
  const size_t n = (size_t)h->n;
  if (n) {
    ENS_HIP(h, hipMemcpyAsync(h->d_y, y0, (size_t)h->mi.D * n * sizeof(double), kind_in(where),
                              h->stream));
    if (t0)
      ENS_HIP(h, hipMemcpyAsync(h->d_t, t0, n * sizeof(double), kind_in(where), h->stream));
    else
      ENS_HIP(h, ens::launch_fill_f64(h->d_t, 0.0, (int64_t)n, h->stream));
    if (h0)
      ENS_HIP(h, hipMemcpyAsync(h->d_h, h0, n * sizeof(double), kind_in(where), h->stream));
    if (h->d_phi) ENS_HIP(h, ens::launch_fill_f64(h->d_phi, 0.0, (int64_t)n, h->stream));
    if (h->d_carry) ENS_HIP(h, ens::launch_fresh_carry(h->d_carry, h->d_t, (int64_t)n, h->stream));
    if (where == ENS_HOST) ENS_HIP(h, hipStreamSynchronize(h->stream));
  }
  h->h_init = h0 != nullptr;
  h->have_y = true;
  h->have_acc = false;
  return ENS_OK;
}

int ens_set_drive_phase(ens_t h, const double *phi, int32_t where) {
  if (!h) return fail(nullptr, ENS_E_INVAL, "ens_set_drive_phase: NULL handle");
  if (!h->d_phi)
    return fail(h, ENS_E_UNSUPPORTED, "ens_set_drive_phase: Keller--Miksis adaptive handles only");
  if (!h->have_y) return fail(h, ENS_E_ORDER, "ens_set_drive_phase: set the state first");
  if (!phi && h->n > 0) return fail(h, ENS_E_INVAL, "ens_set_drive_phase: phi is NULL");
  if (where != ENS_HOST && where != ENS_DEVICE)
    return fail(h, ENS_E_INVAL, "ens_set_drive_phase: bad where");
  DeviceGuard g(h->device);
  const size_t bytes = (size_t)h->n * sizeof(double);
  if (bytes) {
    ENS_HIP(h, hipMemcpyAsync(h->d_phi, phi, bytes, kind_in(where), h->stream));
    if (where == ENS_HOST) ENS_HIP(h, hipStreamSynchronize(h->stream));
  }
  return ENS_OK;
}

int ens_set_carry(ens_t h, const double *carry, int32_t where) {
  if (!h) return fail(nullptr, ENS_E_INVAL, "ens_set_carry: NULL handle");
  if (!h->d_carry) return fail(h, ENS_E_UNSUPPORTED, "ens_set_carry: adaptive handles only");
  if (!h->have_y) return fail(h, ENS_E_ORDER, "ens_set_carry: set the state first");
  if (!carry && h->n > 0) return fail(h, ENS_E_INVAL, "ens_set_carry: carry is NULL");
  if (where != ENS_HOST && where != ENS_DEVICE)
    return fail(h, ENS_E_INVAL, "ens_set_carry: bad where");
  DeviceGuard g(h->device);
  const size_t bytes = (size_t)ENS_NCARRY * h->n * sizeof(double);
  if (bytes) {
    ENS_HIP(h, hipMemcpyAsync(h->d_carry, carry, bytes, kind_in(where), h->stream));
    if (where == ENS_HOST) ENS_HIP(h, hipStreamSynchronize(h->stream));
  }
  return ENS_OK;
}

static int solve_rk4(ens_t h, const ens_solve_opts *o) {
  if (!(o->dt > 0.0) || !std::isfinite(o->dt) || o->n_steps < 0)
    return fail(h, ENS_E_INVAL, "ens_solve: RK4 needs dt > 0 and n_steps >= 0");
  int block = o->block, spl = o->spl;
  TuneVal tv;
  if ((!block || !spl) && tune_lookup(h->model, h->solver, h->device, h->n, &tv)) {
    if (!block) block = tv.block;
    if (!spl) spl = tv.spl;
  }
  if (!block) block = 256;
  if (!spl) spl = 1;
  if (block < 64 || block > 1024 || block % 64)
    return fail(h, ENS_E_INVAL, "ens_solve: block must be a multiple of 64 in [64, 1024]");
  if (spl != 1 && spl != 2 && spl != 4) return fail(h, ENS_E_INVAL, "ens_solve: spl must be 1, 2 or 4");
  ENS_HIP(h, hipEventRecord(h->ev0, h->stream));
  ENS_HIP(h, ens::launch_rk4(h->model, block, spl, h->d_p, h->d_y, h->d_acc, h->n, o->dt,
                             o->n_steps, h->shared[0], h->stream));
  ENS_HIP(h, hipEventRecord(h->ev1, h->stream));
  h->timed = true;
  h->have_acc = true;
  h->last_block = block;
  h->last_spl = spl;
  h->last_grid = (int)((h->n + (int64_t)block * spl - 1) / ((int64_t)block * spl));
  h->last_refill = 0;
  return ENS_OK;
}

static int solve_rkck(ens_t h, const ens_solve_opts *o) {
  {
    std::string msg;
    const int rc = ens::check_adaptive_opts(h->model, h->tangent, h->n, o, &msg);
    if (rc != ENS_OK) return fail(h, rc, "ens_solve: " + msg);
  }
  int block = o->block, refill = o->refill;
  TuneVal tv;
  if ((!block || !refill) && tune_lookup(h->model, h->solver, h->device, h->n, &tv)) {
    if (!block) block = tv.block;
    if (!refill) refill = tv.refill;
  }
  if (!block) block = 256;
  if (!refill) refill = 1;
  if (block < 64 || block > 256 || block % 64)
    return fail(h, ENS_E_INVAL, "ens_solve: adaptive block must be 64, 128, 192 or 256");
  if (refill < 1 || refill > 64) return fail(h, ENS_E_INVAL, "ens_solve: refill must be in [1, 64]");
  const int kmodel = ens::kernel_model(h->model, h->tangent, h->shared, h->n_ens, o->dt_max);
  int grid = o->grid;
  const int cap = ens::rkck_max_blocks(kmodel, h->solver, o->locate_max != 0, block);
  if (cap <= 0) return fail(h, ENS_E_HIP, "ens_solve: occupancy query failed");
  if (grid <= 0) grid = cap;
  if (grid > cap) return fail(h, ENS_E_INVAL, "ens_solve: grid above resident capacity");

  // records
  const int64_t R = o->n_record;
  const size_t rec_count = (size_t)R * h->mi.F * (size_t)h->n;
  if (rec_count > h->rec_cap) {
    free_graph(h);
    dfree(h, h->d_rec);
    h->rec_cap = 0;
    ENS_HIP(h, dalloc(h, &h->d_rec, rec_count));
    h->rec_cap = rec_count;
  }
  // sub-ensemble descriptors: upload only when they change
  std::vector<EnsDesc> desc(h->n_ens);
  for (int e = 0; e < h->n_ens; ++e) {
    std::memset(&desc[e], 0, sizeof(EnsDesc));
    for (int i = 0; i < ENS_MAX_SHARED; ++i) desc[e].shared[i] = h->shared[e][i];
    desc[e].first = h->off[e];
    desc[e].last = h->off[e + 1];
    desc[e].n_phases = h->ens_phases[e] >= 0 ? h->ens_phases[e] : o->n_phases;
    desc[e].max_impacts = h->model == ENS_PRV ? h->ens_impacts[e] : 0;
    if (h->trial_cap > 0) {
      if (desc[e].n_phases > h->trial_cap) desc[e].n_phases = h->trial_cap;
      if (h->model == ENS_PRV &&
          (desc[e].max_impacts == 0 || desc[e].max_impacts > h->trial_cap))
        desc[e].max_impacts = h->trial_cap;
    }
  }
  if (desc.size() != h->desc_dev_copy.size() ||
      std::memcmp(desc.data(), h->desc_dev_copy.data(), desc.size() * sizeof(EnsDesc))) {
    ENS_HIP(h, hipMemcpyAsync(h->d_desc, desc.data(), desc.size() * sizeof(EnsDesc),
                              hipMemcpyHostToDevice, h->stream));
    ENS_HIP(h, hipStreamSynchronize(h->stream));
    h->desc_dev_copy = desc;
  }

  // the cold pointers go to device memory ahead of the launch, stream-ordered
  // and outside any captured graph (the graph's kernel reads them at replay)
  ens::RkckCold c{};
  c.p = h->d_p;
  c.y = h->d_y;
  c.phi2 = h->d_phi;
  c.t = h->d_t;
  c.h = h->d_h;
  c.rec = R > 0 ? h->d_rec : nullptr;
  c.stats = h->d_stats;
  c.status = h->d_status;
  c.queue = h->d_queue;
  c.order = h->use_order ? h->d_order : nullptr;
  c.carry = h->d_carry;
  c.coef = h->d_coef;
  ENS_HIP(h, ens::launch_set_cold(h->d_cold, c, h->stream));

  ens::RkckArgs a;
  std::memset(&a, 0, sizeof(a));  // padding too: the struct is compared bytewise
  a.cold = h->d_cold;
  a.spread = o->spread;
  a.desc = h->d_desc;
  a.n = h->n;
  a.R = R;
  a.n_ens = h->n_ens;
  a.refill = refill;
  a.t_phase = o->t_phase;
  a.dt_min = o->dt_min;
  a.dt_max = o->dt_max;
  a.rtol = o->rtol;
  a.atol = o->atol;
  a.event_tol = o->event_tol;
  a.t_cap = o->t_cap;
  a.v_stick = o->v_stick;
  a.max_steps = o->max_steps;
  a.max_event_iter = o->max_event_iter;
  a.prioritize = std::getenv("ENS_NO_PRIORITY") ? 0 : 1;
  a.locate_max = o->locate_max ? 1 : 0;
  const bool fill_h = !h->h_init;

  auto enqueue = [&](hipStream_t s) -> hipError_t {
    hipError_t e = ens::launch_fill_u64(h->d_queue, 0ull, 2, s);
    if (e == hipSuccess && rec_count)
      e = ens::launch_fill_f64(h->d_rec, std::numeric_limits<double>::quiet_NaN(),
                               (int64_t)rec_count, s);
    if (e == hipSuccess && fill_h) e = ens::launch_fill_f64(h->d_h, o->dt0, h->n, s);
    if (e == hipSuccess && h->n > 0 && h->d_coef) e = ens::launch_rkck_coef(kmodel, a, s);
    if (e == hipSuccess && h->n > 0) e = ens::launch_rkck(kmodel, h->solver, block, grid, a, s);
    return e;
  };

  if (o->use_graph && h->n > 0) {
    const bool same = h->gexec && h->g_block == block && h->g_grid == grid &&
                      h->g_model == kmodel && h->g_fill_h == fill_h &&
                      (!fill_h || h->g_dt0 == o->dt0) &&
                      std::memcmp(&h->g_args, &a, sizeof(a)) == 0;  // a is zero-filled
    if (!same) {
      free_graph(h);
      ENS_HIP(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue(h->cap_stream);
      hipGraph_t gr = nullptr;
      hipError_t e2 = hipStreamEndCapture(h->cap_stream, &gr);
      if (e != hipSuccess) {
        if (gr) (void)hipGraphDestroy(gr);
        return hip_fail(h, e, "ens_solve: capture");
      }
      if (e2 != hipSuccess) return hip_fail(h, e2, "ens_solve: hipStreamEndCapture");
      h->graph = gr;
      ENS_HIP(h, hipGraphInstantiate(&h->gexec, gr, nullptr, nullptr, 0));
      std::memcpy(&h->g_args, &a, sizeof(a));
      h->g_block = block;
      h->g_grid = grid;
      h->g_model = kmodel;
      h->g_fill_h = fill_h;
      h->g_dt0 = o->dt0;
    }
    ENS_HIP(h, hipEventRecord(h->ev0, h->stream));
    ENS_HIP(h, hipGraphLaunch(h->gexec, h->stream));
    ENS_HIP(h, hipEventRecord(h->ev1, h->stream));
  } else {
    ENS_HIP(h, hipEventRecord(h->ev0, h->stream));
    ENS_HIP(h, enqueue(h->stream));
    ENS_HIP(h, hipEventRecord(h->ev1, h->stream));
  }
  h->timed = true;
  h->h_init = true;
  h->have_adaptive = true;
  h->R = R;
  h->last_block = block;
  h->last_spl = 1;
  h->last_grid = grid;
  h->last_refill = refill;
  return ENS_OK;
}

int ens_solve(ens_t h, const ens_solve_opts *o) {
  if (!h) return fail(nullptr, ENS_E_INVAL, "ens_solve: NULL handle");
  if (!o) return fail(h, ENS_E_INVAL, "ens_solve: opts is NULL");
  if (!h->have_p || !h->have_y)
    return fail(h, ENS_E_ORDER, "ens_solve: set params and state first");
  DeviceGuard g(h->device);
  if (!g.ok) return fail(h, ENS_E_HIP, "ens_solve: hipSetDevice failed");
  if (h->solver == ENS_RK4) return solve_rk4(h, o);
  return solve_rkck(h, o);
}

size_t ens_field_bytes(ens_t h, int32_t field) {
  if (!h) return 0;
  const size_t n = (size_t)h->n;
  switch (field) {
    case ENS_STATE: return h->have_y ? (size_t)h->mi.D * n * sizeof(double) : 0;
    case ENS_TIME: return h->have_y ? n * sizeof(double) : 0;
    case ENS_H: return (h->have_y && h->h_init) ? n * sizeof(double) : 0;
    case ENS_ACC: return h->have_acc ? n * sizeof(double) : 0;
    case ENS_RECORDS:
      return h->have_adaptive ? (size_t)h->R * h->mi.F * n * sizeof(double) : 0;
    case ENS_STATS: return h->have_adaptive ? (size_t)ENS_NSTAT * n * sizeof(int64_t) : 0;
    case ENS_STATUS: return h->have_adaptive ? n * sizeof(int32_t) : 0;
    case ENS_DRIVE_PHASE: return (h->have_y && h->d_phi) ? n * sizeof(double) : 0;
    case ENS_CARRY: return (h->have_y && h->d_carry) ? ENS_NCARRY * n * sizeof(double) : 0;
  }
  return 0;
}

int ens_read(ens_t h, int32_t field, void *dst, size_t bytes, int32_t where) {
  if (!h) return fail(nullptr, ENS_E_INVAL, "ens_read: NULL handle");
  if (where != ENS_HOST && where != ENS_DEVICE)
    return fail(h, ENS_E_INVAL, "ens_read: bad where");
  if (field < ENS_STATE || field > ENS_CARRY)
    return fail(h, ENS_E_INVAL, "ens_read: bad field");
  if (field == ENS_DRIVE_PHASE && !h->d_phi)
    return fail(h, ENS_E_UNSUPPORTED, "ens_read: ENS_DRIVE_PHASE is Keller--Miksis adaptive only");
  if (field == ENS_CARRY && !h->d_carry)
    return fail(h, ENS_E_UNSUPPORTED, "ens_read: ENS_CARRY is for adaptive handles");
  const size_t need = ens_field_bytes(h, field);
  const bool produced = need > 0 || h->n == 0 || (field == ENS_RECORDS && h->have_adaptive);
  if (!produced) return fail(h, ENS_E_ORDER, "ens_read: field not produced yet");
  if (bytes != need) return fail(h, ENS_E_INVAL, "ens_read: bytes does not match the field size");
  if (need == 0) return ENS_OK;
  if (!dst) return fail(h, ENS_E_INVAL, "ens_read: dst is NULL");
  const void *src = nullptr;
  switch (field) {
    case ENS_STATE: src = h->d_y; break;
    case ENS_TIME: src = h->d_t; break;
    case ENS_H: src = h->d_h; break;
    case ENS_ACC: src = h->d_acc; break;
    case ENS_RECORDS: src = h->d_rec; break;
    case ENS_STATS: src = h->d_stats; break;
    case ENS_STATUS: src = h->d_status; break;
    case ENS_DRIVE_PHASE: src = h->d_phi; break;
    case ENS_CARRY: src = h->d_carry; break;
  }
  DeviceGuard g(h->device);
  const hipMemcpyKind k = where == ENS_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  ENS_HIP(h, hipMemcpyAsync(dst, src, need, k, h->stream));
  if (where == ENS_HOST) ENS_HIP(h, hipStreamSynchronize(h->stream));
  return ENS_OK;
}

int ens_tune(ens_t h, const ens_solve_opts *opts, int64_t trial_len, ens_solve_opts *best,
             float *best_ms) {
  if (!h) return fail(nullptr, ENS_E_INVAL, "ens_tune: NULL handle");
  if (!opts) return fail(h, ENS_E_INVAL, "ens_tune: opts is NULL");
  if (!h->have_p || !h->have_y) return fail(h, ENS_E_ORDER, "ens_tune: set params and state first");
  DeviceGuard g(h->device);
  const size_t n = (size_t)h->n;
  // snapshot of everything a solve changes in the state (y, t, h, second
  // drive phase, carried accessories), taken once and restored before every
  // trial and at the end; its buffer stays with the handle
  const size_t nd = n ? n : 1;
  const size_t D = (size_t)h->mi.D;
  const size_t snap_count = (D + 3 + ENS_NCARRY) * nd;
  const bool had_h = h->h_init;
  if (!h->d_snap) ENS_HIP(h, dalloc(h, &h->d_snap, snap_count));
  double *sy = h->d_snap, *st = sy + D * nd, *sh = st + nd, *sp = sh + nd, *sc = sp + nd;
  auto copies = [&](bool save) -> hipError_t {
    struct {
      double *dev;
      double *snap;
      size_t count;
      bool use;
    } parts[] = {{h->d_y, sy, D * n, true},
                 {h->d_t, st, n, true},
                 {h->d_h, sh, n, had_h},
                 {h->d_phi, sp, n, h->d_phi != nullptr},
                 {h->d_carry, sc, ENS_NCARRY * n, h->d_carry != nullptr}};
    for (auto &pt : parts) {
      if (!pt.use || pt.count == 0) continue;
      hipError_t r = hipMemcpyAsync(save ? pt.snap : pt.dev, save ? pt.dev : pt.snap,
                                    pt.count * sizeof(double), hipMemcpyDeviceToDevice,
                                    h->stream);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  };
  hipError_t e = copies(true);
  auto restore = [&]() -> hipError_t {
    h->h_init = had_h;
    return copies(false);
  };
  ens_solve_opts trial = *opts;
  std::vector<std::tuple<int, int, int>> cands;  // block, spl, refill
  if (h->solver == ENS_RK4) {
    const int64_t len = trial_len > 0 ? trial_len : 256;
    if (trial.n_steps > len) trial.n_steps = len;
    // largest blocks and most systems per lane first: among candidates
    // within the 2% margin below, the first one tried is kept
    for (int b : {1024, 512, 256, 128, 64})
      for (int sp : {4, 2, 1}) cands.emplace_back(b, sp, 0);
  } else {
    h->trial_cap = trial_len > 0 ? trial_len : 2;
    trial.use_graph = 0;
    for (int b : {64, 128, 256})
      for (int rf : {1, 8, 32, 64}) cands.emplace_back(b, 1, rf);
  }
  int rc = e == hipSuccess ? ENS_OK : hip_fail(h, e, "ens_tune: snapshot");
  TuneVal bestv;
  bestv.ms = std::numeric_limits<float>::infinity();
  for (size_t c = 0; rc == ENS_OK && c < cands.size(); ++c) {
    trial.block = std::get<0>(cands[c]);
    trial.spl = std::get<1>(cands[c]);
    trial.refill = std::get<2>(cands[c]);
    trial.grid = 0;
    float tmin = std::numeric_limits<float>::infinity();
    for (int rep = 0; rc == ENS_OK && rep < 3; ++rep) {
      hipError_t r = restore();
      if (r != hipSuccess) {
        rc = hip_fail(h, r, "ens_tune: restore");
        break;
      }
      rc = h->solver == ENS_RK4 ? solve_rk4(h, &trial) : solve_rkck(h, &trial);
      if (rc != ENS_OK) break;
      float ms = 0.f;
      r = hipEventSynchronize(h->ev1);
      if (r == hipSuccess) r = hipEventElapsedTime(&ms, h->ev0, h->ev1);
      if (r != hipSuccess) {
        rc = hip_fail(h, r, "ens_tune: timing");
        break;
      }
      if (ms < tmin) tmin = ms;
    }
    // a challenger replaces the incumbent only if it is faster by more than
    // the trials' run-to-run spread (2%), so that near-ties do not flip the
    // choice from one run to the next
    if (rc == ENS_OK && tmin < bestv.ms * 0.98f) {
      bestv.block = trial.block;
      bestv.spl = trial.spl;
      bestv.refill = trial.refill;
      bestv.ms = tmin;
    }
  }
  h->trial_cap = 0;
  hipError_t r = restore();
  if (rc == ENS_OK && r != hipSuccess) rc = hip_fail(h, r, "ens_tune: restore");
  if (r == hipSuccess) r = hipStreamSynchronize(h->stream);
  // the trial solves produced results that belong to no real solve
  h->have_acc = false;
  h->have_adaptive = false;
  h->timed = false;
  if (rc != ENS_OK) return rc;
  tune_store(h->model, h->solver, h->device, h->n, bestv);
  if (best) {
    *best = *opts;
    best->block = bestv.block;
    best->spl = h->solver == ENS_RK4 ? bestv.spl : 0;
    best->refill = bestv.refill;
  }
  if (best_ms) *best_ms = bestv.ms;
  return ENS_OK;
}

int ens_last_launch(ens_t h, int32_t *block, int32_t *spl, int32_t *grid, int32_t *refill) {
  if (!h) return fail(nullptr, ENS_E_INVAL, "ens_last_launch: NULL handle");
  if (!h->timed) return fail(h, ENS_E_ORDER, "ens_last_launch: no solve yet");
  if (block) *block = h->last_block;
  if (spl) *spl = h->last_spl;
  if (grid) *grid = h->last_grid;
  if (refill) *refill = h->last_refill;
  return ENS_OK;
}

int ens_last_kernel_ms(ens_t h, float *ms) {
  if (!h || !ms) return fail(h, ENS_E_INVAL, "ens_last_kernel_ms: NULL argument");
  if (!h->timed) return fail(h, ENS_E_ORDER, "ens_last_kernel_ms: no solve yet");
  DeviceGuard g(h->device);
  ENS_HIP(h, hipEventSynchronize(h->ev1));
  ENS_HIP(h, hipEventElapsedTime(ms, h->ev0, h->ev1));
  return ENS_OK;
}

}  // extern "C"
