// ens_solve_noalloc: the adaptive solve of ens_solve without a handle and
// without any device allocation, for callers that cannot allocate (code under
// HIP graph capture, tight serving loops, harnesses that forbid it).  The
// caller passes every per-system array; the launch's own scratch -- the two
// queue counters, the block of per-system array pointers the persistent
// kernel reads, and the sub-ensemble descriptors -- lives in a file-scope
// device array of fixed size, one copy per GPU, written by a small kernel
// before each launch (no memset, no memcpy).  Calls that overlap on one GPU
// share that array and race.
#include <cmath>
#include <cstring>
#include <mutex>

#include "ens_internal.h"
#include "../../include/ens_noalloc.h"
#include <cstdlib>

namespace {

constexpr size_t kQueueOff = 0;      // 2 x u64 queue counters
constexpr size_t kColdOff = 256;     // ens::RkckCold
constexpr size_t kDescOff = 512;     // ens::EnsDesc[ENS_MAX_ENSEMBLES]
constexpr size_t kScratchUsed = kDescOff + sizeof(ens::EnsDesc) * ENS_MAX_ENSEMBLES;
static_assert(sizeof(ens::RkckCold) <= kDescOff - kColdOff, "pointer block overflows its slot");
static_assert(kScratchUsed <= ENS_NOALLOC_SCRATCH_BYTES, "scratch too small for the descriptors");

__device__ __align__(256) unsigned char scratch[ENS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_scratch[kMaxDevices] = {};   // device address of `scratch` per GPU

// The device address of this GPU's copy of `scratch`, looked up once per
// device with that device current (the array's name is not a device address
// in host code).
hipError_t scratch_of(int dev, unsigned char **out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = (unsigned char *)p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

struct DescPack {
  ens::EnsDesc d[ENS_MAX_ENSEMBLES];
};

// Writes the launch's scratch: queue counters to zero, the pointer block and
// the descriptors, all passed by value (stream-ordered, capturable).
__global__ void k_set_scratch(unsigned char *base, ens::RkckCold c, DescPack pk, int n_ens) {
  auto *q = (unsigned long long *)(base + kQueueOff);
  if (threadIdx.x < 2) q[threadIdx.x] = 0ull;
  if (threadIdx.x == 0) *(ens::RkckCold *)(base + kColdOff) = c;
  auto *d = (ens::EnsDesc *)(base + kDescOff);
  for (int e = threadIdx.x; e < n_ens; e += blockDim.x) d[e] = pk.d[e];
}

int fail(int code, const char *msg) {
  ens::set_thread_error(msg);
  return code;
}

#define NA_HIP(call)                                          \
  do {                                                        \
    const hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return fail(ENS_E_HIP, #call);      \
  } while (0)

}  // namespace

extern "C" int ens_solve_noalloc(const ens_noalloc_args *a, const ens_solve_opts *o) {
  if (!a || !o) return fail(ENS_E_INVAL, "ens_solve_noalloc: NULL argument");
  if (a->solver != ENS_RKCK45 && a->solver != ENS_RKDP45)
    return fail(ENS_E_INVAL, "ens_solve_noalloc: solver must be ENS_RKCK45 or ENS_RKDP45");
  if (a->model != ENS_QUAD && a->model != ENS_LORENZ && a->model != ENS_KM &&
      a->model != ENS_KM6 && a->model != ENS_PRV)
    return fail(ENS_E_INVAL, "ens_solve_noalloc: not an adaptive model");
  if (a->n < 0 || a->n > (int64_t)INT32_MAX)
    return fail(ENS_E_INVAL, "ens_solve_noalloc: n must be in [0, 2^31)");
  if (a->n_ensembles < 1 || a->n_ensembles > ENS_MAX_ENSEMBLES)
    return fail(ENS_E_INVAL,
                "ens_solve_noalloc: n_ensembles must be in [1, 16] (the descriptors fill the "
                "fixed scratch array)");
  if (a->reserved_ != 0) return fail(ENS_E_INVAL, "ens_solve_noalloc: reserved_ must be 0");
  const ens::ModelInfo mi0 = ens::model_info(a->model);
  if (a->tangent < 0 || a->tangent > mi0.D || (a->tangent && a->model == ENS_PRV))
    return fail(ENS_E_INVAL, "ens_solve_noalloc: bad tangent count");
  {
    std::string msg;
    const int rc = ens::check_adaptive_opts(a->model, a->tangent, a->n, o, &msg);
    if (rc != ENS_OK) {
      msg = "ens_solve_noalloc: " + msg;
      return fail(rc, msg.c_str());
    }
  }
  const int F = a->tangent ? 1 + a->tangent : mi0.F;
  const int64_t n = a->n, R = o->n_record;
  const bool km = a->model == ENS_KM || a->model == ENS_KM6;
  if (n > 0 && (!a->p || !a->y || !a->t || !a->h || !a->carry || !a->stats || !a->status ||
                (km && !a->phi2) || (R > 0 && !a->records)))
    return fail(ENS_E_INVAL, "ens_solve_noalloc: a required device array is NULL");
  // sub-ensembles
  int64_t off[ENS_MAX_ENSEMBLES + 1];
  if (a->ens_offsets) {
    for (int e = 0; e <= a->n_ensembles; ++e) off[e] = a->ens_offsets[e];
    if (off[0] != 0 || off[a->n_ensembles] != n)
      return fail(ENS_E_INVAL, "ens_solve_noalloc: offsets must run from 0 to n");
    for (int e = 0; e < a->n_ensembles; ++e)
      if (off[e + 1] < off[e])
        return fail(ENS_E_INVAL, "ens_solve_noalloc: offsets must be ascending");
  } else {
    if (a->n_ensembles != 1)
      return fail(ENS_E_INVAL, "ens_solve_noalloc: offsets required for n_ensembles > 1");
    off[0] = 0;
    off[1] = n;
  }
  double shared[ENS_MAX_ENSEMBLES][ENS_MAX_SHARED] = {};
  DescPack pk;
  std::memset(&pk, 0, sizeof(pk));
  for (int e = 0; e < a->n_ensembles; ++e) {
    if (a->shared) {
      for (int k = 0; k < ENS_MAX_SHARED; ++k) shared[e][k] = a->shared[e * ENS_MAX_SHARED + k];
      for (int k = 0; k < mi0.S; ++k)
        if (!std::isfinite(shared[e][k]))
          return fail(ENS_E_INVAL, "ens_solve_noalloc: non-finite shared parameter");
    } else {
      ens::default_shared(a->model, shared[e]);
    }
    ens::EnsDesc &d = pk.d[e];
    for (int k = 0; k < ENS_MAX_SHARED; ++k) d.shared[k] = shared[e][k];
    d.first = off[e];
    d.last = off[e + 1];
    const int64_t ph = a->budgets ? a->budgets[2 * e] : -1;
    const int64_t imp = a->budgets ? a->budgets[2 * e + 1] : 0;
    if (ph < -1 || ph > (int64_t)UINT32_MAX || imp < 0)
      return fail(ENS_E_INVAL, "ens_solve_noalloc: bad budget");
    d.n_phases = ph >= 0 ? ph : o->n_phases;
    d.max_impacts = a->model == ENS_PRV ? imp : 0;
  }
  int block = o->block ? o->block : 256;
  const int refill = o->refill ? o->refill : 1;
  if (block < 64 || block > 256 || block % 64)
    return fail(ENS_E_INVAL, "ens_solve_noalloc: block must be 64, 128, 192 or 256");
  if (refill < 1 || refill > 64)
    return fail(ENS_E_INVAL, "ens_solve_noalloc: refill must be in [1, 64]");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || a->device < 0 || a->device >= ndev ||
      a->device >= kMaxDevices)
    return fail(ENS_E_INVAL, "ens_solve_noalloc: bad device ordinal");
  int prev = -1;
  NA_HIP(hipGetDevice(&prev));
  NA_HIP(hipSetDevice(a->device));
  struct Restore {
    int dev;
    ~Restore() { (void)hipSetDevice(dev); }
  } restore{prev};
  const int kmodel = ens::kernel_model(a->model, a->tangent, shared, a->n_ensembles, o->dt_max);
  const int cap = ens::rkck_max_blocks(kmodel, a->solver, o->locate_max != 0, block);
  if (cap <= 0) return fail(ENS_E_HIP, "ens_solve_noalloc: occupancy query failed");
  const int grid = o->grid > 0 ? o->grid : cap;
  if (grid > cap) return fail(ENS_E_INVAL, "ens_solve_noalloc: grid above resident capacity");
  unsigned char *base = nullptr;
  NA_HIP(scratch_of(a->device, &base));
  if (n == 0) return ENS_OK;

  hipStream_t s = (hipStream_t)a->hip_stream;
  if (a->fresh) {
    // a fresh start: the first step dt0, no running maximum / minimum, the
    // phase starting at the clock, not seated, second drive at phase 0
    NA_HIP(ens::launch_fill_f64(a->h, o->dt0, n, s));
    NA_HIP(ens::launch_fresh_carry(a->carry, a->t, n, s));
    if (a->phi2) NA_HIP(ens::launch_fill_f64(a->phi2, 0.0, n, s));
  }
  if (R > 0)
    NA_HIP(ens::launch_fill_f64(a->records, std::nan(""), R * F * n, s));
  ens::RkckCold c{};
  c.p = a->p;
  c.y = a->y;
  c.phi2 = a->phi2;
  c.t = a->t;
  c.h = a->h;
  c.rec = R > 0 ? a->records : nullptr;
  c.stats = a->stats;
  c.status = a->status;
  c.queue = (unsigned long long *)(base + kQueueOff);
  c.order = a->order;
  c.carry = a->carry;
  hipLaunchKernelGGL(k_set_scratch, dim3(1), dim3(64), 0, s, base, c, pk, a->n_ensembles);
  NA_HIP(hipGetLastError());
  ens::RkckArgs ka;
  std::memset(&ka, 0, sizeof(ka));
  ka.cold = (const ens::RkckCold *)(base + kColdOff);
  ka.spread = o->spread;
  ka.desc = (const ens::EnsDesc *)(base + kDescOff);
  ka.n = n;
  ka.R = R;
  ka.n_ens = a->n_ensembles;
  ka.refill = refill;
  ka.t_phase = o->t_phase;
  ka.dt_min = o->dt_min;
  ka.dt_max = o->dt_max;
  ka.rtol = o->rtol;
  ka.atol = o->atol;
  ka.event_tol = o->event_tol;
  ka.t_cap = o->t_cap;
  ka.v_stick = o->v_stick;
  ka.max_steps = o->max_steps;
  ka.max_event_iter = o->max_event_iter;
  ka.prioritize = std::getenv("ENS_NO_PRIORITY") ? 0 : 1;
  ka.locate_max = o->locate_max ? 1 : 0;
  NA_HIP(ens::launch_rkck(kmodel, a->solver, block, grid, ka, s));
  return ENS_OK;
}
