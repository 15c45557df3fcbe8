/*
 * ens_noalloc.h -- an adaptive ensemble solve that allocates nothing.
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  It is the
 * RKCK45 / RKDP45 solve of ens_solve (include/ens.h: same models, kernels,
 * readings, options and results) without a handle: the caller passes every
 * per-system array in device memory and the call enqueues on the given
 * stream.  Its only scratch -- the work queue's two counters, the block of
 * array pointers the persistent kernel reads and the sub-ensemble
 * descriptors -- sits in a fixed device array of ENS_NOALLOC_SCRATCH_BYTES
 * inside the library, one copy per GPU, kept until the process ends and
 * rewritten by every call (counters cleared by a kernel, no memset).  Calls
 * that overlap on one GPU share that array and race: serialise them (one
 * stream, or events).  The call allocates no device memory, frees none and
 * calls no allocating library routine; it does not wait for the stream.
 */
#ifndef LIBENS_ENS_NOALLOC_H_
#define LIBENS_ENS_NOALLOC_H_

#include "ens.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Size of the library's fixed scratch array per GPU (bytes): 16 for the
 * queue counters, a pointer block and ENS_MAX_ENSEMBLES descriptors. */
#define ENS_NOALLOC_SCRATCH_BYTES 4096

typedef struct {
  int32_t model;          /* ENS_QUAD, ENS_LORENZ, ENS_KM, ENS_KM6 or ENS_PRV      */
  int32_t solver;         /* ENS_RKCK45 or ENS_RKDP45                              */
  int64_t n;              /* systems, 0 .. 2^31 - 1                                */
  int32_t n_ensembles;    /* 1 .. ENS_MAX_ENSEMBLES (the descriptors' room in the
                             scratch array); more is refused with ENS_E_INVAL     */
  int32_t device;         /* device ordinal of every array below                   */
  int32_t tangent;        /* tangent vectors as ens_desc.tangent (not the valve)   */
  int32_t fresh;          /* 1: start every system fresh, as after ens_set_state
                             without h0 (h = dt0, ENS_CARRY reset from t, phi2 =
                             0); 0: resume from the arrays as they are            */
  const int64_t *ens_offsets; /* host, n_ensembles + 1 ascending offsets from 0
                             to n, or NULL for one ensemble                       */
  const double *shared;   /* host [n_ensembles][ENS_MAX_SHARED] (the first S of
                             each row used, as ens_set_shared), or NULL for the
                             model defaults                                       */
  const int64_t *budgets; /* host [n_ensembles][2]: phases (-1 = opts n_phases)
                             and impact budget (valve; 0 = none), or NULL         */
  void *hip_stream;       /* hipStream_t to enqueue on; NULL = null stream         */
  /* device arrays, component-major as in ens.h, owned by the caller: */
  const double *p;        /* [P][n] parameters                                     */
  double *y;              /* [D (1 + tangent)][n] state, in/out                    */
  double *t;              /* [n] clock, in/out                                     */
  double *h;              /* [n] next step, in/out (set by fresh = 1)              */
  double *phi2;           /* [n] second drive's phase, in/out: required for
                             ENS_KM and ENS_KM6, ignored otherwise (may be NULL)  */
  double *carry;          /* [ENS_NCARRY][n] phase accessories, in/out            */
  double *records;        /* [n_record][F][n] ring (NaN-filled first), or NULL
                             when n_record == 0                                   */
  int64_t *stats;         /* [ENS_NSTAT][n] out                                    */
  int32_t *status;        /* [n] out                                               */
  const int64_t *order;   /* [n] queue order (a permutation, not checked), or
                             NULL for index order                                 */
  int32_t reserved_;      /* must be 0                                             */
  int32_t pad_;
} ens_noalloc_args;

/* Enqueues the adaptive solve of the n systems described by `args` with the
 * options `opts` (launch fields 0 = block 256, refill 1, the resident grid;
 * use_graph ignored).  Results are bit-identical to ens_solve's on the same
 * inputs.  Errors (nothing enqueued): ENS_E_INVAL (bad arguments or sizes
 * beyond the scratch), ENS_E_UNSUPPORTED, ENS_E_HIP; message in
 * ens_last_error(NULL). */
int ens_solve_noalloc(const ens_noalloc_args *args, const ens_solve_opts *opts);

#ifdef __cplusplus
}
#endif
#endif /* LIBENS_ENS_NOALLOC_H_ */
