"""Thin Python binding of libens (C ABI in include/ens.h).

Argument marshalling only: every step of the integration runs in the HIP
library.  Device buffers handed to the library are torch CUDA (HIP) tensors;
torch provides device memory and the stream, nothing else.  If libens.so is
missing, loading raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libens.so")

# enums (include/ens.h)
ENS_OK, ENS_E_INVAL, ENS_E_NOMEM, ENS_E_HIP, ENS_E_ORDER, ENS_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
ENS_QUAD, ENS_LORENZ, ENS_KM, ENS_PRV, ENS_DIV, ENS_SIN, ENS_KM6 = 0, 1, 2, 3, 4, 5, 6
ENS_RK4, ENS_RKCK45, ENS_RKDP45 = 0, 1, 2
ENS_HOST, ENS_DEVICE = 0, 1
(ENS_STATE, ENS_TIME, ENS_H, ENS_ACC, ENS_RECORDS, ENS_STATS, ENS_STATUS, ENS_DRIVE_PHASE,
 ENS_CARRY) = range(9)
ENS_CARRY_YMAX, ENS_CARRY_YMIN, ENS_CARRY_TPS, ENS_CARRY_SEATED = range(4)
ENS_NCARRY = 4
ENS_SYS_OK, ENS_SYS_DT_MIN, ENS_SYS_MAX_STEPS, ENS_SYS_NONFINITE = 0, 1, 2, 4
ENS_SYS_SETTLED, ENS_SYS_EVENT_ITER, ENS_SYS_SEATED = 8, 16, 32
ENS_ST_ACCEPTED, ENS_ST_REJECTED, ENS_ST_NRHS, ENS_ST_IMPACTS, ENS_ST_PHASES, ENS_ST_EVRETRY = range(6)
ENS_NSTAT = 6
ENS_MAX_ENSEMBLES = 16
ENS_MAX_SHARED = 16

MODEL_DIMS = {ENS_QUAD: (1, 1, 0, 1), ENS_LORENZ: (3, 1, 2, 1),
              ENS_KM: (2, 2, 11, 1), ENS_PRV: (3, 1, 4, 2),
              ENS_DIV: (1, 1, 0, 1), ENS_SIN: (1, 1, 0, 1),
              ENS_KM6: (2, 6, 7, 1)}   # D, P, S, F


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class ens_desc(C.Structure):
    _fields_ = [("model", C.c_int32), ("solver", C.c_int32), ("n", C.c_int64),
                ("n_ensembles", C.c_int32), ("device", C.c_int32),
                ("ens_offsets", C.POINTER(C.c_int64)), ("hip_stream", C.c_void_p),
                ("tangent", C.c_int32), ("reserved_", C.c_int32),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", C.c_void_p)]


class ens_solve_opts(C.Structure):
    _fields_ = [("dt", C.c_double), ("n_steps", C.c_int64),
                ("t_phase", C.c_double), ("dt0", C.c_double), ("dt_min", C.c_double),
                ("dt_max", C.c_double), ("rtol", C.c_double), ("atol", C.c_double),
                ("event_tol", C.c_double), ("t_cap", C.c_double), ("v_stick", C.c_double),
                ("n_phases", C.c_int64), ("n_record", C.c_int64), ("max_steps", C.c_int64),
                ("max_event_iter", C.c_int32), ("block", C.c_int32), ("spl", C.c_int32),
                ("refill", C.c_int32), ("grid", C.c_int32), ("use_graph", C.c_int32),
                ("locate_max", C.c_int32), ("reserved_", C.c_int32), ("spread", C.c_int64)]


_lib = None


def load():
    """Load libens.so; raises RuntimeError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libens.so not found at {LIB_PATH}: run __graft_entry__.build()")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7);
    # loading torch first makes libens bind to that one instead of bringing a
    # second runtime into the process
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    L.ens_create.argtypes = [C.POINTER(ens_desc), C.POINTER(vp)]
    L.ens_destroy.argtypes = [vp]
    L.ens_last_error.argtypes = [vp]
    L.ens_last_error.restype = C.c_char_p
    L.ens_set_params.argtypes = [vp, vp, i32]
    L.ens_set_shared.argtypes = [vp, i32, dp, i32]
    L.ens_set_budget.argtypes = [vp, i32, i64, i64]
    L.ens_set_state.argtypes = [vp, vp, vp, vp, i32]
    L.ens_set_drive_phase.argtypes = [vp, vp, i32]
    L.ens_set_carry.argtypes = [vp, vp, i32]
    L.ens_default_opts.argtypes = [C.POINTER(ens_solve_opts)]
    L.ens_default_opts.restype = None
    L.ens_solve.argtypes = [vp, C.POINTER(ens_solve_opts)]
    L.ens_read.argtypes = [vp, i32, vp, C.c_size_t, i32]
    L.ens_field_bytes.argtypes = [vp, i32]
    L.ens_field_bytes.restype = C.c_size_t
    L.ens_last_launch.argtypes = [vp] + [C.POINTER(i32)] * 4
    L.ens_last_kernel_ms.argtypes = [vp, C.POINTER(C.c_float)]
    L.ens_tune.argtypes = [vp, C.POINTER(ens_solve_opts), i64, C.POINTER(ens_solve_opts),
                           C.POINTER(C.c_float)]
    L.ens_set_params_gather.argtypes = [vp, vp, i64, vp]
    L.ens_set_order.argtypes = [vp, vp, i32]
    L.ens_order_by_work.argtypes = [vp]
    L.ens_micro_fma.argtypes = [i32, i64, C.POINTER(C.c_double), C.POINTER(C.c_float)]
    _lib = L
    return L


def micro_fma(device: int = 0, iters: int = 1 << 16):
    """Sustained FP64 FMA rate of the device (TFLOP/s, ms); see ens_micro_fma."""
    tf = C.c_double()
    ms = C.c_float()
    _check(load().ens_micro_fma(int(device), int(iters), C.byref(tf), C.byref(ms)))
    return tf.value, ms.value


class EnsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libens error {code}: {msg}")
        self.code = code


def _check(rc, handle=None):
    if rc != ENS_OK:
        msg = load().ens_last_error(handle)
        raise EnsError(rc, msg.decode() if msg else "")


def default_opts(**kw) -> ens_solve_opts:
    o = ens_solve_opts()
    load().ens_default_opts(C.byref(o))
    names = {f[0] for f in ens_solve_opts._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown solve option {k!r}")
        setattr(o, k, v)
    return o


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class Ensemble:
    """One libens handle: n systems of one model, solved on one device."""

    def __init__(self, model: int, solver: int, n: int,
                 offsets: Optional[Sequence[int]] = None, device: int = 0, stream=None,
                 tangent: int = 0, allocator=None):
        """allocator: None (the library's hipMalloc / hipFree) or a pair of
        callables (alloc(nbytes) -> device address, free(address)) through
        which the handle obtains and releases all its device memory."""
        L = load()
        self.model, self.solver, self.n = int(model), int(solver), int(n)
        # an unknown model is passed through: ens_create rejects it
        self.D, self.P, self.S, self.F = MODEL_DIMS.get(self.model, (0, 0, 0, 0))
        self.tangent = int(tangent)   # tangent vectors (True = 1)
        if self.tangent:   # state [y; v_1 .. v_K], records (y1max, K log growths)
            self.D, self.F = self.D * (1 + self.tangent), 1 + self.tangent
        self.device = int(device)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(self.device)
        self._stream = stream
        self.stream_ptr = int(getattr(stream, "cuda_stream", stream) or 0)
        d = ens_desc()
        d.model, d.solver, d.n = self.model, self.solver, self.n
        d.device = self.device
        d.hip_stream = self.stream_ptr
        d.tangent = self.tangent
        self._alloc_fns = None
        if allocator is not None:
            ua, uf = allocator
            # the C callbacks stay referenced as long as the handle lives
            self._alloc_fns = (ALLOC_FN(lambda nb, ctx: int(ua(int(nb))) or None),
                               FREE_FN(lambda ptr, ctx: uf(int(ptr))))
            d.alloc, d.free = self._alloc_fns
        self._offs = None
        if offsets is not None:
            self._offs = (C.c_int64 * len(offsets))(*[int(v) for v in offsets])
            d.n_ensembles = len(offsets) - 1
            d.ens_offsets = C.cast(self._offs, C.POINTER(C.c_int64))
        else:
            d.n_ensembles = 1
        h = C.c_void_p()
        _check(L.ens_create(C.byref(d), C.byref(h)))
        self.h = h
        self.n_ensembles = d.n_ensembles

    # -- marshalling helpers
    def _in(self, arr, shape):
        """(pointer, where, keepalive) for an input array of the given shape."""
        if arr is None:
            return None, ENS_HOST, None
        if _is_torch(arr) and arr.is_cuda:
            import torch
            t = arr.to(dtype=torch.float64).contiguous()
            if t.numel() != int(np.prod(shape)):
                raise ValueError(f"expected {shape}, got {tuple(arr.shape)}")
            return C.c_void_p(t.data_ptr()), ENS_DEVICE, t
        a = np.ascontiguousarray(np.asarray(arr, dtype=np.float64))
        if a.size != int(np.prod(shape)):
            raise ValueError(f"expected {shape}, got {a.shape}")
        return C.c_void_p(a.ctypes.data), ENS_HOST, a

    # Device inputs are copied stream-ordered; the binding keeps the source
    # tensors alive until the next call that replaces them.
    def set_params(self, p):
        ptr, where, keep = self._in(p, (self.P, self.n))
        _check(load().ens_set_params(self.h, ptr, where), self.h)
        self._keep_p = keep

    def set_order(self, order):
        """Queue order of the adaptive solver: the k-th system taken is
        order[k] (a permutation of 0..n-1, int64, host or device); None
        restores the index order."""
        if order is None:
            _check(load().ens_set_order(self.h, None, ENS_HOST), self.h)
            return
        if _is_torch(order) and order.is_cuda:
            import torch
            t = order.to(dtype=torch.int64).contiguous()
            if t.numel() != self.n:
                raise ValueError(f"expected {self.n} entries, got {t.numel()}")
            _check(load().ens_set_order(self.h, C.c_void_p(t.data_ptr()), ENS_DEVICE), self.h)
            return
        a = np.ascontiguousarray(np.asarray(order, dtype=np.int64))
        if a.size != self.n:
            raise ValueError(f"expected {self.n} entries, got {a.size}")
        _check(load().ens_set_order(self.h, C.c_void_p(a.ctypes.data), ENS_HOST), self.h)

    def order_by_work(self):
        """Longest-first queue order from the last adaptive solve's step counts."""
        _check(load().ens_order_by_work(self.h), self.h)

    def set_shared(self, ensemble: int, shared):
        a = np.ascontiguousarray(np.asarray(shared, dtype=np.float64))
        _check(load().ens_set_shared(self.h, int(ensemble),
                                     a.ctypes.data_as(C.POINTER(C.c_double)), int(a.size)), self.h)

    def set_budget(self, ensemble: int, n_phases: int = -1, max_impacts: int = 0):
        _check(load().ens_set_budget(self.h, int(ensemble), int(n_phases), int(max_impacts)), self.h)

    def set_state(self, y0, t0=None, h0=None):
        py, wy, ky = self._in(y0, (self.D, self.n))
        pt, wt, kt = self._in(t0, (self.n,))
        ph, wh, kh = self._in(h0, (self.n,))
        wheres = {w for w, a in ((wy, y0), (wt, t0), (wh, h0)) if a is not None}
        if len(wheres) > 1:
            raise ValueError("y0, t0 and h0 must all be host or all device arrays")
        _check(load().ens_set_state(self.h, py, pt, ph, wy), self.h)
        self._keep_state = (ky, kt, kh)

    def set_drive_phase(self, phi):
        """Keller--Miksis: the second drive's phase per system (cycles), e.g.
        the ENS_DRIVE_PHASE output of an earlier solve, to resume it."""
        p, w, k = self._in(phi, (self.n,))
        _check(load().ens_set_drive_phase(self.h, p, w), self.h)
        self._keep_phi = k

    def set_carry(self, carry):
        """Adaptive solvers: the carried phase accessories [ENS_NCARRY][n]
        (the ENS_CARRY output of a solve), after set_state, to resume a solve
        that stopped inside a phase."""
        p, w, k = self._in(carry, (ENS_NCARRY, self.n))
        _check(load().ens_set_carry(self.h, p, w), self.h)
        self._keep_carry = k

    def solve(self, opts: Optional[ens_solve_opts] = None, **kw):
        o = opts if opts is not None else default_opts(**kw)
        if opts is not None and kw:
            for k, v in kw.items():
                setattr(o, k, v)
        _check(load().ens_solve(self.h, C.byref(o)), self.h)
        return o

    _FIELD_DTYPE = {ENS_STATS: np.int64, ENS_STATUS: np.int32}

    def _shape(self, field):
        n = self.n
        if field == ENS_STATE:
            return (self.D, n)
        if field == ENS_RECORDS:
            nb = load().ens_field_bytes(self.h, field)
            R = nb // (8 * self.F * n) if n else 0
            return (R, self.F, n)
        if field == ENS_STATS:
            return (ENS_NSTAT, n)
        if field == ENS_CARRY:
            return (ENS_NCARRY, n)
        return (n,)

    def read(self, field: int, device: bool = False):
        """Result field as a numpy array (host) or a torch tensor (device)."""
        L = load()
        nbytes = L.ens_field_bytes(self.h, field)
        shape = self._shape(field)
        dt = self._FIELD_DTYPE.get(field, np.float64)
        if device:
            import torch
            tdt = {np.int64: torch.int64, np.int32: torch.int32}.get(dt, torch.float64)
            out = torch.empty(shape, dtype=tdt, device=f"cuda:{self.device}")
            _check(L.ens_read(self.h, field, C.c_void_p(out.data_ptr()), nbytes, ENS_DEVICE), self.h)
            return out
        out = np.empty(shape, dtype=dt)
        _check(L.ens_read(self.h, field, C.c_void_p(out.ctypes.data), nbytes, ENS_HOST), self.h)
        return out

    def tune(self, opts: Optional[ens_solve_opts] = None, trial_len: int = 0, **kw):
        """Run the library's autotuner on the current problem; returns
        (opts with the chosen launch fields, trial milliseconds)."""
        o = opts if opts is not None else default_opts(**kw)
        best = ens_solve_opts()
        ms = C.c_float()
        _check(load().ens_tune(self.h, C.byref(o), int(trial_len), C.byref(best), C.byref(ms)),
               self.h)
        return best, float(ms.value)

    def last_kernel_ms(self) -> float:
        ms = C.c_float()
        _check(load().ens_last_kernel_ms(self.h, C.byref(ms)), self.h)
        return float(ms.value)

    def last_launch(self):
        v = [C.c_int32() for _ in range(4)]
        _check(load().ens_last_launch(self.h, *[C.byref(x) for x in v]), self.h)
        return dict(zip(("block", "spl", "grid", "refill"), (x.value for x in v)))

    def close(self):
        if getattr(self, "h", None):
            _check(load().ens_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
