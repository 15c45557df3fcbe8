"""Python access to the C oracle (TEST INFRASTRUCTURE ONLY).

The oracle is a plain serial FP64 CPU implementation of the integrators
(see oracle.c for what it follows and the readings it takes).  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import this
package; the GPU library never does.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields

import numpy as np

from . import build as _build

QUAD, LORENZ, KM, PRV, DIV, SIN, KM6 = 0, 1, 2, 3, 4, 5, 6
SYS_OK, SYS_DT_MIN, SYS_MAX_STEPS, SYS_NONFINITE = 0, 1, 2, 4
SYS_SETTLED, SYS_EVENT_ITER, SYS_SEATED = 8, 16, 32
ST_ACCEPTED, ST_REJECTED, ST_NRHS, ST_IMPACTS, ST_PHASES, ST_EVRETRY = range(6)
NSTAT = 6
# rows of the carried accessories (orc_rkck45_ext): running phase y1max, y1min,
# phase start time, valve seated (1/0)
CARRY_YMAX, CARRY_YMIN, CARRY_TPS, CARRY_SEATED = range(4)
NCARRY = 4
CASH_KARP, DORMAND_PRINCE = 0, 1

_lib = None
_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)


class _Opts(C.Structure):
    _fields_ = [("t_phase", C.c_double), ("dt0", C.c_double), ("dt_min", C.c_double),
                ("dt_max", C.c_double), ("rtol", C.c_double), ("atol", C.c_double),
                ("event_tol", C.c_double), ("t_cap", C.c_double), ("v_stick", C.c_double),
                ("n_phases", C.c_int64), ("n_record", C.c_int64),
                ("max_impacts", C.c_int64), ("max_steps", C.c_int64),
                ("max_event_iter", C.c_int32), ("scheme", C.c_int32),
                ("locate_max", C.c_int32), ("lyapunov", C.c_int32)]


@dataclass
class Opts:
    """Adaptive-solver options; defaults are the readings used for every workload."""
    t_phase: float = 1.0
    dt0: float = 1e-2
    dt_min: float = 1e-14
    dt_max: float = 0.1
    rtol: float = 1e-10
    atol: float = 1e-10
    event_tol: float = 1e-6
    t_cap: float = 50.0
    v_stick: float = 1e-9
    n_phases: int = 1
    n_record: int = 1
    max_impacts: int = 0
    max_steps: int = 0
    max_event_iter: int = 20
    scheme: int = 0                 # CASH_KARP or DORMAND_PRINCE
    locate_max: int = 0             # KM: maxima located on the step interpolant
    lyapunov: int = 0               # tangents of the variational equation (Lyapunov)

    def _c(self) -> _Opts:
        o = _Opts()
        for f in fields(self):
            setattr(o, f.name, getattr(self, f.name))
        return o


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB selects another build of the same source (the sanitized
        # one of the CPU sanitizer test)
        path = os.environ.get("ORACLE_LIB") or _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        L.orc_rhs.argtypes = [C.c_int, C.c_double, _dp, _dp, _dp, _dp]
        L.orc_km_coeffs.argtypes = [_dp, _dp, _dp]
        L.orc_rk4.argtypes = [C.c_int, C.c_int64, _dp, _dp, _dp, C.c_double, C.c_int64,
                              _dp, _dp, C.c_int]
        L.orc_rkck45.argtypes = [C.c_int, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp,
                                 C.POINTER(_Opts), _dp, _dp, _dp, _dp, _dp, _i64p, _i32p,
                                 C.c_int]
        L.orc_rkck45_ext.argtypes = [C.c_int, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp,
                                     C.POINTER(_Opts), _dp, _dp, _dp, _dp, _dp, _i64p, _i32p,
                                     _dp, _dp, _dp, C.c_int]
        L.orc_rkck_step.argtypes = [C.c_int, C.c_double, _dp, _dp, _dp, C.c_double, _dp, _dp]
        L.orc_rkck_tableau.argtypes = [_dp, _dp, _dp, _dp]
        L.orc_rkdp_step.argtypes = [C.c_int, C.c_double, _dp, _dp, _dp, C.c_double, _dp, _dp]
        L.orc_rkdp_tableau.argtypes = [_dp, _dp, _dp, _dp]
        L.orc_jacobian.argtypes = [C.c_int, C.c_double, _dp, _dp, _dp, _dp]
        for f in ("orc_dim", "orc_nparam", "orc_nshared", "orc_nrec_fields"):
            getattr(L, f).argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def dim(model):
    return lib().orc_dim(model)


def nparam(model):
    return lib().orc_nparam(model)


def nrec_fields(model):
    return lib().orc_nrec_fields(model)


def _shared(model, shared):
    ns = lib().orc_nshared(model)
    sh = _f64(np.zeros(max(ns, 1)) if shared is None else shared)
    if sh.size < ns:
        raise ValueError(f"model {model} needs {ns} shared parameters")
    return sh


def rhs(model, t, y, p, shared=None):
    y = _f64(y)
    p = _f64(p)
    sh = _shared(model, shared)
    out = np.zeros(dim(model))
    if lib().orc_rhs(model, float(t), _ptr(y), _ptr(p), _ptr(sh), _ptr(out)):
        raise ValueError("bad model")
    return out


def jacobian(model, t, y, p, shared=None):
    y = _f64(y)
    p = _f64(p)
    sh = _shared(model, shared)
    D = dim(model)
    out = np.zeros(D * D)
    if lib().orc_jacobian(model, float(t), _ptr(y), _ptr(p), _ptr(sh), _ptr(out)):
        raise ValueError("bad model")
    return out.reshape(D, D)


def km_coeffs(p, shared):
    p = _f64(p)
    sh = _f64(shared)
    out = np.zeros(13)
    lib().orc_km_coeffs(_ptr(p), _ptr(sh), _ptr(out))
    return out


def rk4(model, params, shared, y0, dt, nsteps, nthreads=1):
    """Fixed-step RK4 over an ensemble.  Returns (y[D][n], y1max[n])."""
    D = dim(model)
    y0 = _f64(y0)
    n = y0.shape[-1]
    y0 = y0.reshape(D, n)
    params = _f64(params).reshape(nparam(model), n)
    sh = _shared(model, shared)
    y = np.empty((D, n))
    ymax = np.empty(n)
    rc = lib().orc_rk4(model, n, _ptr(params), _ptr(sh), _ptr(y0), float(dt), int(nsteps),
                       _ptr(y), _ptr(ymax), int(nthreads))
    if rc:
        raise ValueError("orc_rk4 rejected its arguments")
    return y, ymax


@dataclass
class AdaptiveResult:
    y: np.ndarray        # [D][n]
    t: np.ndarray        # [n]
    h: np.ndarray        # [n]
    records: np.ndarray  # [R][F][n], ring: phase k in slot k % R
    stats: np.ndarray    # [NSTAT][n] int64
    status: np.ndarray   # [n] int32
    phi: np.ndarray      # [n] Keller--Miksis: second drive's phase at the phase start
    carry: np.ndarray    # [NCARRY][n] running phase y1max, y1min, phase start, seated
    hx: np.ndarray       # [2][n] smallest, largest accepted step (phase-end cuts excluded)


def rkck45(model, params, shared, y0, opts: Opts, t0=None, h0=None, nthreads=1, phi0=None,
           carry0=None):
    """Adaptive solve of an ensemble through its phases with the scheme of
    opts.scheme (Cash--Karp by default).  phi0 (Keller--Miksis): the second
    drive's phase in cycles at the start of the current phase (0 if None).
    carry0: a previous result's `carry` (None: every system starts fresh);
    with y, t, h, phi and carry passed back a solve resumes exactly."""
    D = dim(model) * (1 + int(opts.lyapunov))
    y0 = _f64(y0)
    n = y0.shape[-1]
    y0 = y0.reshape(D, n)
    params = _f64(params).reshape(nparam(model), n)
    sh = _shared(model, shared)
    t0 = None if t0 is None else _f64(t0).reshape(n)
    h0 = None if h0 is None else _f64(h0).reshape(n)
    phi0 = None if phi0 is None else _f64(phi0).reshape(n)
    R = int(opts.n_record)
    F = 1 + int(opts.lyapunov) if opts.lyapunov else nrec_fields(model)
    y = np.empty((D, n))
    t = np.empty(n)
    h = np.empty(n)
    phi = np.empty(n)
    rec = np.full((max(R, 0), F, n), np.nan)
    stats = np.zeros((NSTAT, n), dtype=np.int64)
    status = np.zeros(n, dtype=np.int32)
    carry0 = None if carry0 is None else _f64(carry0).reshape(NCARRY, n)
    carry = np.empty((NCARRY, n))
    hx = np.empty((2, n))
    o = opts._c()
    rc = lib().orc_rkck45_ext(model, n, _ptr(params), _ptr(sh), _ptr(y0), _ptr(t0), _ptr(h0),
                              _ptr(phi0), C.byref(o), _ptr(y), _ptr(t), _ptr(h), _ptr(phi),
                              _ptr(rec) if R > 0 else None,
                              stats.ctypes.data_as(_i64p), status.ctypes.data_as(_i32p),
                              _ptr(carry0), _ptr(carry), _ptr(hx), int(nthreads))
    if rc:
        raise ValueError("orc_rkck45 rejected its arguments")
    return AdaptiveResult(y, t, h, rec, stats, status, phi, carry, hx)


def rkck_step(model, t, y, p, shared, h):
    """One Cash--Karp step without error control: (y5, y4)."""
    y = _f64(y)
    p = _f64(p)
    sh = _shared(model, shared)
    y5 = np.zeros(dim(model))
    y4 = np.zeros(dim(model))
    lib().orc_rkck_step(model, float(t), _ptr(y), _ptr(p), _ptr(sh), float(h), _ptr(y5), _ptr(y4))
    return y5, y4


def rkck_tableau():
    a = np.zeros((6, 6))
    b5 = np.zeros(6)
    b4 = np.zeros(6)
    c = np.zeros(6)
    lib().orc_rkck_tableau(_ptr(a), _ptr(b5), _ptr(b4), _ptr(c))
    return a, b5, b4, c


def rkdp45(model, params, shared, y0, opts: Opts, t0=None, h0=None, nthreads=1, phi0=None,
           carry0=None):
    """Adaptive Dormand--Prince solve (first same as last) of an ensemble."""
    o = Opts(**{f.name: getattr(opts, f.name) for f in fields(opts)})
    o.scheme = DORMAND_PRINCE
    return rkck45(model, params, shared, y0, o, t0, h0, nthreads, phi0, carry0)


def rkdp_step(model, t, y, p, shared, h):
    """One Dormand--Prince step without error control: (y5, y4)."""
    y = _f64(y)
    p = _f64(p)
    sh = _shared(model, shared)
    y5 = np.zeros(dim(model))
    y4 = np.zeros(dim(model))
    lib().orc_rkdp_step(model, float(t), _ptr(y), _ptr(p), _ptr(sh), float(h), _ptr(y5), _ptr(y4))
    return y5, y4


def rkdp_tableau():
    a = np.zeros((7, 7))
    b5 = np.zeros(7)
    b4 = np.zeros(7)
    c = np.zeros(7)
    lib().orc_rkdp_tableau(_ptr(a), _ptr(b5), _ptr(b4), _ptr(c))
    return a, b5, b4, c
