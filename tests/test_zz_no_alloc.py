"""ens_solve_noalloc (include/ens_noalloc.h) through the C ABI: the handle-free
adaptive solve that allocates nothing, against ens_solve on the same inputs
(bit for bit: the same kernels), on two calls in a row with the second one
smaller, a resumed call, and its size limit."""
import ctypes as C

import numpy as np
import pytest

from paper_2011_01740_amd import inputs as I

pytestmark = pytest.mark.gpu


class NoallocArgs(C.Structure):
    _fields_ = [("model", C.c_int32), ("solver", C.c_int32), ("n", C.c_int64),
                ("n_ensembles", C.c_int32), ("device", C.c_int32), ("tangent", C.c_int32),
                ("fresh", C.c_int32), ("ens_offsets", C.c_void_p), ("shared", C.c_void_p),
                ("budgets", C.c_void_p), ("hip_stream", C.c_void_p), ("p", C.c_void_p),
                ("y", C.c_void_p), ("t", C.c_void_p), ("h", C.c_void_p), ("phi2", C.c_void_p),
                ("carry", C.c_void_p), ("records", C.c_void_p), ("stats", C.c_void_p),
                ("status", C.c_void_p), ("order", C.c_void_p), ("reserved_", C.c_int32),
                ("pad_", C.c_int32)]


def _lib():
    import torch
    from paper_2011_01740_amd import ens
    assert torch.cuda.is_available()
    L = ens.load()
    L.ens_solve_noalloc.argtypes = [C.POINTER(NoallocArgs), C.POINTER(ens.ens_solve_opts)]
    return ens, L


def _handle_solve(ens, model, solver, P, y0, opts_list, offsets=None, shared=None, budgets=None):
    n = y0.shape[-1]
    outs = []
    with ens.Ensemble(model, solver, n, offsets=offsets) as e:
        e.set_params(P)
        if shared is not None:
            for k, sh in enumerate(shared):
                e.set_shared(k, sh)
        if budgets is not None:
            for k, (ph, imp) in enumerate(budgets):
                e.set_budget(k, ph, imp)
        e.set_state(y0)
        for o in opts_list:
            e.solve(**o)
            r = {"y": e.read(ens.ENS_STATE), "t": e.read(ens.ENS_TIME), "h": e.read(ens.ENS_H),
                 "rec": e.read(ens.ENS_RECORDS), "stats": e.read(ens.ENS_STATS),
                 "status": e.read(ens.ENS_STATUS), "carry": e.read(ens.ENS_CARRY)}
            if model in (ens.ENS_KM, ens.ENS_KM6):
                r["phi"] = e.read(ens.ENS_DRIVE_PHASE)
            outs.append(r)
    return outs


class Buffers:
    """Caller-owned device arrays for one no-alloc problem (torch tensors)."""

    def __init__(self, ens, model, P, y0, R):
        import torch
        D, Pn, S, F = ens.MODEL_DIMS[model]
        n = y0.shape[-1]
        dev = "cuda:0"
        self.n, self.R, self.F = n, R, F
        self.p = torch.tensor(np.asarray(P, dtype=np.float64), device=dev).contiguous()
        self.y = torch.tensor(np.asarray(y0, dtype=np.float64), device=dev).contiguous()
        self.t = torch.zeros(n, dtype=torch.float64, device=dev)
        self.h = torch.zeros(n, dtype=torch.float64, device=dev)
        self.phi = torch.zeros(n, dtype=torch.float64, device=dev)
        self.carry = torch.zeros((4, n), dtype=torch.float64, device=dev)
        self.rec = torch.zeros((max(R, 1), F, n), dtype=torch.float64, device=dev)
        self.stats = torch.zeros((6, n), dtype=torch.int64, device=dev)
        self.status = torch.zeros(n, dtype=torch.int32, device=dev)

    def args(self, ens, model, solver, fresh, offsets=None, shared=None, budgets=None):
        import torch
        a = NoallocArgs()
        a.model, a.solver, a.n, a.device, a.fresh = model, solver, self.n, 0, fresh
        self._keep = []
        if offsets is not None:
            off = np.asarray(offsets, dtype=np.int64)
            self._keep.append(off)
            a.ens_offsets = off.ctypes.data
            a.n_ensembles = len(offsets) - 1
        else:
            a.n_ensembles = 1
        if shared is not None:
            sh = np.zeros((a.n_ensembles, ens.ENS_MAX_SHARED))
            for k, row in enumerate(shared):
                sh[k, :len(row)] = row
            self._keep.append(sh)
            a.shared = sh.ctypes.data
        if budgets is not None:
            b = np.asarray(budgets, dtype=np.int64).reshape(-1)
            self._keep.append(b)
            a.budgets = b.ctypes.data
        a.hip_stream = torch.cuda.current_stream(0).cuda_stream
        a.p, a.y, a.t, a.h = (self.p.data_ptr(), self.y.data_ptr(), self.t.data_ptr(),
                              self.h.data_ptr())
        a.phi2, a.carry = self.phi.data_ptr(), self.carry.data_ptr()
        a.records = self.rec.data_ptr() if self.R > 0 else None
        a.stats, a.status = self.stats.data_ptr(), self.status.data_ptr()
        return a

    def read(self, km):
        import torch
        torch.cuda.synchronize()
        r = {"y": self.y.cpu().numpy(), "t": self.t.cpu().numpy(), "h": self.h.cpu().numpy(),
             "rec": self.rec[:self.R].cpu().numpy(), "stats": self.stats.cpu().numpy(),
             "status": self.status.cpu().numpy(), "carry": self.carry.cpu().numpy()}
        if km:
            r["phi"] = self.phi.cpu().numpy()
        return r


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_noalloc_equals_ens_solve_on_two_calls_the_second_smaller():
    ens, L = _lib()
    # first call: a Keller--Miksis grid, Cash--Karp, 3 phases, a 3-slot ring
    P, y0 = I.km_grid(40, 40)
    opts = dict(n_phases=3, n_record=3)
    ref = _handle_solve(ens, ens.ENS_KM, ens.ENS_RKCK45, P, y0, [opts])[0]
    bk = Buffers(ens, ens.ENS_KM, P, y0, 3)
    o = ens.default_opts(**opts)
    assert L.ens_solve_noalloc(C.byref(bk.args(ens, ens.ENS_KM, ens.ENS_RKCK45, 1)),
                               C.byref(o)) == 0, L.ens_last_error(None)
    _same(bk.read(True), ref)
    # second call, smaller: a batched valve ensemble (two sub-ensembles with
    # their own budgets and shared parameters), Dormand--Prince
    Pv, yv = I.prv_linspace(300, 0.5, 6.0)
    offs = [0, 120, 300]
    shared = [list(I.PRV_DEFAULT), [1.25, 10.0, 20.0, 0.7]]
    budgets = [(6, 0), (-1, 5)]
    optv = dict(n_phases=9, n_record=4)
    refv = _handle_solve(ens, ens.ENS_PRV, ens.ENS_RKDP45, Pv, yv, [optv], offsets=offs,
                         shared=shared, budgets=budgets)[0]
    bv = Buffers(ens, ens.ENS_PRV, Pv, yv, 4)
    o = ens.default_opts(**optv)
    a = bv.args(ens, ens.ENS_PRV, ens.ENS_RKDP45, 1, offsets=offs, shared=shared,
                budgets=budgets)
    assert L.ens_solve_noalloc(C.byref(a), C.byref(o)) == 0, L.ens_last_error(None)
    _same(bv.read(False), refv)


def test_noalloc_resumes_like_a_second_ens_solve():
    ens, L = _lib()
    P, y0 = I.prv_linspace(200, 0.3, 7.0)
    o1 = dict(n_phases=5, n_record=5, max_steps=700)
    o2 = dict(n_phases=4, n_record=4)
    ref = _handle_solve(ens, ens.ENS_PRV, ens.ENS_RKCK45, P, y0, [o1, o2])
    b = Buffers(ens, ens.ENS_PRV, P, y0, 5)
    assert L.ens_solve_noalloc(C.byref(b.args(ens, ens.ENS_PRV, ens.ENS_RKCK45, 1)),
                               C.byref(ens.default_opts(**o1))) == 0
    _same(b.read(False), ref[0])
    b.R = 4
    assert L.ens_solve_noalloc(C.byref(b.args(ens, ens.ENS_PRV, ens.ENS_RKCK45, 0)),
                               C.byref(ens.default_opts(**o2))) == 0
    _same(b.read(False), ref[1])


def test_noalloc_refuses_sizes_beyond_its_scratch():
    ens, L = _lib()
    P, y0 = I.km_grid(4, 4)
    b = Buffers(ens, ens.ENS_KM, P, y0, 1)
    a = b.args(ens, ens.ENS_KM, ens.ENS_RKCK45, 1)
    a.n_ensembles = 17
    assert L.ens_solve_noalloc(C.byref(a), C.byref(ens.default_opts())) == ens.ENS_E_INVAL
    assert b"scratch" in L.ens_last_error(None)
    a = b.args(ens, ens.ENS_KM, ens.ENS_RK4, 1)
    assert L.ens_solve_noalloc(C.byref(a), C.byref(ens.default_opts())) == ens.ENS_E_INVAL
