"""Solves that stop inside an integration phase and resume it, on the GPU
(through the C ABI), against one uninterrupted solve and against the oracle;
and the caller-supplied allocator of ens_desc."""
import numpy as np
import pytest

import oracle as O
from paper_2011_01740_amd import inputs as I
from tests.parity import CK_ATOL, CK_RTOL, close, per_system

pytestmark = pytest.mark.gpu

PRV_SH = list(I.PRV_DEFAULT)


def _ens():
    import torch
    from paper_2011_01740_amd import ens
    assert torch.cuda.is_available()
    return ens


def _read_all(ens, e):
    return {k: e.read(f) for k, f in (("y", ens.ENS_STATE), ("t", ens.ENS_TIME),
                                      ("h", ens.ENS_H), ("rec", ens.ENS_RECORDS),
                                      ("stats", ens.ENS_STATS), ("status", ens.ENS_STATUS),
                                      ("carry", ens.ENS_CARRY))}


def test_valve_resume_inside_a_phase_equals_one_solve():
    """Valves stopped by an impact budget (inside a Poincare phase) and solved
    on by a second ens_solve give the uninterrupted solve's records and final
    state bit for bit; both match the oracle's split run."""
    ens = _ens()
    N = 10
    P, y0 = I.prv_linspace(256, 0.3, 7.0)
    n = P.shape[1]
    with ens.Ensemble(ens.ENS_PRV, ens.ENS_RKCK45, n) as e:
        e.set_params(P)
        e.set_state(y0)
        e.solve(n_phases=N, n_record=N)
        whole = _read_all(ens, e)
    with ens.Ensemble(ens.ENS_PRV, ens.ENS_RKCK45, n) as e:
        e.set_params(P)
        e.set_state(y0)
        e.set_budget(0, N, 3)
        e.solve(n_phases=N, n_record=N)
        a = _read_all(ens, e)
        e.set_budget(0, N, 0)
        e.solve(n_phases=N, n_record=N)        # continues from the library state
        b = _read_all(ens, e)
    p1 = a["stats"][O.ST_PHASES]
    assert (a["stats"][O.ST_IMPACTS] == 3).any() and (p1 < N).all()
    # the second solve runs N more phases: its first N - p1 are the rest of
    # the uninterrupted solve's N
    for i in range(n):
        k = int(p1[i])
        np.testing.assert_array_equal(a["rec"][:k, :, i], whole["rec"][:k, :, i])
        np.testing.assert_array_equal(b["rec"][:N - k, :, i], whole["rec"][k:, :, i])
    for key in ("stats",):
        for row in (O.ST_ACCEPTED, O.ST_REJECTED, O.ST_IMPACTS):
            # second solve ran further (N phases): at least the whole's remainder
            assert (a[key][row] <= whole[key][row]).all()
    # against the oracle, split the same way
    ra = O.rkck45(O.PRV, P, PRV_SH, y0, O.Opts(n_phases=N, n_record=N, max_impacts=3), nthreads=8)
    rb = O.rkck45(O.PRV, P, PRV_SH, ra.y, O.Opts(n_phases=N, n_record=N), t0=ra.t, h0=ra.h,
                  carry0=ra.carry, nthreads=8)
    ok = (per_system(close(b["y"], rb.y, CK_RTOL, CK_ATOL))
          & per_system(close(b["rec"], rb.records, CK_RTOL, CK_ATOL))
          & per_system(close(a["carry"][:3], ra.carry[:3], CK_RTOL, CK_ATOL)
                       | (a["carry"][:3] == ra.carry[:3])))
    # the valve is mildly chaotic for some q: most of the ensemble must agree
    assert ok.mean() > 0.9, ok.mean()
    np.testing.assert_array_equal(a["carry"][O.CARRY_SEATED], ra.carry[O.CARRY_SEATED])


@pytest.mark.parametrize("solver", ["ck", "dp"])
def test_seated_valve_resumes_seated(solver):
    ens = _ens()
    s = ens.ENS_RKCK45 if solver == "ck" else ens.ENS_RKDP45
    y0 = np.array([[1e-20], [0.0], [9.9]])
    P = np.array([[1.0]])
    with ens.Ensemble(ens.ENS_PRV, s, 1) as e:
        e.set_params(P)
        e.set_state(y0)
        e.solve(n_phases=2, n_record=2)
        whole = _read_all(ens, e)
    with ens.Ensemble(ens.ENS_PRV, s, 1) as e:
        e.set_params(P)
        e.set_state(y0)
        e.set_budget(0, 2, 1)
        e.solve(n_phases=2, n_record=2)
        a = _read_all(ens, e)
        assert a["carry"][O.CARRY_SEATED, 0] == 1.0 and a["status"][0] & O.SYS_SEATED
        # hand the stopped system to a fresh handle: state, clock, step and carry
        with ens.Ensemble(ens.ENS_PRV, s, 1) as f:
            f.set_params(P)
            f.set_state(a["y"], a["t"], a["h"])
            f.set_carry(a["carry"])
            f.solve(n_phases=2 - int(a["stats"][O.ST_PHASES, 0]), n_record=2)
            b = _read_all(ens, f)
    np.testing.assert_array_equal(b["y"], whole["y"])
    assert b["t"][0] == whole["t"][0]
    assert b["stats"][O.ST_IMPACTS, 0] + 1 == whole["stats"][O.ST_IMPACTS, 0]


def test_km_step_cap_inside_a_phase_resumes_the_running_maximum():
    ens = _ens()
    P, y0 = I.km_grid(16, 16)
    n = P.shape[1]
    N = 4
    with ens.Ensemble(ens.ENS_KM, ens.ENS_RKCK45, n) as e:
        e.set_params(P)
        e.set_state(y0)
        e.solve(n_phases=N, n_record=N)
        whole = _read_all(ens, e)
    cap = 150
    with ens.Ensemble(ens.ENS_KM, ens.ENS_RKCK45, n) as e:
        e.set_params(P)
        e.set_state(y0)
        e.solve(n_phases=N, n_record=N, max_steps=cap)
        a = _read_all(ens, e)
        e.solve(n_phases=N, n_record=N)
        b = _read_all(ens, e)
    p1 = a["stats"][O.ST_PHASES]
    stopped = (a["status"] & O.SYS_MAX_STEPS) != 0
    assert stopped.mean() > 0.5
    for i in range(n):
        k = int(p1[i])
        np.testing.assert_array_equal(b["rec"][:N - k, :, i], whole["rec"][k:, :, i])
    # the carried maximum of a stopped system is the oracle's
    r = O.rkck45(O.KM, P, I.KM_WATER, y0, O.Opts(n_phases=N, n_record=N, max_steps=cap),
                 nthreads=8)
    np.testing.assert_array_equal(r.stats[O.ST_PHASES], p1)
    ok = per_system(close(a["carry"][[O.CARRY_YMAX, O.CARRY_TPS]],
                          r.carry[[O.CARRY_YMAX, O.CARRY_TPS]], CK_RTOL, CK_ATOL)
                    | (a["carry"][[O.CARRY_YMAX, O.CARRY_TPS]]
                       == r.carry[[O.CARRY_YMAX, O.CARRY_TPS]]))
    # the cap cuts each system at its 150th attempt: where the GPU's and the
    # oracle's accept / reject sequences differ by one attempt (FMA rounding,
    # a few systems) the cut falls on another step point
    same = ((a["stats"][O.ST_ACCEPTED] == r.stats[O.ST_ACCEPTED])
            & (a["stats"][O.ST_REJECTED] == r.stats[O.ST_REJECTED]))
    assert same.mean() >= 0.97, same.mean()
    assert ok[same].all(), np.nonzero(same & ~ok)[0][:8]
    # no minimum is kept for Keller--Miksis: +inf on both sides
    np.testing.assert_array_equal(a["carry"][O.CARRY_YMIN], r.carry[O.CARRY_YMIN])


def test_set_state_starts_fresh_phases():
    ens = _ens()
    P, y0 = I.prv_linspace(8, 1.0, 3.0)
    t0 = np.linspace(0.0, 2.0, 8)
    with ens.Ensemble(ens.ENS_PRV, ens.ENS_RKCK45, 8) as e:
        e.set_params(P)
        e.set_state(y0, t0)
        c = e.read(ens.ENS_CARRY)
    assert np.all(c[O.CARRY_YMAX] == -np.inf) and np.all(c[O.CARRY_YMIN] == np.inf)
    np.testing.assert_array_equal(c[O.CARRY_TPS], t0)
    assert np.all(c[O.CARRY_SEATED] == 0.0)


def test_caller_allocator_gets_every_buffer_and_results_do_not_change():
    """ens_desc.alloc / free: every device buffer of the handle comes from the
    caller (torch's caching allocator here), none from hipMalloc, and the
    solve is bit-identical to one on library-allocated buffers."""
    import torch
    ens = _ens()
    live = {}
    calls = {"alloc": 0, "free": 0}

    def alloc(nbytes):
        t = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
        live[t.data_ptr()] = t
        calls["alloc"] += 1
        return t.data_ptr()

    def free(ptr):
        calls["free"] += 1
        live.pop(ptr)

    P, y0 = I.km_grid(24, 24)
    n = P.shape[1]
    out = []
    for allocator in (None, (alloc, free)):
        with ens.Ensemble(ens.ENS_KM, ens.ENS_RKCK45, n, allocator=allocator) as e:
            e.set_params(P)
            e.set_state(y0)
            e.solve(n_phases=2, n_record=2)
            e.order_by_work()
            e.solve(n_phases=3, n_record=3, use_graph=1)
            out.append(_read_all(ens, e))
            if allocator is not None:
                assert calls["alloc"] >= 10 and len(live) == calls["alloc"] - calls["free"]
                # the pilot, its ordering and the second solve allocated
                # nothing beyond the record ring's growth
                assert calls["alloc"] <= 20
    assert calls["free"] == calls["alloc"] and not live
    for k in out[0]:
        np.testing.assert_array_equal(out[0][k], out[1][k])


def test_order_by_work_allocates_nothing_after_create():
    import torch
    ens = _ens()
    seen = []

    def alloc(nbytes):
        t = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
        seen.append(t)
        return t.data_ptr()

    def free(ptr):
        pass

    P, y0 = I.km_grid(16, 16)
    with ens.Ensemble(ens.ENS_KM, ens.ENS_RKCK45, P.shape[1], allocator=(alloc, free)) as e:
        e.set_params(P)
        e.set_state(y0)
        e.solve(n_phases=1, n_record=4)
        k = len(seen)
        e.order_by_work()
        e.solve(n_phases=3, n_record=4)
        assert len(seen) == k
