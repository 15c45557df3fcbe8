"""GPU parity of the persistent adaptive Cash--Karp kernel against the oracle,
plus the properties of the work queue (through the C ABI)."""
import numpy as np
import pytest

import oracle as O
from paper_2011_01740_amd import inputs as I
from tests.parity import CK_ATOL, CK_RTOL, PERTURB, close, per_system, sensitivity_mask

pytestmark = pytest.mark.gpu

SHARED = {0: None, 1: [I.LORENZ_SIGMA, I.LORENZ_BETA], 2: list(I.KM_WATER), 3: list(I.PRV_DEFAULT)}


def _ens():
    import torch
    from paper_2011_01740_amd import ens
    assert torch.cuda.is_available()
    return ens


class Res:
    pass


def gpu_ck(model, P, y0, opts, t0=None, h0=None, shared=None, offsets=None, budgets=None,
           solves=1, solver=None, phi0=None, tangent=False, **launch):
    ens = _ens()
    n = y0.shape[-1]
    solver = ens.ENS_RKCK45 if solver is None else solver
    with ens.Ensemble(model, solver, n, offsets=offsets, tangent=tangent) as e:
        e.set_params(P)
        if shared is not None:
            for k in range(e.n_ensembles):
                e.set_shared(k, shared[k] if isinstance(shared[0], (list, tuple, np.ndarray)) else shared)
        if budgets is not None:
            for k, (ph, imp) in enumerate(budgets):
                e.set_budget(k, ph, imp)
        e.set_state(y0, t0, h0)
        if phi0 is not None:
            e.set_drive_phase(phi0)
        kw = dict(t_phase=opts.t_phase, dt0=opts.dt0, dt_min=opts.dt_min, dt_max=opts.dt_max,
                  rtol=opts.rtol, atol=opts.atol, event_tol=opts.event_tol, t_cap=opts.t_cap,
                  v_stick=opts.v_stick, n_phases=opts.n_phases, n_record=opts.n_record,
                  max_steps=opts.max_steps, max_event_iter=opts.max_event_iter)
        kw.update(launch)
        for _ in range(solves):
            e.solve(**kw)
        r = Res()
        r.y = e.read(ens.ENS_STATE)
        r.t = e.read(ens.ENS_TIME)
        r.h = e.read(ens.ENS_H)
        r.records = e.read(ens.ENS_RECORDS)
        r.stats = e.read(ens.ENS_STATS)
        r.status = e.read(ens.ENS_STATUS)
        r.phi = e.read(ens.ENS_DRIVE_PHASE) if model in (2, 6) else None
        r.launch = e.last_launch()
        r.ms = e.last_kernel_ms()
        return r


def oracle_pair(model, P, sh, y0, opts, nthreads=8):
    a = O.rkck45(model, P, sh, y0, opts, nthreads=nthreads)
    b = O.rkck45(model, P, sh, y0 * (1 + PERTURB), opts, nthreads=nthreads)
    keep = sensitivity_mask([a.y, a.records], [b.y, b.records], 1e-9, 1e-11)
    return a, keep


def check_parity(g, a, keep, min_keep=0.5, step_match=0.99):
    ok = (per_system(close(g.y, a.y, CK_RTOL, CK_ATOL))
          & per_system(close(g.records, a.records, CK_RTOL, CK_ATOL)))
    bad = keep & ~ok
    assert not bad.any(), np.nonzero(bad)[0][:10]
    assert keep.mean() >= min_keep, keep.mean()
    same_steps = (g.stats[O.ST_ACCEPTED] == a.stats[O.ST_ACCEPTED]) & \
                 (g.stats[O.ST_REJECTED] == a.stats[O.ST_REJECTED])
    assert same_steps[keep].mean() >= step_match, same_steps[keep].mean()
    assert np.array_equal(g.stats[O.ST_PHASES], a.stats[O.ST_PHASES])
    assert np.array_equal(g.status & ~O.SYS_DT_MIN, a.status & ~O.SYS_DT_MIN)


def test_quad_adaptive_matches_oracle():
    P, y0 = I.quad_linspace(1000, 0.1, 1.0)
    o = O.Opts(t_phase=0.5, n_phases=4, n_record=4)
    g = gpu_ck(0, P, y0, o)
    a = O.rkck45(O.QUAD, P, None, y0, o)
    check_parity(g, a, np.ones(1000, bool), step_match=0.999)


def test_km_grid_matches_oracle():
    P, y0 = I.km_grid(24, 24)
    o = O.Opts(n_phases=6, n_record=6)
    g = gpu_ck(2, P, y0, o)
    a, keep = oracle_pair(O.KM, P, I.KM_WATER, y0, o)
    check_parity(g, a, keep, min_keep=0.8)
    assert np.all(g.stats[O.ST_NRHS] == 6 * (g.stats[O.ST_ACCEPTED] + g.stats[O.ST_REJECTED]))


def test_prv_matches_oracle():
    P, y0 = I.prv_linspace(256)
    o = O.Opts(n_phases=40, n_record=8)
    g = gpu_ck(3, P, y0, o)
    a, keep = oracle_pair(O.PRV, P, I.PRV_DEFAULT, y0, o)
    check_parity(g, a, keep, min_keep=0.5, step_match=0.95)
    same_imp = g.stats[O.ST_IMPACTS] == a.stats[O.ST_IMPACTS]
    assert same_imp[keep].all()


def test_prv_closed_form_events_on_gpu():
    """beta = 0 valve: GPU event location agrees with the oracle tightly."""
    sh = [0.25, 10.0, 0.0, 0.8]
    P = np.array([[1.0, 2.0]])
    y0 = np.array([[10.0, 6.0], [0.0, 0.0], [10.5, 10.5]])
    o = O.Opts(n_phases=6, n_record=6, event_tol=1e-9, t_cap=1e9)
    g = gpu_ck(3, P, y0, o, shared=sh)
    a = O.rkck45(O.PRV, P, sh, y0, o)
    assert np.array_equal(g.stats[O.ST_IMPACTS], a.stats[O.ST_IMPACTS])
    assert close(g.records, a.records, 1e-9, 1e-9).all()
    assert close(g.t, a.t, 1e-9, 1e-9).all()


@pytest.mark.parametrize("scheme", [O.CASH_KARP, O.DORMAND_PRINCE])
def test_prv_seating_and_lift_off_on_gpu(scheme):
    """A valve dropped from 1e-20 lands slower than v_stick and seats; while
    seated the chamber fills until y3 = delta and the valve lifts off.  The
    seated right-hand side must hold y1 = y2 = 0 exactly and fill y3 at
    beta q, as the oracle does."""
    ens = _ens()
    solver = ens.ENS_RKDP45 if scheme == O.DORMAND_PRINCE else ens.ENS_RKCK45
    P = np.array([[1.0, 1.0, 2.0]])
    y0 = np.array([[1e-20, 1e-20, 1e-20], [0.0, 0.0, 0.0], [9.9, 9.5, 9.9]])
    # one impact: the state right after seating
    o1 = O.Opts(n_phases=2, n_record=2, max_impacts=1, scheme=scheme)
    g = gpu_ck(3, P, y0, o1, solver=solver, budgets=[(2, 1)])
    a = O.rkck45(O.PRV, P, I.PRV_DEFAULT, y0, o1)
    # the first two seat; the third (q = 2) lands fast enough to rebound
    seated = np.array([True, True, False])
    assert np.array_equal((a.status & O.SYS_SEATED) != 0, seated)
    assert np.array_equal((g.status & O.SYS_SEATED) != 0, seated)
    assert np.all(g.y[0] == 0.0) and np.all(g.y[1, seated] == 0.0)
    assert close(g.y, a.y, CK_RTOL, CK_ATOL).all()
    # two phases: seated, filled, lifted off, next local maximum
    o2 = O.Opts(n_phases=2, n_record=2, scheme=scheme)
    g = gpu_ck(3, P, y0, o2, solver=solver)
    a = O.rkck45(O.PRV, P, I.PRV_DEFAULT, y0, o2)
    assert np.array_equal(g.status, a.status)
    assert np.array_equal(g.stats[O.ST_PHASES], a.stats[O.ST_PHASES])
    assert np.array_equal(g.stats[O.ST_IMPACTS], a.stats[O.ST_IMPACTS])
    assert close(g.records, a.records, CK_RTOL, CK_ATOL).all()
    assert close(g.y, a.y, CK_RTOL, CK_ATOL).all()
    assert close(g.t, a.t, CK_RTOL, CK_ATOL).all()


@pytest.mark.parametrize("second_drive", [False, True])
def test_km_long_phase_matches_oracle(second_drive):
    """One phase of 200 acoustic cycles: the forcing angle runs to 400
    half-turns within the phase (the second drive's, at f2 = 150 kHz, to
    ~3000), so the kernel's reduction of the drive angles to the nearest
    quarter turn covers hundreds of turns.  Small drives keep the response
    near-linear (insensitive) so the oracle's own rounding of the large
    radian arguments does not matter."""
    P, y0 = I.km_grid(4, 4, pa_lo=2e3, pa_hi=2e4)
    sh = list(I.KM_WATER)
    if second_drive:
        sh[8], sh[9], sh[10] = 5e3, 150e3, 0.7
    o = O.Opts(t_phase=200.0, n_phases=1, n_record=1)
    g = gpu_ck(2, P, y0, o, shared=sh)
    a, keep = oracle_pair(O.KM, P, np.array(sh), y0, o)
    # values to the adaptive tolerance; over the thousands of steps of one
    # long phase an accept/reject decision at E ~ 1 may fall differently
    # (the oracle divides and rounds a radian argument up to ~1257), so the
    # step counts need only agree for most systems
    check_parity(g, a, keep, min_keep=0.9, step_match=0.75)
    assert np.all(g.stats[O.ST_PHASES] == 1)


def test_resume_is_bit_identical():
    P, y0 = I.km_grid(8, 8)
    full = gpu_ck(2, P, y0, O.Opts(n_phases=4, n_record=4))
    half = gpu_ck(2, P, y0, O.Opts(n_phases=2, n_record=2))
    rest = gpu_ck(2, P, half.y, O.Opts(n_phases=2, n_record=2), t0=half.t, h0=half.h)
    assert np.array_equal(full.y, rest.y) and np.array_equal(full.h, rest.h)
    assert np.array_equal(full.records[2:], rest.records)
    # consecutive solves on one handle continue from the library-owned state
    two = gpu_ck(2, P, y0, O.Opts(n_phases=2, n_record=2), solves=2)
    assert np.array_equal(two.y, full.y)


def test_permutation_invariance():
    P, y0 = I.km_grid(16, 16)
    o = O.Opts(n_phases=3, n_record=3)
    g = gpu_ck(2, P, y0, o)
    perm = np.random.default_rng(5).permutation(P.shape[1])
    gp = gpu_ck(2, P[:, perm], y0[:, perm], o)
    assert np.array_equal(gp.y, g.y[:, perm])
    assert np.array_equal(gp.records, g.records[:, :, perm])
    assert np.array_equal(gp.stats, g.stats[:, perm])


@pytest.mark.parametrize("launch", [dict(refill=64), dict(refill=7, block=64),
                                    dict(grid=1, block=64), dict(block=128, grid=3)])
def test_refill_and_grid_invariance(launch):
    P, y0 = I.prv_linspace(300)
    o = O.Opts(n_phases=12, n_record=4)
    ref = gpu_ck(3, P, y0, o)
    g = gpu_ck(3, P, y0, o, **launch)
    assert np.array_equal(g.y, ref.y) and np.array_equal(g.records, ref.records)
    assert np.array_equal(g.stats, ref.stats)


def test_graph_replays_match_eager():
    ens = _ens()
    P, y0 = I.km_grid(8, 8)
    o = dict(n_phases=2, n_record=2)
    eager = gpu_ck(2, P, y0, O.Opts(**o))
    n = P.shape[1]
    with ens.Ensemble(ens.ENS_KM, ens.ENS_RKCK45, n) as e:
        e.set_params(P)
        for rep in range(3):
            e.set_state(y0)
            e.solve(use_graph=1, **o)
            y = e.read(ens.ENS_STATE)
            rec = e.read(ens.ENS_RECORDS)
            assert np.array_equal(y, eager.y), rep
            assert np.array_equal(rec, eager.records), rep


def test_batched_sub_ensembles_equal_separate_launches():
    """Three valve ensembles with their own q draws and budgets in one
    graph-captured launch give what three separate launches give."""
    sizes, budgets = [40, 70, 100], [(30, 30), (20, 20), (10, 10)]
    Ps, ys = [], []
    for k, m in enumerate(sizes):
        P, y0 = I.prv_random(m, seed=3 + k)
        Ps.append(P)
        ys.append(y0)
    P = np.concatenate(Ps, axis=1)
    y0 = np.concatenate(ys, axis=1)
    off = np.concatenate([[0], np.cumsum(sizes)])
    o = O.Opts(n_phases=999, n_record=8)
    g = gpu_ck(3, P, y0, o, offsets=off, budgets=budgets, use_graph=1)
    for k in range(3):
        s = gpu_ck(3, Ps[k], ys[k], O.Opts(n_phases=999, n_record=8), budgets=[budgets[k]])
        sl = slice(off[k], off[k + 1])
        assert np.array_equal(g.y[:, sl], s.y)
        assert np.array_equal(g.records[:, :, sl], s.records)
        assert np.array_equal(g.stats[:, sl], s.stats)


def test_status_words():
    P = np.array([[1.2e5, 1.2e5, 1.2e5], [20e3, 20e3, 20e3]])
    y0 = np.array([[1.0, np.nan, 1.0], [0.0, 0.0, 0.0]])
    o = O.Opts(n_phases=5, n_record=1, max_steps=100)
    g = gpu_ck(2, P, y0, o)
    a = O.rkck45(O.KM, P, I.KM_WATER, y0, o)
    assert g.status[0] & O.SYS_MAX_STEPS and g.status[1] & O.SYS_NONFINITE
    assert np.array_equal(g.status, a.status)
    o2 = O.Opts(n_phases=1, n_record=1, dt_min=1e-3, dt_max=1e-3, dt0=1e-3)
    g2 = gpu_ck(2, P[:, :1], y0[:, :1], o2)
    assert g2.status[0] & O.SYS_DT_MIN


def test_zero_phases_and_empty():
    P, y0 = I.km_grid(2, 2)
    g = gpu_ck(2, P, y0, O.Opts(n_phases=0, n_record=0))
    assert np.array_equal(g.y, y0)
    assert np.all(g.stats == 0)


def test_issue_priority_does_not_change_results(monkeypatch):
    """Waves raising their issue priority by remaining work (the Keller--Miksis
    kernel does by default) reorder only the hardware's scheduling: records,
    state and counters are bit-identical with it switched off."""
    P, y0 = I.km_grid(48, 48)
    o = O.Opts(n_phases=5, n_record=5)
    ref = gpu_ck(2, P, y0, o, grid=8, block=64)
    monkeypatch.setenv("ENS_NO_PRIORITY", "1")
    g = gpu_ck(2, P, y0, o, grid=8, block=64)
    assert np.array_equal(g.y, ref.y) and np.array_equal(g.records, ref.records)
    assert np.array_equal(g.stats, ref.stats) and np.array_equal(g.status, ref.status)


def test_queue_order_does_not_change_results():
    """A permuted queue order (ens_set_order) changes which lane takes which
    system and when, never a system's arithmetic; bad orders are refused."""
    ens = _ens()
    P, y0 = I.km_grid(40, 40)
    n = P.shape[1]
    o = O.Opts(n_phases=4, n_record=4)
    ref = gpu_ck(2, P, y0, o, grid=4, block=64)
    for order in (np.arange(n)[::-1], np.random.default_rng(3).permutation(n)):
        with ens.Ensemble(ens.ENS_KM, ens.ENS_RKCK45, n) as e:
            e.set_params(P)
            e.set_state(y0)
            e.set_order(order)
            e.solve(n_phases=4, n_record=4, grid=4, block=64)
            assert np.array_equal(e.read(ens.ENS_RECORDS), ref.records)
            assert np.array_equal(e.read(ens.ENS_STATE), ref.y)
            assert np.array_equal(e.read(ens.ENS_STATS), ref.stats)
    with ens.Ensemble(ens.ENS_KM, ens.ENS_RKCK45, n) as e:
        bad = np.arange(n)
        bad[5] = 6
        with pytest.raises(ens.EnsError):
            e.set_order(bad)
        bad[5] = n
        with pytest.raises(ens.EnsError):
            e.set_order(bad)
        e.set_order(None)


def test_longest_first_continuation_is_bit_identical():
    """Pilot phases, ens_order_by_work, then the remaining phases: the same
    state, step size and records as one uninterrupted solve."""
    ens = _ens()
    P, y0 = I.km_grid(32, 32)
    n = P.shape[1]
    full = gpu_ck(2, P, y0, O.Opts(n_phases=6, n_record=3), grid=4, block=64)
    with ens.Ensemble(ens.ENS_KM, ens.ENS_RKCK45, n) as e:
        e.set_params(P)
        e.set_state(y0)
        with pytest.raises(ens.EnsError):
            e.order_by_work()           # no adaptive solve yet
        e.solve(n_phases=3, n_record=3, grid=4, block=64)
        pilot = e.read(ens.ENS_STATS)
        e.order_by_work()
        e.solve(n_phases=3, n_record=3, grid=4, block=64)
        assert np.array_equal(e.read(ens.ENS_STATE), full.y)
        assert np.array_equal(e.read(ens.ENS_H), full.h)
        assert np.array_equal(e.read(ens.ENS_RECORDS), full.records)
        rest = e.read(ens.ENS_STATS)
    # per-solve counters add up to the uninterrupted solve's
    for row in (O.ST_ACCEPTED, O.ST_REJECTED, O.ST_PHASES):
        assert np.array_equal(pilot[row] + rest[row], full.stats[row])



# ------------------------------------------------------------ Dormand--Prince
def _dp():
    return _ens().ENS_RKDP45


def test_dp_quad_matches_oracle():
    P, y0 = I.quad_linspace(1000, 0.1, 1.0)
    o = O.Opts(t_phase=0.5, n_phases=4, n_record=4, scheme=O.DORMAND_PRINCE)
    g = gpu_ck(0, P, y0, o, solver=_dp())
    a = O.rkck45(O.QUAD, P, None, y0, o)
    check_parity(g, a, np.ones(1000, bool), step_match=0.999)
    assert np.array_equal(g.stats[O.ST_NRHS], a.stats[O.ST_NRHS])


def test_dp_km_grid_matches_oracle():
    P, y0 = I.km_grid(24, 24)
    o = O.Opts(n_phases=6, n_record=6, scheme=O.DORMAND_PRINCE)
    g = gpu_ck(2, P, y0, o, solver=_dp())
    a, keep = oracle_pair(O.KM, P, I.KM_WATER, y0, o)
    check_parity(g, a, keep, min_keep=0.8)
    # first same as last: 6 per attempt plus one per phase start
    assert np.all(g.stats[O.ST_NRHS] == 6 * (g.stats[O.ST_ACCEPTED] + g.stats[O.ST_REJECTED])
                  + g.stats[O.ST_PHASES])
    same = g.stats[O.ST_NRHS] == a.stats[O.ST_NRHS]
    assert same[keep].mean() >= 0.99


def test_dp_prv_matches_oracle():
    P, y0 = I.prv_linspace(256)
    o = O.Opts(n_phases=40, n_record=8, scheme=O.DORMAND_PRINCE)
    g = gpu_ck(3, P, y0, o, solver=_dp())
    a, keep = oracle_pair(O.PRV, P, I.PRV_DEFAULT, y0, o)
    check_parity(g, a, keep, min_keep=0.5, step_match=0.95)
    assert (g.stats[O.ST_IMPACTS] == a.stats[O.ST_IMPACTS])[keep].all()
    assert (g.stats[O.ST_NRHS] == a.stats[O.ST_NRHS])[keep].mean() >= 0.95


def test_dp_prv_closed_form_events_on_gpu():
    sh = [0.25, 10.0, 0.0, 0.8]
    P = np.array([[1.0, 2.0]])
    y0 = np.array([[10.0, 6.0], [0.0, 0.0], [10.5, 10.5]])
    o = O.Opts(n_phases=6, n_record=6, event_tol=1e-9, t_cap=1e9, scheme=O.DORMAND_PRINCE)
    g = gpu_ck(3, P, y0, o, shared=sh, solver=_dp())
    a = O.rkck45(O.PRV, P, sh, y0, o)
    assert np.array_equal(g.stats[O.ST_IMPACTS], a.stats[O.ST_IMPACTS])
    assert close(g.records, a.records, 1e-9, 1e-9).all()
    assert close(g.t, a.t, 1e-9, 1e-9).all()


def test_dp_resume_and_refill_invariance():
    P, y0 = I.km_grid(8, 8)
    dp = _dp()
    full = gpu_ck(2, P, y0, O.Opts(n_phases=4, n_record=4), solver=dp)
    half = gpu_ck(2, P, y0, O.Opts(n_phases=2, n_record=2), solver=dp)
    rest = gpu_ck(2, P, half.y, O.Opts(n_phases=2, n_record=2), t0=half.t, h0=half.h, solver=dp)
    assert np.array_equal(full.y, rest.y) and np.array_equal(full.h, rest.h)
    assert np.array_equal(full.records[2:], rest.records)
    alt = gpu_ck(2, P, y0, O.Opts(n_phases=4, n_record=4), solver=dp, refill=7, block=64)
    assert np.array_equal(alt.y, full.y) and np.array_equal(alt.stats, full.stats)


@pytest.mark.parametrize("scheme", [O.CASH_KARP, O.DORMAND_PRINCE])
def test_located_maxima_match_oracle(scheme):
    """locate_max: Keller--Miksis y1max also takes the maxima located on the
    step interpolant; the steps themselves do not change."""
    ens = _ens()
    solver = ens.ENS_RKDP45 if scheme == O.DORMAND_PRINCE else ens.ENS_RKCK45
    P, y0 = I.km_grid(24, 24)
    o = O.Opts(n_phases=6, n_record=6, scheme=scheme, locate_max=1)
    g = gpu_ck(2, P, y0, o, solver=solver, locate_max=1)
    plain = gpu_ck(2, P, y0, o, solver=solver)
    a, keep = oracle_pair(O.KM, P, I.KM_WATER, y0, o)
    check_parity(g, a, keep, min_keep=0.8)
    assert (g.stats[O.ST_NRHS] == a.stats[O.ST_NRHS])[keep].mean() >= 0.99
    assert np.array_equal(g.y, plain.y) and np.array_equal(g.h, plain.h)
    assert np.array_equal(g.stats[O.ST_ACCEPTED], plain.stats[O.ST_ACCEPTED])
    assert np.all(g.records >= plain.records)      # the step points are still included
    assert (g.records > plain.records).mean() > 0.5
    with pytest.raises(ens.EnsError):
        gpu_ck(3, *I.prv_linspace(4), O.Opts(n_phases=2), solver=solver, locate_max=1)


def test_km_sweep_records_come_back_in_phase_order():
    """A pilot whose remainder is not a multiple of the ring: the records are
    rotated into phase order and equal the uninterrupted solve's."""
    from paper_2011_01740_amd import workloads as W
    P, y0 = I.km_grid(8, 8)
    a = W.km_sweep(8, 8, n_phases=20, n_record=8, pilot=5)
    b = W.km_sweep(8, 8, n_phases=20, n_record=8)
    assert np.array_equal(a.records, b.records) and np.array_equal(a.y, b.y)
    o = O.Opts(n_phases=20, n_record=20)
    ref = O.rkck45(O.KM, P, I.KM_WATER, y0, o, nthreads=8)
    ok = close(b.records, ref.records[12:], CK_RTOL, CK_ATOL)
    assert ok.mean() > 0.9


def test_spread_head_does_not_change_results():
    """Queue positions [0, spread) go to the first wave slot of each SIMD:
    only the placement changes, not a bit of any result."""
    ens = _ens()
    # valve batch: the largest-budget sub-ensemble first
    Ps, ys, off = [], [], [0]
    for m, seed in ((700, 3), (1500, 4), (2600, 5)):
        P, y0 = I.prv_random(m, seed=seed)
        Ps.append(P)
        ys.append(y0)
        off.append(off[-1] + m)
    P, y0 = np.concatenate(Ps, axis=1), np.concatenate(ys, axis=1)
    budgets = [(60, 60), (12, 12), (3, 3)]
    o = O.Opts(n_phases=60, n_record=4)
    sh = [list(I.PRV_DEFAULT)] * 3
    ref = gpu_ck(3, P, y0, o, shared=sh, offsets=off, budgets=budgets)
    for spread in (700, 1, off[-1]):
        g = gpu_ck(3, P, y0, o, shared=sh, offsets=off, budgets=budgets, spread=spread)
        # (slots of phases a short-budget system never reached hold NaN)
        assert np.array_equal(g.y, ref.y)
        assert np.array_equal(g.records, ref.records, equal_nan=True)
        assert np.array_equal(g.stats, ref.stats) and np.array_equal(g.status, ref.status)
    # Keller--Miksis, spread over a small grid and a single block
    P, y0 = I.km_grid(12, 12)
    o = O.Opts(n_phases=3, n_record=3)
    ref = gpu_ck(2, P, y0, o)
    for launch in (dict(spread=50), dict(spread=144, grid=1), dict(spread=7, block=64, refill=5)):
        g = gpu_ck(2, P, y0, o, **launch)
        assert np.array_equal(g.y, ref.y) and np.array_equal(g.records, ref.records)
    with pytest.raises(ens.EnsError):
        gpu_ck(2, P, y0, o, spread=145)
