"""Parity at the workloads' full sizes, in the launches the workload runners use,
on a seeded sample of systems the oracle integrates one by one."""
import numpy as np
import pytest

import oracle as O
from paper_2011_01740_amd import inputs as I
from tests.parity import CK_ATOL, CK_RTOL, PERTURB, close, per_system, sensitivity_mask

pytestmark = pytest.mark.gpu
THREADS = 16


def _sample(n, k, seed, extra=()):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.asarray(extra, dtype=np.int64), rng.integers(0, n, k)]))


@pytest.mark.parametrize("scheme", [O.CASH_KARP, O.DORMAND_PRINCE])
def test_keller_miksis_512x512_1024_cycles(scheme):
    """2^18 systems, every one of the 1024 cycle maxima recorded (both
    adaptive schemes)."""
    from paper_2011_01740_amd import ens
    from paper_2011_01740_amd import workloads as W
    solver = ens.ENS_RKDP45 if scheme == O.DORMAND_PRINCE else ens.ENS_RKCK45
    r = W.km_sweep(512, 512, n_phases=1024, solver=solver)
    n = 512 * 512
    assert r.records.shape == (1024, 1, n)
    assert np.all((r.status & ~O.SYS_DT_MIN) == 0)
    assert np.all(r.stats[O.ST_PHASES] == 1024)
    P, y0 = I.km_grid(512, 512)
    idx = _sample(n, 40, 31, extra=[0, 511, n - 512, n - 1, 300 * 512 + 17])
    o = O.Opts(n_phases=1024, n_record=1024, scheme=scheme)
    a = O.rkck45(O.KM, P[:, idx], I.KM_WATER, y0[:, idx], o, nthreads=THREADS)
    b = O.rkck45(O.KM, P[:, idx], I.KM_WATER, y0[:, idx] * (1 + PERTURB), o, nthreads=THREADS)
    keep = sensitivity_mask([a.y, a.records], [b.y, b.records], 1e-9, 1e-11)
    ok = (per_system(close(r.y[:, idx], a.y, CK_RTOL, CK_ATOL))
          & per_system(close(r.records[:, :, idx], a.records, CK_RTOL, CK_ATOL)))
    assert not (keep & ~ok).any(), idx[keep & ~ok]
    assert keep.mean() >= 0.5, keep.mean()
    # non-parity-set systems still agree on what the screening uses: the label
    lab_g = r.records[-64:, 0, idx].max(axis=0) >= 2
    lab_o = a.records[-64:, 0, :].max(axis=0) >= 2
    assert (lab_g == lab_o).mean() >= 0.9


def test_relief_valve_three_ensembles_one_graph_launch():
    """2^15 + 2^16 + 2^17 systems with their own seeds and budgets (phases or
    impacts, whichever first) in one graph-captured persistent launch.  The
    budgets are the workload's divided by 100 (the full-budget launch runs
    minutes: its 2^15 long systems run serially, see bench.py --case prv)."""
    from paper_2011_01740_amd import workloads as W
    ensm = tuple((m, K // 100, s) for m, K, s in W.PRV_ENSEMBLES)
    r = W.prv_batched(ensm, n_record=32)
    P, y0, off = W.prv_inputs(ensm)
    # terminal / informative bits only; EVENT_ITER (secant retries capped, e.g. at
    # near-grazing impacts) stays rare
    allowed = O.SYS_DT_MIN | O.SYS_SETTLED | O.SYS_EVENT_ITER
    assert np.all((r.status & ~allowed) == 0)
    assert ((r.status & O.SYS_EVENT_ITER) != 0).mean() < 0.01
    for k, (m, K, seed) in enumerate(ensm):
        sl = slice(off[k], off[k + 1])
        ph, imp = r.stats[O.ST_PHASES, sl], r.stats[O.ST_IMPACTS, sl]
        settled = (r.status[sl] & O.SYS_SETTLED) != 0
        # every system stopped at its budget (or settled)
        assert np.all((ph == K) | (imp == K) | settled)
        idx = off[k] + _sample(m, 12, 40 + k, extra=[0, m - 1])
        o = O.Opts(n_phases=K, n_record=32, max_impacts=K)
        a = O.rkck45(O.PRV, P[:, idx], I.PRV_DEFAULT, y0[:, idx], o, nthreads=THREADS)
        b = O.rkck45(O.PRV, P[:, idx], I.PRV_DEFAULT, y0[:, idx] * (1 + PERTURB), o,
                     nthreads=THREADS)
        keep = sensitivity_mask([a.y, a.records], [b.y, b.records], 1e-9, 1e-11)
        ok = (per_system(close(r.y[:, idx], a.y, CK_RTOL, CK_ATOL))
              & per_system(close(r.records[:, :, idx], a.records, CK_RTOL, CK_ATOL)))
        assert not (keep & ~ok).any(), (k, idx[keep & ~ok])
        assert np.array_equal(r.stats[O.ST_IMPACTS, idx][keep], a.stats[O.ST_IMPACTS][keep])
        assert np.array_equal(r.status[idx][keep] & ~O.SYS_DT_MIN, a.status[keep] & ~O.SYS_DT_MIN)


def test_relief_valve_full_budgets_one_graph_launch():
    """The valve workload as specified: 2^15 systems with budget 10^5, 2^16
    with 10^4 and 2^17 with 10^3 (Poincare phases or impacts, whichever
    first), in one graph-captured persistent launch (~10^12 attempted steps).
    The oracle integrates a seeded sample of each ensemble, the system with
    the most attempted steps included, with the same budgets; systems its own
    1e-13 perturbation moves are checked for invariants only."""
    from paper_2011_01740_amd import workloads as W
    ensm = W.PRV_ENSEMBLES
    r = W.prv_batched(ensm, n_record=32)
    P, y0, off = W.prv_inputs(ensm)
    allowed = O.SYS_DT_MIN | O.SYS_SETTLED | O.SYS_EVENT_ITER
    assert np.all((r.status & ~allowed) == 0)
    assert ((r.status & O.SYS_EVENT_ITER) != 0).mean() < 0.01
    att = r.stats[O.ST_ACCEPTED] + r.stats[O.ST_REJECTED] + r.stats[O.ST_EVRETRY]
    assert att.sum() > 5e11
    for k, (m, K, seed) in enumerate(ensm):
        sl = slice(off[k], off[k + 1])
        ph, imp = r.stats[O.ST_PHASES, sl], r.stats[O.ST_IMPACTS, sl]
        settled = (r.status[sl] & O.SYS_SETTLED) != 0
        assert np.all((ph == K) | (imp == K) | settled)
        # impacting valves (q up to ~7.5, Sec. 4.3) reach the impact budget,
        # the others the phase budget or settle
        longest = int(np.argmax(att[sl]))
        idx = off[k] + _sample(m, 10, 60 + k, extra=[0, m - 1, longest])
        o = O.Opts(n_phases=K, n_record=32, max_impacts=K)
        a = O.rkck45(O.PRV, P[:, idx], I.PRV_DEFAULT, y0[:, idx], o, nthreads=THREADS)
        b = O.rkck45(O.PRV, P[:, idx], I.PRV_DEFAULT, y0[:, idx] * (1 + PERTURB), o,
                     nthreads=THREADS)
        keep = sensitivity_mask([a.y, a.records], [b.y, b.records], 1e-9, 1e-11)
        ok = (per_system(close(r.y[:, idx], a.y, CK_RTOL, CK_ATOL))
              & per_system(close(r.records[:, :, idx], a.records, CK_RTOL, CK_ATOL)))
        assert not (keep & ~ok).any(), (k, idx[keep & ~ok])
        # in the parity set every count and status bit agrees; outside it the
        # budget that ended a system is reached on both sides
        for row in (O.ST_PHASES, O.ST_IMPACTS):
            assert np.array_equal(r.stats[row, idx][keep], a.stats[row][keep])
        assert np.array_equal(r.status[idx][keep] & ~O.SYS_DT_MIN,
                              a.status[keep] & ~O.SYS_DT_MIN)
        hit_imp = a.stats[O.ST_IMPACTS] == K
        assert np.all(r.stats[O.ST_IMPACTS, idx][hit_imp] == K)
        hit_ph = (a.stats[O.ST_PHASES] == K) & ~hit_imp
        assert np.all((r.stats[O.ST_PHASES, idx][hit_ph] == K)
                      | (r.stats[O.ST_IMPACTS, idx][hit_ph] == K))
        # the rest: bounded, finite, minimum at the seat (0) or above it
        assert np.isfinite(r.records[:, :, idx]).all()
        assert (r.records[:, 1, idx] >= 0.0).all()
