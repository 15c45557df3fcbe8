"""The usage example of the README, run as written (smaller sizes), with its
outputs checked for shape and against the oracle on a few systems."""
import numpy as np
import pytest

import oracle as O
from paper_2011_01740_amd import inputs as I
from tests.parity import CK_ATOL, CK_RTOL, PERTURB, close, per_system, sensitivity_mask

pytestmark = pytest.mark.gpu


def test_usage_example():
    from paper_2011_01740_amd import ens

    P, y0 = I.lorenz_random(1 << 12, seed=1)
    with ens.Ensemble(ens.ENS_LORENZ, ens.ENS_RK4, P.shape[1]) as e:
        e.set_params(P)
        e.set_state(y0)
        e.solve(dt=0.01, n_steps=1000)
        y = e.read(ens.ENS_STATE)
        xmax = e.read(ens.ENS_ACC)
    assert y.shape == (3, 1 << 12) and xmax.shape == (1 << 12,)
    # rho < 13.9 in the first systems of the seeded draw: non-chaotic, so the
    # textbook oracle agrees to the fixed-step tolerance
    idx = np.flatnonzero(P[0] < 13.0)[:8]
    oy, om = O.rk4(O.LORENZ, P[:, idx], [I.LORENZ_SIGMA, I.LORENZ_BETA], y0[:, idx], 0.01, 1000)
    assert np.all(np.abs(y[:, idx] - oy) <= 1e-10 * np.abs(oy) + 1e-12)
    assert np.all(np.abs(xmax[idx] - om) <= 1e-10 * np.abs(om) + 1e-12)

    P, y0 = I.km_grid(8, 8)
    with ens.Ensemble(ens.ENS_KM, ens.ENS_RKCK45, P.shape[1]) as e:
        e.set_params(P)
        e.set_state(y0)
        e.solve(n_phases=16, n_record=8, rtol=1e-10, atol=1e-10)
        rec = e.read(ens.ENS_RECORDS)
        stats = e.read(ens.ENS_STATS)
        status = e.read(ens.ENS_STATUS)
    assert rec.shape == (8, 1, 64) and stats.shape == (ens.ENS_NSTAT, 64)
    assert np.all((status & ~ens.ENS_SYS_DT_MIN) == 0)
    assert np.all(stats[ens.ENS_ST_PHASES] == 16)
    # the records of every tenth system against the oracle (insensitive ones)
    idx = np.arange(0, 64, 10)
    o = O.Opts(n_phases=16, n_record=8)
    a = O.rkck45(O.KM, P[:, idx], I.KM_WATER, y0[:, idx], o)
    b = O.rkck45(O.KM, P[:, idx], I.KM_WATER, y0[:, idx] * (1 + PERTURB), o)
    keep = sensitivity_mask([a.records], [b.records], 1e-9, 1e-11)
    ok = per_system(close(rec[:, :, idx], a.records, CK_RTOL, CK_ATOL))
    assert keep.any() and not (keep & ~ok).any()
