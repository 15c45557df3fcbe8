"""The library autotuner: it restores the state it started from, its choice is
one of the candidates, and later solves with automatic launch fields use it."""
import numpy as np
import pytest

from paper_2011_01740_amd import inputs as I

pytestmark = pytest.mark.gpu


def _ens():
    import torch
    from paper_2011_01740_amd import ens
    assert torch.cuda.is_available()
    return ens


def test_rk4_tune_restores_state_and_is_used():
    ens = _ens()
    P, y0 = I.lorenz_random(5000, seed=21)
    with ens.Ensemble(ens.ENS_LORENZ, ens.ENS_RK4, 5000) as e:
        e.set_params(P)
        e.set_state(y0)
        best, ms = e.tune(dt=0.01, n_steps=400)
        assert best.block in (64, 128, 256, 512, 1024) and best.spl in (1, 2, 4) and ms > 0
        assert np.array_equal(e.read(ens.ENS_STATE), y0)
        e.solve(dt=0.01, n_steps=400)
        launch = e.last_launch()
        assert (launch["block"], launch["spl"]) == (best.block, best.spl)
        y = e.read(ens.ENS_STATE)
    with ens.Ensemble(ens.ENS_LORENZ, ens.ENS_RK4, 5000) as e:
        e.set_params(P)
        e.set_state(y0)
        e.solve(dt=0.01, n_steps=400, block=256, spl=1)
        assert np.array_equal(e.read(ens.ENS_STATE), y)


def test_adaptive_tune_restores_state():
    ens = _ens()
    P, y0 = I.prv_linspace(700)
    with ens.Ensemble(ens.ENS_PRV, ens.ENS_RKCK45, 700) as e:
        e.set_params(P)
        e.set_state(y0)
        best, ms = e.tune(n_phases=30, n_record=4)
        assert best.block in (64, 128, 256) and best.refill in (1, 8, 32, 64)
        assert np.array_equal(e.read(ens.ENS_STATE), y0)
        e.solve(n_phases=30, n_record=4)
        assert e.last_launch()["refill"] == best.refill
        y = e.read(ens.ENS_STATE)
        st = e.read(ens.ENS_STATS)
    with ens.Ensemble(ens.ENS_PRV, ens.ENS_RKCK45, 700) as e:
        e.set_params(P)
        e.set_state(y0)
        e.solve(n_phases=30, n_record=4, block=64, refill=64)
        assert np.array_equal(e.read(ens.ENS_STATE), y)
        assert np.array_equal(e.read(ens.ENS_STATS), st)
