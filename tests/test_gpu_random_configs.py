"""Seeded random configurations of the adaptive solvers against the oracle:
model, scheme, size, tolerances, phase length, ring length (also longer than
the run), step cap, located maxima, tangent, second drive, and launch shape
(block, refill threshold, grid, spread head), each drawn per case.  Parity is checked on
the systems whose oracle result is insensitive to a 1e-13 perturbation of
the initial state; on those, state, records, status, phases and (for >= 95%)
step counts must agree."""
import numpy as np
import pytest

import oracle as O
from paper_2011_01740_amd import inputs as I
from tests.parity import CK_ATOL, CK_RTOL, close, per_system
from tests.test_gpu_rkck import _ens, gpu_ck, oracle_pair

pytestmark = pytest.mark.gpu

N_CASES = 24


def draw(seed):
    rng = np.random.default_rng(1000 + seed)
    model = int(rng.choice([0, 1, 2, 3, 6]))
    n = int(rng.integers(1, 2000))
    c = dict(model=model, n=n, scheme=int(rng.integers(0, 2)))
    tol = float(rng.choice([1e-6, 1e-8, 1e-10]))
    o = dict(rtol=tol, atol=tol, n_phases=int(rng.integers(0, 6)),
             n_record=int(rng.integers(0, 8)), dt_max=float(rng.choice([0.05, 0.1, 0.2])),
             max_steps=int(rng.choice([0, 0, 400])))
    if model != 3:
        o["t_phase"] = float(rng.choice([1.0, 0.37]))
        c["tangent"] = bool(rng.random() < 0.3)
    if model in (2, 6) and not c.get("tangent"):
        o["locate_max"] = int(rng.random() < 0.3)
    c["launch"] = dict(block=int(rng.choice([64, 128, 192, 256])),
                       refill=int(rng.choice([1, 7, 64])), grid=int(rng.choice([0, 1, 3])),
                       spread=int(rng.choice([0, n // 3, n])))
    # inputs
    if model == 0:
        P, y0 = I.quad_linspace(n, 0.1, 1.0)
        sh = None
    elif model == 1:
        P, y0 = I.lorenz_random(n, seed=seed, hi=15.0)
        sh = [I.LORENZ_SIGMA, I.LORENZ_BETA]
    elif model == 3:
        P, y0 = I.prv_random(n, seed=seed)
        sh = list(I.PRV_DEFAULT)
    else:
        pa = rng.uniform(0.2e5, 1.2e5, n)
        f = np.exp(rng.uniform(np.log(20e3), np.log(1e6), n))
        P = np.vstack([pa, f])
        y0 = np.vstack([np.ones(n), np.zeros(n)])
        sh = list(I.KM_WATER)
        if rng.random() < 0.4:                     # second drive
            sh[8], sh[9], sh[10] = 0.4e5, float(rng.uniform(50e3, 400e3)), 0.3
        if model == 6:
            P = np.vstack([P, np.tile(np.array([[sh[8]], [sh[9]], [sh[10]], [sh[7]]]), (1, n))])
            P[2] = rng.uniform(0.0, 0.6e5, n)
            sh = sh[:7]
    if c.get("tangent"):
        y0 = np.vstack([y0, np.full_like(y0, 1.0 / np.sqrt(y0.shape[0]))])
        o["lyapunov"] = 1
    return c, o, P, y0, sh


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_configuration_matches_oracle(seed):
    ens = _ens()
    c, o, P, y0, sh = draw(seed)
    print("case", seed, c, o, flush=True)
    opts = O.Opts(scheme=c["scheme"], **o)
    solver = ens.ENS_RKDP45 if c["scheme"] == O.DORMAND_PRINCE else ens.ENS_RKCK45
    g = gpu_ck(c["model"], P, y0, opts, shared=sh, solver=solver,
               tangent=c.get("tangent", False), locate_max=o.get("locate_max", 0),
               **c["launch"])
    a, keep = oracle_pair(c["model"], P, None if sh is None else np.array(sh), y0, opts)
    ok = per_system(close(g.y, a.y, CK_RTOL, CK_ATOL))
    if opts.n_record > 0:
        ok &= per_system(close(g.records, a.records, CK_RTOL, CK_ATOL))
    assert not (keep & ~ok).any(), np.nonzero(keep & ~ok)[0][:10]
    assert np.array_equal(g.status[keep] & ~O.SYS_DT_MIN, a.status[keep] & ~O.SYS_DT_MIN)
    assert np.array_equal(g.stats[O.ST_PHASES][keep], a.stats[O.ST_PHASES][keep])
    same = (g.stats[O.ST_ACCEPTED] == a.stats[O.ST_ACCEPTED]) & \
           (g.stats[O.ST_REJECTED] == a.stats[O.ST_REJECTED])
    if keep.any():
        assert same[keep].mean() >= 0.95, same[keep].mean()
    # most systems of every case are in the parity set
    assert keep.mean() >= 0.3, keep.mean()
