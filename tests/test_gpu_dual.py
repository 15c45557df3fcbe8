"""GPU parity of the dual-frequency Keller--Miksis drive (Sec. 4.2: p_inf
carries P_A1 sin(omega1 t) + P_A2 sin(omega2 t + theta)) against the oracle,
through the C ABI.  The second drive runs on the absolute time, so its phase
is part of each system's state (ENS_DRIVE_PHASE) and is carried across the
integration phases and across solves."""
import numpy as np
import pytest

import oracle as O
from paper_2011_01740_amd import inputs as I
from tests.test_gpu_rkck import _ens, check_parity, gpu_ck, oracle_pair

pytestmark = pytest.mark.gpu


def dual_shared(pa2=0.5e5, f2=150e3, theta=0.7):
    sh = list(I.KM_WATER)
    sh[8], sh[9], sh[10] = pa2, f2, theta
    return sh


def _solver(ens, scheme):
    return ens.ENS_RKDP45 if scheme == O.DORMAND_PRINCE else ens.ENS_RKCK45


# dt_max 0.1 runs the fast arithmetic (fifth root, angle addition for the
# first drive), 0.2 the general one (exp/log, sincospi for both drives)
@pytest.mark.parametrize("scheme,locate,dt_max", [
    (O.CASH_KARP, 0, 0.1), (O.DORMAND_PRINCE, 0, 0.1), (O.CASH_KARP, 1, 0.1),
    (O.DORMAND_PRINCE, 1, 0.1), (O.CASH_KARP, 0, 0.2), (O.DORMAND_PRINCE, 1, 0.2)])
def test_dual_km_grid_matches_oracle(scheme, locate, dt_max):
    ens = _ens()
    sh = dual_shared()
    # f1 over [20 kHz, 1 MHz]: C11 = f2 / f1 from 7.5 down to 0.15, mostly
    # not an integer, so the second drive's phase moves from phase to phase
    P, y0 = I.km_grid(20, 20)
    o = O.Opts(n_phases=6, n_record=6, scheme=scheme, locate_max=locate, dt_max=dt_max)
    g = gpu_ck(2, P, y0, o, shared=sh, solver=_solver(ens, scheme), locate_max=locate)
    a, keep = oracle_pair(O.KM, P, np.array(sh), y0, o)
    check_parity(g, a, keep, min_keep=0.7)
    # the drive's phase: same roundings on both sides (a multiply and an add,
    # then the reduction modulo 1)
    assert np.array_equal(g.phi, a.phi)
    assert np.all((g.phi >= 0.0) & (g.phi < 1.0))
    assert np.mean(g.phi != 0.0) > 0.9


def test_dual_km_resume_and_consecutive_solves_are_bit_identical():
    sh = dual_shared()
    P, y0 = I.km_grid(8, 8)
    full = gpu_ck(2, P, y0, O.Opts(n_phases=4, n_record=4), shared=sh)
    half = gpu_ck(2, P, y0, O.Opts(n_phases=2, n_record=2), shared=sh)
    rest = gpu_ck(2, P, half.y, O.Opts(n_phases=2, n_record=2), t0=half.t, h0=half.h,
                  phi0=half.phi, shared=sh)
    assert np.array_equal(full.y, rest.y) and np.array_equal(full.h, rest.h)
    assert np.array_equal(full.phi, rest.phi)
    assert np.array_equal(full.records[2:], rest.records)
    # the library keeps the drive's phase between solves on one handle
    two = gpu_ck(2, P, y0, O.Opts(n_phases=2, n_record=2), shared=sh, solves=2)
    assert np.array_equal(two.y, full.y) and np.array_equal(two.phi, full.phi)
    # the wrong continuation (drive restarted) differs: the phase matters
    cold = gpu_ck(2, P, half.y, O.Opts(n_phases=2, n_record=2), t0=half.t, h0=half.h,
                  shared=sh)
    assert not np.array_equal(cold.y, full.y)


def test_dual_and_single_drive_sub_ensembles_in_one_launch():
    """A single-frequency sub-ensemble beside a dual one runs on the variant
    that carries the second drive; both match the oracle."""
    P, y0 = I.km_grid(12, 12)
    n = P.shape[1]
    off = [0, n // 2, n]
    shs = [list(I.KM_WATER), dual_shared(pa2=0.8e5, f2=310e3, theta=-1.1)]
    o = O.Opts(n_phases=4, n_record=4)
    g = gpu_ck(2, P, y0, o, shared=shs, offsets=off)
    for k in range(2):
        sl = slice(off[k], off[k + 1])
        a, keep = oracle_pair(O.KM, P[:, sl], np.array(shs[k]), y0[:, sl], o)
        sub = type(g)()
        sub.y, sub.records, sub.stats, sub.status = (g.y[:, sl], g.records[:, :, sl],
                                                     g.stats[:, sl], g.status[sl])
        check_parity(sub, a, keep, min_keep=0.7)
        assert np.array_equal(g.phi[sl], a.phi)


def test_drive_phase_field_and_errors():
    ens = _ens()
    P, y0 = I.km_grid(2, 2)
    with ens.Ensemble(2, ens.ENS_RKCK45, 4) as e:
        e.set_params(P)
        with pytest.raises(ens.EnsError):
            e.set_drive_phase(np.zeros(4))          # before the state
        e.set_state(y0)
        assert np.array_equal(e.read(ens.ENS_DRIVE_PHASE), np.zeros(4))
        e.set_drive_phase(np.full(4, 0.25))
        assert np.array_equal(e.read(ens.ENS_DRIVE_PHASE), np.full(4, 0.25))
        e.set_state(y0)                             # a new state restarts the drive
        assert np.array_equal(e.read(ens.ENS_DRIVE_PHASE), np.zeros(4))
        with pytest.raises(ValueError):
            e.set_drive_phase(np.zeros(3))
    Pp, yp = I.prv_linspace(4)
    with ens.Ensemble(3, ens.ENS_RKCK45, 4) as e:
        e.set_params(Pp)
        e.set_state(yp)
        with pytest.raises(ens.EnsError):
            e.set_drive_phase(np.zeros(4))
        with pytest.raises(ens.EnsError):
            e.read(ens.ENS_DRIVE_PHASE)


def km6_grid(n_side, seed=3):
    """All six control parameters per system: (P_A1, f1) on the usual grid,
    (P_A2, f2, theta, R_E) drawn per system."""
    P, y0 = I.km_grid(n_side, n_side)
    n = P.shape[1]
    rng = np.random.default_rng(seed)
    extra = np.vstack([rng.uniform(0.0, 0.8e5, n),
                       np.exp(rng.uniform(np.log(50e3), np.log(400e3), n)),
                       rng.uniform(-np.pi, np.pi, n),
                       rng.uniform(5e-6, 15e-6, n)])
    return np.vstack([P, extra]), y0


@pytest.mark.parametrize("scheme,dt_max", [(O.CASH_KARP, 0.1), (O.DORMAND_PRINCE, 0.1),
                                           (O.CASH_KARP, 0.2)])
def test_km6_per_system_sweep_matches_oracle(scheme, dt_max):
    ens = _ens()
    P6, y0 = km6_grid(16)
    fluid = list(I.KM_WATER[:7])
    o = O.Opts(n_phases=5, n_record=5, scheme=scheme, dt_max=dt_max)
    g = gpu_ck(6, P6, y0, o, shared=fluid, solver=_solver(ens, scheme))
    a, keep = oracle_pair(O.KM6, P6, np.array(fluid), y0, o)
    check_parity(g, a, keep, min_keep=0.7)
    assert np.array_equal(g.phi, a.phi)


def test_km6_equals_km_with_the_same_values():
    """Per-system second-drive parameters that happen to be equal give the
    same bits as the shared ones."""
    sh = dual_shared()
    P, y0 = I.km_grid(10, 10)
    n = P.shape[1]
    P6 = np.vstack([P, np.tile(np.array([sh[8], sh[9], sh[10], sh[7]]).reshape(4, 1), (1, n))])
    o = O.Opts(n_phases=4, n_record=4)
    a = gpu_ck(2, P, y0, o, shared=sh)
    b = gpu_ck(6, P6, y0, o, shared=sh[:7])
    assert np.array_equal(a.y, b.y) and np.array_equal(a.records, b.records)
    assert np.array_equal(a.stats, b.stats) and np.array_equal(a.phi, b.phi)
