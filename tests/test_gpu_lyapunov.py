"""GPU parity of the variational-equation mode (ens_desc.tangent): the tangent
dy rides along each system, both under error control, and at every phase
end log |dy| is recorded and dy rescaled to unit length (Benettin's
renormalisation for the largest Lyapunov exponent, inside the kernel)."""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle as O
from paper_2011_01740_amd import inputs as I
from tests.test_gpu_dual import dual_shared, km6_grid
from tests.test_gpu_rkck import _ens, check_parity, gpu_ck, oracle_pair

pytestmark = pytest.mark.gpu

LOR = [I.LORENZ_SIGMA, I.LORENZ_BETA]


def _solver(ens, scheme):
    return ens.ENS_RKDP45 if scheme == O.DORMAND_PRINCE else ens.ENS_RKCK45


def with_tangent(y0):
    D, n = y0.shape
    return np.vstack([y0, np.full((D, n), 1.0 / np.sqrt(D))])


@pytest.mark.parametrize("scheme", [O.CASH_KARP, O.DORMAND_PRINCE])
def test_km_tangent_matches_oracle(scheme):
    ens = _ens()
    P, y0 = I.km_grid(16, 16)
    Y0 = with_tangent(y0)
    o = O.Opts(n_phases=6, n_record=6, scheme=scheme, lyapunov=1)
    g = gpu_ck(2, P, Y0, o, solver=_solver(ens, scheme), tangent=True)
    a, keep = oracle_pair(O.KM, P, I.KM_WATER, Y0, o)
    check_parity(g, a, keep, min_keep=0.7)
    assert g.y.shape == (4, P.shape[1]) and g.records.shape[1] == 2
    np.testing.assert_allclose(np.linalg.norm(g.y[2:], axis=0), 1.0, rtol=1e-14)


@pytest.mark.parametrize("model,shared,P,y0", [
    (2, dual_shared(), *I.km_grid(12, 12)),
    (6, list(I.KM_WATER[:7]), *km6_grid(12)),
])
def test_dual_drive_tangent_matches_oracle(model, shared, P, y0):
    Y0 = with_tangent(y0)
    o = O.Opts(n_phases=5, n_record=5, lyapunov=1)
    g = gpu_ck(model, P, Y0, o, shared=shared, tangent=True)
    a, keep = oracle_pair(model, P, np.array(shared), Y0, o)
    check_parity(g, a, keep, min_keep=0.6)
    assert np.array_equal(g.phi, a.phi)


def test_lorenz_and_quadratic_tangent():
    # Lorenz: short horizon (parity) and the attractor's exponent
    P = np.array([[28.0, 28.0, 14.0, 0.5]])
    y0 = np.array([[1.0, -3.0, 2.0, 0.3], [1.0, 4.0, 1.0, 0.2], [20.0, 25.0, 5.0, 0.1]])
    Y0 = with_tangent(y0)
    o = O.Opts(n_phases=8, n_record=8, lyapunov=1, dt_max=0.05)
    g = gpu_ck(1, P, Y0, o, shared=LOR, tangent=True)
    a, keep = oracle_pair(O.LORENZ, P, LOR, Y0, o)
    check_parity(g, a, keep, min_keep=0.5)
    long = gpu_ck(1, P[:, :2], Y0[:, :2], O.Opts(n_phases=1000, n_record=1000, lyapunov=1,
                                                  dt_max=0.05), shared=LOR, tangent=True)
    lam = long.records[100:, 1, :].mean(axis=0)
    assert np.all(np.abs(lam - 0.9056) < 0.03), lam
    # dx/dt = x^2 - 1 from -1/2: log growth = -2 log(cosh(T + a) / cosh(a))
    q = gpu_ck(0, np.array([[1.0]]), np.array([[-0.5], [1.0]]),
               O.Opts(n_phases=5, n_record=5, rtol=1e-12, atol=1e-12, lyapunov=1),
               tangent=True)
    a_ = np.arctanh(0.5)
    T = np.arange(1, 6)
    np.testing.assert_allclose(np.cumsum(q.records[:, 1, 0]),
                               -2.0 * np.log(np.cosh(T + a_) / np.cosh(a_)), atol=1e-9)


def test_fixed_point_growth_is_the_matrix_exponential():
    o = O.Opts(n_phases=6, n_record=6, rtol=1e-12, atol=1e-12, lyapunov=1)
    g = gpu_ck(2, np.array([[0.0], [50e3]]), np.array([[1.0], [0.0], [0.6], [0.8]]), o,
               tangent=True)
    J = O.jacobian(O.KM, 0.0, [1.0, 0.0], [0.0, 50e3], I.KM_WATER)
    want = np.log(np.linalg.norm(expm(J * 6.0) @ np.array([0.6, 0.8])))
    assert g.records[:, 1, 0].sum() == pytest.approx(want, abs=1e-8)


def test_tangent_resume_and_errors():
    ens = _ens()
    P, y0 = I.km_grid(6, 6)
    Y0 = with_tangent(y0)
    full = gpu_ck(2, P, Y0, O.Opts(n_phases=4, n_record=4, lyapunov=1), tangent=True)
    two = gpu_ck(2, P, Y0, O.Opts(n_phases=2, n_record=2, lyapunov=1), tangent=True, solves=2)
    assert np.array_equal(full.y, two.y) and np.array_equal(full.records[2:], two.records)
    with pytest.raises(ens.EnsError):
        ens.Ensemble(1, ens.ENS_RK4, 4, tangent=True)
    with pytest.raises(ens.EnsError):
        ens.Ensemble(3, ens.ENS_RKCK45, 4, tangent=True)
    with pytest.raises(ens.EnsError):
        gpu_ck(2, P, Y0, O.Opts(n_phases=1), tangent=True, locate_max=1)


def with_frame(y0, K):
    """K orthonormal starting tangents per system (a fixed rotation of e_1..e_K)."""
    D, n = y0.shape
    Q = np.linalg.qr(np.arange(1.0, D * D + 1).reshape(D, D) + np.eye(D) * D * D)[0]
    return np.vstack([y0] + [np.tile(Q[:, j:j + 1], (1, n)) for j in range(K)])


@pytest.mark.parametrize("scheme", [O.CASH_KARP, O.DORMAND_PRINCE])
def test_km_spectrum_matches_oracle(scheme):
    ens = _ens()
    P, y0 = I.km_grid(12, 12)
    Y0 = with_frame(y0, 2)
    o = O.Opts(n_phases=5, n_record=5, scheme=scheme, lyapunov=2)
    g = gpu_ck(2, P, Y0, o, solver=_solver(ens, scheme), tangent=2)
    a, keep = oracle_pair(O.KM, P, I.KM_WATER, Y0, o)
    check_parity(g, a, keep, min_keep=0.7)
    assert g.records.shape[1] == 3 and g.y.shape[0] == 6
    # the frame is orthonormal after the last renormalisation (one Gram--Schmidt
    # pass on tangents that a phase has turned nearly parallel: ~1e-10)
    v1, v2 = g.y[2:4], g.y[4:6]
    np.testing.assert_allclose((v1 * v2).sum(axis=0), 0.0, atol=1e-8)
    np.testing.assert_allclose(np.linalg.norm(v2, axis=0), 1.0, rtol=1e-14)


def test_dual_and_km6_spectrum_match_oracle():
    for model, shared, (P, y0) in ((2, dual_shared(), I.km_grid(10, 10)),
                                   (6, list(I.KM_WATER[:7]), km6_grid(10))):
        Y0 = with_frame(y0, 2)
        o = O.Opts(n_phases=4, n_record=4, lyapunov=2)
        g = gpu_ck(model, P, Y0, o, shared=shared, tangent=2)
        a, keep = oracle_pair(model, P, np.array(shared), Y0, o)
        check_parity(g, a, keep, min_keep=0.6)


def test_lorenz_spectrum_on_gpu():
    P = np.array([[28.0, 28.0, 14.0, 0.5]])
    y0 = np.array([[1.0, -3.0, 2.0, 0.3], [1.0, 4.0, 1.0, 0.2], [20.0, 25.0, 5.0, 0.1]])
    for K in (2, 3):
        Y0 = with_frame(y0, K)
        o = O.Opts(n_phases=6, n_record=6, lyapunov=K, dt_max=0.05)
        g = gpu_ck(1, P, Y0, o, shared=LOR, tangent=K)
        a, keep = oracle_pair(O.LORENZ, P, LOR, Y0, o)
        check_parity(g, a, keep, min_keep=0.5)
    long = gpu_ck(1, P[:, :2], with_frame(y0[:, :2], 3),
                  O.Opts(n_phases=400, n_record=400, lyapunov=3, dt_max=0.05),
                  shared=LOR, tangent=3)
    per_phase = long.records[:, 1:, :].sum(axis=1)
    tr = -(10.0 + 1.0 + 8.0 / 3.0)
    assert np.abs(per_phase - tr).max() < 1e-3 * abs(tr)
    lam = long.records[50:, 1:, :].mean(axis=0)
    assert np.all(np.abs(lam[0] - 0.9056) < 0.05) and np.all(np.abs(lam[1]) < 0.03), lam
    ens = _ens()
    with pytest.raises(ens.EnsError):
        ens.Ensemble(0, ens.ENS_RKCK45, 4, tangent=2)   # more tangents than D
