"""Pins of the oracle's Runge--Kutta schemes against mathematics.

* Cash--Karp 5(4): the coefficients the oracle uses must satisfy every
  order condition of order <= 5 (fifth-order weights) and <= 4 (embedded
  weights), checked in exact rational arithmetic, while the embedded weights
  must fail order 5.
* One step on the linear test equation y' = lambda y multiplies by the
  scheme's stability polynomial (classic RK4 and both Cash--Karp solutions).
* Observed convergence orders on a nonlinear problem with a closed form
  (the introductory example of Sec. 3, dx/dt = x^2 - p).
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_2011_01740_amd import inputs as I


def _rat(x):
    f = Fraction(x).limit_denominator(1 << 20)
    # the double must be the correctly rounded value of that small rational
    assert float(f) == x, (x, f)
    return f


def _tab():
    a, b5, b4, c = O.rkck_tableau()
    A = [[_rat(v) for v in row] for row in a]
    return A, [_rat(v) for v in b5], [_rat(v) for v in b4], [_rat(v) for v in c]


def _order_conditions(A, b, c):
    """Elementary-weight conditions of all 17 rooted trees with <= 5 nodes."""
    s = len(b)

    def Av(v):
        return [sum(A[i][j] * v[j] for j in range(s)) for i in range(s)]

    def dot(u, v):
        return sum(x * y for x, y in zip(u, v))

    def mul(u, v):
        return [x * y for x, y in zip(u, v)]

    one = [Fraction(1)] * s
    c2 = mul(c, c)
    c3 = mul(c2, c)
    c4 = mul(c3, c)
    Ac = Av(c)
    Ac2 = Av(c2)
    AAc = Av(Ac)
    conds = {
        1: [(dot(b, one), Fraction(1))],
        2: [(dot(b, c), Fraction(1, 2))],
        3: [(dot(b, c2), Fraction(1, 3)), (dot(b, Ac), Fraction(1, 6))],
        4: [(dot(b, c3), Fraction(1, 4)), (dot(b, mul(c, Ac)), Fraction(1, 8)),
            (dot(b, Ac2), Fraction(1, 12)), (dot(b, AAc), Fraction(1, 24))],
        5: [(dot(b, c4), Fraction(1, 5)), (dot(b, mul(c2, Ac)), Fraction(1, 10)),
            (dot(b, mul(c, Ac2)), Fraction(1, 15)), (dot(b, mul(c, AAc)), Fraction(1, 30)),
            (dot(b, mul(Ac, Ac)), Fraction(1, 20)), (dot(b, Av(c3)), Fraction(1, 20)),
            (dot(b, Av(mul(c, Ac))), Fraction(1, 40)), (dot(b, Av(Ac2)), Fraction(1, 60)),
            (dot(b, Av(AAc)), Fraction(1, 120))],
    }
    return conds


def test_cash_karp_row_sums_equal_nodes():
    A, _, _, c = _tab()
    for i in range(6):
        assert sum(A[i]) == c[i]
        assert all(A[i][j] == 0 for j in range(i, 6))  # explicit scheme


def test_cash_karp_fifth_order_weights_satisfy_all_17_conditions():
    A, b5, _, c = _tab()
    conds = _order_conditions(A, b5, c)
    n = 0
    for order, lst in conds.items():
        for got, want in lst:
            assert got == want, (order, got, want)
            n += 1
    assert n == 17


def test_cash_karp_embedded_weights_are_order_four_exactly():
    A, _, b4, c = _tab()
    conds = _order_conditions(A, b4, c)
    for order in (1, 2, 3, 4):
        for got, want in conds[order]:
            assert got == want, (order, got, want)
    assert all(got != want for got, want in conds[5])


def _lorenz_z_decay(z0, h, step):
    """Lorenz with x = y = 0 reduces to z' = -beta z, a linear test equation."""
    sh = np.array([I.LORENZ_SIGMA, I.LORENZ_BETA])
    return step(np.array([0.0, 0.0, z0]), sh, h)


@pytest.mark.parametrize("h", [0.01, 0.1, 0.3, 0.7])
def test_rk4_step_is_stability_polynomial(h):
    # R(w) = 1 + w + w^2/2 + w^3/6 + w^4/24 for classic RK4
    def step(y0, sh, h):
        y, _ = O.rk4(O.LORENZ, np.array([[0.0]]), sh, y0.reshape(3, 1), h, 1)
        return y[:, 0]

    z0 = 1.7
    y = _lorenz_z_decay(z0, h, step)
    w = -I.LORENZ_BETA * h
    R = 1 + w + w**2 / 2 + w**3 / 6 + w**4 / 24
    assert y[0] == 0.0 and y[1] == 0.0
    assert y[2] == pytest.approx(z0 * R, rel=4e-15, abs=1e-300)


@pytest.mark.parametrize("h", [0.01, 0.1, 0.3, 0.7])
def test_cash_karp_step_is_stability_polynomial(h):
    sh = np.array([I.LORENZ_SIGMA, I.LORENZ_BETA])
    z0 = 1.3
    y5, y4 = O.rkck_step(O.LORENZ, 0.0, np.array([0.0, 0.0, z0]), np.array([0.0]), sh, h)
    w = -I.LORENZ_BETA * h
    base = 1 + w + w**2 / 2 + w**3 / 6 + w**4 / 24
    R5 = base + w**5 / 120 + w**6 / 800
    R4 = base + 10517 / 1228800 * w**5 + 1771 / 1638400 * w**6
    assert y5[2] == pytest.approx(z0 * R5, rel=4e-15)
    assert y4[2] == pytest.approx(z0 * R4, rel=1e-14)


def _quad_exact(p, t, x0=-0.5):
    """Closed form of dx/dt = x^2 - p (Sec. 3) from x(0) = x0 < 0."""
    s = np.sqrt(p)
    z = -x0 / s
    if z < 1:
        return -s * np.tanh(s * t + np.arctanh(z))
    return -s / np.tanh(s * t + 0.5 * np.log((z + 1) / (z - 1)))


def test_rk4_global_order_four_on_closed_form():
    p = np.array([[0.7]])
    y0 = np.array([[-0.5]])
    T = 2.0
    errs = []
    for k in range(4):
        n = 50 * 2**k
        y, _ = O.rk4(O.QUAD, p, None, y0, T / n, n)
        errs.append(abs(y[0, 0] - _quad_exact(0.7, T)))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for r in ratios:
        assert 14.0 < r < 18.0, ratios


def test_cash_karp_fixed_step_orders_five_and_four():
    p = np.array([0.7])
    T = 2.0
    e5, e4 = [], []
    for k in range(4):
        n = 40 * 2**k
        h = T / n
        x5 = np.array([-0.5])
        x4 = np.array([-0.5])
        for j in range(n):
            x5, _ = O.rkck_step(O.QUAD, j * h, x5, p, None, h)
            _, x4 = O.rkck_step(O.QUAD, j * h, x4, p, None, h)
        e5.append(abs(x5[0] - _quad_exact(0.7, T)))
        e4.append(abs(x4[0] - _quad_exact(0.7, T)))
    r5 = [e5[i] / e5[i + 1] for i in range(2)]
    r4 = [e4[i] / e4[i + 1] for i in range(3)]
    for r in r5:
        assert 28.0 < r < 36.0, r5
    for r in r4:
        assert 14.0 < r < 18.0, r4


def test_quad_sweep_matches_closed_form():
    # the paper's introductory sweep: p in [0.1, 1], x0 = -0.5, 1000 steps of 0.01
    import json, os
    here = os.path.dirname(__file__)
    g = json.load(open(os.path.join(here, "golden", "paper_numbers.json")))["quad_intro_example"]
    P, y0 = I.quad_linspace(64, g["p_lo"], g["p_hi"])
    y, ymax = O.rk4(O.QUAD, P, None, y0, g["dt"], g["n_steps"])
    T = g["dt"] * g["n_steps"]
    for i in range(P.shape[1]):
        ex = _quad_exact(P[0, i], T)
        assert abs(y[0, i] - ex) < 1e-8 * max(1.0, abs(ex)), (P[0, i], y[0, i], ex)
        # x^2 - p: for p > 1/4 the solution decreases from -0.5, so the max is x0
        if P[0, i] > 0.25:
            assert ymax[i] == -0.5


def test_quad_quarter_is_an_exact_equilibrium():
    y, ymax = O.rk4(O.QUAD, np.array([[0.25]]), None, np.array([[-0.5]]), 0.01, 1000)
    assert y[0, 0] == -0.5 and ymax[0] == -0.5


# --------------------------------------------------------- Dormand--Prince 5(4)
def _dp_tab():
    a, b5, b4, c = O.rkdp_tableau()
    A = [[_rat(v) for v in row] for row in a]
    return A, [_rat(v) for v in b5], [_rat(v) for v in b4], [_rat(v) for v in c]


def test_dormand_prince_rows_and_first_same_as_last():
    A, b5, _, c = _dp_tab()
    for i in range(7):
        assert sum(A[i]) == c[i]
        assert all(A[i][j] == 0 for j in range(i, 7))
    # the seventh stage evaluates f at the fifth-order result (FSAL)
    assert A[6][:6] == b5[:6] and b5[6] == 0 and c[6] == 1


def test_dormand_prince_fifth_order_weights_satisfy_all_17_conditions():
    A, b5, _, c = _dp_tab()
    conds = _order_conditions(A, b5, c)
    assert sum(len(v) for v in conds.values()) == 17
    for order, lst in conds.items():
        for got, want in lst:
            assert got == want, (order, got, want)


def test_dormand_prince_embedded_weights_are_order_four_exactly():
    A, _, b4, c = _dp_tab()
    conds = _order_conditions(A, b4, c)
    for order in (1, 2, 3, 4):
        for got, want in conds[order]:
            assert got == want, (order, got, want)
    assert any(got != want for got, want in conds[5])


@pytest.mark.parametrize("h", [0.01, 0.1, 0.3, 0.7])
def test_dormand_prince_step_is_stability_polynomial(h):
    # the propagated fifth-order solution of DOPRI5 has R(w) = sum_k<=5 w^k/k!
    # + w^6/600 (Hairer, Norsett, Wanner, Solving ODEs I, Sec. II.5)
    sh = np.array([I.LORENZ_SIGMA, I.LORENZ_BETA])
    z0 = 1.3
    y5, y4 = O.rkdp_step(O.LORENZ, 0.0, np.array([0.0, 0.0, z0]), np.array([0.0]), sh, h)
    w = -I.LORENZ_BETA * h
    R5 = 1 + w + w**2 / 2 + w**3 / 6 + w**4 / 24 + w**5 / 120 + w**6 / 600
    assert y5[2] == pytest.approx(z0 * R5, rel=4e-15)
    # the embedded solution agrees with exp(w) through w^4 only
    base = 1 + w + w**2 / 2 + w**3 / 6 + w**4 / 24
    assert abs(y4[2] / z0 - base) < 0.02 * abs(w) ** 5 + 1e-15


def test_dormand_prince_fixed_step_orders_five_and_four():
    p = np.array([0.7])
    T = 2.0
    e5, e4 = [], []
    for k in range(4):
        n = 40 * 2**k
        h = T / n
        x5 = np.array([-0.5])
        x4 = np.array([-0.5])
        for j in range(n):
            x5, _ = O.rkdp_step(O.QUAD, j * h, x5, p, None, h)
            _, x4 = O.rkdp_step(O.QUAD, j * h, x4, p, None, h)
        e5.append(abs(x5[0] - _quad_exact(0.7, T)))
        e4.append(abs(x4[0] - _quad_exact(0.7, T)))
    r5 = [e5[i] / e5[i + 1] for i in range(2)]
    r4 = [e4[i] / e4[i + 1] for i in range(3)]
    for r in r5:
        assert 28.0 < r < 36.0, r5
    for r in r4:
        assert 14.0 < r < 18.0, r4
