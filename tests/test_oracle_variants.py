"""Pins of the oracle's division and transcendental variants of the
introductory example (Sec. 3.3), dx/dt = 1/x - p x and dx/dt = p sin x, by
their closed-form solutions, with classic RK4 at a fixed step (Sec. 3).

  1/x - p x :  u = x^2 obeys u' = 2 - 2 p u, so
               x(t) = sqrt(1/p + (x0^2 - 1/p) exp(-2 p t))          (x0 > 0)
  p sin x   :  dx / sin x = p dt integrates to log tan(x/2) = p t + C, so
               x(t) = 2 atan(tan(x0/2) exp(p t))                    (0 < x0 < pi)
"""
import numpy as np
import pytest

import oracle as O


def div_exact(x0, p, t):
    return np.sqrt(1.0 / p + (x0 * x0 - 1.0 / p) * np.exp(-2.0 * p * t))


def sin_exact(x0, p, t):
    return 2.0 * np.arctan(np.tan(0.5 * x0) * np.exp(p * t))


CASES = [(O.DIV, div_exact, (0.5, 2.0), (0.5, 2.0)),
         (O.SIN, sin_exact, (0.2, 3.0), (-1.0, 1.0))]


@pytest.mark.parametrize("model,exact,xr,pr", CASES)
def test_rk4_follows_closed_form(model, exact, xr, pr):
    rng = np.random.default_rng(11)
    n = 64
    x0 = rng.uniform(*xr, n)
    p = rng.uniform(*pr, n)
    T, steps = 2.0, 2000
    y, ymax = O.rk4(model, p.reshape(1, n), None, x0.reshape(1, n), T / steps, steps)
    want = exact(x0, p, T)
    np.testing.assert_allclose(y[0], want, rtol=1e-11, atol=0)
    # the running maximum over the step points: the solutions are monotone
    np.testing.assert_allclose(ymax, np.maximum(x0, want), rtol=1e-11, atol=0)


@pytest.mark.parametrize("model,exact,xr,pr", CASES)
def test_rk4_is_fourth_order(model, exact, xr, pr):
    x0 = np.array([[0.5 * (xr[0] + xr[1])]])
    p = np.array([[pr[1]]])
    T = 2.0
    errs = []
    for steps in (20, 40, 80):
        y, _ = O.rk4(model, p, None, x0, T / steps, steps)
        errs.append(abs(y[0, 0] - exact(x0[0, 0], p[0, 0], T)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13.0 < r1 < 19.0 and 13.0 < r2 < 19.0, (r1, r2)


def test_fixed_points():
    # 1/x - p x vanishes at x = 1/sqrt(p); p sin x at x = pi
    for p in (0.25, 1.0, 4.0):
        assert abs(O.rhs(O.DIV, 0.0, [1.0 / np.sqrt(p)], [p])[0]) < 1e-15
    y, _ = O.rk4(O.SIN, np.array([[0.7]]), None, np.array([[np.pi]]), 0.01, 100)
    assert abs(y[0, 0] - np.pi) < 1e-13
