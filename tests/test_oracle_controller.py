"""Exact pins of the oracle's step-size controller (a reading: the paper does
not print its controller; Sec. 4.2.2 only says the packages differ there).

The readings under test: the error ratio E = max_i |err_i| / (atol + rtol
max(|y_i|, |y5_i|)); accept iff E <= 1 or h <= dt_min; factor 0.9 E^(-1/5)
(5 when E = 0), clamped to [0.2, 5] after an accepted and to [0.2, 1] after
a rejected step, then h clamped to [dt_min, dt_max]; a step cut short to land
on a phase end, once accepted, hands the next phase the untruncated proposal.

The probe is the Lorenz system (Sec. 4.1) started on its z axis: with x = y =
0 it reduces to z' = -beta z, so one Cash--Karp step multiplies z by the
stability polynomial R5(w), w = -beta h, and the embedded solution by R4(w).
Both polynomials are written out here as exact rationals and are pinned to
the oracle's one-step results in test_oracle_tableau.py; E follows from them
in closed form, independently of the oracle's tableau arithmetic.  Then a
safety factor of 0.8, an exponent of -1/4, a growth clamp after rejections,
a step restarted from its truncated length or a propagated fourth-order
solution each move the expected numbers by several percent.

Also pinned: the paper's Dormand--Prince step counts and step-size extremes
at 20 / 100 / 500 kHz (Sec. 4.2, the bubble time series), and the Adam
update beyond its first step (constant gradients).
"""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle as O
from oracle import mlp as M
from paper_2011_01740_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_numbers.json")))
SH = np.array([I.LORENZ_SIGMA, I.LORENZ_BETA])
BETA = I.LORENZ_BETA
RTOL = ATOL = 1e-10


def _R(w):
    """Cash--Karp stability polynomials at w (exact rationals): (R5, R4)."""
    w = Fr(w)
    base = 1 + w + w**2 / 2 + w**3 / 6 + w**4 / 24
    R5 = base + w**5 / 120 + w**6 / 800
    R4 = base + Fr(10517, 1228800) * w**5 + Fr(1771, 1638400) * w**6
    return R5, R4


def _expected_E(h, z0=1.0):
    """Error ratio of one step of z' = -beta z from z0 with step h."""
    R5, R4 = _R(-BETA * h)
    z5 = R5 * Fr(z0)
    err = abs((R5 - R4) * Fr(z0))
    return float(err / (Fr(ATOL) + Fr(RTOL) * max(abs(Fr(z0)), abs(z5)))), float(z5)


def _h_for_E(E, z0=1.0):
    """The step whose error ratio is E (bisection on the closed form)."""
    lo, hi = 1e-6, 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _expected_E(mid, z0)[0] < E:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _one_attempt(h0, z0=1.0, t0=0.0, **kw):
    o = O.Opts(n_phases=kw.pop("n_phases", 1), n_record=1, max_steps=kw.pop("max_steps", 1),
               t_phase=kw.pop("t_phase", 1e3), dt_max=kw.pop("dt_max", 10.0),
               dt_min=kw.pop("dt_min", 1e-14), rtol=RTOL, atol=ATOL, **kw)
    y0 = np.array([[0.0], [0.0], [z0]])
    return O.rkck45(O.LORENZ, np.array([[5.0]]), SH, y0, o, t0=np.array([t0]),
                    h0=np.array([h0]))


@pytest.mark.parametrize("E", [3e-4, 1e-3, 0.05, 0.5, 0.99])
def test_accepted_step_factor_is_09_E_to_minus_one_fifth(E):
    h0 = _h_for_E(E)
    Ee, z5 = _expected_E(h0)
    assert Ee == pytest.approx(E, rel=1e-9)
    r = _one_attempt(h0)
    assert r.stats[O.ST_ACCEPTED, 0] == 1 and r.stats[O.ST_REJECTED, 0] == 0
    fac = min(max(0.9 * Ee ** -0.2, 0.2), 5.0)
    # E comes out of a sum that cancels to ~1e-9 of its terms: ~1e-7 relative
    assert r.h[0] == pytest.approx(h0 * fac, rel=2e-6)
    # the fifth-order solution is the one propagated
    assert r.y[2, 0] == pytest.approx(z5, rel=1e-14)
    assert r.y[0, 0] == 0.0 and r.y[1, 0] == 0.0
    assert r.t[0] == h0


@pytest.mark.parametrize("E", [1.05, 3.0, 30.0, 1e3, 1e5])
def test_rejected_step_factor_is_clamped_to_02_1(E):
    h0 = _h_for_E(E)
    Ee, _ = _expected_E(h0)
    r = _one_attempt(h0)
    assert r.stats[O.ST_ACCEPTED, 0] == 0 and r.stats[O.ST_REJECTED, 0] == 1
    fac = min(max(0.9 * Ee ** -0.2, 0.2), 1.0)
    assert r.h[0] == pytest.approx(h0 * fac, rel=2e-6)
    # a rejected step leaves the state and the clock where they were
    assert r.y[2, 0] == 1.0 and r.t[0] == 0.0
    assert r.status[0] & O.SYS_MAX_STEPS


def test_zero_error_gives_factor_five_then_the_dt_max_clamp():
    r = _one_attempt(0.03, z0=0.0)
    assert r.h[0] == 5 * 0.03
    r = _one_attempt(0.03, z0=0.0, dt_max=0.1)
    assert r.h[0] == 0.1


def test_accept_at_the_dt_min_floor():
    # E >> 1 at h = dt_min: taken anyway, flagged, the proposal clamped to dt_min
    h0 = _h_for_E(5e3)
    Ee, z5 = _expected_E(h0)
    assert Ee > 1
    r = _one_attempt(h0, dt_min=h0)
    assert r.stats[O.ST_ACCEPTED, 0] == 1 and r.stats[O.ST_REJECTED, 0] == 0
    assert r.status[0] & O.SYS_DT_MIN
    assert r.y[2, 0] == pytest.approx(z5, rel=1e-14)
    assert r.h[0] == h0


def test_truncated_step_hands_the_next_phase_the_untruncated_proposal():
    h0 = _h_for_E(0.05)
    cut = 0.3 * h0
    t0 = 1.0 - cut
    r = _one_attempt(h0, t0=t0, t_phase=1.0, max_steps=0)
    assert r.stats[O.ST_ACCEPTED, 0] == 1 and r.stats[O.ST_PHASES, 0] == 1
    assert r.t[0] == 0.0
    # not h_cut * clamp(0.9 E(h_cut)^(-1/5)): the proposal made before the cut
    assert r.h[0] == h0
    Ec, z5 = _expected_E(1.0 - t0)
    assert r.y[2, 0] == pytest.approx(z5, rel=1e-14)
    # the next phase's first attempt is taken with h0 from t = 0
    r2 = _one_attempt(h0, t0=t0, t_phase=1.0, n_phases=2, max_steps=2)
    assert r2.stats[O.ST_ACCEPTED, 0] == 2
    assert r2.t[0] == h0
    E2, _ = _expected_E(h0, z5)
    assert r2.h[0] == pytest.approx(h0 * min(max(0.9 * E2 ** -0.2, 0.2), 5.0), rel=2e-6)


def test_rejected_truncated_step_continues_from_the_cut_length():
    h0 = _h_for_E(1e4)
    cut = 0.5 * h0
    r = _one_attempt(h0, t0=1.0 - cut, t_phase=1.0)
    assert r.stats[O.ST_REJECTED, 0] == 1 and r.stats[O.ST_PHASES, 0] == 0
    h_cut = 1.0 - (1.0 - cut)
    Ec, _ = _expected_E(h_cut)
    assert Ec > 1
    assert r.h[0] == pytest.approx(h_cut * min(max(0.9 * Ec ** -0.2, 0.2), 1.0), rel=2e-6)


def test_dormand_prince_uses_the_same_controller():
    # DP's stability polynomials differ, so only the structure is compared:
    # the proposal after one accepted step is h0 * 0.9 E^(-1/5) with E from
    # DP's own embedded pair (y5, y4), taken from the oracle's single step
    h0 = 0.008
    y = np.array([0.0, 0.0, 1.0])
    y5, y4 = O.rkdp_step(O.LORENZ, 0.0, y, np.array([5.0]), SH, h0)
    E = abs(y5[2] - y4[2]) / (ATOL + RTOL * max(1.0, abs(y5[2])))
    assert 1e-3 < E < 1
    r = _one_attempt(h0, scheme=O.DORMAND_PRINCE)
    assert r.stats[O.ST_ACCEPTED, 0] == 1
    # y5 - y4 differs from h sum (b5 - b4) k in the last bits of a cancelling sum
    assert r.h[0] == pytest.approx(h0 * min(max(0.9 * E ** -0.2, 0.2), 5.0), rel=1e-4)


# ------------------------------------------------------------------ Sec. 4.2, the time series
def _km_two_phases_after_transient(scheme):
    sh = np.array(I.KM_WATER_PAPER)
    fs = np.array([20e3, 100e3, 500e3])
    P = np.vstack([np.full(fs.size, 1.5e5), fs])
    y0 = np.vstack([np.ones(fs.size), np.zeros(fs.size)])
    r = O.rkck45(O.KM, P, sh, y0, O.Opts(n_phases=1024, scheme=scheme), nthreads=3)
    return O.rkck45(O.KM, P, sh, r.y, O.Opts(n_phases=2, n_record=2, scheme=scheme),
                    t0=r.t, h0=r.h, carry0=r.carry, nthreads=3)


def test_dormand_prince_step_counts_and_extremes_match_the_papers_time_series():
    """Sec. 4.2: with Dormand--Prince at tolerance 1e-10 (Julia's controller,
    not printed), two phases after the transient take about 6800 / 1800 /
    300 steps at 20 / 100 / 500 kHz, and at 20 kHz the steps range from
    2.2e-9 to 1.2e-3.  Soft pins: the counts within 20%, the extremes within
    a factor 10 (measured here: -12%, -10%, -13%; 1.1e-8 and 5.3e-3)."""
    g = GOLD["km_dp_steps_two_phases"]
    r = _km_two_phases_after_transient(O.DORMAND_PRINCE)
    acc = r.stats[O.ST_ACCEPTED]
    for got, want in zip(acc, g["steps"]):
        assert abs(got / want - 1) < 0.20, (acc, g["steps"])
    x = GOLD["km_step_sizes_20khz"]
    h_min, h_max = r.hx[0, 0], r.hx[1, 0]
    assert x["h_min"] / 10 < h_min < x["h_min"] * 10, h_min
    assert x["h_max"] / 10 < h_max < x["h_max"] * 10, h_max
    # the collapse at 20 kHz needs steps five orders of magnitude apart
    assert h_max / h_min > 1e4
    # smoother dynamics at higher frequency: fewer steps, larger smallest step
    assert acc[0] > acc[1] > acc[2]
    assert r.hx[0, 0] < r.hx[0, 1] < r.hx[0, 2]


# ------------------------------------------------------------------ Adam beyond its first step
def test_adam_with_constant_gradients_steps_lr_sign_g_every_time():
    """With a constant gradient both bias-corrected moments are exact at every
    step (m_hat = g, v_hat = g^2), so each update is lr g / (|g| + eps); a
    wrong bias correction (or none) makes the early steps differ."""
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    p = [np.zeros(4)]
    m = [np.zeros(4)]
    v = [np.zeros(4)]
    lr = 0.01
    step = lr * g / (np.abs(g) + 1e-8)
    for t in range(1, 51):
        p, m, v = M.adam_step(p, [g], m, v, t, lr=lr)
        assert np.allclose(p[0], -t * step, rtol=1e-9, atol=0), t
        assert np.allclose(m[0], (1 - 0.9 ** t) * g, rtol=1e-12)
        assert np.allclose(v[0], (1 - 0.999 ** t) * g * g, rtol=1e-12)


def test_adam_alternating_gradient_matches_closed_form_moments():
    """g_t = (-1)^(t+1) c: m_t = (1 - b1) c sum_k b1^(t-k) (-1)^(k+1) in closed
    form, v_t = (1 - b2^t) c^2, so the t-th update is known exactly."""
    c = np.array([2.0, -0.25])
    b1, b2, lr, eps = 0.9, 0.999, 0.003, 1e-8
    p, m, v = [np.zeros(2)], [np.zeros(2)], [np.zeros(2)]
    want_p = np.zeros(2)
    for t in range(1, 31):
        g = c if t % 2 else -c
        p, m, v = M.adam_step(p, [g], m, v, t, lr=lr, b1=b1, b2=b2, eps=eps)
        # geometric sum with ratio -b1: (1 - b1) c (-1)^(t+1) (1 - (-b1)^t) / (1 + b1)
        mt = (1 - b1) * c * (-1) ** (t + 1) * (1 - (-b1) ** t) / (1 + b1)
        vt = (1 - b2 ** t) * c * c
        want_p = want_p - lr * (mt / (1 - b1 ** t)) / (np.sqrt(vt / (1 - b2 ** t)) + eps)
        assert np.allclose(m[0], mt, rtol=1e-12)
        assert np.allclose(v[0], vt, rtol=1e-12)
        assert np.allclose(p[0], want_p, rtol=1e-10, atol=1e-15)


# ------------------------------------------------------------------ Sec. 3.2.2, FLOP accounting
def test_flop_accounting_of_the_introductory_rk4_kernel():
    """The profiler listing of Sec. 3.2.2 counts 15360000 FP64 adds, no
    multiplies and 153600000 FMAs for the introductory example; the RK4 step
    of dx/dt = x^2 - p is 10 FMAs and one add per system (21 flop), so the
    listing is 1000 steps of 15360 systems, and the largest FLOP efficiency
    those instructions allow (an add counts 1 flop in an FMA's issue slot) is
    the 95% the paper states."""
    g = GOLD["tab2_flop_accounting"]
    fma_per_step, add_per_step = 10, 1
    steps = g["dp_fma"] // fma_per_step
    assert steps * add_per_step == g["dp_add"] and g["dp_mul"] == 0
    assert steps == 15360 * 1000
    flop = 2 * g["dp_fma"] + g["dp_add"] + g["dp_mul"]
    assert flop == 21 * steps
    ceiling = flop / (2 * (g["dp_fma"] + g["dp_add"] + g["dp_mul"]))
    assert round(ceiling, 2) == g["max_efficiency"]
