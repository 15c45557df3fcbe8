"""Seeded synthetic inputs for the ensemble workloads.

This module is the only code shared by the CPU oracle and the GPU path.  It
holds no arithmetic of the integration method: it only produces parameter
sweeps, initial conditions and the physical constants that the paper lists
for each model.  Everything here is plain numpy.

Workloads (the paper's own synthetic parameter sweeps):

* Lorenz (Sec. 4.1): the parameter p swept over [0, 21]; initial condition
  (10, 10, 10); classic RK4 with a fixed step.
* Keller--Miksis (Sec. 4.2): sinusoidal pressure drive, amplitude p_A and
  frequency f swept on a grid (f logarithmically spaced, as in the paper's
  frequency-response study); bubble starts at rest at its equilibrium radius.
* Pressure-relief valve (Sec. 4.3): dimensionless flow rate q in [0.2, 10].

Random draws use SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the k-th uniform of system i
under seed s is the first output of a SplitMix64 generator whose state starts
at s * 2**40 + i * 8 + k, shifted right by 11 bits and scaled by 2**-53.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "splitmix64_uniform",
    "LORENZ_SIGMA", "LORENZ_BETA", "LORENZ_BETA_PAPER",
    "KM_WATER", "KM_WATER_PAPER",
    "PRV_DEFAULT",
    "lorenz_linspace", "lorenz_random",
    "km_grid", "km_axes",
    "prv_random", "prv_linspace",
    "quad_linspace",
    "mlp_init",
]

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_MIX1 = np.uint64(0xBF58476D1CE4E5B9)
_MIX2 = np.uint64(0x94D049BB133111EB)


def _splitmix64_first(state: np.ndarray) -> np.ndarray:
    """First output of SplitMix64 started from ``state`` (uint64, wrapping)."""
    with np.errstate(over="ignore"):
        z = state + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _MIX1
        z = (z ^ (z >> np.uint64(27))) * _MIX2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_uniform(seed: int, index: np.ndarray, k: int) -> np.ndarray:
    """Uniform doubles in [0, 1): draw ``k`` of systems ``index`` under ``seed``."""
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = (np.uint64(seed) << np.uint64(40)) + idx * np.uint64(8) + np.uint64(k)
    bits = _splitmix64_first(state) >> np.uint64(11)
    return bits.astype(np.float64) * (2.0 ** -53)


# ---------------------------------------------------------------- constants
# Lorenz coefficients (Sec. 4.1).  The paper prints 2.666 for the z-damping
# coefficient; the classic value 8/3 is the default, 2.666 is kept as the
# paper-literal alternative.
LORENZ_SIGMA = 10.0
LORENZ_BETA = 8.0 / 3.0
LORENZ_BETA_PAPER = 2.666

# Keller--Miksis material constants, SI units.  Order of the fields matches
# the shared-parameter layout of both implementations:
# (rho_L, c_L, p_V, sigma, mu_L, gamma, P_inf, R_E, P_A2, f2, theta)
KM_FIELDS = ("rho_L", "c_L", "p_V", "sigma", "mu_L", "gamma", "P_inf", "R_E",
             "P_A2", "f2", "theta")
# Water at 25 C as used by the sweeps (single-frequency drive).
KM_WATER = (997.0, 1497.0, 3166.0, 0.0728, 8.9e-4, 1.4, 1.0e5, 10.0e-6,
            0.0, 0.0, 0.0)
# The values printed in Sec. 4.2 (used to compare with Tab. 4 work counts).
KM_WATER_PAPER = (997.1, 1497.3, 3166.8, 0.072, 8.902e-4, 1.4, 1.0e5, 10.0e-6,
                  0.0, 0.0, 0.0)

# Pressure-relief valve constants of Sec. 4.3: (kappa, delta, beta, r).
PRV_DEFAULT = (1.25, 10.0, 20.0, 0.8)


# ---------------------------------------------------------------- sweeps
def quad_linspace(n: int, lo: float = 0.1, hi: float = 1.0):
    """Introductory example of Sec. 3: p on an equidistant grid, x0 = -0.5."""
    p = np.linspace(lo, hi, n, dtype=np.float64)
    y0 = np.full((1, n), -0.5, dtype=np.float64)
    return p.reshape(1, n), y0


def lorenz_linspace(n: int, lo: float = 0.0, hi: float = 21.0):
    """Lorenz sweep of Sec. 4.1: p on an inclusive equidistant grid, IC (10,10,10)."""
    p = np.linspace(lo, hi, n, dtype=np.float64).reshape(1, n)
    y0 = np.full((3, n), 10.0, dtype=np.float64)
    return p, y0


def lorenz_random(n: int, seed: int = 1, lo: float = 0.0, hi: float = 21.0,
                  ic_halfwidth: float = 1.0, first: int = 0):
    """Lorenz sweep with p ~ U[lo, hi] and IC 10 + U[-1, 1] per component.

    Draw 0 of each system gives p, draws 1..3 the IC offsets.  ``first`` lets a
    caller generate a contiguous slice [first, first + n) of a larger ensemble.
    """
    idx = np.arange(first, first + n, dtype=np.uint64)
    p = lo + (hi - lo) * splitmix64_uniform(seed, idx, 0)
    y0 = np.empty((3, n), dtype=np.float64)
    for c in range(3):
        y0[c] = 10.0 + ic_halfwidth * (2.0 * splitmix64_uniform(seed, idx, 1 + c) - 1.0)
    return p.reshape(1, n), y0


def km_axes(n_pa: int, n_f: int, pa_lo=0.2e5, pa_hi=1.2e5, f_lo=20e3, f_hi=1e6):
    """Grid axes: pressure amplitude linear [Pa], frequency geometric [Hz]."""
    pa = np.linspace(pa_lo, pa_hi, n_pa, dtype=np.float64)
    f = np.geomspace(f_lo, f_hi, n_f, dtype=np.float64)
    return pa, f


def km_grid(n_pa: int, n_f: int, **kw):
    """Keller--Miksis sweep on an (n_pa x n_f) grid; system index = i_pa * n_f + i_f.

    Neighbouring systems have neighbouring parameters (the paper's advice for
    limiting divergence inside a wavefront, Sec. 3.2.1).  IC: bubble at rest at
    its equilibrium radius, (y1, y2) = (1, 0).
    """
    pa, f = km_axes(n_pa, n_f, **kw)
    P = np.empty((2, n_pa * n_f), dtype=np.float64)
    P[0] = np.repeat(pa, n_f)
    P[1] = np.tile(f, n_pa)
    y0 = np.empty((2, n_pa * n_f), dtype=np.float64)
    y0[0] = 1.0
    y0[1] = 0.0
    return P, y0


def prv_random(n: int, seed: int, lo: float = 0.2, hi: float = 10.0, first: int = 0):
    """Relief-valve sweep, q ~ U[lo, hi]; IC (0.2, 0, 10.2) (valve at rest, forces balanced)."""
    idx = np.arange(first, first + n, dtype=np.uint64)
    q = lo + (hi - lo) * splitmix64_uniform(seed, idx, 0)
    y0 = np.empty((3, n), dtype=np.float64)
    y0[0] = 0.2
    y0[1] = 0.0
    y0[2] = 10.2
    return q.reshape(1, n), y0


def prv_linspace(n: int, lo: float = 0.2, hi: float = 10.0):
    """Relief-valve sweep on the paper's uniform grid of q."""
    q = np.linspace(lo, hi, n, dtype=np.float64).reshape(1, n)
    y0 = np.empty((3, n), dtype=np.float64)
    y0[0] = 0.2
    y0[1] = 0.0
    y0[2] = 10.2
    return q, y0


def mlp_init(seed: int = 4, dims=(2, 256, 256, 256, 64), ff_scale: float = 16.0):
    """Initial surrogate parameters, packed W1, b1, W2, b2, ... (float64; both
    implementations round as they need).  Layer 1 is the fixed random
    Fourier-feature map: dims[1] / 2 frequency vectors f_k ~ N(0, ff_scale^2 I)
    (rows k and k + dims[1] / 2 of W1), phases b1 = 0 (sine) and pi / 2
    (cosine).  The trained layers: He-uniform U[-sqrt(6/fan_in),
    sqrt(6/fan_in)] weights (shape (out, in), row-major), zero biases."""
    rng = np.random.default_rng(seed)
    half = dims[1] // 2
    F = rng.normal(size=(half, dims[0])) * ff_scale
    parts = [np.vstack([F, F]).ravel(),
             np.concatenate([np.zeros(half), np.full(dims[1] - half, np.pi / 2)])]
    for i in range(1, len(dims) - 1):
        lim = (6.0 / dims[i]) ** 0.5
        parts.append(rng.uniform(-lim, lim, size=(dims[i + 1], dims[i])).ravel())
        parts.append(np.zeros(dims[i + 1]))
    return np.concatenate(parts)
