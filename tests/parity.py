"""Parity helpers shared by the GPU tests.

Tolerances (written out here, applied element by element):
* fixed-step RK4, non-chaotic systems:   |gpu - oracle| <= 1e-10 |oracle| + 1e-12
* adaptive Cash--Karp, endpoint and every recorded value:
                                         |gpu - oracle| <= 1e-7 |oracle| + 1e-9
Chaotic systems amplify the last-bit differences between the GPU's fused
multiply-adds and the oracle's separately rounded operations, so parity is
checked on the "parity set": systems whose own oracle result moves by less
than 1e-11 (fixed step) or 1e-9 (adaptive) when the initial condition is
perturbed by 1e-13 relative.  The others are checked for invariants only.
"""
import numpy as np

RK4_RTOL, RK4_ATOL = 1e-10, 1e-12
CK_RTOL, CK_ATOL = 1e-7, 1e-9
PERTURB = 1e-13


def close(g, o, rtol, atol):
    g = np.asarray(g)
    o = np.asarray(o)
    both_nan = np.isnan(g) & np.isnan(o)
    # the tolerance applies where the oracle is finite; an infinite oracle
    # value needs the same infinity
    with np.errstate(invalid="ignore"):
        ok = np.isfinite(o) & (np.abs(g - o) <= rtol * np.abs(o) + atol)
    return ok | both_nan | (g == o)


def per_system(mask):
    """Collapse a [..., n] boolean array to [n] (all components true)."""
    m = np.asarray(mask)
    return m.reshape(-1, m.shape[-1]).all(axis=0)


def sensitivity_mask(a_list, b_list, rtol, atol):
    """Systems whose oracle outputs agree between the nominal and perturbed runs."""
    m = None
    for a, b in zip(a_list, b_list):
        s = per_system(close(b, a, rtol, atol))
        m = s if m is None else (m & s)
    return m
