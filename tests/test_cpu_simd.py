"""The benchmark's vectorised CPU Lorenz code against the oracle (both CPU)."""
import numpy as np
import pytest

import oracle as O
from paper_2011_01740_amd import inputs as I

LOR = [I.LORENZ_SIGMA, I.LORENZ_BETA]


@pytest.fixture(scope="module")
def B():
    import bench_cpu
    import os
    if not os.path.exists(bench_cpu.LIB):
        bench_cpu.build()
    return bench_cpu


@pytest.mark.parametrize("n", [0, 1, 31, 32, 33, 1000])
def test_matches_oracle_on_the_non_chaotic_range(B, n):
    P, y0 = I.lorenz_linspace(max(n, 1), 0.0, 12.0)
    P, y0 = P[:, :n], y0[:, :n]
    Y, M = B.lorenz_rk4(P, y0, 0.01, 1000, *LOR, nthreads=4)
    oy, om = O.rk4(O.LORENZ, P, LOR, y0, 0.01, 1000)
    assert np.all(np.abs(Y - oy) <= 1e-10 * np.abs(oy) + 1e-12)
    assert np.all(np.abs(M - om) <= 1e-10 * np.abs(om) + 1e-12)


def test_threads_do_not_change_results(B):
    P, y0 = I.lorenz_random(3000, seed=2)
    a = B.lorenz_rk4(P, y0, 0.01, 200, *LOR, nthreads=1)
    b = B.lorenz_rk4(P, y0, 0.01, 200, *LOR, nthreads=8)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_zero_steps_returns_the_initial_state(B):
    P, y0 = I.lorenz_random(100, seed=3)
    Y, M = B.lorenz_rk4(P, y0, 0.01, 0, *LOR, nthreads=2)
    assert np.array_equal(Y, y0) and np.array_equal(M, y0[0])
