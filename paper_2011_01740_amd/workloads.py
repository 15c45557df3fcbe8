"""The paper's ensemble workloads, set up through the libens binding.

Each function builds the seeded synthetic inputs (``inputs``), hands them to
the library as device tensors, runs the solve on the current torch stream and
returns the results with the measured kernel time.  Nothing here computes any
part of the method.

* ``lorenz``     -- Lorenz sweep with classic RK4 (Sec. 4.1)
* ``km_sweep``   -- Keller--Miksis (p_A, f) grid, adaptive Cash--Karp, one
                    record per acoustic cycle (Sec. 4.2)
* ``prv_batched``-- several relief-valve ensembles with their own q draws
                    and phase/impact budgets, solved in one graph-captured
                    persistent launch (Sec. 4.3)
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

from . import ens
from . import inputs as I


@dataclass
class Result:
    y: np.ndarray
    t: Optional[np.ndarray] = None
    h: Optional[np.ndarray] = None
    acc: Optional[np.ndarray] = None
    records: Optional[np.ndarray] = None
    stats: Optional[np.ndarray] = None
    status: Optional[np.ndarray] = None
    kernel_ms: float = 0.0
    wall_s: float = 0.0
    launch: Dict[str, int] = field(default_factory=dict)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def lorenz(n: int, n_steps: int, seed: Optional[int] = 1, dt: float = 0.01, **launch) -> Result:
    """Lorenz RK4 sweep: seeded random p and IC (seed) or the linspace sweep (seed None)."""
    import torch
    P, y0 = I.lorenz_random(n, seed=seed) if seed is not None else I.lorenz_linspace(n)
    with ens.Ensemble(ens.ENS_LORENZ, ens.ENS_RK4, n) as e:
        e.set_params(_dev(P))
        e.set_state(_dev(y0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e.solve(dt=dt, n_steps=n_steps, **launch)
        ms = e.last_kernel_ms()
        wall = time.perf_counter() - t0
        return Result(y=e.read(ens.ENS_STATE), acc=e.read(ens.ENS_ACC), kernel_ms=ms,
                      wall_s=wall, launch=e.last_launch())


def scalar_rk4(model: int, n: int, n_steps: int = 1000, dt: float = 0.01, **launch) -> Result:
    """The introductory example (ENS_QUAD) or its division (ENS_DIV) and
    transcendental (ENS_SIN) variants with fixed-step RK4: p on an equidistant
    grid in [0.1, 1], x0 = -0.5 (Sec. 3, Sec. 3.3)."""
    import torch
    P, y0 = I.quad_linspace(n)
    with ens.Ensemble(model, ens.ENS_RK4, n) as e:
        e.set_params(_dev(P))
        e.set_state(_dev(y0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e.solve(dt=dt, n_steps=n_steps, **launch)
        ms = e.last_kernel_ms()
        wall = time.perf_counter() - t0
        return Result(y=e.read(ens.ENS_STATE), acc=e.read(ens.ENS_ACC), kernel_ms=ms,
                      wall_s=wall, launch=e.last_launch())


def _adaptive(model, P, y0, opts, offsets=None, shared=None, budgets=None, read_records=True,
              rest_opts=None, solver=None, tangent=False):
    """One solve with opts; or, with rest_opts, a pilot solve with opts, the
    queue ordered longest-first by its step counts (ens_order_by_work) and a
    second solve with rest_opts (stats summed, status bits or-ed, kernel
    times added)."""
    import torch
    n = y0.shape[-1]
    solver = ens.ENS_RKCK45 if solver is None else solver
    with ens.Ensemble(model, solver, n, offsets=offsets, tangent=tangent) as e:
        e.set_params(_dev(P))
        if shared is not None:
            for k, sh in enumerate(shared):
                e.set_shared(k, sh)
        if budgets is not None:
            for k, (ph, imp) in enumerate(budgets):
                e.set_budget(k, ph, imp)
        e.set_state(_dev(y0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e.solve(opts)
        ms = e.last_kernel_ms()
        stats0, status0 = 0, 0
        if rest_opts is not None:
            stats0, status0 = e.read(ens.ENS_STATS), e.read(ens.ENS_STATUS)
            e.order_by_work()
            e.solve(rest_opts)
            ms += e.last_kernel_ms()
        wall = time.perf_counter() - t0
        return Result(y=e.read(ens.ENS_STATE), t=e.read(ens.ENS_TIME), h=e.read(ens.ENS_H),
                      records=e.read(ens.ENS_RECORDS) if read_records else None,
                      stats=stats0 + e.read(ens.ENS_STATS),
                      status=status0 | e.read(ens.ENS_STATUS),
                      kernel_ms=ms, wall_s=wall, launch=e.last_launch())


def km_sweep(n_pa: int, n_f: int, n_phases: int = 1024, n_record: Optional[int] = None,
             shared: Sequence[float] = I.KM_WATER, rtol: float = 1e-10, atol: float = 1e-10,
             P: Optional[np.ndarray] = None, pilot: int = 0, pilot_grid: int = 0,
             solver: Optional[int] = None, tangent: bool = False, **launch) -> Result:
    """Keller--Miksis sweep over an (n_pa x n_f) grid (p_A linear in [0.2, 1.2]
    bar, f geometric in [20 kHz, 1 MHz]), IC (1, 0), one y1max record per
    acoustic cycle (the last n_record cycles).  P overrides the grid.  With
    pilot > 0 (and n_phases - pilot >= n_record) the first `pilot` cycles run
    in index order and the rest longest-first (on pilot_grid blocks; 0: all);
    the records come back in phase order either way.
    solver: ENS_RKCK45 (default) or ENS_RKDP45.  tangent: the variational
    equation rides along from dy = (1, 1)/sqrt 2, and each record gains the
    phase's log growth (the largest Lyapunov exponent is its mean)."""
    if P is None:
        P, y0 = I.km_grid(n_pa, n_f)
    else:
        y0 = np.vstack([np.ones(P.shape[1]), np.zeros(P.shape[1])])
    if tangent:
        y0 = np.vstack([y0, np.full_like(y0, 1.0 / np.sqrt(2.0))])
    R = n_phases if n_record is None else n_record
    if 0 < pilot and n_phases - pilot >= R:
        o = ens.default_opts(n_phases=pilot, n_record=R, rtol=rtol, atol=atol, **launch)
        rest = dict(launch, grid=pilot_grid or launch.get("grid", 0))
        o2 = ens.default_opts(n_phases=n_phases - pilot, n_record=R, rtol=rtol, atol=atol, **rest)
        r = _adaptive(ens.ENS_KM, P, y0, o, shared=[list(shared)], rest_opts=o2,
                      solver=solver, tangent=tangent)
        m = n_phases - pilot
    else:
        o = ens.default_opts(n_phases=n_phases, n_record=R, rtol=rtol, atol=atol, **launch)
        r = _adaptive(ens.ENS_KM, P, y0, o, shared=[list(shared)], solver=solver,
                      tangent=tangent)
        m = n_phases
    # the ring's oldest slot is m % R: rotate the phases into order
    if r.records is not None and R > 0:
        r.records = np.roll(r.records, -(m % R), axis=0)
    return r


PRV_ENSEMBLES: Tuple[Tuple[int, int, int], ...] = ((1 << 15, 100000, 3), (1 << 16, 10000, 4),
                                                   (1 << 17, 1000, 5))


def prv_inputs(ensembles=PRV_ENSEMBLES):
    Ps, ys = [], []
    for m, _, seed in ensembles:
        P, y0 = I.prv_random(m, seed=seed)
        Ps.append(P)
        ys.append(y0)
    off = np.concatenate([[0], np.cumsum([m for m, _, _ in ensembles])]).astype(np.int64)
    return np.concatenate(Ps, axis=1), np.concatenate(ys, axis=1), off


def prv_batched(ensembles=PRV_ENSEMBLES, n_record: int = 32, use_graph: int = 1,
                solver: Optional[int] = None, spread: Optional[int] = None,
                **launch) -> Result:
    """Relief-valve ensembles (size, budget K, seed): each system runs until K
    Poincare phases or K impacts, whichever comes first; the last n_record
    phases (y1max, y1min) are kept.  One persistent launch for all.  spread
    (default: the first ensemble, which holds the largest budget): queue head
    handed out one wave per SIMD."""
    P, y0, off = prv_inputs(ensembles)
    budgets = [(K, K) for _, K, _ in ensembles]
    if spread is None:
        spread = ensembles[0][0] if len(ensembles) > 1 else 0
    o = ens.default_opts(n_phases=max(K for _, K, _ in ensembles), n_record=n_record,
                         use_graph=use_graph, spread=spread, **launch)
    return _adaptive(ens.ENS_PRV, P, y0, o, offsets=off, budgets=budgets, solver=solver)
