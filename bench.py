#!/usr/bin/env python3
"""Throughput benchmark of the ensemble integrator on one MI355X.

Workload: the paper's Lorenz parameter sweep (Sec. 4.1) at scale --
2^23 independent Lorenz systems, p ~ U[0, 21] and IC 10 + U[-1, 1] (seeded
SplitMix64), classic RK4 with dt = 0.01 for 10^4 steps, FP64.  One benchmark
step is one full pass: reset the state from the resident initial conditions
and integrate all systems for all 10^4 steps (final state and running max of
x written back).

Output: one JSON line with system-steps/s, the FP64 roofline of the RK4
kernel (71 algorithmic flop per system-step, peak 78.6 TFLOP/s), and the CPU
oracle timed on a bounded sample of the same workload on the host's cores.
The same line carries the Keller--Miksis half of the metric (Sec. 4.2): the
512 x 512 x 1024-cycle sweep (`km_sweep`, with the oracle on a sub-grid) and
the surrogate-screened 4096 x 4096 sweep against the plain sweep of all its
points (`km_screened`).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 vector peak (256 CU x 2.4 GHz x 128)
# Lorenz RK4, textbook step: 4 x 8 (RHS: sigma (y - x) 2, x (rho - z) - y 3,
# x y - beta z 3) + 3 x 6 (stage inputs y + (h/2) k: a multiply and an add per
# component) + 21 (update y + h/6 (k1 + 2 k2 + 2 k3 + k4): 7 per component)
FLOP_PER_STEP = 71
HW_FLOP_PER_STEP = 70            # what the kernel executes: 33 FMA (x 2) + 4 subtractions
BYTES_PER_SYSTEM = 8 * 8         # reads p, x, y, z; writes x, y, z, max x
BF16_PEAK_TFLOPS = 2500.0        # MI355X dense BF16 matrix peak
# the surrogate network's matrix products per point: 2 x (256 x 256 + 256 x 256
# + 64 x 256) multiply-adds (the 2 -> 256 feature layer runs on the vector unit)
SCREEN_FLOP_PER_POINT = 2 * (256 * 256 + 256 * 256 + 64 * 256)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lorenz_rk4_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2011_01740_amd", "csrc", "rk4.hip")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(n, nsteps):
    """HBM bytes per launch from the committed counter run, if it was taken
    on the current kernel source at this size; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash() or t.get("n") != n or t.get("n_steps") != nsteps:
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(n_total, nsteps, dt, seed, target_s=12.0):
    """The oracle (plain serial FP64 C, one thread per system batch) on the
    first m systems of the same seeded ensemble, m sized for ~target_s."""
    import oracle as O
    from paper_2011_01740_amd import inputs as I

    threads = max(1, min(os.cpu_count() or 1, 16))
    sh = [I.LORENZ_SIGMA, I.LORENZ_BETA]
    probe = 64 * threads
    P, y0 = I.lorenz_random(probe, seed=seed)
    t0 = time.perf_counter()
    O.rk4(O.LORENZ, P, sh, y0, dt, nsteps, nthreads=threads)
    dt_probe = time.perf_counter() - t0
    m = int(probe * max(1.0, target_s / max(dt_probe, 1e-3)))
    m = max(probe, min(m, n_total))
    P, y0 = I.lorenz_random(m, seed=seed)
    t0 = time.perf_counter()
    O.rk4(O.LORENZ, P, sh, y0, dt, nsteps, nthreads=threads)
    el = time.perf_counter() - t0
    return {"value": m * nsteps / el, "unit": "system-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {m} of the {n_total} systems, all {nsteps} steps, {el:.1f} s"}


def cpu_simd_baseline(n_total, nsteps, dt, seed, target_s=6.0):
    """Context beside the oracle: the vectorised, unrolled CPU code of the
    same workload (bench_cpu, the paper's Sec. 3.1 CPU techniques) on the
    first m systems of the same seeded ensemble, m sized for ~target_s."""
    import bench_cpu as B
    from paper_2011_01740_amd import inputs as I

    threads = max(1, min(os.cpu_count() or 1, 16))
    probe = 4096 * threads
    P, y0 = I.lorenz_random(probe, seed=seed)
    t0 = time.perf_counter()
    B.lorenz_rk4(P, y0, dt, nsteps, I.LORENZ_SIGMA, I.LORENZ_BETA, threads)
    dt_probe = time.perf_counter() - t0
    m = int(probe * max(1.0, target_s / max(dt_probe, 1e-3)))
    m = max(probe, min(m, n_total))
    P, y0 = I.lorenz_random(m, seed=seed)
    t0 = time.perf_counter()
    B.lorenz_rk4(P, y0, dt, nsteps, I.LORENZ_SIGMA, I.LORENZ_BETA, threads)
    el = time.perf_counter() - t0
    rate = m * nsteps / el
    return {"value": rate, "unit": "system-steps/s", "cores": threads,
            "kind": "vectorised CPU code (8-wide FP64 SIMD, 4 vectors per iteration, OpenMP)",
            "gflops": FLOP_PER_STEP * rate / 1e9,
            "sample": f"first {m} of the {n_total} systems, all {nsteps} steps, {el:.1f} s"}


def _threads():
    return max(1, min(os.cpu_count() or 1, 16))


def km_cpu_baseline(G, n_phases, side, solver="ck", shared=None):
    """The oracle on a side x side sub-grid (evenly spaced rows and columns)
    of the G x G Keller--Miksis grid, all n_phases cycles."""
    import numpy as np

    import oracle as O
    from paper_2011_01740_amd import inputs as I
    P, y0 = I.km_grid(G, G)
    rows = np.linspace(0, G - 1, side).round().astype(np.int64)
    idx = (rows[:, None] * G + rows[None, :]).ravel()
    th = _threads()
    t0 = time.perf_counter()
    scheme = O.DORMAND_PRINCE if solver == "dp" else O.CASH_KARP
    sh = I.KM_WATER if shared is None else shared
    a = O.rkck45(O.KM, P[:, idx], sh, y0[:, idx],
                 O.Opts(n_phases=n_phases, n_record=1, scheme=scheme), nthreads=th)
    el = time.perf_counter() - t0
    steps = float(a.stats[O.ST_ACCEPTED].sum() + a.stats[O.ST_REJECTED].sum())
    return {"value": steps / el, "unit": "attempted steps/s", "cores": th, "kind": "oracle",
            "sample": f"{side} x {side} evenly spaced points of the {G} x {G} grid, all "
                      f"{n_phases} cycles, {el:.1f} s"}


def prv_cpu_baseline(ensembles, m_each, solver="ck"):
    """The oracle on the first m_each systems of each valve ensemble, with the
    ensemble's budget."""
    import numpy as np

    import oracle as O
    from paper_2011_01740_amd import inputs as I
    from paper_2011_01740_amd import workloads as W
    P, y0, off = W.prv_inputs(ensembles)
    th = _threads()
    steps, el = 0.0, 0.0
    for k, (m, K, _) in enumerate(ensembles):
        sl = slice(off[k], off[k] + min(m, m_each))
        t0 = time.perf_counter()
        a = O.rkck45(O.PRV, P[:, sl], I.PRV_DEFAULT, y0[:, sl],
                     O.Opts(n_phases=K, n_record=1, max_impacts=K,
                            scheme=O.DORMAND_PRINCE if solver == "dp" else O.CASH_KARP),
                     nthreads=th)
        el += time.perf_counter() - t0
        steps += float(a.stats[O.ST_ACCEPTED].sum() + a.stats[O.ST_REJECTED].sum()
                       + a.stats[O.ST_EVRETRY].sum())
    return {"value": steps / el, "unit": "attempted steps/s", "cores": th, "kind": "oracle",
            "sample": f"first {m_each} systems of each ensemble with its budget, {el:.1f} s"}


def lane_busy(steps, att, launch):
    """Share of the lane-attempt slots of an adaptive launch that carried an
    attempt: attempted steps / (resident lanes x the longest system's
    attempts), taking every attempt as equally long.  1 means no lane idled
    while the longest system ran; the rest is the tail."""
    lanes = int(launch["grid"]) * int(launch["block"])
    return float(steps) / max(lanes * int(att.max()), 1)


def km_sweep_line(args):
    """The Keller--Miksis sweep of the paper's Sec. 4.2 study on a 512 x 512
    (p_A, f) grid, 1024 acoustic cycles, per-cycle maximum radius: a 16-cycle
    pilot in index order, then the rest with the queue longest-first.  Timed
    around the two launches (HIP events) and on the wall clock; the oracle
    beside it on an evenly spaced sub-grid."""
    from paper_2011_01740_amd import workloads as W
    r = W.km_sweep(args.km_grid, args.km_grid, n_phases=args.km_phases, n_record=64,
                   pilot=16, pilot_grid=256)
    att = r.stats[0] + r.stats[1]
    steps = int(att.sum())
    line = {"workload": f"keller_miksis_rkck45_{args.km_grid}x{args.km_grid}x{args.km_phases}",
            "systems": args.km_grid * args.km_grid, "cycles": args.km_phases,
            "time_s": r.kernel_ms / 1e3, "wall_s": r.wall_s,
            "attempted_steps": steps, "attempted_steps_per_s": steps / r.kernel_ms * 1e3,
            "accepted_steps_per_s": float(r.stats[0].sum()) / r.kernel_ms * 1e3,
            "rhs_per_s": float(r.stats[2].sum()) / r.kernel_ms * 1e3,
            "attempts_max_over_mean": float(att.max() / max(att.mean(), 1e-30)),
            "lane_busy_fraction": lane_busy(steps, att, r.launch),
            "status_ok_frac": float(((r.status & ~1) == 0).mean()),
            "launch": r.launch}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = km_cpu_baseline(args.km_grid, args.km_phases, 16)
    return line


def km_screened_line(args):
    """The surrogate-screened 4096 x 4096 Keller--Miksis sweep (training sweep
    of the 512 x 512 grid, network training, calibration, screening, re-solve)
    against the plain FP64 sweep of all 2^24 points, which also judges every
    screened label; plus the screen without the network beside it."""
    from paper_2011_01740_amd import surrogate as S
    cfg = S.Config(train_grid=args.km_grid, screen_grid=args.sur_screen,
                   n_phases=args.km_phases, epochs=args.sur_epochs, judge_n=0,
                   target_wrong=args.sur_target)
    rep = S.run(cfg, log=lambda *a: print(*a, file=sys.stderr, flush=True))
    return {"workload": f"keller_miksis_screened_{args.sur_screen}x{args.sur_screen}",
            "points": rep.n_screen, "plain_s": rep.plain_time_s,
            "screened_s": rep.screened_time_s, "speedup": rep.speedup,
            "speedup_excl_training_sweep": rep.speedup_excl_data,
            "wrong_frac": rep.judge_wrong_frac, "resolve_frac": rep.resolve_frac,
            "network_alone_wrong_frac": rep.network_only_wrong_frac,
            "judged_points": rep.judge_points, "times_s": rep.times_s,
            "screen_rule": rep.extra.get("rule", "network"),
            "compare": rep.compare}


def run_case(case, args):
    """Single launches for counter runs: a 1 GiB device copy (the scale of the
    FETCH_SIZE / WRITE_SIZE counters), a Keller--Miksis grid, or the valve
    batch with reduced budgets.  Prints one JSON line."""
    import torch

    from paper_2011_01740_amd import workloads as W

    torch.cuda.set_device(0)
    if case == "copy":
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.fill_(0.0)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"case": "copy", "bytes_read": a.numel() * 8,
                          "bytes_written": a.numel() * 8}), flush=True)
    elif case == "km":
        from paper_2011_01740_amd import ens
        import numpy as np

        from paper_2011_01740_amd import inputs as I
        solver = ens.ENS_RKDP45 if args.solver == "dp" else ens.ENS_RKCK45
        sh = list(I.KM_WATER)
        sh[8], sh[9], sh[10] = args.km_pa2, args.km_f2, args.km_theta
        r = W.km_sweep(args.km_grid, args.km_grid, n_phases=args.km_phases,
                       n_record=args.km_record or None, pilot=args.km_pilot,
                       pilot_grid=args.km_blocks, solver=solver, shared=sh,
                       tangent=args.km_tangent)
        att = r.stats[0] + r.stats[1]
        steps = int(att.sum())
        line = {"case": "km", "solver": args.solver, "grid": args.km_grid,
                "phases": args.km_phases,
                "second_drive": {"P_A2": args.km_pa2, "f2": args.km_f2, "theta": args.km_theta},
                "tangent": bool(args.km_tangent),
                "pilot": args.km_pilot, "blocks_after_pilot": args.km_blocks,
                "kernel_ms": r.kernel_ms, "attempted_steps": steps,
                "steps_per_s": steps / r.kernel_ms * 1e3,
                "accepted_per_s": float(r.stats[0].sum()) / r.kernel_ms * 1e3,
                "rhs_per_s": float(r.stats[2].sum()) / r.kernel_ms * 1e3,
                "attempts_max_over_mean": float(att.max() / max(att.mean(), 1e-30)),
                "attempts_max": int(att.max()),
                "lane_busy_fraction": lane_busy(steps, att, r.launch),
                "us_per_attempt_longest": r.kernel_ms * 1e3 / max(int(att.max()), 1),
                "launch": r.launch}
        if args.km_tangent:
            # largest Lyapunov exponent per system: mean log growth per unit tau
            lam = r.records[:, 1, :].mean(axis=0)
            line["lyapunov"] = {"positive_fraction": float((lam > 0).mean()),
                                "max": float(lam.max()), "median": float(np.median(lam))}
        if args.cpu_sample:
            line["cpu_baseline"] = km_cpu_baseline(args.km_grid, args.km_phases, args.cpu_sample,
                                                   args.solver, sh)
        print(json.dumps(line), flush=True)
    elif case == "surrogate":
        from paper_2011_01740_amd import surrogate as S
        cfg = S.Config(train_grid=args.sur_train, screen_grid=args.sur_screen,
                       n_phases=args.sur_phases, epochs=args.sur_epochs, judge_n=args.sur_judge,
                       target_wrong=args.sur_target)
        rep = S.run(cfg, log=lambda *a: print(*a, file=sys.stderr, flush=True))
        d = {k: v for k, v in rep.__dict__.items() if k != "extra"}
        d["case"] = "surrogate"
        print(json.dumps(d), flush=True)
    elif case == "screen":
        # the screening forward alone: the seeded network (the weights' values
        # do not change the work) over the sweep grid, timed with HIP events
        # on the handle's stream around each sur_screen call (the fused
        # network kernel, the three weight-layout kernels and the compaction)
        import numpy as np

        from paper_2011_01740_amd import inputs as I
        from paper_2011_01740_amd import sur
        G = args.sur_screen
        P, _ = I.km_grid(G, G)
        lo = np.array([P[0].min(), np.log(P[1].min())])
        hi = np.array([P[0].max(), np.log(P[1].max())])
        Pd = torch.from_numpy(P).cuda()
        st = torch.cuda.current_stream()
        times = []
        with sur.Surrogate(max_batch=4096, stream=st) as s:
            s.set_params(I.mlp_init(4))
            s.set_norm(lo, hi, np.zeros(64), np.ones(64))
            for rep in range(args.warmup + args.steps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(st)
                s.screen(Pd, 0.05, 0.5, 0.1)
                e1.record(st)
                e1.synchronize()
                if rep >= args.warmup:
                    times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        flop = SCREEN_FLOP_PER_POINT * G * G
        print(json.dumps({"case": "screen", "points": G * G, "screen_ms": ms,
                          "screen_ms_all": times, "mfma_flop": flop,
                          "tflops": flop / ms / 1e9,
                          "frac_of_bf16_peak": flop / ms / 1e9 / BF16_PEAK_TFLOPS}), flush=True)
    elif case == "micro":
        # the (B, N) table of the introductory example and its division and
        # sine variants: one JSON line per configuration
        from paper_2011_01740_amd import ens
        models = {"quad": ens.ENS_QUAD, "div": ens.ENS_DIV, "sin": ens.ENS_SIN}
        for name in args.micro_models.split(","):
            for n in (int(v) for v in args.micro_n.split(",")):
                for block in (int(v) for v in args.micro_blocks.split(",")):
                    for spl in (int(v) for v in args.micro_spl.split(",")):
                        W.scalar_rk4(models[name], min(n, 4096), 10, block=block, spl=spl)
                        r = W.scalar_rk4(models[name], n, args.micro_steps, block=block, spl=spl)
                        rate = n * args.micro_steps / r.kernel_ms * 1e3
                        line = {"case": "micro", "model": name, "n": n, "block": block,
                                "spl": spl, "n_steps": args.micro_steps,
                                "kernel_ms": r.kernel_ms, "system_steps_per_s": rate}
                        if name == "quad":
                            # 11 FMA per step in the accumulated stage form
                            line["tflops"] = 22.0 * rate / 1e12
                            line["frac_of_spec_fp64"] = 22.0 * rate / 78.6e12
                        print(json.dumps(line), flush=True)
    elif case == "prv":
        from paper_2011_01740_amd import ens
        ensm = tuple((m, max(1, K // args.prv_div), sd) for m, K, sd in W.PRV_ENSEMBLES)
        if args.prv_n:   # one ensemble of the first sub-ensemble's kind (latency studies)
            ensm = ((args.prv_n, max(1, W.PRV_ENSEMBLES[0][1] // args.prv_div),
                     W.PRV_ENSEMBLES[0][2]),)
        launch = {"grid": args.prv_grid} if args.prv_grid else {}
        r = W.prv_batched(ensm, solver=ens.ENS_RKDP45 if args.solver == "dp" else None,
                          spread=args.prv_spread if args.prv_spread >= 0 else None, **launch)
        steps = int(r.stats[0].sum() + r.stats[1].sum() + r.stats[5].sum())
        att = r.stats[0] + r.stats[1] + r.stats[5]
        line = {"case": "prv", "solver": args.solver, "budget_divisor": args.prv_div,
                "ensembles": [list(e) for e in ensm],
                "attempts_max": int(att.max()),
                "lane_busy_fraction": lane_busy(steps, att, r.launch),
                "us_per_attempt_longest": r.kernel_ms * 1e3 / max(int(att.max()), 1),
                "kernel_ms": r.kernel_ms, "attempted_steps": steps,
                "steps_per_s": steps / r.kernel_ms * 1e3,
                "impacts_per_s": float(r.stats[3].sum()) / r.kernel_ms * 1e3,
                "phases_per_s": float(r.stats[4].sum()) / r.kernel_ms * 1e3,
                "launch": r.launch}
        if args.cpu_sample:
            line["cpu_baseline"] = prv_cpu_baseline(ensm, args.cpu_sample, args.solver)
        print(json.dumps(line), flush=True)
    else:
        r = W.lorenz(args.n, args.n_steps, block=args.block, spl=args.spl)
        print(json.dumps({"case": "lorenz", "n": args.n, "n_steps": args.n_steps,
                          "kernel_ms": r.kernel_ms,
                          "system_steps_per_s": args.n * args.n_steps / r.kernel_ms * 1e3}),
              flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--case", choices=["bench", "lorenz", "km", "prv", "copy", "surrogate", "micro",
                                       "screen"],
                    default="bench",
                    help="bench: the benchmark line; others: one launch for counter runs")
    ap.add_argument("--km-grid", type=int, default=512)
    ap.add_argument("--km-phases", type=int, default=1024)
    ap.add_argument("--km-pilot", type=int, default=0,
                    help="cycles before the longest-first queue order (0: one solve)")
    ap.add_argument("--km-blocks", type=int, default=0,
                    help="persistent blocks after the pilot (0: resident capacity)")
    ap.add_argument("--km-record", type=int, default=0, help="record ring (0: all cycles)")
    ap.add_argument("--micro-models", default="quad,div,sin")
    ap.add_argument("--micro-n", default="65536",
                    help="comma-separated ensemble sizes for --case micro")
    ap.add_argument("--micro-blocks", default="256", help="comma-separated block sizes")
    ap.add_argument("--micro-spl", default="1", help="comma-separated systems per lane")
    ap.add_argument("--micro-steps", type=int, default=1000)
    ap.add_argument("--km-pa2", type=float, default=0.0,
                    help="second drive amplitude P_A2 [Pa] (0: single frequency)")
    ap.add_argument("--km-f2", type=float, default=0.0, help="second drive frequency f2 [Hz]")
    ap.add_argument("--km-theta", type=float, default=0.0, help="second drive phase shift [rad]")
    ap.add_argument("--km-tangent", action="store_true",
                    help="integrate the variational equation (largest Lyapunov exponent)")
    ap.add_argument("--solver", choices=["ck", "dp"], default="ck",
                    help="km/prv cases: Cash--Karp or Dormand--Prince 5(4)")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="km/prv cases: time the oracle on a sample (km: side of a sub-grid, "
                         "prv: systems per ensemble; 0: off)")
    ap.add_argument("--prv-div", type=int, default=100)
    ap.add_argument("--prv-n", type=int, default=0,
                    help="one valve ensemble of this size (the first ensemble's budget / div)")
    ap.add_argument("--prv-grid", type=int, default=0, help="persistent blocks (0: capacity)")
    ap.add_argument("--prv-spread", type=int, default=-1,
                    help="queue head spread one wave per SIMD (-1: the first ensemble)")
    ap.add_argument("--sur-train", type=int, default=512)
    ap.add_argument("--sur-screen", type=int, default=4096)
    ap.add_argument("--sur-phases", type=int, default=1024)
    ap.add_argument("--sur-epochs", type=int, default=200)
    ap.add_argument("--sur-judge", type=int, default=0)   # 0: every point (the plain time)
    ap.add_argument("--sur-target", type=float, default=0.002,
                    help="hold-out wrong fraction the screening flags are calibrated to")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 23)
    ap.add_argument("--n-steps", type=int, default=10000)
    ap.add_argument("--dt", type=float, default=0.01)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--spl", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-km", action="store_true",
                    help="leave the Keller--Miksis sweep and the screened sweep out of the line")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path. "
              "The systems are independent, so an ensemble would shard by contiguous "
              "index ranges, one process per GPU.", file=sys.stderr)
        return 2
    if args.case != "bench":
        return run_case(args.case, args)

    import torch

    from paper_2011_01740_amd import ens
    from paper_2011_01740_amd import inputs as I

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    n, nsteps, dt, seed = args.n, args.n_steps, args.dt, 1

    P, y0 = I.lorenz_random(n, seed=seed)
    P_d = torch.from_numpy(P).to(dev)
    y0_d = torch.from_numpy(y0).to(dev)
    stream = torch.cuda.current_stream(dev)
    e = ens.Ensemble(ens.ENS_LORENZ, ens.ENS_RK4, n, stream=stream)
    e.set_params(P_d)
    opts = ens.default_opts(dt=dt, n_steps=nsteps, block=args.block, spl=args.spl)
    tuned_ms = None
    if not args.block and not args.spl:
        # library autotuner on trials of 1000 steps of this problem (untimed;
        # ~10 ms each, so that run-to-run noise stays below its 2% margin)
        e.set_state(y0_d)
        opts, tuned_ms = e.tune(opts, trial_len=1000)

    for _ in range(args.warmup):
        e.set_state(y0_d)
        e.solve(opts)
    torch.cuda.synchronize()

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        e.set_state(y0_d)
        evs[k][0].record(stream)
        e.solve(opts)
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    avg_kern_s = sum(kern_ms) / len(kern_ms) / 1e3
    launch = e.last_launch()
    ymax = e.read(ens.ENS_ACC, device=True)
    finite = bool(torch.isfinite(ymax).all().item())
    e.close()
    # the FP64 FMA rate the chip sustains (independent FMA chains): the peak
    # the clock under dense FP64 load allows, beside the published one
    fma_tflops, _ = ens.micro_fma(0, 1 << 16)

    sys_steps = n * nsteps
    value = sys_steps * args.steps / wall
    achieved = FLOP_PER_STEP * sys_steps / avg_kern_s / 1e12
    hw_tflops = HW_FLOP_PER_STEP * sys_steps / avg_kern_s / 1e12   # as the chain counts
    line = {
        "metric": "system-steps/s",
        "value": value,
        "unit": "system-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "lorenz_rk4_fixed_step", "systems": n, "rk4_steps": nsteps,
                   "dt": dt, "p_range": [0.0, 21.0], "ic": "10 + U[-1,1]", "seed": seed,
                   "block": launch["block"], "systems_per_lane": launch["spl"],
                   "autotuned": tuned_ms is not None},
        "fp64_peak_frac": achieved / FP64_PEAK_TFLOPS,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(n, nsteps),
                     "fma_chain_tflops": fma_tflops,
                     "hardware_flop_per_step": HW_FLOP_PER_STEP,
                     "hardware_tflops": hw_tflops,
                     "frac_of_fma_chain": hw_tflops / fma_tflops,
                     "kernel": "k_rk4_lorenz", "kernel_ms": avg_kern_s * 1e3,
                     "algorithmic_flop_per_launch": FLOP_PER_STEP * sys_steps,
                     "algorithmic_bytes_per_launch": BYTES_PER_SYSTEM * n},
        "finite": finite,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(n, nsteps, dt, seed)
        try:
            line["cpu_simd"] = cpu_simd_baseline(n, nsteps, dt, seed)
        except (OSError, RuntimeError) as exc:   # context only: never fail the line
            line["cpu_simd"] = {"error": str(exc)}
    if not args.no_km:
        print("bench: Keller--Miksis sweep", file=sys.stderr, flush=True)
        line["km_sweep"] = km_sweep_line(args)
        print("bench: screened Keller--Miksis sweep and its plain sweep", file=sys.stderr,
              flush=True)
        line["km_screened"] = km_screened_line(args)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
