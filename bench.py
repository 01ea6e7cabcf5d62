#!/usr/bin/env python3
"""Benchmark of the exponential propagator's hot path on one MI355X.

Workload (default): linear steel cantilever 80x8x8 hex8 (6,561 nodes, 19,440 free DOFs),
E = 200 GPa, nu = 0.3, rho = 7800, x = 0 clamped, tip traction 1e5 Pa (-z), initial
velocity N(0, (1e-3 m/s)^2) per free DOF (seed 0), dt = 1e-4 s, Krylov tol 1e-10, FP64.
As in the paper's production runs (Sec. 6.2), the subspace size is calibrated on the
warm-up steps by the adaptive error estimate and then held fixed for the timed steps.

One JSON line on stdout.  value = DOF-matvecs/s = free DOFs x Hbar applications / s.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--dt", type=float, default=1e-4)
    ap.add_argument("--m-max", type=int, default=64)
    ap.add_argument("--precision", default="f64", choices=["f64", "mixed_f32"])
    ap.add_argument("--workgroups", type=int, default=0)
    ap.add_argument("--adaptive", action="store_true", help="keep the adaptive subspace choice while timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(prob, n_free, m, k, s_x=8):
    """Algorithmic HBM bytes of one projection launch (k substeps of m Arnoldi steps).

    Operator apply (per application): read x (u- and v-part, 2*3n), write y (2*3n),
    connectivity (32 B per element), M^{-1/2} (3n) and the load vector (3n).
    Arnoldi-MGS (per projection): step j reads v_1..v_j and writes v_{j+1}: L*m(m+1)/2 reads
    and L*(m+1) writes; the combination reads m vectors and writes one.  L = 2*3n + 1.
    """
    n3 = 3 * prob.n_nodes
    L = 2 * n3 + 1
    per_mv = (4 * n3 + 2 * n3) * s_x + 32 * prob.n_elems
    per_proj = m * per_mv + s_x * L * (m * (m + 1) // 2 + (m + 1) + m + 1)
    return k * per_proj


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "described in DESIGN.md but not built)"}))
        sys.exit(2)
    import torch
    from workloads import config
    from paper_2405_05213_amd import solver_from_problem

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    over = {"dt": args.dt}
    prob = config(args.config, **over)
    n_free = prob.n_free
    stream = torch.cuda.current_stream()

    # --- calibration on the warm-up steps: adaptive m (error estimate), then fixed m
    cal = solver_from_problem(prob, m_max=args.m_max, precision=args.precision, workgroups=args.workgroups,
                              stream=stream.cuda_stream)
    nwarm = max(1, args.warmup)
    cal.step(prob.dt, nwarm)
    cal.sync()
    lg = cal.step_log(nwarm)
    m_cal = int(lg["m_corr"][-1])
    k_cal = int(lg["k_corr"][-1])
    log(args, f"calibrated: m={m_cal} k={k_cal} (eps {lg['eps_corr'][-1]:.2e})")
    if args.adaptive:
        ctx = cal
    else:
        del cal
        ctx = solver_from_problem(prob, m_max=args.m_max, m_fixed=m_cal, k_fixed=k_cal, precision=args.precision,
                                  workgroups=args.workgroups, stream=stream.cuda_stream)
        ctx.step(prob.dt, nwarm)
    ctx.sync()
    e_ref = ctx.energy()
    st0 = ctx.stats()

    # --- timed steps: HIP events on the stream the kernels run on
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        ctx.step(prob.dt, 1)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.sync()
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    gpu_s = float(step_ms.sum()) / 1e3
    st1 = ctx.stats()
    matvecs = st1["matvecs"] - st0["matvecs"]
    ke, se, we = ctx.energy()
    e0 = e_ref[0] + e_ref[1] - e_ref[2]
    e1 = ke + se - we
    e_scale = max(e_ref[0] + e_ref[1], ke + se)
    energy_err = abs(e1 - e0) / e_scale
    dof_mv_s = n_free * matvecs / gpu_s
    steps_s = args.steps / gpu_s

    # --- roofline of the dominant kernel (the persistent projection kernel, one launch per step)
    m_used = st1["m"]
    k_used = st1["k"]
    alg = algorithmic_bytes(prob, n_free, m_used, k_used)
    launch_s = float(np.mean(step_ms)) / 1e3
    achieved = alg / launch_s / 1e9
    result = {
        "metric": "DOF-matvecs/s (+ time-steps/s) at fixed energy error",
        "value": dof_mv_s,
        "unit": "DOF-matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(np.mean(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "f64" else "f64 (Krylov) / f32 (operator)",
        "data": "synthetic",
        "config": {
            "workload": f"{args.config}: linear steel cantilever {prob.grid[0]}x{prob.grid[1]}x{prob.grid[2]} hex8, "
                        f"{n_free} free DOFs, dt={prob.dt:g} s, tol={prob.tol:g}",
            "dt": prob.dt, "m": m_used, "substeps": k_used, "m_mode": "adaptive" if args.adaptive else
            "calibrated then fixed", "precision": args.precision, "free_dofs": n_free,
        },
        "time_steps_per_s": steps_s,
        "energy_rel_err": energy_err,
        "wall_s": wall,
        "roofline": {
            "kernel": "k_expv (persistent Arnoldi-MGS projection incl. operator applies)",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "alg_bytes_per_launch": alg, "avg_launch_ms": launch_s * 1e3,
        },
    }

    # --- the oracle on the host cores, a bounded sample of the same workload
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(prob, m_used, k_used, args)
    print(json.dumps(result))


def cpu_baseline(prob, m, k, args):
    from threadpoolctl import threadpool_limits
    from oracle.stepper import Propagator
    with threadpool_limits(1):
        orc = Propagator(prob, m_max=max(m, 1), m_fixed=m, k_fixed=k)
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds or n == 0:
            orc.step(prob.dt)
            n += 1
        dt = time.perf_counter() - t0
    return {"value": prob.n_free * orc.matvecs / dt, "unit": "DOF-matvecs/s", "cores": 1, "kind": "oracle",
            "time_steps_per_s": n / dt,
            "sample": f"{n} steps of the same workload (m={m}, k={k} fixed) by the NumPy FP64 oracle, 1 thread, "
                      f"{platform.processor() or platform.machine()}"}


if __name__ == "__main__":
    main()
