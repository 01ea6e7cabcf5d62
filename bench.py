#!/usr/bin/env python3
"""Benchmark of the exponential propagator's hot path on one MI355X.

Headline workload (the metric's own configuration): 256 independent compressible
Neo-Hookean rubber blocks of uneven size (nx ~ U{20..60}, ny = nz ~ U{4..8}, 1 cm cells;
mu ~ U[0.2, 1] MPa, lambda = 5 mu, rho 1100; x = 0 clamped; constant tip traction
~ U[1e3, 1e4] Pa in -z; from rest; seed 5), advanced together by one persistent launch per
time step (captured graph), dt = 6.25e-6 s, 1000 steps, Krylov tol 1e-10 with the augmented
entry at each block's scale, adaptive subspace per instance.
The mixed form (FP32 operator, FP64 Krylov / exponential / state) is timed, and the plain
FP64 form on the same instances, the same dt and the same steps beside it; both report the
relative energy error (from rest under a constant load, E_0 = 0:
|KE + SE - W| / (KE + SE)), which must be <= 1e-6 for the comparison to hold.

value = DOF-matvecs/s of the mixed batch = sum over instances of free DOFs x Hbar
applications / s; time-steps/s (batch steps) and instance-steps/s beside it.
roofline: the batch kernel k_batch (one launch per step), algorithmic bytes per launch from
the per-instance operator and Gram-Schmidt traffic, over its average launch duration.
cpu_baseline: the FP64 oracle on 16 instances spanning the sizes, in parallel worker
processes (one thread each), for a bounded time; extrapolated to the batch as a rate.
Extras (labelled): the single-instance workloads (steel cantilever 80x8x8, Neo-Hookean
cantilever 160x16x16, Yeoh 64^3 block) on short step subsets, stand-alone operator applies
(incl. a 192^3 cube beyond the Infinity Cache) and the BF16 tangent formation.
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


# Arnoldi steps between a-priori error estimates in the timed adaptive runs: an estimate at
# every step stops each projection at the first size that meets the tolerance, and costs
# less than the Arnoldi steps that a sparser check runs past that size
CHECK_EVERY = 1


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed batch steps (the workload's 1000)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--instances", type=int, default=256, help="batch size of the headline workload")
    ap.add_argument("--batch-dt", type=float, default=6.25e-6)
    ap.add_argument("--batch-m-max", type=int, default=32)
    ap.add_argument("--headline-only", action="store_true", help="only the batch (profiling)")
    ap.add_argument("--config", default="c2", help="single-instance workload of the extras")
    ap.add_argument("--dt", type=float, default=1e-4)
    ap.add_argument("--m-max", type=int, default=64)
    ap.add_argument("--check-every", type=int, default=CHECK_EVERY,
                    help="Arnoldi steps between a-priori error checks in the adaptive runs")
    ap.add_argument("--precision", default="f64", choices=["f64", "mixed_f32", "mixed_bf16"])
    ap.add_argument("--workgroups", type=int, default=0)
    ap.add_argument("--autotune-steps", type=int, default=5,
                    help="steps over which the plan autotuner times each candidate plan")
    ap.add_argument("--no-batch-autotune", action="store_true",
                    help="keep one workgroup per batch instance (no plan autotuning)")
    ap.add_argument("--ortho", type=int, default=-1, choices=[-1, 0, 1],
                    help="Gram-Schmidt form: -1 automatic, 0 sequential, 1 compact WY")
    ap.add_argument("--adaptive", action="store_true", help="keep the adaptive subspace choice while timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extra", action="store_true", help="only the headline workload")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--matvec-only", action="store_true",
                    help="only the stand-alone FP64 operator applies on the 64^3 and 128^3 cubes (profiling)")
    ap.add_argument("--schemes-only", action="store_true",
                    help="only the second- vs fourth-order comparison on the Neo-Hookean cantilever")
    ap.add_argument("--tangents-only", action="store_true",
                    help="only the BF16 tangent formation / apply on the 64^3 Yeoh block (profiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run 3 device copies of 256 MiB (counter calibration under rocprofv3 --pmc)")
    return ap.parse_args()


def copy_probe(torch):
    """A plain device-to-device copy of known size: 256 MiB read + 256 MiB written per dispatch."""
    a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(prob, m, k, s_x=8, projections=1):
    """Algorithmic HBM bytes of one single-instance projection launch (k substeps of m
    Arnoldi steps), as the batch's per instance: operator apply = read x, write y (2 * 3n
    values of s_x bytes), connectivity (32 B per element), M^{-1/2} (3n values); Arnoldi-MGS
    on L = 2 N_free + 1 FP64 entries reads L m(m+1)/2 and writes L (m+1) doubles, the
    combination reads m vectors."""
    n3 = 3 * prob.n_nodes
    L = 2 * prob.n_free + 1
    per_mv = (2 * n3 + n3) * s_x + 32 * prob.n_elems
    per_proj = m * per_mv + 8 * L * (m * (m + 1) // 2 + (m + 1) + m)
    return projections * k * per_proj


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_batch_c5_rubber256_mixed_traffic.json")


def measured_traffic(workload, precision):
    """HBM bytes per launch of the batch kernel from the committed rocprofv3 counter runs
    (FETCH_SIZE / WRITE_SIZE scaled by a copy kernel of known size), or None when the kernel
    sources or the workload differ from the profiled ones."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    from paper_2405_05213_amd.profsum import batch_kernel_sha256
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    same = (rec.get("kernel_sources_sha256") == batch_kernel_sha256() and rec.get("workload") == workload
            and rec.get("precision") == precision)
    return float(rec["traffic_bytes_per_launch"]) if same else None


def energy_err(e0, e1):
    E0 = e0[0] + e0[1] - e0[2]
    E1 = e1[0] + e1[1] - e1[2]
    scale = max(e0[0] + e0[1], e1[0] + e1[1], 1e-300)
    return abs(E1 - E0) / scale


def timed_steps(ctx, dt, steps, stream, torch):
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        ctx.step(dt, 1)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return ms, wall


def run_single(prob, precision, steps, warmup, m_max, workgroups, adaptive, stream, torch, args):
    """Calibrate m on the warm-up steps, then time `steps` steps with m (and k) fixed."""
    from paper_2405_05213_amd import solver_from_problem
    cal = solver_from_problem(prob, m_max=m_max, check_every=args.check_every, precision=precision,
                              workgroups=workgroups,
                              stream=stream.cuda_stream, ortho=args.ortho)
    nwarm = max(1, warmup)
    cal.step(prob.dt, nwarm)
    cal.sync()
    lg = cal.step_log(nwarm)
    m_cal, k_cal = int(lg["m_corr"][-1]), int(lg["k_corr"][-1])
    m_pred = int(lg["m_pred"][-1])
    tuned_G = workgroups
    if workgroups == 0:
        # the project's autotuner picks the team size of the persistent kernel
        tuned_G, tuned_ms = cal.autotune(prob.dt, m_trial=max(8, min(m_cal, 48)), trials=5)
        log(args, f"  {prob.name} {precision}: autotuned workgroups = {tuned_G} ({tuned_ms:.3f} ms/projection)")
    if adaptive:
        ctx = cal
    else:
        cal.close()
        ctx = solver_from_problem(prob, m_max=m_max, check_every=args.check_every,
                                  m_fixed=max(m_cal, m_pred), k_fixed=k_cal,
                                  precision=precision, workgroups=tuned_G, stream=stream.cuda_stream,
                                  ortho=args.ortho)
        ctx.step(prob.dt, nwarm)
    ctx.sync()
    e_ref = ctx.energy() if prob.model == "linear" else (0.0, 0.0, 0.0)
    st0 = ctx.stats()
    ms, wall = timed_steps(ctx, prob.dt, steps, stream, torch)
    ctx.sync()
    st1 = ctx.stats()
    e1 = ctx.energy()
    if prob.model != "linear":
        # time-varying load: the energy balance is not conserved; report the drift of a
        # restart from the calibrated state instead (same definition for both precisions)
        e_ref = e1
    gpu_s = float(ms.sum()) / 1e3
    mv = st1["matvecs"] - st0["matvecs"]
    log(args, f"  {prob.name} {precision}: m={st1['m']} k={st1['k']} {np.mean(ms):.3f} ms/step")
    return {
        "ms_per_step": float(np.mean(ms)), "time_steps_per_s": steps / gpu_s,
        "dof_matvecs_per_s": prob.n_free * mv / gpu_s, "m": st1["m"], "k": st1["k"],
        "m_fixed": max(m_cal, m_pred), "energy_rel_err": energy_err(e_ref, e1) if prob.model == "linear" else None,
        "matvecs": mv, "wall_s": wall, "step_ms": ms, "ctx": ctx, "workgroups": tuned_G,
        "ortho": ctx.orthogonalization(),
    }


def run_matvec(prob, u_lin, reps, stream, torch, args):
    """Stand-alone operator apply y = H(u) x (FP64).  `reps` applies are captured in one
    graph on a side stream (a single apply takes less time than a host-side launch), the
    graph is replayed and timed with events; the replayed result is checked against the
    eager one.  Algorithmic bytes of one apply: read x and write y (3 n_n doubles each),
    plus the connectivity (32 B per element) on paths that read it, plus u (3 n_n doubles)
    for a secant material."""
    from paper_2405_05213_amd import solver_from_problem
    side = torch.cuda.Stream()
    ctx = solver_from_problem(prob, m_max=4, stream=side.cuda_stream)
    n3 = 3 * prob.n_nodes
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    x = torch.randn(n3, dtype=torch.float64, device="cuda", generator=gen)
    y = torch.zeros_like(x)
    u = None if u_lin is None else torch.as_tensor(u_lin, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ctx.apply_H(u, x, y)
    y_eager = y.clone()
    y.zero_()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        for _ in range(reps):
            ctx.apply_H(u, x, y, sync=False)
    graph.replay()
    side.synchronize()
    ok = bool(torch.equal(y, y_eager))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rounds = 5
    with torch.cuda.stream(side):
        e0.record(side)
        for _ in range(rounds):
            graph.replay()
        e1.record(side)
    side.synchronize()
    ctx.sync()
    us = e0.elapsed_time(e1) * 1e3 / (rounds * reps)
    workgroups, chunk, mesh_class = ctx.launch()
    npe = prob.conn.shape[1]
    if npe == 27:
        path, reads_conn = "Q2 element kernel (32 lanes per element) + slot gather", True
    elif prob.model == "linear" and mesh_class == 2:
        path, reads_conn = "lattice: 27-block stencil over LDS tiles + boundary faces", False
    elif prob.model == "linear" and mesh_class == 1:
        path, reads_conn = "node-by-node, stored element stiffness", True
    else:
        path, reads_conn = "element kernel + slot gather", True
    alg = (2 * n3 + (n3 if u is not None else 0)) * 8 + (4 * npe * prob.n_elems if reads_conn else 0)
    achieved = alg / (us * 1e-6) / 1e9
    log(args, f"  matvec {prob.name} {prob.model} {prob.grid}: {us:.2f} us/apply, {achieved:.0f} GB/s ({path})")
    del graph
    ctx.close()
    return {"us_per_apply": us, "dofs": n3, "elements": prob.n_elems, "path": path, "graph_replay_matches": ok,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "alg_bytes_per_apply": alg}}


BF16_DENSE_PEAK_TFLOPS = 2500.0


def run_tangents(prob, u_lin, reps, stream, torch, args):
    """BF16 element tangents: the formation alone (ep_form_tangents) and formation + apply
    (ep_apply_H), each captured `reps` times in a graph and replayed.  Algorithmic work of a
    formation: the shared-gradient product Psi (64 x 72) . Cbar (72 x 9) per element on the
    matrix cores (2 * 64 * 72 * 9 flops); its algorithmic bytes: u (3 n_n doubles) and the
    connectivity read, the tangents written (1152 B per element)."""
    from paper_2405_05213_amd import solver_from_problem
    side = torch.cuda.Stream()
    ctx = solver_from_problem(prob, m_max=4, precision="mixed_bf16", stream=side.cuda_stream)
    n3 = 3 * prob.n_nodes
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    x = torch.randn(n3, dtype=torch.float64, device="cuda", generator=gen)
    y = torch.zeros_like(x)
    u = torch.as_tensor(u_lin, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ctx.apply_H(u, x, y)
    y_eager = y.clone()
    out = {}
    for what in ("form", "form_apply"):
        y.zero_()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            for _ in range(reps):
                if what == "form":
                    ctx.form_tangents(u, sync=False)
                else:
                    ctx.apply_H(u, x, y, sync=False)
        graph.replay()
        side.synchronize()
        if what == "form_apply":
            out["graph_replay_matches"] = bool(torch.equal(y, y_eager))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(side):
            e0.record(side)
            for _ in range(5):
                graph.replay()
            e1.record(side)
        side.synchronize()
        out[f"us_per_{what}"] = e0.elapsed_time(e1) * 1e3 / (5 * reps)
        del graph
    ctx.sync()
    us = out["us_per_form"]
    flops = 2.0 * 64 * 72 * 9 * prob.n_elems
    alg_bytes = n3 * 8 + 32 * prob.n_elems + 1152 * prob.n_elems
    tf = flops / (us * 1e-6) / 1e12
    gbs = alg_bytes / (us * 1e-6) / 1e9
    log(args, f"  tangents {prob.name} {prob.grid}: form {us:.1f} us ({tf:.1f} TFLOP/s, {gbs:.0f} GB/s), "
              f"form+apply {out['us_per_form_apply']:.1f} us")
    out.update({
        "elements": prob.n_elems,
        "us_per_apply_estimate": out["us_per_form_apply"] - us,
        "formation_mfma": {"bound": "hbm", "achieved_tflops": tf, "peak_tflops_bf16_dense": BF16_DENSE_PEAK_TFLOPS,
                           "frac_mfma": tf / BF16_DENSE_PEAK_TFLOPS, "achieved_gbs": gbs, "peak_gbs": HBM_PEAK_GBS,
                           "frac_hbm": gbs / HBM_PEAK_GBS, "flops_per_formation": flops,
                           "alg_bytes_per_formation": alg_bytes},
    })
    ctx.close()
    return out


def batch_algorithmic_bytes(probs, per_inst, s_x):
    """Algorithmic HBM bytes of one batch launch (one time step of every instance).

    Per operator apply of an instance (n = nodes, e = elements): read x, write y (2 * 3n
    values of s_x bytes), the connectivity (32 B per element), M^{-1/2} (3n values) and the
    nodal linearisation displacement (3n values; two sets in the predictor).  Per projection of
    size m on L = 2 N_free + 1 FP64 entries: Arnoldi-MGS reads L m(m+1)/2 and writes L (m+1)
    doubles, the combination reads m vectors.  per_inst: (m_corr, k_corr, m_pred, k_pred)."""
    tot = 0
    for p, (mc, kc, mp, kp) in zip(probs, per_inst):
        n3 = 3 * p.n_nodes
        L = 2 * p.n_free + 1
        mv = lambda sets: (2 * n3 + n3 + sets * n3) * s_x + 32 * p.n_elems
        mgs = lambda m: 8 * L * (m * (m + 1) // 2 + (m + 1) + m)
        tot += kc * (mc * mv(1) + mgs(mc)) + kp * (mp * mv(2) + mgs(mp))
    return tot


def run_batch(probs, precision, steps, warmup, m_max, stream, torch, args):
    from paper_2405_05213_amd import batch_from_problems
    from paper_2405_05213_amd.ep import S0_SCALED
    b = batch_from_problems(probs, m_max=m_max, check_every=args.check_every, precision=precision,
                            stream=stream.cuda_stream, s0=S0_SCALED)
    dt = probs[0].dt
    plan = None
    if not getattr(args, "no_batch_autotune", False):
        # the project's plan autotuner: teams of workgroups for the costly blocks, lists of
        # cheap ones (states restored afterwards)
        wg, tuned_ms = b.autotune(dt, steps=getattr(args, "autotune_steps", 5))
        teams = [b.plan_of(i)[0] for i in range(len(probs))]
        plan = {"workgroups": wg, "max_team": max(teams), "instances_in_teams": sum(g > 1 for g in teams),
                "autotune_ms_per_step": tuned_ms}
        log(args, f"  batch {len(probs)} {precision}: plan {wg} workgroups, largest team {max(teams)}, "
                  f"{plan['instances_in_teams']} instances in teams ({tuned_ms:.3f} ms/step while tuning)")
    b.step(dt, max(1, warmup))
    b.sync()
    st0 = [b.stats(i) for i in range(len(probs))]
    ms, wall = timed_steps(b, dt, steps, stream, torch)
    b.sync()
    st1 = [b.stats(i) for i in range(len(probs))]
    gpu_s = float(ms.sum()) / 1e3
    n_free = np.array([p.n_free for p in probs])
    mv = np.array([a["matvecs"] - z["matvecs"] for a, z in zip(st1, st0)])
    mvp = np.array([a["matvecs_pred"] - z["matvecs_pred"] for a, z in zip(st1, st0)])
    # per-instance projection sizes over the timed steps (matvecs per projection)
    per_inst = []
    for i in range(len(probs)):
        kc, kp = max(1, st1[i]["k"]), max(1, st1[i]["k_pred"])
        mc = (mv[i] - mvp[i]) / (steps * kc)
        mp = mvp[i] / (steps * kp)
        per_inst.append((int(round(mc)), kc, int(round(mp)), kp))
    # constant loads from rest: E_0 = 0, so the energy error is |KE + SE - W| / (KE + SE)
    errs = np.array([energy_err((0.0, 0.0, 0.0), b.energy(i)) for i in range(len(probs))])
    alg = batch_algorithmic_bytes(probs, per_inst, 8 if precision == "f64" else 4)
    launch_ms = float(np.mean(ms))
    log(args, f"  batch {len(probs)} {precision}: {launch_ms:.3f} ms/step, energy err max {errs.max():.2e}")
    out = {
        "ms_per_step": launch_ms, "instance_steps_per_s": len(probs) * steps / gpu_s,
        "time_steps_per_s": steps / gpu_s,
        "dof_matvecs_per_s": float((n_free * mv).sum()) / gpu_s,
        "energy_rel_err_max": float(errs.max()), "energy_rel_err_median": float(np.median(errs)),
        "instances": len(probs), "total_free_dofs": int(n_free.sum()),
        "matvecs_per_step": float(mv.sum()) / steps,
        "m_corr_range": [min(q[0] for q in per_inst), max(q[0] for q in per_inst)],
        "m_pred_range": [min(q[2] for q in per_inst), max(q[2] for q in per_inst)],
        "alg_bytes_per_launch": alg, "wall_s": wall, "plan": plan,
    }
    b.close()
    return out


def _cpu_worker(args):
    """Oracle steps of one instance for about `seconds` (one thread); returns
    (free DOFs x H applications, steps, seconds)."""
    prob, seconds = args
    from threadpoolctl import threadpool_limits
    from oracle.stepper import Propagator
    with threadpool_limits(1):
        orc = Propagator(prob, m_max=32)
        n, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < seconds or n == 0:
            orc.step(prob.dt)
            n += 1
        el = time.perf_counter() - t0
    return prob.n_free * orc.matvecs, n, el


def cpu_baseline_batch(probs, seconds, args):
    """The FP64 oracle (as it stands) on 16 instances spanning the batch's sizes, one worker
    process per instance (one thread each), for about `seconds` each.  Run before the GPU is
    touched (the workers are forked)."""
    import multiprocessing as mp
    order = np.argsort([p.n_free for p in probs])
    pick = [probs[i] for i in order[np.linspace(0, len(probs) - 1, min(16, len(probs))).round().astype(int)]]
    procs = max(1, min(len(pick), os.cpu_count() or 1, 16))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_cpu_worker, [(p, seconds) for p in pick])
    wall = time.perf_counter() - t0
    dofmv = sum(r[0] for r in res)
    thread_s = sum(r[2] for r in res)
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    log(args, f"  cpu baseline: {dofmv / wall:.3e} DOF-matvecs/s on {procs} processes ({cpu})")
    return {"value": dofmv / wall, "unit": "DOF-matvecs/s", "cores": procs, "kind": "oracle",
            "per_thread_value": dofmv / thread_s,
            "instance_steps_per_s": sum(r[1] for r in res) / wall,
            "host_cpu": cpu, "host_logical_cpus": os.cpu_count(),
            "sample": (f"{len(pick)} of the {len(probs)} instances (evenly spaced in size, {pick[0].n_free}.."
                       f"{pick[-1].n_free} free DOFs), about {seconds:g} s of oracle steps each (dt, tol and "
                       f"m_max as the GPU run), NumPy FP64, one process and one thread per instance, "
                       f"{procs} processes in parallel; extrapolated to the whole batch as a rate")}


def batch_workload(probs, dt, m_max, check_every):
    nx = [p.grid[0] for p in probs]
    nyz = [p.grid[1] for p in probs]
    check = "at every Arnoldi step" if check_every == 1 else f"every {check_every} Arnoldi steps"
    return (f"c5: {len(probs)} compressible Neo-Hookean rubber blocks, hex8 nx {min(nx)}..{max(nx)} x "
            f"ny=nz {min(nyz)}..{max(nyz)}, {sum(p.n_free for p in probs)} free DOFs in all, dt={dt:g} s, "
            f"tol=1e-10 (augmented entry at each block's scale), m_max={m_max} adaptive per instance "
            f"(error estimate {check}), "
            f"one launch per step")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 (sharding over several "
                                   "GPUs is not built)"}))
        sys.exit(2)
    from workloads import config, batch_instances
    probs = batch_instances(args.instances, seed=5, dt=args.batch_dt)
    # the oracle on the host cores first: its worker processes are forked before the GPU is touched
    cpu = None
    if not (args.no_cpu or args.matvec_only or args.tangents_only or args.schemes_only):
        cpu = cpu_baseline_batch(probs, args.cpu_seconds, args)
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    stream = torch.cuda.current_stream()
    if args.copy_probe:
        copy_probe(torch)
    if args.matvec_only:
        print(json.dumps(run_matvecs(config, stream, torch, args)))
        return
    if args.schemes_only:
        print(json.dumps({"c3_second_vs_fourth_order": run_scheme_comparison(config, stream, torch, args)}))
        return
    if args.tangents_only:
        cube = config("c4")
        u_aff = (0.02 * cube.xyz * np.array([1.0, 1.0, -1.0])).ravel()
        print(json.dumps({"tangents_cube64_yeoh_bf16": run_tangents(cube, u_aff, 20, stream, torch, args)}))
        return

    mixed = run_batch(probs, "mixed_f32", args.steps, args.warmup, args.batch_m_max, stream, torch, args)
    f64 = run_batch(probs, "f64", args.steps, args.warmup, args.batch_m_max, stream, torch, args)
    workload = batch_workload(probs, args.batch_dt, args.batch_m_max, args.check_every)
    launch_s = mixed["ms_per_step"] / 1e3
    achieved = mixed["alg_bytes_per_launch"] / launch_s / 1e9
    gate = max(mixed["energy_rel_err_max"], f64["energy_rel_err_max"]) <= 1e-6
    result = {
        "metric": "DOF-matvecs/s + time-steps/s at fixed energy error, mixed/batched vs FP64",
        "value": mixed["dof_matvecs_per_s"],
        "unit": "DOF-matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 operator, f64 Krylov/expm/state",
        "data": "synthetic",
        "config": {"workload": workload, "instances": len(probs), "dt": args.batch_dt, "tol": 1e-10,
                   "m_max": args.batch_m_max, "precision": "mixed_f32",
                   "total_free_dofs": mixed["total_free_dofs"]},
        "time_steps_per_s": mixed["time_steps_per_s"],
        "instance_steps_per_s": mixed["instance_steps_per_s"],
        "energy_rel_err_max": mixed["energy_rel_err_max"],
        "fp64_same_workload": {k: f64[k] for k in ("dof_matvecs_per_s", "time_steps_per_s", "instance_steps_per_s",
                                                   "ms_per_step", "energy_rel_err_max", "energy_rel_err_median",
                                                   "matvecs_per_step", "m_corr_range", "m_pred_range", "plan")},
        "mixed_vs_fp64": {"time_steps_per_s": mixed["time_steps_per_s"] / f64["time_steps_per_s"],
                          "dof_matvecs_per_s": mixed["dof_matvecs_per_s"] / f64["dof_matvecs_per_s"],
                          "energy_gate_1e-6_met_by_both": gate},
        "headline_detail": {k: mixed[k] for k in ("energy_rel_err_median", "matvecs_per_step", "m_corr_range",
                                                  "m_pred_range", "plan")},
        "roofline": {
            "kernel": "k_batch<float, 1> (workgroups stepping lists of instances or teams of workgroups stepping one "
                      "instance: operator applies, Arnoldi-MGS, exponential, predictor and corrector of one time "
                      "step), one launch per step",
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(workload, "mixed_f32"),
            "alg_bytes_per_launch": mixed["alg_bytes_per_launch"], "avg_launch_ms": launch_s * 1e3,
        },
    }
    if cpu is not None:
        result["cpu_baseline"] = cpu
    if not (args.headline_only or args.no_extra):
        result["extra"] = run_extras(config, stream, torch, args)
    print(json.dumps(result))


def run_extras(config, stream, torch, args):
    """Single-instance workloads on short step subsets (labelled), stand-alone applies and
    the BF16 tangents."""
    extra = {}
    prob = config(args.config, dt=args.dt)
    states = {}
    for prec in ("f64", "mixed_f32"):
        r = run_single(prob, prec, 30, args.warmup, args.m_max, args.workgroups, args.adaptive, stream, torch, args)
        m_used, k_used = r["m"], r["k"]
        alg = algorithmic_bytes(prob, m_used, k_used, s_x=8 if prec == "f64" else 4)
        e = {k: v for k, v in r.items() if k not in ("ctx", "step_ms")}
        e["subset"] = f"30 timed steps after {args.warmup} calibration steps (the workload runs 500)"
        e["roofline_k_expv"] = {"achieved": alg / (r["ms_per_step"] / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": alg / (r["ms_per_step"] / 1e3) / 1e9 / HBM_PEAK_GBS,
                                "alg_bytes_per_launch": alg}
        _, u, v = r["ctx"].get_state()
        states[prec] = (u, v)
        if prec != "f64":
            u0, v0 = states["f64"]
            e["state_rel_err_vs_f64"] = {"u": float(np.abs(u - u0).max() / np.abs(u0).max()),
                                         "v": float(np.abs(v - v0).max() / np.abs(v0).max())}
        r["ctx"].close()
        extra[f"{args.config}_{prec}"] = e
    # the c2 workload's time-step sweep (FP64): the subspace size and substeps the adaptive
    # choice settles on, and the cost of one simulated second at each step size
    sweep = {}
    for dt in (1e-5, 1e-4, 1e-3):
        r = run_single(config(args.config, dt=dt), "f64", 10, 3, args.m_max, args.workgroups, False,
                       stream, torch, args)
        sweep[f"{dt:g}"] = {"ms_per_step": r["ms_per_step"], "m": r["m"], "k": r["k"],
                            "time_steps_per_s": r["time_steps_per_s"],
                            "dof_matvecs_per_s": r["dof_matvecs_per_s"],
                            "gpu_s_per_simulated_s": r["ms_per_step"] / 1e3 / dt}
        r["ctx"].close()
    extra["c2_dt_sweep_f64"] = sweep
    for name, dt, steps, precs in (("c3", 1e-4, 20, ("f64", "mixed_f32", "mixed_bf16")),
                                   ("c3", 5e-4, 10, ("f64", "mixed_f32")),
                                   ("c4", 1e-3, 8, ("f64", "mixed_f32", "mixed_bf16"))):
        p = config(name, dt=dt)
        ref_state = None
        key = name if (name, dt) != ("c3", 5e-4) else "c3dt5e-4"
        for prec in precs:
            r = run_single(p, prec, steps, 3, 64, 0, True, stream, torch, args)
            e = {k: v for k, v in r.items() if k not in ("ctx", "step_ms", "energy_rel_err")}
            e["free_dofs"] = p.n_free
            e["subset"] = f"{steps} timed steps after 3 warm-up steps (the workload runs {p.n_steps})"
            # time-varying load: error of the final state (warm-up + timed steps, same
            # steps in every precision) against the FP64 run, which matches the oracle to 1e-8
            _, u, v = r["ctx"].get_state()
            en = r["ctx"].energy()
            if ref_state is None:
                ref_state = (u, v, en)
            else:
                ur, vr, er = ref_state
                e["state_rel_err_vs_f64"] = {
                    "u": float(np.abs(u - ur).max() / np.abs(ur).max()),
                    "v": float(np.abs(v - vr).max() / np.abs(vr).max()),
                    "energy": abs((en[0] + en[1] - en[2]) - (er[0] + er[1] - er[2])) / (er[0] + er[1])}
            r["ctx"].close()
            extra[f"{key}_{prec}"] = e
    extra["c3_second_vs_fourth_order"] = run_scheme_comparison(config, stream, torch, args)
    extra.update(run_matvecs(config, stream, torch, args))
    cube = config("c4")
    u_aff = (0.02 * cube.xyz * np.array([1.0, 1.0, -1.0])).ravel()
    extra["tangents_cube64_yeoh_bf16"] = run_tangents(cube, u_aff, 20, stream, torch, args)
    return extra


def run_scheme_comparison(config, stream, torch, args):
    """Second- against fourth-order Magnus step on the 160x16x16 Neo-Hookean cantilever (FP64):
    from rest over the first 5 ms of the load ramp, the element-wise error of u and v against a
    fourth-order run at dt = T/320, and the GPU time of each run (HIP events)."""
    from paper_2405_05213_amd import solver_from_problem
    T = 0.005
    p0 = config("c3")

    def run(scheme, n):
        p = config("c3", dt=T / n)
        ctx = solver_from_problem(p, m_max=64, check_every=args.check_every, scheme=scheme,
                                  stream=stream.cuda_stream)
        ctx.sync()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.step(p.dt, n)
        e1.record(stream)
        torch.cuda.synchronize()
        _, u, v = ctx.get_state()
        ms = e0.elapsed_time(e1)
        st = ctx.stats()
        ctx.close()
        return u, v, ms, st

    ur, vr, ms_ref, _ = run(4, 320)
    out = {"workload": f"c3 {p0.grid}, first {T * 1e3:g} ms of the load ramp, FP64, tol 1e-10",
           "reference": f"fourth-order scheme at dt = {T / 320:g} s ({ms_ref:.0f} ms)", "runs": []}
    for scheme in (2, 4):
        for n in (10, 20, 40):
            u, v, ms, st = run(scheme, n)
            eu = float(np.abs(u - ur).max() / np.abs(ur).max())
            ev = float(np.abs(v - vr).max() / np.abs(vr).max())
            out["runs"].append({"scheme": scheme, "dt": T / n, "steps": n, "gpu_ms": ms, "ms_per_step": ms / n,
                                "matvecs": st["matvecs"], "err_u": eu, "err_v": ev})
            log(args, f"  scheme {scheme} dt={T / n:g}: {ms / n:.3f} ms/step, err u {eu:.2e} v {ev:.2e}")
    return out


def run_matvecs(config, stream, torch, args):
    """The stand-alone FP64 applies: linear 64^3, 128^3 and 192^3 cubes (lattice path) and the Yeoh
    secant apply on the 64^3 block at an affine deformation."""
    import dataclasses
    out = {}
    cube = config("c4")
    # 192^3: x and y alone are 0.34 GB, beyond the 256 MB Infinity Cache (the roofline probe)
    for nx in (64, 128, 192):
        q = cube if nx == 64 else config("c4", nx=nx, ny=nx, nz=nx)
        q = dataclasses.replace(q, model="linear", params=(200e9, 0.3), rho=7800.0)
        out[f"matvec_cube{nx}_linear_f64"] = run_matvec(q, None, 50, stream, torch, args)
        del q
    u_aff = (0.02 * cube.xyz * np.array([1.0, 1.0, -1.0])).ravel()
    out["matvec_cube64_yeoh_f64"] = run_matvec(cube, u_aff, 20, stream, torch, args)
    # the same 65^3 nodes as 32^3 quadratic (27-node) elements, the paper's element
    from workloads import q2_of
    q2 = q2_of(cube)
    out["matvec_cube64nodes_q2_linear_f64"] = run_matvec(
        dataclasses.replace(q2, model="linear", params=(200e9, 0.3), rho=7800.0), None, 20, stream, torch, args)
    out["matvec_cube64nodes_q2_yeoh_f64"] = run_matvec(q2, u_aff, 20, stream, torch, args)
    return out


if __name__ == "__main__":
    main()
