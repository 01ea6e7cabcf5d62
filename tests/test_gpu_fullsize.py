"""Parity at the full workload sizes, in the launch configuration the benchmark uses
(needs an MI355X).  Where a whole oracle step would take minutes (the 64^3 block), the
operator and the energies are compared at full size instead."""
import dataclasses

import numpy as np
import pytest

from workloads import config
from oracle.stepper import Propagator
from tests.gpu_util import pair, maxrel, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("prec,tol_u,tol_v", [("f64", 1e-8, 1e-8), ("mixed_f32", 5e-6, 5e-5)])
def test_c2_full_step(prec, tol_u, tol_v):
    """80x8x8 linear cantilever, dt = 1e-4, the benchmark's calibrated mode (m = 48, 4 substeps).
    FP32 operator: measured u 8e-7, v 9.5e-6 (the steel beam's small net forces amplify the
    FP32 rounding of the element forces, most in the velocity); tolerances about 5x that."""
    say(f"[full] c2 one step m=48 k=4 {prec}")
    p = config("c2")
    ctx, orc = pair(p, m_max=64, m_fixed=48, k_fixed=4, precision=prec)
    ctx.step(p.dt, 1)
    t, u, v = ctx.get_state()
    orc.step(p.dt)
    eu, ev = maxrel(u, orc.u()), maxrel(v, orc.v())
    say(f"  rel err u {eu:.2e} v {ev:.2e}")
    assert eu < tol_u and ev < tol_v


@pytest.mark.parametrize("prec,tol", [("f64", 1e-8), ("mixed_f32", 5e-8), ("mixed_bf16", 5e-4)])
def test_c3_full_step(prec, tol):
    """160x16x16 compressible Neo-Hookean cantilever, first predictor-corrector step.  Measured:
    FP32 operator 4e-9 / 8e-9, BF16 tangents 4e-5 / 8e-5 (u / v); tolerances about 5x that."""
    say(f"[full] c3 one step {prec}")
    p = config("c3")
    ctx, orc = pair(p, m_max=64, precision=prec)
    ctx.step(p.dt, 1)
    t, u, v = ctx.get_state()
    orc.step(p.dt)
    eu, ev = maxrel(u, orc.u()), maxrel(v, orc.v())
    say(f"  rel err u {eu:.2e} v {ev:.2e}")
    assert eu < tol and ev < tol
    if prec == "f64":
        assert ctx.step_log(1)["m_corr"][0] == orc.log[0]["corr"]["m"][0]


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("mixed_f32", 3e-6), ("mixed_bf16", 1e-2)])
def test_c4_full_operator_and_energy(prec, tol):
    """64^3 decoupled Neo-Hookean (Yeoh) block: H(u) x at a deformed state, full size."""
    say(f"[full] c4 operator {prec}")
    p = config("c4")
    ctx, orc = pair(p, m_max=16, precision=prec)
    rng = np.random.default_rng(21)
    n3 = 3 * p.n_nodes
    u = np.zeros(n3)
    u[orc.free] = 2e-3 * rng.normal(size=orc.N)
    x = np.zeros(n3)
    x[orc.free] = rng.normal(size=orc.N)
    y = torch.zeros(n3, dtype=torch.float64, device=DEV)
    ctx.apply_H(_t(u), _t(x), y)
    ref = orc.fem.H_apply(u, x)
    assert maxrel(y.cpu().numpy()[orc.free], ref[orc.free]) < tol
    # energies of a deformed, moving state
    v = np.zeros(n3)
    v[orc.free] = 1e-3 * rng.normal(size=orc.N)
    ctx.set_state(0.05, u, v)
    ke, se, we = ctx.energy()
    o = Propagator(p.with_(u0=u, v0=v))
    o.t = 0.05
    ko, so, wo = o.energies()
    assert abs(ke - ko) <= 1e-12 * ko and abs(se - so) <= 1e-11 * so and abs(we - wo) <= 1e-12 * abs(wo)


def test_lattice_apply_many_tiles():
    """Linear lattice whose 79 x 71 x 87 interior nodes make 3 x 9 x 22 = 594 tiles of the
    stencil apply (each cut in x, y and z at the far end), more tiles than the machine holds
    at once: H x on all DOFs against the oracle."""
    say("[full] lattice 80x72x88 apply")
    p = dataclasses.replace(config("c4", nx=80, ny=72, nz=88), model="linear", params=(200e9, 0.3), rho=7800.0)
    ctx, orc = pair(p, m_max=4)
    assert ctx.launch()[2] == 2                        # the lattice path
    x = np.random.default_rng(22).normal(size=3 * p.n_nodes)
    y = torch.zeros(3 * p.n_nodes, dtype=torch.float64, device=DEV)
    ctx.apply_H(None, _t(x), y)
    err = maxrel(y.cpu().numpy(), orc.fem.H_apply(None, x))
    say(f"  rel err {err:.2e}")
    assert err < 1e-12


@pytest.mark.parametrize("prec,tol", [("f64", 1e-8), ("mixed_f32", 1e-8)])
def test_c5_full_batch_sampled(prec, tol):
    """The 256-instance rubber batch in the benchmark's configuration (m_max 32, adaptive with
    an error estimate at every Arnoldi step, dt 6.25e-6, augmented entry at each block's
    scale, launch plan chosen by the plan autotuner as the benchmark does): five steps, then
    the smallest, a middle and the largest instance and the smallest one stepped by a team
    against the oracle run on their own."""
    from paper_2405_05213_amd import batch_from_problems
    from paper_2405_05213_amd.ep import S0_SCALED
    from workloads import batch_instances
    say(f"[full] c5 batch of 256, {prec}")
    probs = batch_instances(256, seed=5)
    b = batch_from_problems(probs, m_max=32, check_every=1, precision=prec, s0=S0_SCALED)
    wg, ms = b.autotune(probs[0].dt, steps=5)
    teams = [b.plan_of(i)[0] for i in range(len(probs))]
    say(f"  plan: {wg} workgroups, largest team {max(teams)}, {sum(g > 1 for g in teams)} instances in teams")
    n = 5
    b.step(probs[0].dt, n)
    sizes = [p.n_nodes for p in probs]
    pick = [int(np.argmin(sizes)), 128, int(np.argmax(sizes))]
    in_teams = [i for i in range(len(probs)) if teams[i] > 1]
    if in_teams:
        pick.append(min(in_teams, key=lambda i: sizes[i]))
    for i in pick:
        p = probs[i]
        t, u, v = b.get_state(i)
        orc = Propagator(p, m_max=32, check_every=1, s0="scaled")
        orc.run(p.dt, n)
        eu, ev = maxrel(u, orc.u()), maxrel(v, orc.v())
        say(f"  instance {i} ({p.n_nodes} nodes, team {teams[i]}): rel err u {eu:.2e} v {ev:.2e}")
        assert eu < tol and ev < tol
    b.close()


# ---------------------------------------------------------------------------------------
# Several steps at full size against stored oracle results (tests/golden/fullsize_*.json,
# written by tests/golden/make_fullsize_golden.py, which runs only the oracle): a seeded
# sample of 2048 free DOFs of u and v, element-wise error normalised by max |u|, max |v| of
# the oracle over all DOFs, plus the energies and, in FP64, the subspace sizes.
# ---------------------------------------------------------------------------------------
def _golden(case):
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"fullsize_{case}.json")) as fh:
        return json.load(fh)


# (case, precision, tol u, tol v, tol energy)
GOLDEN_CASES = [
    ("c2dt1e-3", "f64", 1e-8, 1e-8, 1e-8),        # one step at dt = 1e-3: m = 56, 32 substeps
    ("c2dt1e-3", "mixed_f32", 1e-4, 1e-3, 1e-5),
    ("c3", "f64", 1e-8, 1e-8, 1e-8),              # three steps: the two-point predictor runs
    ("c3", "mixed_f32", 1e-6, 1e-6, 1e-6),
    ("c4", "f64", 1e-8, 1e-8, 1e-8),              # three steps of the 64^3 Yeoh block
    ("c4", "mixed_f32", 1e-6, 1e-6, 1e-6),
]


@pytest.mark.parametrize("case,prec,tol_u,tol_v,tol_e", GOLDEN_CASES)
def test_fullsize_steps_against_stored_oracle(case, prec, tol_u, tol_v, tol_e):
    from paper_2405_05213_amd import solver_from_problem
    g = _golden(case)
    say(f"[full] {case} {g['steps']} steps {prec} {g['krylov']}")
    p = config(g["workload"], **g["overrides"])
    ctx = solver_from_problem(p, precision=prec, **g["krylov"])
    ctx.step(p.dt, g["steps"])
    t, u, v = ctx.get_state()
    idx = np.asarray(g["dofs"])
    eu = maxrel(u[idx], np.asarray(g["u"]), g["max_abs_u"])
    ev = maxrel(v[idx], np.asarray(g["v"]), g["max_abs_v"])
    ke, se, we = ctx.energy()
    ko, so, wo = g["energies"]
    ee = abs((ke + se - we) - (ko + so - wo)) / (ko + so)
    say(f"  element-wise err u {eu:.2e} v {ev:.2e}, energy {ee:.2e}")
    assert abs(t - g["t"]) < 1e-15
    assert eu < tol_u and ev < tol_v and ee < tol_e
    if prec == "f64":
        log = ctx.step_log(g["steps"])
        assert list(log["m_corr"]) == g["m_corr"] and list(log["k_corr"]) == g["k_corr"]
        if g["m_pred"]:
            assert list(log["m_pred"]) == g["m_pred"]
    ctx.close()
