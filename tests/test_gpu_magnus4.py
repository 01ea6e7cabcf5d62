"""The fourth-order scheme (ep_set_scheme(ctx, 4): the two-term Magnus step) against the
oracle's step4, element by element (needs an MI355X)."""
import numpy as np
import pytest

from oracle.stepper import Propagator
from tests.gpu_util import maxrel, say, svk_of, yeoh_rubber_of
from workloads import config

pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(model):
    if model == "linear":     # the load ramps, so A_1 != A_2 and the commutator acts
        p = config("c1", dt=2e-4)
        return p.with_(knots_t=np.array([0.0, 0.01]), knots_s=np.array([0.0, 1.0]))
    if model == "nh":
        return config("c3", nx=8, ny=2, nz=2, dt=5e-4)
    if model == "svk":
        return svk_of(config("c3", nx=8, ny=2, nz=2, dt=5e-4))
    if model == "yeoh":
        return config("c4", nx=3, ny=3, nz=3, dt=2e-3)
    return yeoh_rubber_of(config("c4", nx=3, ny=3, nz=3, dt=2e-3))


@pytest.mark.parametrize("ortho", [0, 1])
@pytest.mark.parametrize("mode", ["fixed", "adaptive"])
@pytest.mark.parametrize("model", ["linear", "nh", "svk", "yeoh", "yeoh3"])
def test_fourth_order_steps_match_oracle(model, mode, ortho):
    from paper_2405_05213_amd import solver_from_problem
    p = _case(model)
    say(f"[magnus4] {model} {mode} ortho={ortho}")
    # fixed m: 24 converges for the soft solids; the steel beam at this dt needs 40 (at m = 24
    # its projection is far from converged, eps ~ 0.04, and a 1e-18 change of the input moves
    # the oracle's own result by 1e-2)
    mf = 40 if model == "linear" else 24
    kw = dict(m_max=48) if mode == "adaptive" else dict(m_max=48, m_fixed=mf, k_fixed=1)
    ctx = solver_from_problem(p, scheme=4, ortho=ortho, **kw)
    orc = Propagator(p, **kw)
    n = 8
    ctx.step(p.dt, n)
    for _ in range(n):
        orc.step4(p.dt)
    t, u, v = ctx.get_state()
    eu, ev = maxrel(u, orc.u()), maxrel(v, orc.v())
    say(f"  err u {eu:.2e} v {ev:.2e}")
    assert abs(t - orc.t) < 1e-15
    assert eu < 1e-8 and ev < 1e-8
    if mode == "adaptive":
        log = ctx.step_log(n)
        assert np.array_equal(log["m_corr"], np.array([r["corr"]["m"][0] for r in orc.log]))
    ctx.close()


@pytest.mark.parametrize("model", ["nh", "yeoh"])
def test_fourth_order_fp32_operator(model):
    """FP32 element kernels, FP64 Krylov: against the FP64 oracle at a stated tolerance."""
    from paper_2405_05213_amd import solver_from_problem
    p = _case(model)
    say(f"[magnus4 mixed_f32] {model}")
    ctx = solver_from_problem(p, scheme=4, precision="mixed_f32", m_max=48, m_fixed=24, k_fixed=1)
    orc = Propagator(p, m_max=48, m_fixed=24, k_fixed=1)
    n = 8
    ctx.step(p.dt, n)
    for _ in range(n):
        orc.step4(p.dt)
    t, u, v = ctx.get_state()
    eu, ev = maxrel(u, orc.u()), maxrel(v, orc.v())
    say(f"  err u {eu:.2e} v {ev:.2e}")
    assert eu < 1e-6 and ev < 1e-6
    ctx.close()


def test_set_state_restarts_the_extrapolation():
    """After ep_set_state the first step predicts with the Taylor polynomial again: the same
    steps from the same state give the same result."""
    from paper_2405_05213_amd import solver_from_problem
    p = _case("nh")
    ctx = solver_from_problem(p, scheme=4, m_max=48)
    ctx.step(p.dt, 3)
    _, u1, v1 = ctx.get_state()
    ctx.set_state(0.0, p.u0, p.v0)
    ctx.step(p.dt, 3)
    _, u2, v2 = ctx.get_state()
    assert np.array_equal(u1, u2) and np.array_equal(v1, v2)
    ctx.close()
