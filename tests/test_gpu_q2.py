"""Quadratic 27-node hexahedra on the GPU (ep_set_mesh_hex27) against the oracle, element by
element (needs an MI355X)."""
import numpy as np
import pytest

from oracle.stepper import Propagator
from tests.gpu_util import maxrel, pair, say, svk_of, yeoh_rubber_of
from workloads import config, distort, q2_of

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _case(model, distorted=False):
    if model == "linear":
        p = q2_of(config("c1", nx=10, ny=2, nz=2))
    elif model == "nh":
        p = q2_of(config("c3", nx=8, ny=2, nz=2, dt=5e-4))
    elif model == "svk":
        p = svk_of(q2_of(config("c3", nx=8, ny=2, nz=2, dt=5e-4)))
    elif model == "yeoh":
        p = q2_of(config("c4", nx=4, ny=4, nz=4, dt=2e-3))
    else:
        p = yeoh_rubber_of(q2_of(config("c4", nx=4, ny=4, nz=4, dt=2e-3)))
    # interior nodes moved by up to 0.1 of the smallest node spacing: curved elements with
    # det J > 0 at every Gauss and Gauss-Lobatto point (0.2 folds a corner of the 2x2x2 block)
    return distort(p, 0.1, seed=6) if distorted else p


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("mixed_f32", 3e-6)])
@pytest.mark.parametrize("model", ["linear", "nh", "svk", "yeoh", "yeoh3"])
@pytest.mark.parametrize("distorted", [False, True])
def test_q2_apply_H_matches_oracle(model, distorted, prec, tol):
    say(f"[q2 apply_H] {model} distorted={distorted} {prec}")
    p = _case(model, distorted)
    ctx, orc = pair(p, precision=prec)
    assert ctx.launch()[2] == (0 if distorted else 1)          # congruent unless distorted
    rng = np.random.default_rng(8)
    n3 = 3 * p.n_nodes
    x = rng.normal(size=n3)
    u = None if model == "linear" else rng.normal(size=n3)
    if u is not None:
        u *= 0.05 / np.abs(orc.fem.grad(u)).max()
    y = torch.zeros(n3, dtype=torch.float64, device=DEV)
    ctx.apply_H(None if u is None else _t(u), _t(x), y)
    ref = orc.fem.H_apply(u, x)
    err = maxrel(y.cpu().numpy(), ref)
    say(f"  err {err:.2e}")
    assert err < tol
    ctx.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-8), ("mixed_f32", 1e-6)])
@pytest.mark.parametrize("model", ["linear", "nh", "svk", "yeoh", "yeoh3"])
def test_q2_steps_match_oracle(model, prec, tol):
    """FP64 and FP32 element kernels.  The steel cantilever in FP32 carries the amplified
    rounding of its element forces (a smooth bending field is a small difference of large
    forces, as with hex8): measured u 4.3e-7, v 1.5e-5 after 20 steps; tolerance 1e-4 there."""
    if model == "linear" and prec == "mixed_f32":
        tol = 1e-4
    say(f"[q2 steps] {model} {prec}")
    p = _case(model)
    kw = dict(m_max=64)
    ctx, orc = pair(p, precision=prec, **kw)
    n = 6 if model != "linear" else 20
    ctx.step(p.dt, n)
    orc.run(p.dt, n)
    t, u, v = ctx.get_state()
    eu, ev = maxrel(u, orc.u()), maxrel(v, orc.v())
    say(f"  err u {eu:.2e} v {ev:.2e}")
    assert abs(t - orc.t) < 1e-15
    assert eu < tol and ev < tol
    ke, se, we = ctx.energy()
    ko, so, wo = orc.energies()
    assert abs((ke + se - we) - (ko + so - wo)) <= tol * (ko + so)
    if prec == "f64":
        log = ctx.step_log(n)
        assert np.array_equal(log["m_corr"], np.array([r["corr"]["m"][0] for r in orc.log]))
    ctx.close()


def test_q2_refuses_the_unsupported_modes():
    from paper_2405_05213_amd import ep as epmod
    from paper_2405_05213_amd import solver_from_problem
    p = _case("nh")
    for kw in (dict(precision="mixed_bf16"), dict(scheme=4)):
        with pytest.raises(epmod.EPError) as e:
            solver_from_problem(p, **kw)
        assert e.value.code == epmod.EP_ERR_ARG
