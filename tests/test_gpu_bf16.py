"""Stored BF16 element tangents (EP_PREC_MIXED_BF16) against the FP64 oracle (needs an MI355X).

The tangents keep 8 significant bits, so these compare at a stated tolerance rather than to
rounding: for random inputs the operator error is about 2e-3 relative (the BF16 rounding
model run on the CPU gives 1.6e-3 on the linear cantilever and 2.3e-3 on the Neo-Hookean
and Yeoh meshes below), and after 12 predictor-corrector steps the displacement and
velocity differ from the oracle by 1e-3 to 2e-3.  A wrong fragment layout or index in the
matrix-core formation gives errors of order one."""
import numpy as np
import pytest

from workloads import config, distort
from tests.gpu_util import pair, maxrel, say, svk_of

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL_OP = 1e-2
TOL_TRAJ = 1e-2


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


# (model, workload, overrides, displacement amplitude relative to the mesh extent);
# 19x3x2 = 114 elements leaves a partly filled formation workgroup and a partly filled
# group of 8 (its elements are smaller, hence the smaller random displacement that keeps
# det F > 0)
CASES = [("linear", "c1", {}, 0.0), ("nh", "c3", dict(nx=8, ny=2, nz=2), 0.03),
         ("nh", "c3", dict(nx=19, ny=3, nz=2), 0.01), ("yeoh", "c4", dict(nx=4, ny=3, nz=3), 0.03),
         ("svk", "c3", dict(nx=8, ny=2, nz=2), 0.03)]


@pytest.mark.parametrize("model,name,over,amp", CASES)
def test_apply_H_bf16(model, name, over, amp):
    """y = H(u) x from the stored tangents at a deformed state (rest state for linear)."""
    say(f"[bf16 apply_H] {model} {name} {over}")
    p = config(name, **over)
    if model == "svk":
        p = svk_of(p)
    ctx, orc = pair(p, precision="mixed_bf16")
    rng = np.random.default_rng(3)
    n3 = 3 * p.n_nodes
    x = rng.normal(size=n3)
    u = None if model == "linear" else amp * rng.normal(size=n3) * (p.xyz.max() - p.xyz.min())
    y = torch.zeros(n3, dtype=torch.float64, device=DEV)
    ctx.apply_H(None if u is None else _t(u), _t(x), y)
    ref = orc.fem.H_apply(u, x)
    err = maxrel(y.cpu().numpy(), ref)
    say(f"  rel err {err:.2e}")
    assert err < TOL_OP


def test_apply_H_bf16_tangents_follow_the_state():
    """The tangents are re-formed for each linearisation point: the rest state after a
    deformed one gives the linear operator again."""
    say("[bf16 apply_H] re-formation")
    p = config("c3", nx=8, ny=2, nz=2)
    ctx, orc = pair(p, precision="mixed_bf16")
    rng = np.random.default_rng(4)
    n3 = 3 * p.n_nodes
    x = rng.normal(size=n3)
    u = 0.02 * rng.normal(size=n3) * (p.xyz.max() - p.xyz.min())
    y = torch.zeros(n3, dtype=torch.float64, device=DEV)
    ctx.apply_H(_t(u), _t(x), y)
    assert maxrel(y.cpu().numpy(), orc.fem.H_apply(u, x)) < TOL_OP
    ctx.apply_H(None, _t(x), y)
    assert maxrel(y.cpu().numpy(), orc.fem.H_apply(np.zeros(n3), x)) < TOL_OP
    ctx.apply_H(_t(u), _t(x), y)
    assert maxrel(y.cpu().numpy(), orc.fem.H_apply(u, x)) < TOL_OP


@pytest.mark.parametrize("model,name,over", [("nh", "c3", dict(nx=8, ny=2, nz=2, dt=5e-4)),
                                              ("yeoh", "c4", dict(nx=3, ny=3, nz=3, dt=2e-3))])
@pytest.mark.parametrize("ortho", [0, 1])
def test_steps_bf16(model, name, over, ortho):
    """12 predictor-corrector steps (tangents of the extrapolated predictor operator and of the
    midpoint operator formed every step) against the FP64 oracle."""
    say(f"[bf16 steps] {model} {name} {over} ortho={ortho}")
    p = config(name, **over)
    n = 12
    ctx, orc = pair(p, m_max=48, m_fixed=24, k_fixed=1, ortho=ortho, precision="mixed_bf16")
    ctx.step(p.dt, n)
    t, u, v = ctx.get_state()
    orc.run(p.dt, n)
    eu, ev = maxrel(u, orc.u()), maxrel(v, orc.v())
    say(f"  rel err u {eu:.2e} v {ev:.2e}")
    assert eu < TOL_TRAJ and ev < TOL_TRAJ


def test_bf16_needs_congruent_mesh():
    """A distorted mesh has element-dependent gradients: no shared left factor, refused."""
    from paper_2405_05213_amd import ep as epmod
    say("[bf16] distorted mesh refused")
    p = distort(config("c3", nx=8, ny=2, nz=2), 0.2, seed=5)
    with pytest.raises(epmod.EPError) as e:
        pair(p, precision="mixed_bf16")
    assert e.value.code == epmod.EP_ERR_ARG
