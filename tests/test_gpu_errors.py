"""Device-side failures reach the caller as sticky errors (needs an MI355X): the next
synchronising call returns them, they stay until ep_set_state, and the context is usable
again after it.  The conditions are made by the inputs; every kernel ends normally."""
import numpy as np
import pytest

from workloads import config
from tests.gpu_util import pair, maxrel, say

pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ep():
    from paper_2405_05213_amd import ep as epmod
    return epmod


def test_inverted_state_is_a_sticky_error():
    """The free end of the Neo-Hookean cantilever pushed back through three element layers:
    det F <= 0 in those elements, so the secant operator cannot be formed."""
    epmod = _ep()
    say("[errors] inverted state")
    p = config("c3", nx=8, ny=2, nz=2)
    ctx, orc = pair(p, m_max=48)
    n3 = 3 * p.n_nodes
    x = p.xyz[:, 0]
    u = np.zeros(n3)
    u[3 * np.where(x == x.max())[0]] = -3.0 * (x.max() - x.min()) / 8
    ctx.set_state(0.0, u, np.zeros(n3))
    ctx.step(p.dt, 2)
    with pytest.raises(epmod.EPError) as e:
        ctx.sync()
    assert e.value.code == epmod.EP_ERR_INVERTED
    ctx.step(p.dt, 1)                                  # still failed: nothing advances
    with pytest.raises(epmod.EPError) as e:
        ctx.get_state()
    assert e.value.code == epmod.EP_ERR_INVERTED
    # a new state clears the error and the predictor history
    ctx.set_state(0.0, p.u0, p.v0)
    ctx.step(p.dt, 3)
    t, u1, v1 = ctx.get_state()
    orc.run(p.dt, 3)
    assert maxrel(u1, orc.u()) < 1e-8 and maxrel(v1, orc.v()) < 1e-8


def test_krylov_not_converged_is_a_sticky_error():
    """A step 100 times the linear cantilever's with at most 4 Krylov vectors and no
    substeps cannot meet the tolerance."""
    epmod = _ep()
    say("[errors] Krylov not converged")
    p = config("c1")
    ctx, orc = pair(p, m_max=4, max_substeps=1)
    ctx.step(100 * p.dt, 1)
    with pytest.raises(epmod.EPError) as e:
        ctx.sync()
    assert e.value.code == epmod.EP_ERR_KRYLOV
    ctx.set_state(0.0, p.u0, p.v0)
    ctx.step(1e-8, 2)                                  # steps 4 vectors resolve (tau omega_max ~ 1e-3)
    t, u1, v1 = ctx.get_state()
    assert np.isfinite(u1).all() and abs(t - 2e-8) < 1e-20


def test_batch_failure_stays_with_its_instance():
    """One of three batched Neo-Hookean instances starts inverted: it fails alone, the others
    match the oracle, and a new state for it clears the failure."""
    epmod = _ep()
    from paper_2405_05213_amd import batch_from_problems
    from oracle.stepper import Propagator
    from workloads import batch_instances
    say("[errors] batch instance failure")
    probs = batch_instances(n_inst=3, seed=5, dt=2e-4, nx_range=(4, 8), nyz_range=(2, 3))
    kw = dict(m_max=40, m_fixed=20, k_fixed=2)
    b = batch_from_problems(probs, **kw)
    bad = 1
    q = probs[bad]
    x = q.xyz[:, 0]
    u = np.zeros(3 * q.n_nodes)
    u[3 * np.where(x == x.max())[0]] = -3.0 * (x.max() - x.min()) / 4
    b.set_state(bad, 0.0, u, np.zeros_like(u))
    n = 3
    b.step(q.dt, n)
    with pytest.raises(epmod.EPError) as e:
        b.get_state(bad)
    assert e.value.code == epmod.EP_ERR_INVERTED
    for i, p in enumerate(probs):
        if i == bad:
            continue
        t, ui, vi = b.get_state(i)
        orc = Propagator(p, **kw)
        orc.run(p.dt, n)
        assert maxrel(ui, orc.u()) < 1e-8 and maxrel(vi, orc.v()) < 1e-8
    b.set_state(bad, 0.0, q.u0, q.v0)
    b.step(q.dt, n)
    t, ub, vb = b.get_state(bad)
    orc = Propagator(q, **kw)
    orc.run(q.dt, n)
    assert maxrel(ub, orc.u()) < 1e-8 and maxrel(vb, orc.v()) < 1e-8


def test_batch_autotune_failure_puts_the_batch_back():
    """The plan autotuner meets a device error in its first timing run (an instance whose
    state inverts elements): it returns that error with one workgroup per instance and the
    states it started from, and the batch steps on normally once that instance is reset."""
    epmod = _ep()
    from paper_2405_05213_amd import batch_from_problems
    from workloads import batch_instances
    say("[errors] batch autotune failure")
    probs = batch_instances(n_inst=3, seed=5, dt=2e-4, nx_range=(4, 8), nyz_range=(2, 3))
    b = batch_from_problems(probs, m_max=40)
    bad = 1
    q = probs[bad]
    x = q.xyz[:, 0]
    u = np.zeros(3 * q.n_nodes)
    u[3 * np.where(x == x.max())[0]] = -3.0 * (x.max() - x.min()) / 4
    b.set_state(bad, 0.0, u, np.zeros_like(u))
    before = [b.get_state(i) for i in range(3)]
    with pytest.raises(epmod.EPError) as e:
        b.autotune(q.dt, steps=2)
    assert e.value.code == epmod.EP_ERR_INVERTED
    assert all(b.plan_of(i)[0] == 1 for i in range(3)) and b.plan_of(0)[1] == 3
    for (t0, u0, v0), (t1, u1, v1) in zip(before, [b.get_state(i) for i in range(3)]):
        assert t0 == t1 and np.array_equal(u0, u1) and np.array_equal(v0, v1)
    b.set_state(bad, 0.0, q.u0, q.v0)
    b.step(q.dt, 2)
    for i in range(3):
        assert b.get_state(i)[0] == pytest.approx(2 * q.dt)
    b.close()
