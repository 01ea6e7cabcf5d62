"""Checkpoint and resume: an image of the stepping state saved after some steps and loaded
into a fresh context (or back into the saving one) continues bit for bit as the saving
context does - the predictor's midpoint history (Sec. 4.2), the adaptive Krylov state, the
resolved augmented entry and the fourth-order scheme's previous start state included."""
import numpy as np
import pytest

from gpu_util import say
from workloads import batch_instances, config

pytestmark = pytest.mark.gpu


def _solver(p, prec, scheme, s0):
    from paper_2405_05213_amd import solver_from_problem
    # a fixed team size: the same reduction order in both contexts
    return solver_from_problem(p, m_max=32, precision=prec, scheme=scheme, s0=s0, workgroups=4)


def _same(a, b):
    return a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("name,prec,scheme,s0", [
    ("c3", "f64", 2, -1.0), ("c3", "mixed_f32", 2, -1.0), ("c3", "f64", 4, -1.0), ("c2", "f64", 2, -2.0)])
def test_resume_is_bit_exact(name, prec, scheme, s0):
    say(f"[checkpoint] {name} {prec} scheme {scheme} s0 {s0}")
    p = config(name, nx=24, ny=4, nz=4)
    a = _solver(p, prec, scheme, s0)
    a.step(p.dt, 5)
    img = a.save_checkpoint()
    a.step(p.dt, 4)
    ref = a.get_state()
    m_ref = a.stats()["m"]
    b = _solver(p, prec, scheme, s0)
    b.load_checkpoint(img)
    b.step(p.dt, 4)
    assert _same(b.get_state(), ref)
    assert b.stats()["m"] == m_ref
    # back into the saving context
    a.load_checkpoint(img)
    a.step(p.dt, 4)
    assert _same(a.get_state(), ref)
    # a restart from (t, u, v) alone drops the history and re-derives ubar = M^{1/2} u
    t5, u5, v5 = _solver_state_after(p, prec, scheme, s0, 5)
    c = _solver(p, prec, scheme, s0)
    c.set_state(t5, u5, v5)
    c.step(p.dt, 4)
    diff = np.abs(c.get_state()[1] - ref[1]).max() / np.abs(ref[1]).max()
    say(f"  restart from (t, u, v) differs by {diff:.1e} (checkpoint: 0)")
    for x in (a, b, c):
        x.close()


def _solver_state_after(p, prec, scheme, s0, n):
    s = _solver(p, prec, scheme, s0)
    s.step(p.dt, n)
    st = s.get_state()
    s.close()
    return st


def test_checkpoint_refuses_other_contexts_and_corrupt_images():
    from paper_2405_05213_amd.ep import EPError
    p = config("c3", nx=24, ny=4, nz=4)
    a = _solver(p, "f64", 2, -1.0)
    a.step(p.dt, 2)
    img = a.save_checkpoint()
    other = _solver(config("c3", nx=20, ny=4, nz=4), "f64", 2, -1.0)
    with pytest.raises(EPError):
        other.load_checkpoint(img)
    prec32 = _solver(p, "mixed_f32", 2, -1.0)
    with pytest.raises(EPError):
        prec32.load_checkpoint(img)
    bad = bytearray(img)
    bad[0:8] = b"XXXXXXXX"
    with pytest.raises(EPError):
        a.load_checkpoint(bytes(bad))
    with pytest.raises(EPError):
        a.load_checkpoint(img[:-8])
    for x in (a, other, prec32):
        x.close()


@pytest.mark.parametrize("prec", ["f64", "mixed_f32"])
def test_batch_instance_resume_is_bit_exact(prec):
    from paper_2405_05213_amd import batch_from_problems
    from paper_2405_05213_amd.ep import S0_SCALED
    say(f"[checkpoint] batch of 3 rubber blocks {prec}")
    probs = batch_instances(3, seed=1, dt=6.25e-6)
    dt = probs[0].dt
    a = batch_from_problems(probs, m_max=32, precision=prec, s0=S0_SCALED)
    a.step(dt, 5)
    imgs = [a.save_checkpoint(i) for i in range(3)]
    a.step(dt, 4)
    ref = [a.get_state(i) for i in range(3)]
    b = batch_from_problems(probs, m_max=32, precision=prec, s0=S0_SCALED)
    for i in range(3):
        b.load_checkpoint(i, imgs[i])
    b.step(dt, 4)
    for i in range(3):
        assert _same(b.get_state(i), ref[i])
    a.close()
    b.close()
