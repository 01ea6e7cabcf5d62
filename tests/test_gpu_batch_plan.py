"""Launch plans of the batch: instances stepped one after the other by one workgroup (lists)
and large instances stepped by a team of workgroups, and the plan autotuner (needs an MI355X)."""
import numpy as np
import pytest

from oracle.stepper import Propagator
from tests.gpu_util import maxrel, say
from workloads import batch_instances, config

pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _probs(dt=2e-4):
    probs = batch_instances(n_inst=3, seed=5, dt=dt, nx_range=(4, 8), nyz_range=(2, 3))
    probs.append(config("c4", nx=3, ny=3, nz=3, dt=dt))
    # slices beyond the LDS budget on one workgroup, inside it on a team of 4 or more
    probs += batch_instances(n_inst=1, seed=9, dt=dt, nx_range=(40, 40), nyz_range=(8, 8))
    return probs


def _states(b, n):
    return [b.get_state(i) for i in range(n)]


@pytest.mark.parametrize("prec", ["f64", "mixed_f32"])
def test_one_list_is_bit_identical_to_one_workgroup_per_instance(prec):
    from paper_2405_05213_amd import batch_from_problems
    probs = _probs()
    say(f"[batch plan] one list of {len(probs)} instances, {prec}")
    a = batch_from_problems(probs, m_max=32, precision=prec)
    a.step(probs[0].dt, 5)
    ref = _states(a, len(probs))
    b = batch_from_problems(probs, m_max=32, precision=prec)
    b.plan(max_workgroups=1)
    # one list per material model (one launch per model)
    assert b.plan_of(0) == (1, len({p.model for p in probs}))
    b.step(probs[0].dt, 5)
    for (t0, u0, v0), (t1, u1, v1) in zip(ref, _states(b, len(probs))):
        assert t0 == t1 and np.array_equal(u0, u1) and np.array_equal(v0, v1)
    a.close()
    b.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-8), ("mixed_f32", 1e-5)])
def test_teams_match_the_oracle(prec, tol):
    from paper_2405_05213_amd import batch_from_problems
    probs = _probs()
    dt = probs[0].dt
    b = batch_from_problems(probs, m_max=32, precision=prec)
    b.plan(max_workgroups=0, serial=0.0)            # room for teams: the costly instances get them
    teams = [b.plan_of(i)[0] for i in range(len(probs))]
    say(f"[batch plan] teams {teams}, {b.plan_of(0)[1]} workgroups, {prec}")
    assert max(teams) > 1
    n = 6
    b.step(dt, n)
    for i, p in enumerate(probs):
        t, u, v = b.get_state(i)
        orc = Propagator(p, m_max=32)
        orc.run(dt, n)
        eu, ev = maxrel(u, orc.u()), maxrel(v, orc.v())
        say(f"  instance {i} team {teams[i]} nodes {p.n_nodes}: u {eu:.1e} v {ev:.1e}")
        assert abs(t - orc.t) < 1e-15
        assert eu < tol and ev < tol
    b.close()


def test_mixed_plan_and_autotune_leave_the_states_and_match_the_oracle():
    from paper_2405_05213_amd import batch_from_problems
    probs = _probs()
    dt = probs[0].dt
    b = batch_from_problems(probs, m_max=32)
    b.step(dt, 2)
    before = _states(b, len(probs))
    w, ms = b.autotune(dt, steps=3)
    say(f"[batch plan] autotune: {w} workgroups, {ms:.3f} ms/step, teams "
        f"{[b.plan_of(i)[0] for i in range(len(probs))]}")
    for (t0, u0, v0), (t1, u1, v1) in zip(before, _states(b, len(probs))):
        assert t0 == t1 and np.array_equal(u0, u1) and np.array_equal(v0, v1)
    # lists and teams in one launch: at most four workgroups per launch for five instances
    b.plan(max_workgroups=4, serial=0.0)
    teams = [b.plan_of(i)[0] for i in range(len(probs))]
    assert b.plan_of(0)[1] <= 4 * len({p.model for p in probs})
    b.step(dt, 4)
    for i, p in enumerate(probs):
        t, u, v = b.get_state(i)
        orc = Propagator(p, m_max=32)
        orc.run(dt, 6)
        assert maxrel(u, orc.u()) < 1e-8 and maxrel(v, orc.v()) < 1e-8, (i, teams)
    b.close()
