"""HIP path vs the CPU oracle, element by element, on seeded workloads (needs an MI355X)."""
import numpy as np
import pytest

from workloads import config, distort
from oracle import krylov
from tests.gpu_util import from_gpu_vec, pair, maxrel, say, svk_of, to_gpu_vec, yeoh_rubber_of

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _np(t):
    return t.detach().cpu().numpy()


CASES_H = [
    ("linear", "c1", {}, False),
    ("linear", "c1", {}, True),
    ("linear", "c1", {}, "renumbered"),
    ("linear", "c1", dict(nx=19, ny=9, nz=5), False),
    ("linear", "bar", dict(nx=16), False),                 # lattice with no interior nodes
    ("linear", "c1", dict(nx=33, ny=9, nz=6), False),      # interior tiles cut in x, y and z
    ("nh", "c3", dict(nx=8, ny=2, nz=2), False),
    ("nh", "c3", dict(nx=8, ny=2, nz=2), True),
    ("yeoh", "c4", dict(nx=4, ny=3, nz=3), True),
    ("svk", "c3", dict(nx=8, ny=2, nz=2), False),
    ("svk", "c3", dict(nx=8, ny=2, nz=2), True),
    ("yeoh3", "c4", dict(nx=4, ny=3, nz=3), True),
    # uniformly sheared lattices: every element the same parallelepiped (congruent) with a
    # full J^{-1}, which must not take the diagonal form of axis-aligned boxes
    ("nh", "c3", dict(nx=8, ny=2, nz=2), "sheared"),
    ("yeoh", "c4", dict(nx=4, ny=3, nz=3), "sheared"),
    ("linear", "c1", {}, "sheared"),
]


def sheared(p):
    """The problem on the lattice mapped by a fixed shear (an affine map of the whole mesh)."""
    S = np.array([[1.0, 0.3, 0.1], [0.0, 1.0, 0.2], [0.0, 0.0, 1.0]])
    return p.with_(xyz=p.xyz @ S.T, name=p.name + "-sheared")


@pytest.mark.parametrize("model,name,over,distorted", CASES_H)
@pytest.mark.parametrize("prec", ["f64", "mixed_f32"])
def test_apply_H_matches_oracle(model, name, over, distorted, prec):
    """Operator apply (weak-form term 2 with the secant split): y = H(u) x on all DOFs."""
    say(f"[apply_H] {model} {name} {over} distorted={distorted} prec={prec}")
    p = config(name, **over)
    if model == "svk":
        p = svk_of(p)
    elif model == "yeoh3":
        p = yeoh_rubber_of(p)
    if distorted == "renumbered":
        p = renumbered(p)
    elif distorted == "sheared":
        p = sheared(p)
    elif distorted:
        p = distort(p, 0.2, seed=5)
    ctx, orc = pair(p, precision=prec)
    rng = np.random.default_rng(3)
    n3 = 3 * p.n_nodes
    x = rng.normal(size=n3)
    # linearisation point: random nodal displacements of 3 % of the extent (0.3 % on the
    # sheared lattice, whose skewed cells then reach random strains of about 30 %, where the
    # FP32 operator's error grows to 9e-6 in the nodal and the modal element form alike)
    amp = 0.003 if distorted == "sheared" else 0.03
    u = None if model == "linear" else amp * rng.normal(size=n3) * (p.xyz.max() - p.xyz.min())
    y = torch.zeros(n3, dtype=torch.float64, device=DEV)
    ctx.apply_H(None if u is None else _t(u), _t(x), y)
    ref = orc.fem.H_apply(u, x)
    tol = 1e-12 if prec == "f64" else 2e-6
    assert maxrel(_np(y), ref) < tol


@pytest.mark.parametrize("m,scale", [(1, 0.3), (6, 0.9), (12, 3.0), (30, 40.0), (48, 1000.0), (64, 250.0), (128, 900.0),
                                     (256, 2000.0)])
def test_expm_matches_oracle(m, scale):
    say(f"[expm] m={m} scale={scale}")
    p = config("c1")
    ctx, _ = pair(p, m_max=256)
    rng = np.random.default_rng(m)
    H = np.triu(rng.normal(size=(m, m)), -1)
    H *= scale / krylov.norm1(H)
    E = ctx.expm(H)
    R = krylov.expm(H)
    assert np.abs(E - R).max() <= 1e-13 * max(1.0, np.abs(R).max()) * max(1.0, scale / 10)


def test_expm_closed_forms():
    """exp(H) on the GPU against closed forms, independent of the oracle: 1 x 1 matrices (the
    scalar exponential, up to 6 squarings), 2 x 2 rotation generators (cos / sin, up to 7
    squarings), the zero matrix (the identity, exactly) and a nilpotent matrix (its finite
    Taylor sum)."""
    import math
    say("[expm] closed forms")
    ctx, _ = pair(config("c1"), m_max=256)
    for h in (-30.0, -1.0, 0.0, 0.5, 3.0, 40.0):
        e = ctx.expm(np.array([[h]]))[0, 0]
        assert abs(e - math.exp(h)) <= 1e-14 * math.exp(h) * max(1.0, abs(h)), h
    for th in (0.3, 5.0, 100.0):
        E = ctx.expm(np.array([[0.0, -th], [th, 0.0]]))
        R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        assert np.abs(E - R).max() <= 1e-15 * max(1.0, th), th
    assert np.array_equal(ctx.expm(np.zeros((5, 5))), np.eye(5))
    N = np.triu(np.random.default_rng(7).normal(size=(6, 6)), 1)
    S, P = np.eye(6), np.eye(6)
    for k in range(1, 6):
        P = P @ N / k
        S = S + P
    assert np.abs(ctx.expm(N) - S).max() <= 1e-14 * np.abs(S).max()


@pytest.mark.parametrize("ortho", [0, 1])
@pytest.mark.parametrize("name,over,workgroups", [("c1", {}, 1), ("c1", {}, 4), ("c2", dict(nx=20, ny=4, nz=4), 0),
                                                  ("c2", dict(nx=20, ny=4, nz=4), 37)])
def test_arnoldi_matches_oracle(name, over, workgroups, ortho):
    """Arnoldi-MGS (sequential and compact-WY forms): same Hessenberg matrix and basis as the
    oracle on the same operator."""
    say(f"[arnoldi] {name} {over} G={workgroups} ortho={ortho}")
    p = config(name, **over)
    ctx, orc = pair(p, m_max=40, workgroups=workgroups, ortho=ortho)
    assert ctx.orthogonalization() == ortho
    rng = np.random.default_rng(7)
    N = orc.N
    w = np.concatenate([orc.Mh * rng.normal(0, 1e-5, N), orc.Mh * rng.normal(0, 1e-2, N), [1.0]])
    L, Lp = ctx.vector_length()
    wg = _t(to_gpu_vec(orc, w, Lp))
    m = 30
    V = torch.zeros((m + 1) * Lp, dtype=torch.float64, device=DEV)
    dt = 1e-4
    H, steps = ctx.arnoldi(None, dt, 1.0, wg, m, V)
    assert steps == m
    pbar = orc.P0bar
    Vo, Ho, beta, so = krylov.arnoldi_mgs(lambda v: orc.A_apply(v, dt, None, pbar), w, m)
    assert so == m
    scale = np.abs(Ho).max()
    assert np.abs(H - Ho).max() <= 1e-9 * scale
    Vg = _np(V).reshape(m + 1, Lp)
    for j in (0, 1, 5, m):
        assert maxrel(from_gpu_vec(orc, Vg[j]), Vo[j]) < 1e-8


@pytest.mark.parametrize("check_every", [4, 1])
@pytest.mark.parametrize("ortho", [0, 1])
@pytest.mark.parametrize("dt,workgroups", [(2e-5, 1), (1e-4, 2), (4e-4, 3)])
def test_expv_matches_oracle(dt, workgroups, ortho, check_every):
    say(f"[expv] c1 dt={dt} G={workgroups} ortho={ortho} check_every={check_every}")
    p = config("c1")
    ctx, orc = pair(p, m_max=48, check_every=check_every, workgroups=workgroups, ortho=ortho)
    rng = np.random.default_rng(11)
    N = orc.N
    w = np.concatenate([orc.Mh * rng.normal(0, 1e-5, N), orc.Mh * rng.normal(0, 1e-2, N), [1.0]])
    L, Lp = ctx.vector_length()
    y = torch.zeros(Lp, dtype=torch.float64, device=DEV)
    m, k, eps = ctx.expv(None, dt, 1.0, _t(to_gpu_vec(orc, w, Lp)), y)
    yo, info = krylov.expv(lambda v, f: orc.A_apply(v, f, None, orc.P0bar), w, dt, tol=p.tol, m_max=48,
                           check_every=check_every, state={})
    assert k == info["k"] and m == info["m"][-1]
    assert maxrel(from_gpu_vec(orc, _np(y)), yo) < 1e-9


@pytest.mark.parametrize("ortho", [0, 1])
@pytest.mark.parametrize("mode", ["fixed", "adaptive", "adaptive_every_step"])
def test_linear_steps_c1(mode, ortho):
    """200 steps of the 10x2x2 linear cantilever (dt 1e-4, tol 1e-10) against the oracle; the
    adaptive runs estimate the error every fourth or every Arnoldi step and must pick the
    oracle's subspace size at every step."""
    say(f"[steps] c1 linear {mode} ortho={ortho}")
    p = config("c1")
    kw = {"fixed": dict(m_max=64, m_fixed=32, k_fixed=1), "adaptive": dict(m_max=64),
          "adaptive_every_step": dict(m_max=64, check_every=1)}[mode]
    kw["ortho"] = ortho
    ctx, orc = pair(p, **kw)
    ctx.step(p.dt, p.n_steps)
    t, u, v = ctx.get_state()
    orc.run(p.dt, p.n_steps)
    assert abs(t - orc.t) < 1e-15
    assert maxrel(u, orc.u()) < 1e-8
    assert maxrel(v, orc.v()) < 1e-8
    ke, se, we = ctx.energy()
    ko, so_, wo = orc.energies()
    assert abs(ke - ko) <= 1e-8 * (ko + so_) and abs(se - so_) <= 1e-8 * (ko + so_)
    assert abs(we - wo) <= 1e-8 * abs(wo)
    if mode != "fixed":
        log = ctx.step_log(p.n_steps)
        mo = np.array([r["corr"]["m"][0] for r in orc.log])
        assert np.array_equal(log["m_corr"], mo)


@pytest.mark.parametrize("model,name,over", [("nh", "c3", dict(nx=8, ny=2, nz=2, dt=5e-4)),
                                              ("yeoh", "c4", dict(nx=3, ny=3, nz=3, dt=2e-3)),
                                              ("svk", "c3", dict(nx=8, ny=2, nz=2, dt=5e-4)),
                                              ("yeoh3", "c4", dict(nx=3, ny=3, nz=3, dt=2e-3))])
@pytest.mark.parametrize("mode", ["fixed", "adaptive"])
@pytest.mark.parametrize("ortho", [0, 1])
def test_nonlinear_steps(model, name, over, mode, ortho):
    """Predictor-corrector steps of the Neo-Hookean / Yeoh / St. Venant-Kirchhoff solids
    against the oracle."""
    say(f"[steps] {model} {name} {over} {mode} ortho={ortho}")
    p = config(name, **over)
    if model == "svk":
        p = svk_of(p)
    elif model == "yeoh3":
        p = yeoh_rubber_of(p)
    n = 12
    kw = dict(m_max=48) if mode == "adaptive" else dict(m_max=48, m_fixed=24, k_fixed=1)
    kw["ortho"] = ortho
    ctx, orc = pair(p, **kw)
    ctx.step(p.dt, n)
    t, u, v = ctx.get_state()
    orc.run(p.dt, n)
    assert maxrel(u, orc.u()) < 1e-8
    assert maxrel(v, orc.v()) < 1e-8
    ke, se, we = ctx.energy()
    ko, so_, wo = orc.energies()
    assert abs(se - so_) <= 1e-8 * (ko + so_ + abs(wo))


def renumbered(p, seed=9):
    """The same mesh with a random node numbering: congruent, not a lattice."""
    import dataclasses
    rng = np.random.default_rng(seed)
    perm = rng.permutation(p.n_nodes)            # new id of old node
    inv = np.argsort(perm)
    clamped = np.sort(3 * perm[np.asarray(p.clamped) // 3] + np.asarray(p.clamped) % 3) if len(p.clamped) else p.clamped
    faces = perm[np.asarray(p.faces)] if len(p.faces) else p.faces
    def vec(v):
        return np.asarray(v).reshape(-1, 3)[inv].ravel()
    return dataclasses.replace(p, xyz=p.xyz[inv], conn=perm[p.conn].astype(p.conn.dtype), clamped=clamped,
                               faces=faces, u0=vec(p.u0), v0=vec(p.v0), grid=None)


@pytest.mark.parametrize("name,over,mode,expect", [("c1", {}, "box", 2), ("c2", dict(nx=20, ny=4, nz=4), "box", 2),
                                                   ("c1", {}, "renumbered", 1), ("c1", {}, "distorted", 0)])
def test_congruence_detection(name, over, mode, expect):
    """Box meshes with coordinates i*h (rounding noise in J) are congruent lattices; a random
    renumbering stays congruent but is no lattice; distorted meshes are neither."""
    say(f"[congruence] {name} {over} {mode}")
    p = config(name, **over)
    if mode == "distorted":
        p = distort(p, 0.2, seed=5)
    elif mode == "renumbered":
        p = renumbered(p)
    ctx, _ = pair(p)
    g, chunk, cong = ctx.launch()
    assert cong == expect
    assert g >= 1 and chunk >= 64 and g * chunk >= 2 * 3 * p.n_nodes + 1


# FP32 operator error on this steel beam (operator parity: 2-3e-6 relative); each step's
# rounding perturbs the energy by about that much, independently of the others
FP32_OP_ERR = 3e-6


@pytest.mark.parametrize("prec,fixed", [("f64", False), ("f64", True), ("mixed_f32", False), ("mixed_f32", True)])
def test_energy_conservation_free_vibration(prec, fixed):
    """Unloaded cantilever with random initial velocity, 60 steps (adaptive subspace, or fixed
    at m = 48 with 2 substeps): the propagator conserves the discrete energy up to the Krylov
    tolerance in FP64 (~1e-8 adaptive, ~3e-9 at the fixed m) and up to the FP32 operator's
    rounding in the mixed form, where each step adds an independent error of about the
    operator's relative error e (2-3e-6 on this beam: a bending field is a small difference of
    large element forces), so the drift is a random walk bounded by about sqrt(n) e: the test
    takes 1.3 sqrt(n) e (3e-5 at n = 60; measured 5e-6 - 1.6e-5, the same at the fixed and the
    adaptive subspace, and of either sign over 20 ... 120 steps).  This is outside the 1e-6
    energy gate of the batched rubber blocks, which their FP32 form meets.  An element kernel
    that loses the deformation to a large common translation drifts 1e-3."""
    say(f"[energy] c2 20x4x4 {prec} {'fixed m' if fixed else 'adaptive'}")
    p = config("c2", nx=20, ny=4, nz=4)
    kw = dict(m_max=64, m_fixed=48, k_fixed=2) if fixed else dict(m_max=64)
    ctx, _ = pair(p, precision=prec, **kw)
    n = 60
    tol = 1e-7 if prec == "f64" else 1.3 * np.sqrt(n) * FP32_OP_ERR
    e0 = ctx.energy()
    ctx.step(p.dt, n)
    e1 = ctx.energy()
    E0, E1 = e0[0] + e0[1] - e0[2], e1[0] + e1[1] - e1[2]
    say(f"  relative energy drift {abs(E1 - E0) / (e0[0] + e0[1]):.2e} (bound {tol:.1e})")
    assert abs(E1 - E0) <= tol * (e0[0] + e0[1])
    ctx.close()


@pytest.mark.parametrize("ortho", [0, 1])
def test_slices_in_device_memory(ortho):
    """A team too small for its Krylov-vector slices to fit in LDS keeps them in device
    memory: same steps as the oracle (and the LDS layout) on a 40x8x8 cantilever."""
    say(f"[slices in device memory] ortho={ortho}")
    p = config("c2", nx=40, ny=8, nz=8)
    ctx, orc = pair(p, m_max=48, workgroups=2, ortho=ortho)
    assert ctx.slices_in_device_memory()
    ref, _ = pair(p, m_max=48, ortho=ortho)
    assert not ref.slices_in_device_memory()
    n = 3
    ctx.step(p.dt, n)
    ref.step(p.dt, n)
    orc.run(p.dt, n)
    _, u, v = ctx.get_state()
    _, ur, vr = ref.get_state()
    assert maxrel(u, orc.u()) < 1e-8 and maxrel(v, orc.v()) < 1e-8
    assert maxrel(u, ur) < 1e-9 and maxrel(v, vr) < 1e-9


# (model, workload, overrides, steps, tolerance on u, tolerance on v).  Measured errors: the
# soft solids 4e-10 - 5e-8; the steel cantilever u 9.5e-7, v 4.1e-5 after 40 steps - its
# smooth bending response is a small difference of large element forces (E = 200 GPa), so the
# FP32 rounding of those forces (about 1e-7 relative) appears amplified about 1e3 times in the
# velocity.  Tolerances keep a margin of about 5 over the measured errors.
MIXED_STEP_CASES = [("linear", "c1", dict(dt=1e-4), 40, 5e-6, 2e-4),
                    ("nh", "c3", dict(nx=8, ny=2, nz=2, dt=5e-4), 12, 1e-6, 1e-6),
                    ("yeoh", "c4", dict(nx=3, ny=3, nz=3, dt=2e-3), 12, 1e-6, 1e-6),
                    ("svk", "c3", dict(nx=8, ny=2, nz=2, dt=5e-4), 12, 1e-6, 1e-6),
                    ("yeoh3", "c4", dict(nx=3, ny=3, nz=3, dt=2e-3), 12, 1e-6, 1e-6)]


@pytest.mark.parametrize("model,name,over,n,tol_u,tol_v", MIXED_STEP_CASES)
def test_steps_mixed_f32(model, name, over, n, tol_u, tol_v):
    """Time steps with the FP32 operator (Krylov, exponential and state in FP64) against the
    FP64 oracle, fixed subspace so that both take the same path.  The operator's FP32
    rounding is the only difference from the FP64 path."""
    say(f"[steps mixed_f32] {model} {name} {over} n={n}")
    p = config(name, **over)
    if model == "svk":
        p = svk_of(p)
    elif model == "yeoh3":
        p = yeoh_rubber_of(p)
    ctx, orc = pair(p, m_max=48, m_fixed=24, k_fixed=1, precision="mixed_f32")
    ctx.step(p.dt, n)
    t, u, v = ctx.get_state()
    orc.run(p.dt, n)
    eu, ev = maxrel(u, orc.u()), maxrel(v, orc.v())
    say(f"  rel err u {eu:.2e} v {ev:.2e}")
    assert eu < tol_u and ev < tol_v


@pytest.mark.parametrize("name,over", [("c2", dict(nx=20, ny=4, nz=4)), ("c3", dict(nx=8, ny=2, nz=2))])
def test_autotune_keeps_state_and_parity(name, over):
    """The launch autotuner times projections of the current operator without touching the
    state, leaves the context on the fastest team size it found, and steps from there agree
    with the oracle."""
    say(f"[autotune] {name} {over}")
    p = config(name, **over)
    ctx, orc = pair(p, m_max=48)
    ctx.step(p.dt, 2)
    t0, u0, v0 = ctx.get_state()
    G, ms = ctx.autotune(p.dt, m_trial=16, trials=2)
    say(f"  G = {G}, {ms:.3f} ms per projection")
    assert G >= 1 and ms > 0.0
    assert ctx.launch()[0] == G
    t1, u1, v1 = ctx.get_state()
    assert t1 == t0 and np.array_equal(u1, u0) and np.array_equal(v1, v0)
    ctx.step(p.dt, 3)
    t, u, v = ctx.get_state()
    orc.run(p.dt, 5)
    assert maxrel(u, orc.u()) < 1e-8 and maxrel(v, orc.v()) < 1e-8


@pytest.mark.parametrize("model,name,over", [("nh", "c3", dict(nx=8, ny=2, nz=2, dt=1e-4)),
                                              ("linear", "c1", dict(dt=1e-5))])
def test_scaled_s0_matches_oracle(model, name, over):
    """ep_set_krylov with s0 = EP_S0_SCALED (augmented entry at the problem's scale, fixed at the
    first step) against the oracle with the same rule, adaptive subspace."""
    from paper_2405_05213_amd.ep import S0_SCALED
    say(f"[steps] scaled s0 {model} {name} {over}")
    p = config(name, **over)
    ctx, orc = pair(p, m_max=48, s0=S0_SCALED)
    n = 10
    ctx.step(p.dt, n)
    orc.run(p.dt, n)
    t, u, v = ctx.get_state()
    eu, ev = maxrel(u, orc.u()), maxrel(v, orc.v())
    say(f"  s0 = {orc.s0:.3e}, err u {eu:.2e} v {ev:.2e}")
    assert eu < 1e-8 and ev < 1e-8
    assert np.array_equal(ctx.step_log(n)["m_corr"], np.array([r["corr"]["m"][0] for r in orc.log]))
