"""Pins of the oracle's constitutive laws and the secant split R(u) = H(u) u."""
import numpy as np
import pytest

from workloads import config, distort
from oracle import fem
from oracle.material import Material, Qmat, jm1, cof, lame_from_E_nu

MODELS = [
    ("nh", (0.4e6, 2.0e6)),
    ("yeoh", (5.0e3, 0.0, 0.0, 2.0e-6)),
    ("yeoh", (100.0, -1.0, 0.01, 0.001)),      # rubber constants printed in Sec. 6.2.3
    ("svk", (1.2e6, 0.8e6)),
]


def _rand_D(rng, n, s=0.25):
    return rng.uniform(-s, s, size=(n, 3, 3))


def test_cofactor_and_det_identity():
    """App. A: det F - 1 = P_e : D, with P_e = Q(D)."""
    rng = np.random.default_rng(1)
    D = _rand_D(rng, 200, 0.6)
    assert np.allclose(jm1(D), np.linalg.det(np.eye(3) + D) - 1.0, atol=1e-14)
    Dinv_ok = np.abs(np.linalg.det(D)) > 1e-3
    c = cof(D[Dinv_ok])
    ref = np.linalg.det(D[Dinv_ok])[:, None, None] * np.linalg.inv(np.swapaxes(D[Dinv_ok], 1, 2))
    assert np.allclose(c, ref, atol=1e-12)
    assert np.allclose(Qmat(np.zeros((1, 3, 3))), np.eye(3))


@pytest.mark.parametrize("model,params", MODELS)
def test_pk1_is_energy_derivative(model, params):
    """P = d psi / d F by central differences (checks the App. A stress of each model)."""
    mat = Material(model, params)
    rng = np.random.default_rng(2)
    D = _rand_D(rng, 20)
    P = mat.pk1(D)
    h = 1e-6
    num = np.zeros_like(P)
    for i in range(3):
        for k in range(3):
            E = np.zeros((3, 3)); E[i, k] = h
            num[:, i, k] = (mat.psi(D + E) - mat.psi(D - E)) / (2 * h)
    scale = np.abs(P).max()
    assert np.abs(num - P).max() <= 1e-7 * scale


@pytest.mark.parametrize("model,params", MODELS)
def test_secant_reproduces_stress(model, params):
    """secant(D, .) is linear and secant(D, D) = P(F): H(u) u = R(u) pointwise."""
    mat = Material(model, params)
    rng = np.random.default_rng(3)
    D = _rand_D(rng, 100)
    P = mat.pk1(D)
    assert np.allclose(mat.secant(D, D), P, rtol=0, atol=1e-13 * np.abs(P).max())
    X1, X2 = _rand_D(rng, 100), _rand_D(rng, 100)
    lhs = mat.secant(D, 2.0 * X1 - 3.0 * X2)
    rhs = 2.0 * mat.secant(D, X1) - 3.0 * mat.secant(D, X2)
    assert np.allclose(lhs, rhs, rtol=0, atol=1e-12 * np.abs(lhs).max())


@pytest.mark.parametrize("model,params", MODELS)
def test_secant_at_rest_is_linear_elasticity(model, params):
    mat = Material(model, params)
    lam, mu = mat.small_strain_lame()
    rng = np.random.default_rng(4)
    X = _rand_D(rng, 50)
    lin = Material("linear", (1.0, 0.25))
    lin.lam, lin.mu = lam, mu
    got = mat.secant(np.zeros_like(X), X)
    assert np.allclose(got, lin.secant(None, X), rtol=0, atol=1e-12 * np.abs(got).max())


@pytest.mark.parametrize("model,params", MODELS)
def test_rigid_rotation_is_stress_free(model, params):
    mat = Material(model, params)
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    ax = np.array([1.0, 2.0, -0.5]); ax /= np.linalg.norm(ax)
    Kx = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    R2 = np.eye(3) + np.sin(1.1) * Kx + (1 - np.cos(1.1)) * Kx @ Kx
    D = np.stack([R - np.eye(3), R2 @ R - np.eye(3)])
    scale = max(abs(p) for p in params if p != 0)
    assert np.abs(mat.pk1(D)).max() < 1e-9 * scale


def test_lame_constants():
    lam, mu = lame_from_E_nu(200e9, 0.3)
    assert np.isclose(mu, 200e9 / 2.6)
    assert np.isclose(lam, 200e9 * 0.3 / (1.3 * 0.4))
    # decoupled Neo-Hookean (Yeoh, C20 = C30 = 0): mu = 2 C10, kappa = 2 / D1
    m = Material("yeoh", (5e3, 0.0, 0.0, 2e-6))
    lam2, mu2 = m.small_strain_lame()
    assert np.isclose(mu2, 1e4) and np.isclose(lam2, 1e6 - 2e4 / 3)


# ---------------------------------------------------------------------------
# mesh-level identities
# ---------------------------------------------------------------------------
def _mesh(model, params):
    p = distort(config("c1", nx=3, ny=2, nz=2), 0.2, seed=11)
    return p, fem.Discretization(p.xyz, p.conn, Material(model, params), 1100.0)


@pytest.mark.parametrize("model,params", MODELS)
def test_H_of_u_times_u_equals_R_of_u(model, params):
    p, d = _mesh(model, params)
    rng = np.random.default_rng(5)
    u = 0.02 * rng.normal(size=3 * p.n_nodes)
    R = d.internal_force(u)
    Hu = d.H_apply(u, u)
    assert np.abs(Hu - R).max() <= 1e-12 * np.abs(R).max()
    # the paper's element form sum B^T S gives the same internal force
    Rv = d.internal_force_voigt(u)
    assert np.abs(Rv - R).max() <= 1e-12 * np.abs(R).max()


@pytest.mark.parametrize("model,params", MODELS[:2])
def test_R_is_gradient_of_strain_energy(model, params):
    p, d = _mesh(model, params)
    rng = np.random.default_rng(6)
    u = 0.02 * rng.normal(size=3 * p.n_nodes)
    R = d.internal_force(u)
    h = 1e-7
    for _ in range(4):
        dirn = rng.normal(size=u.size)
        num = (d.strain_energy(u + h * dirn) - d.strain_energy(u - h * dirn)) / (2 * h)
        assert abs(num - R @ dirn) <= 1e-6 * np.abs(R).max() * np.abs(dirn).sum()


@pytest.mark.parametrize("model,params", MODELS)
def test_H_at_rest_equals_linear_stiffness(model, params):
    p, d = _mesh(model, params)
    K = d.stiffness()                    # assembled sum B^T D B with the small-strain constants
    x = np.random.default_rng(7).normal(size=3 * p.n_nodes)
    Hx = d.H_apply(np.zeros_like(x), x)
    assert np.abs(Hx - K @ x).max() <= 1e-11 * np.abs(Hx).max()
