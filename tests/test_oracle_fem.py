"""Pins of the oracle's finite-element pieces against textbook identities and exact quadrature."""
import numpy as np
import pytest

from workloads import box_mesh, box_face_quads, config, distort
from oracle import fem
from oracle.material import Material, lame_from_E_nu


def test_shape_partition_of_unity_and_kronecker():
    rng = np.random.default_rng(0)
    xi = rng.uniform(-1, 1, size=(50, 3))
    N, dN = fem.shape(xi)
    assert np.allclose(N.sum(-1), 1.0, atol=1e-15)
    assert np.allclose(dN.sum(-2), 0.0, atol=1e-15)
    Nv, _ = fem.shape(fem.XI_NODES)
    assert np.allclose(Nv, np.eye(8), atol=1e-15)
    # derivative against central differences
    h = 1e-6
    for d in range(3):
        e = np.zeros(3); e[d] = h
        Np, _ = fem.shape(xi + e)
        Nm, _ = fem.shape(xi - e)
        assert np.allclose((Np - Nm) / (2 * h), dN[..., d], atol=1e-9)


def test_gauss_rule_exactness():
    P, W = fem.gauss_rule(2)
    assert np.isclose(W.sum(), 8.0)
    # 2-point Gauss integrates x^2 y^2 z^2 exactly over [-1,1]^3 (= (2/3)^3)
    assert np.isclose((W * (P ** 2).prod(1)).sum(), (2.0 / 3.0) ** 3, rtol=1e-14)


def _sheared_element():
    # affine map of the reference cube: X = c + B xi
    B = np.array([[0.3, 0.05, 0.02], [0.01, 0.2, 0.04], [0.03, -0.02, 0.25]])
    X = (fem.XI_NODES @ B.T) + np.array([1.0, 2.0, 3.0])
    return X, B


def test_patch_test_linear_field_on_distorted_mesh():
    """A linear displacement field has the exact constant gradient at every Gauss point,
    and (linear material) produces zero net force at interior nodes."""
    p = distort(config("c1", nx=4, ny=3, nz=3), 0.25, seed=3)
    A = np.array([[1e-3, 2e-4, -3e-4], [5e-4, -1e-3, 2e-4], [1e-4, 3e-4, 2e-3]])
    u = (p.xyz @ A.T).ravel()
    d = fem.Discretization(p.xyz, p.conn, Material("linear", (200e9, 0.3)), 7800.0)
    D = d.grad(u)
    assert np.allclose(D, A, atol=1e-15)
    R = d.internal_force(u)
    lo, hi = p.xyz.min(0), p.xyz.max(0)
    interior = np.all((p.xyz > lo + 1e-9) & (p.xyz < hi - 1e-9), axis=1)
    scale = np.abs(R).max()
    assert np.abs(R.reshape(-1, 3)[interior]).max() <= 1e-10 * scale
    # rigid translation: zero force everywhere
    assert np.abs(d.internal_force(np.tile([1e-3, -2e-3, 5e-4], p.n_nodes))).max() < 1e-6


def test_element_stiffness_nullspace_symmetry_and_exact_quadrature():
    X, B = _sheared_element()
    lam, mu = lame_from_E_nu(200e9, 0.3)
    conn = np.arange(8)[None]
    g2, w2 = fem.geometry(X, conn, 2)
    g3, w3 = fem.geometry(X, conn, 3)
    K2 = fem.element_stiffness(g2[0], w2[0], lam, mu)
    K3 = fem.element_stiffness(g3[0], w3[0], lam, mu)
    assert np.allclose(K2, K2.T, rtol=0, atol=1e-12 * np.abs(K2).max())
    # affine element: integrand is degree <= 2 per direction, 2-point Gauss is exact
    assert np.allclose(K2, K3, rtol=0, atol=1e-12 * np.abs(K2).max())
    ev = np.linalg.eigvalsh(K2)
    assert np.sum(np.abs(ev) < 1e-9 * ev.max()) == 6          # six rigid-body modes
    # rigid rotation about an axis is in the null space
    W = np.array([[0, -1, 2], [1, 0, -3], [-2, 3, 0]], float) * 1e-3
    assert np.abs(K2 @ (X @ W.T).ravel()).max() < 1e-9 * np.abs(K2).max() * 1e-3


def test_lumped_mass_total():
    p = config("c1", nx=5, ny=2, nz=3)
    M = fem.lumped_mass(p.xyz, p.conn, 7800.0)
    V = 1.0 * 0.2 * 0.2
    assert np.isclose(M.sum(), 3 * 7800.0 * V, rtol=1e-14)
    # affine (sheared) element: vertex rule is exact for the volume
    X, B = _sheared_element()
    Me = fem.lumped_mass(X, np.arange(8)[None], 2.0)
    assert np.isclose(Me.sum() / 3, 2.0 * 8 * np.linalg.det(B), rtol=1e-14)
    # uniform box: each element contributes rho V_e / 8 to each of its nodes
    m = M[::3]
    ve = V / p.n_elems
    counts = np.bincount(p.conn.ravel(), minlength=p.n_nodes)
    assert np.allclose(m, counts * 7800.0 * ve / 8.0, rtol=1e-13)


def test_traction_load_resultant_and_distribution():
    nx, ny, nz = 3, 2, 4
    xyz, conn = box_mesh(nx, ny, nz, 1.0, 0.2, 0.4)
    faces = box_face_quads(nx, ny, nz, 0, 1)
    t0 = np.array([0.0, 3.0, -7.0])
    P = fem.traction_load(xyz, faces, t0)
    area = 0.2 * 0.4
    assert np.allclose(P.reshape(-1, 3).sum(0), t0 * area, rtol=1e-14)
    # a uniform traction on a rectangle gives t A_f / 4 to each corner of each face
    Af = area / (ny * nz)
    cnt = np.zeros(xyz.shape[0]); np.add.at(cnt, faces.ravel(), 1)
    assert np.allclose(P.reshape(-1, 3)[:, 2], cnt * t0[2] * Af / 4, rtol=1e-13)


def test_face_orientation_outward():
    nx, ny, nz = 2, 3, 2
    xyz, _ = box_mesh(nx, ny, nz, 1.0, 1.0, 1.0)
    c = xyz.mean(0)
    for axis in range(3):
        for side in (0, 1):
            q = box_face_quads(nx, ny, nz, axis, side)
            X = xyz[q]
            n = np.cross(X[:, 1] - X[:, 0], X[:, 3] - X[:, 0])
            assert np.all(((X.mean(1) - c) * n).sum(1) > 0)
