"""Pins of the oracle's quadratic (27-node, Q2) hexahedron: the paper's element (Sec. 2.2:
quadratic Lagrange interpolation, Gauss quadrature for the internal force and the loads,
Gauss-Lobatto quadrature for a diagonal mass)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import fem
from oracle.material import Material
from oracle.stepper import Propagator
from workloads import config, distort, q2_of

MATS = [("linear", (200e9, 0.3)), ("nh", (0.4e6, 2.0e6)), ("yeoh", (1.0e5, -1.0e3, 10.0, 1.0e-6)),
        ("svk", (2.0e6, 0.4e6))]


def test_shape27_identities():
    rng = np.random.default_rng(0)
    xi = rng.uniform(-1, 1, size=(60, 3))
    N, dN = fem.shape27(xi)
    assert np.allclose(N.sum(-1), 1.0, atol=1e-14)
    assert np.allclose(dN.sum(-2), 0.0, atol=1e-14)
    Nv, _ = fem.shape27(fem.XI_NODES27)
    assert np.allclose(Nv, np.eye(27), atol=1e-15)
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        Np, _ = fem.shape27(xi + e)
        Nm, _ = fem.shape27(xi - e)
        assert np.allclose((Np - Nm) / (2 * h), dN[..., d], atol=1e-8)
    # completeness: every monomial x^i y^j z^k with i, j, k <= 2 is interpolated exactly
    for (i, j, k) in [(2, 2, 2), (1, 2, 0), (2, 0, 1), (0, 0, 0), (1, 1, 1)]:
        f = lambda p: p[..., 0] ** i * p[..., 1] ** j * p[..., 2] ** k
        assert np.allclose(N @ f(fem.XI_NODES27), f(xi), atol=1e-14)


def _q2_box(distorted=False, model="linear", params=(200e9, 0.3)):
    p = q2_of(config("c1", nx=4, ny=4, nz=4))
    if distorted:
        p = distort(p, 0.2, seed=4)       # interior nodes moved: curved quadratic elements
    return p, fem.Discretization(p.xyz, p.conn, Material(model, params), 7800.0, elem="hex27")


def test_patch_test_on_curved_q2_elements():
    """A linear displacement field has its exact gradient at every Gauss point of curved
    isoparametric elements and gives zero net force at interior nodes; a translation gives
    zero force."""
    p, d = _q2_box(distorted=True)
    A = np.array([[1e-3, 2e-4, -3e-4], [5e-4, -1e-3, 2e-4], [1e-4, 3e-4, 2e-3]])
    u = (p.xyz @ A.T).ravel()
    assert np.allclose(d.grad(u), A, atol=1e-14)
    R = d.internal_force(u)
    lo, hi = p.xyz.min(0), p.xyz.max(0)
    interior = np.all((p.xyz > lo + 1e-9) & (p.xyz < hi - 1e-9), axis=1)
    assert interior.sum() > 0
    assert np.abs(R.reshape(-1, 3)[interior]).max() <= 1e-10 * np.abs(R).max()
    assert np.abs(d.internal_force(np.tile([1e-3, -2e-3, 5e-4], p.n_nodes))).max() < 1e-6


def test_q2_element_stiffness_nullspace_symmetry_exact_quadrature():
    """K_e (81 x 81): symmetric, six rigid modes, and on an affine element 3x3x3 Gauss equals
    4x4x4 Gauss (the integrand is of degree 4 per direction)."""
    B = np.array([[0.3, 0.05, 0.02], [0.01, 0.2, 0.04], [0.03, -0.02, 0.25]])
    X = fem.XI_NODES27 @ B.T + np.array([1.0, 2.0, 3.0])
    conn = np.arange(27)[None, :]
    mats = []
    for ng in (3, 4):
        gN, wd = fem.geometry(X, conn, ng, "hex27")
        mats.append(fem.element_stiffness(gN[0], wd[0], 1.2e9, 0.8e9))
    K3, K4 = mats
    assert np.abs(K3 - K4).max() <= 1e-12 * np.abs(K4).max()
    assert np.abs(K3 - K3.T).max() <= 1e-12 * np.abs(K3).max()
    ev = np.linalg.eigvalsh(0.5 * (K3 + K3.T))
    assert np.sum(np.abs(ev) < 1e-9 * ev.max()) == 6


def test_q2_gll_mass_is_diagonal_positive_and_exact_in_total():
    # curved elements: positive nodal masses (3-point Gauss-Lobatto is exact to degree 3 per
    # direction, below det J of a curved Q2 element, so the total is close to rho V, not exact)
    p, d = _q2_box(distorted=True)
    m = d.M[::3]
    assert np.all(m > 0)
    lo, hi = p.xyz.min(0), p.xyz.max(0)      # distortion keeps the outer box
    assert np.isclose(m.sum(), 7800.0 * np.prod(hi - lo), rtol=1e-3)
    # on the undistorted box each element gives its corner / edge / face / centre nodes
    # rho V_e times (1/3, 4/3, 1/3)^3 / 8
    p2, d2 = _q2_box()
    Vt = np.prod(p2.xyz.max(0) - p2.xyz.min(0))
    assert np.isclose(d2.M[::3].sum(), 7800.0 * Vt, rtol=1e-13)
    Ve = Vt / p2.n_elems
    w = np.array([1.0, 4.0, 1.0]) / 3.0
    ref = np.zeros(p2.n_nodes)
    for e in range(p2.n_elems):
        for a in range(27):
            ref[p2.conn[e, a]] += 7800.0 * Ve / 8.0 * w[a % 3] * w[(a // 3) % 3] * w[a // 9]
    assert np.allclose(d2.M[::3], ref, rtol=1e-13)


def test_nine_node_face_load_is_the_consistent_simpson_distribution():
    """A uniform traction t on a flat face of area A loads its 9 nodes with t A (1, 4, 1) (x)
    (1, 4, 1) / 36 (the integrals of the biquadratic shape functions); the resultant is t A."""
    p = q2_of(config("c1", nx=2, ny=2, nz=2))
    assert p.faces.shape == (1, 9)
    t0 = np.array([0.0, 0.0, -1e5])
    P = fem.traction_load(p.xyz, p.faces, t0)
    A = 0.2 * 0.2
    w = np.array([1.0, 4.0, 1.0])
    expect = np.outer(w, w).ravel() / 36.0 * A * t0[2]
    assert np.allclose(P[3 * p.faces[0] + 2], expect, rtol=1e-13)
    assert np.isclose(P[2::3].sum(), A * t0[2], rtol=1e-13)


@pytest.mark.parametrize("model,params", MATS)
def test_q2_H_of_u_times_u_is_R_and_H0_is_K(model, params):
    p, d = _q2_box(distorted=True, model=model, params=params)
    rng = np.random.default_rng(5)
    u = rng.normal(size=3 * p.n_nodes)
    u *= 0.05 / np.abs(d.grad(u)).max()
    R = d.internal_force(u)
    if model != "linear":
        assert np.abs(d.H_apply(u, u) - R).max() <= 1e-12 * np.abs(R).max()
    x = rng.normal(size=3 * p.n_nodes)
    Hx = d.H_apply(np.zeros_like(x) if model != "linear" else None, x)
    assert np.abs(Hx - d.stiffness() @ x).max() <= 1e-11 * np.abs(Hx).max()


def _bar_first_frequency(nx, elem):
    """Lowest frequency of the nx-element bar of length 1 (y / z DOFs and x = 0 clamped):
    a 1D chain (hex8) or 1D quadratic spectral element (hex27, Gauss-Lobatto mass)."""
    p = config("bar", nx=nx if elem == "hex8" else 2 * nx, h=1.0 / (nx if elem == "hex8" else 2 * nx))
    if elem == "hex27":
        # the hex27 bar of nx elements has the nodes of the 2nx x 2 x 2 hex8 box; the bar's
        # cross-section is one Q2 element, so build it from a 2nx x 2 x 2 lattice
        from workloads import box_mesh_q2
        h = 1.0 / nx
        xyz, conn = box_mesh_q2(nx, 1, 1, 1.0, h, h)
        n = xyz.shape[0]
        x0 = np.where(np.abs(xyz[:, 0]) < 1e-12)[0]
        clamped = np.unique(np.concatenate([3 * np.arange(n) + 1, 3 * np.arange(n) + 2, 3 * x0]))
        p = p.with_(xyz=xyz, conn=conn, clamped=clamped.astype(np.int32), elem="hex27", grid=(nx, 1, 1),
                    u0=np.zeros(3 * n), v0=np.zeros(3 * n))
    pr = Propagator(p)
    K = pr.fem.stiffness().toarray()[np.ix_(pr.free, pr.free)]
    Minv = pr.Mih ** 2
    ev = scipy.linalg.eigvalsh(np.sqrt(Minv)[:, None] * K * np.sqrt(Minv)[None, :])
    return float(np.sqrt(ev.min()))


def test_q2_bar_frequency_converges_at_fourth_order():
    """The bar's lowest frequency tends to the continuum pi c / 2 (c^2 = (lambda + 2 mu) / rho):
    the error falls as h^4 with Q2 elements and Gauss-Lobatto mass, h^2 with hex8."""
    lam, mu = 200e9 * 0.3 / (1.3 * 0.4), 200e9 / 2.6
    w_exact = np.pi / 2.0 * np.sqrt((lam + 2 * mu) / 7800.0)
    e27 = [abs(_bar_first_frequency(n, "hex27") - w_exact) / w_exact for n in (2, 4, 8)]
    e8 = [abs(_bar_first_frequency(n, "hex8") - w_exact) / w_exact for n in (4, 8, 16)]
    o27 = np.log2(np.array(e27[:-1]) / np.array(e27[1:]))
    o8 = np.log2(np.array(e8[:-1]) / np.array(e8[1:]))
    assert np.all((o27 > 3.6) & (o27 < 4.5)), (e27, o27)
    assert np.all((o8 > 1.8) & (o8 < 2.3)), (e8, o8)
