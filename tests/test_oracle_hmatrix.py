"""Pin of the oracle's H(u) against the H-matrices printed in App. A.

The oracle applies H(u) as an operator on X = grad x (oracle/material.py, secant).  Here
the printed 3x3 blocks H_AB of App. A are transcribed term by term, with the nodal sums
that define D_e, S_SVK,e, alpha_e, beta_e and P_e written out from the nodal values, and
assembled into the 24 x 24 element matrix at every Gauss point.  Nothing here calls the
oracle's material code: the blocks use only the shape-function gradients of the element.

  * St. Venant-Kirchhoff: App. A, the H-matrix of the St. Venant-Kirchhoff derivation
    (with its leading 1/2).
  * Yeoh: App. A, the last equation, each term multiplied by the 1/2 of the internal
    virtual work dE = (F^T grad w + grad w^T F) / 2 that precedes it (reading recorded
    in the design notes: without it the printed matrix gives H(u) u = 2 R(u)).
  * compressible Neo-Hookean (the paper's "trivially extended"): the Yeoh blocks with mu
    for alpha_e, without the tr C / 3 term, and lambda ln J / (J - 1) for beta_e.

Checks: element matrix times x equals the oracle's H(u) x (element by element, random x);
the printed blocks times u equal R(u) (the stress P = d psi / d F is pinned by finite
differences in test_oracle_material.py, which also checks H(0) against the linear stiffness).
"""
import numpy as np
import pytest

from workloads import config, distort
from oracle import fem
from oracle.material import Material

I = np.eye(3)


def outer(a, b):
    return np.outer(a, b)


def P_e_printed(du):
    """App. A, the matrix P_e, entry by entry; du[i, j] = d u_(i+1) / d X_(j+1)."""
    u = lambda i, j: du[i - 1, j - 1]
    m = lambda a, b, c, d: u(a, b) * u(c, d) / 3.0        # the \dudxm macro
    p = lambda a, b, c, d: 0.5 * (u(a, b) + u(c, d))      # the \dudxp macro
    P = np.empty((3, 3))
    P[0, 0] = 1 + p(2, 2, 3, 3) + m(2, 2, 3, 3) - m(2, 3, 3, 2)
    P[0, 1] = -0.5 * u(2, 1) + m(2, 3, 3, 1) - m(2, 1, 3, 3)
    P[0, 2] = -0.5 * u(3, 1) + m(2, 1, 3, 2) - m(3, 1, 2, 2)
    P[1, 0] = -0.5 * u(1, 2) + m(1, 3, 3, 2) - m(1, 2, 3, 3)
    P[1, 1] = 1 + p(1, 1, 3, 3) + m(1, 1, 3, 3) - m(1, 3, 3, 1)
    P[1, 2] = -0.5 * u(3, 2) + m(1, 2, 3, 1) - m(1, 1, 3, 2)
    P[2, 0] = -0.5 * u(1, 3) + m(1, 2, 2, 3) - m(1, 3, 2, 2)
    P[2, 1] = -0.5 * u(2, 3) + m(1, 3, 2, 1) - m(1, 1, 2, 3)
    P[2, 2] = 1 + p(1, 1, 2, 2) + m(1, 1, 2, 2) - m(1, 2, 2, 1)
    return P


def element_H_printed(model, params, g, ue):
    """24 x 24 block matrix sum_B H_AB at one Gauss point; g (8, 3) = grad_X N, ue (8, 3)."""
    De = sum(outer(ue[A], g[A]) for A in range(8))             # eq. D_e
    F = I + De
    Finv = np.linalg.inv(F)
    FinvT = Finv.T
    H = np.zeros((24, 24))
    if model == "svk":
        lam, mu = params
        S = np.zeros((3, 3))                                     # eq. S_SVK,e, nodal sums
        for A in range(8):
            S += lam * (g[A] @ ue[A]) * I + mu * (outer(ue[A], g[A]) + outer(g[A], ue[A]))
            for B in range(8):
                S += (lam / 2) * (g[A] @ g[B]) * (ue[B] @ ue[A]) * I \
                    + mu * outer(g[A], g[B]) * (ue[A] @ ue[B])
        for A in range(8):
            for B in range(8):
                blk = 0.5 * (lam * outer(g[A], g[B]) @ (2 * I + De.T)
                             + 2 * mu * (g[B] @ g[A]) * I
                             + mu * outer(g[B], g[A]) @ (2 * I + De.T)
                             + mu * De.T * (g[A] @ g[B])
                             + 2 * (g[B] @ S @ g[A]) * I)
                H[3 * A:3 * A + 3, 3 * B:3 * B + 3] = blk
        return H
    J = np.linalg.det(F)
    Ci = Finv @ FinvT
    trFTF = np.trace(F.T @ F)
    Pe = P_e_printed(De)
    if model == "yeoh":
        C10, C20, C30, D1 = params
        z = trFTF * J ** (-2 / 3) - 3
        alpha = 2 * J ** (-2 / 3) * (C10 + 2 * C20 * z + 3 * C30 * z ** 2)   # eq. alpha_e
        beta = 2 * (1 / D1) * J                                             # eq. beta_e
        for A in range(8):
            for B in range(8):
                blk = (2 * alpha * (g[B] @ Finv @ g[A]) * I
                       + 2 * alpha * (FinvT @ outer(g[B], g[A]))
                       - alpha * (g[B] @ (Ci @ De.T) @ g[A]) * I
                       - alpha * De @ Ci @ outer(g[B], g[A])
                       - (2 / 3) * alpha * Ci @ outer(g[A], g[B]) @ (2 * I + De.T)
                       + 2 * alpha * (g[B] @ (I - Ci * trFTF / 3) @ g[A]) * I
                       + (2 * beta) * Ci @ outer(g[A], g[B]) @ Pe.T
                       + (2 * beta) * (J - 1) * (g[A] @ Ci @ g[B]) * I)
                H[3 * A:3 * A + 3, 3 * B:3 * B + 3] = 0.5 * blk
        return H
    if model == "nh":
        mu, lam = params
        S = mu * (I - Ci) + lam * np.log(J) * Ci
        vol = lam * np.log(J) / (J - 1)
        for A in range(8):
            for B in range(8):
                blk = (2 * mu * (g[B] @ Finv @ g[A]) * I
                       + 2 * mu * (FinvT @ outer(g[B], g[A]))
                       - mu * (g[B] @ (Ci @ De.T) @ g[A]) * I
                       - mu * De @ Ci @ outer(g[B], g[A])
                       + 2 * vol * Ci @ outer(g[A], g[B]) @ Pe.T
                       + 2 * (g[B] @ S @ g[A]) * I)
                H[3 * A:3 * A + 3, 3 * B:3 * B + 3] = 0.5 * blk
        return H
    raise ValueError(model)


MODELS = [
    ("svk", (1.2e6, 0.8e6)),
    ("yeoh", (5.0e3, 0.0, 0.0, 2.0e-6)),          # decoupled Neo-Hookean (C20 = C30 = 0)
    ("yeoh", (100.0, -1.0, 0.01, 0.001)),         # rubber constants of Sec. 6.2.3
    ("nh", (0.4e6, 2.0e6)),
]


def _mesh(model, params):
    p = distort(config("c1", nx=2, ny=2, nz=1), 0.2, seed=21)
    return p, fem.Discretization(p.xyz, p.conn, Material(model, params), 1000.0)


def _disp(d, rng, size=0.3):
    """Random nodal displacement scaled so that max |grad u| = size at the Gauss points."""
    u = rng.normal(size=3 * d.n_nodes)
    return u * (size / np.abs(d.grad(u)).max())


def _element_matrices(d, model, params, u):
    """Per element: sum_q w detJ H(q) assembled from the printed blocks."""
    ue_all = d.gather(u)
    out = []
    for e in range(d.conn.shape[0]):
        He = np.zeros((24, 24))
        for q in range(d.gradN.shape[1]):
            He += d.wdet[e, q] * element_H_printed(model, params, d.gradN[e, q], ue_all[e])
        out.append(He)
    return out


def _assemble_apply(d, Hes, x):
    y = np.zeros(3 * d.n_nodes)
    for e, He in enumerate(Hes):
        idx = (3 * d.conn[e][:, None] + np.arange(3)).ravel()
        y[idx] += He @ x[idx]
    return y


@pytest.mark.parametrize("model,params", MODELS)
def test_oracle_H_matches_printed_blocks(model, params):
    p, d = _mesh(model, params)
    rng = np.random.default_rng(31)
    u = _disp(d, rng)
    Hes = _element_matrices(d, model, params, u)
    for _ in range(3):
        x = rng.normal(size=3 * p.n_nodes)
        ref = _assemble_apply(d, Hes, x)
        got = d.H_apply(u, x)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("model,params", MODELS)
def test_printed_blocks_reproduce_internal_force(model, params):
    p, d = _mesh(model, params)
    u = _disp(d, np.random.default_rng(32))
    Hes = _element_matrices(d, model, params, u)
    R = d.internal_force(u)
    assert np.abs(_assemble_apply(d, Hes, u) - R).max() <= 1e-12 * np.abs(R).max()


def test_printed_P_e_is_the_det_identity():
    """App. A: det F - 1 = tr(D^T P_e) for the printed P_e."""
    rng = np.random.default_rng(33)
    for _ in range(50):
        D = rng.uniform(-0.7, 0.7, size=(3, 3))
        assert abs(np.trace(D.T @ P_e_printed(D)) - (np.linalg.det(I + D) - 1)) < 1e-14


@pytest.mark.parametrize("model,params", MODELS)
def test_printed_blocks_differ_from_a_plain_first_piola_split(model, params):
    """The App. A operator is not the Jacobian dP/dF nor a trivially symmetric split:
    at a deformed state H(u) x differs from the tangent stiffness, while both agree at rest
    (guards against a pin that passes for any decomposition)."""
    p, d = _mesh(model, params)
    rng = np.random.default_rng(34)
    u = _disp(d, rng)
    x = rng.normal(size=3 * p.n_nodes)
    h = 1e-6
    tangent = (d.internal_force(u + h * x) - d.internal_force(u - h * x)) / (2 * h)
    Hx = d.H_apply(u, x)
    assert np.abs(Hx - tangent).max() > 1e-3 * np.abs(tangent).max()
