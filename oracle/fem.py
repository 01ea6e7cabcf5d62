"""Hexahedral finite-element pieces of the semi-discrete system (ORACLE, test infrastructure).

Follows Sec. 2.2 of the paper (finite element formulation) for two elements:
  * hex8: trilinear shape functions; internal force by 2x2x2 Gauss; mass by the 2-point
    Gauss-Lobatto rule per direction, whose points are the element's vertices, so M is
    diagonal (the 8-node analogue of the paper's choice);
  * hex27: the paper's quadratic Lagrange hexahedron (interpolation eq. of Sec. 2.2), nodes
    at the local points {-1, 0, 1}^3; internal force by 3x3x3 Gauss; mass by the 3-point
    Gauss-Lobatto rule per direction (points -1, 0, 1, weights 1/3, 4/3, 1/3), whose
    points are the nodes, which makes M diagonal (Sec. 2.2, remark after the semi-discrete
    equation: quadratic Lagrange + Gauss-Lobatto);
  * loads by Gauss quadrature on the element faces (2x2 on 4-node, 3x3 on 9-node quads);
  * the element integrals of the weak-form terms: mass (term 1), internal force
    R(u) = sum B^T S (term 2) and the external force P (term 3).
Arrays are node-major: DOF 3*A + i is component i of node A.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .material import Material, I3

# local coordinates of the 8 vertices, VTK order
XI_NODES = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                     [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)


def shape(xi):
    """Trilinear shape functions at local points xi (..., 3).

    Returns N (..., 8) and dN/dxi (..., 8, 3), N_A = 1/8 prod_d (1 + xi_A,d xi_d).
    """
    xi = np.asarray(xi, dtype=np.float64)
    f = 1.0 + xi[..., None, :] * XI_NODES            # (..., 8, 3)
    N = 0.125 * f[..., 0] * f[..., 1] * f[..., 2]
    dN = np.empty(f.shape)
    dN[..., 0] = 0.125 * XI_NODES[:, 0] * f[..., 1] * f[..., 2]
    dN[..., 1] = 0.125 * XI_NODES[:, 1] * f[..., 0] * f[..., 2]
    dN[..., 2] = 0.125 * XI_NODES[:, 2] * f[..., 0] * f[..., 1]
    return N, dN


# hex27: local node a = i + 3 j + 9 k at (i - 1, j - 1, k - 1)
XI_NODES27 = np.array([[i - 1, j - 1, k - 1] for k in range(3) for j in range(3) for i in range(3)],
                      dtype=np.float64)


def lagrange3(x):
    """Quadratic Lagrange polynomials on the points -1, 0, 1 and their derivatives."""
    x = np.asarray(x, dtype=np.float64)
    l = np.stack([0.5 * x * (x - 1.0), 1.0 - x * x, 0.5 * x * (x + 1.0)], axis=-1)
    dl = np.stack([x - 0.5, -2.0 * x, x + 0.5], axis=-1)
    return l, dl


def shape27(xi):
    """Quadratic Lagrange shape functions of the 27-node hexahedron at local points xi (..., 3).

    N_a = l_i(xi) l_j(eta) l_k(zeta) for a = i + 3 j + 9 k.  Returns N (..., 27) and
    dN/dxi (..., 27, 3).
    """
    xi = np.asarray(xi, dtype=np.float64)
    lx, dx = lagrange3(xi[..., 0])
    ly, dy = lagrange3(xi[..., 1])
    lz, dz = lagrange3(xi[..., 2])
    ii = np.array([a % 3 for a in range(27)])
    jj = np.array([(a // 3) % 3 for a in range(27)])
    kk = np.array([a // 9 for a in range(27)])
    N = lx[..., ii] * ly[..., jj] * lz[..., kk]
    dN = np.stack([dx[..., ii] * ly[..., jj] * lz[..., kk],
                   lx[..., ii] * dy[..., jj] * lz[..., kk],
                   lx[..., ii] * ly[..., jj] * dz[..., kk]], axis=-1)
    return N, dN


ELEMENTS = {
    # name: (shape function, Gauss points per direction for stiffness and loads,
    #        local node coordinates, Gauss-Lobatto weights per direction at the nodes)
    "hex8": (None, 2, XI_NODES, (1.0, 1.0)),
    "hex27": (shape27, 3, XI_NODES27, (1.0 / 3.0, 4.0 / 3.0, 1.0 / 3.0)),
}


def element_shape(elem):
    return shape if elem == "hex8" else ELEMENTS[elem][0]


def gauss_rule(n: int):
    """Tensor Gauss-Legendre rule with n points per direction: points (n^3, 3), weights."""
    x, w = np.polynomial.legendre.leggauss(n)
    P = np.array([[x[i], x[j], x[k]] for k in range(n) for j in range(n) for i in range(n)])
    W = np.array([w[i] * w[j] * w[k] for k in range(n) for j in range(n) for i in range(n)])
    return P, W


def jacobian(Xe, dN):
    """J[..., i, j] = d X_i / d xi_j for element coordinates Xe (n_e, 8, 3)."""
    return np.einsum("eai,...aj->e...ij", Xe, dN)


def geometry(xyz, conn, n_gauss: int = 2, elem: str = "hex8"):
    """Physical shape-function gradients and weights at the volume Gauss points.

    Returns gradN (n_e, Q, n, 3) with gradN[e,q,a,k] = dN_a/dX_k and
    wdet (n_e, Q) = quadrature weight * det J.
    """
    P, W = gauss_rule(n_gauss)
    _, dN = element_shape(elem)(P)                    # (Q, n, 3)
    Xe = xyz[conn]                                    # (n_e, 8, 3)
    J = jacobian(Xe, dN)                              # (n_e, Q, 3, 3)
    detJ = np.linalg.det(J)
    if np.any(detJ <= 0.0):
        raise ValueError("inverted or degenerate element (det J <= 0)")
    Jinv = np.linalg.inv(J)
    gradN = np.einsum("qaj,eqjk->eqak", dN, Jinv)
    return gradN, W[None, :] * detJ


def lumped_mass(xyz, conn, rho, elem: str = "hex8"):
    """Diagonal mass by the nodal Gauss-Lobatto rule: M_A = sum_e rho w_A detJ_e(xi_A), w_A the
    product of the rule's weights at node A (hex8: the vertex rule, w = 1; hex27: 1/3, 4/3, 1/3
    per direction).

    Returned per DOF (each node's value repeated for its 3 components).
    """
    _, _, xin, w1 = ELEMENTS[elem]
    idx = np.rint((xin + 1.0) * (len(w1) - 1) / 2.0).astype(int)   # node's point index per direction
    w1 = np.asarray(w1)
    wA = w1[idx[:, 0]] * w1[idx[:, 1]] * w1[idx[:, 2]]
    _, dN = element_shape(elem)(xin)                  # at the nodes
    J = jacobian(xyz[conn], dN)                       # (n_e, n, 3, 3)
    detJ = np.linalg.det(J)
    m = np.zeros(xyz.shape[0])
    np.add.at(m, conn.ravel(), (rho * wA[None, :] * detJ).ravel())
    return np.repeat(m, 3)


def traction_load(xyz, faces, t0):
    """Consistent nodal force of a dead traction t0 on quad faces, eq. term 3: 2x2 Gauss on
    bilinear 4-node faces, 3x3 Gauss on biquadratic 9-node faces (node p + 3 q at (p-1, q-1))."""
    n = xyz.shape[0]
    P = np.zeros(3 * n)
    faces = np.asarray(faces)
    if len(faces) == 0:
        return P
    Xf = xyz[faces]                                                       # (n_f, nf, 3)
    if faces.shape[1] == 4:
        s_nodes = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)
        g = 1.0 / np.sqrt(3.0)
        pts = [((s, t), 1.0) for (s, t) in ((-g, -g), (g, -g), (g, g), (-g, g))]

        def fshape(s, t):
            N = 0.25 * (1 + s * s_nodes[:, 0]) * (1 + t * s_nodes[:, 1])
            dNs = 0.25 * s_nodes[:, 0] * (1 + t * s_nodes[:, 1])
            dNt = 0.25 * s_nodes[:, 1] * (1 + s * s_nodes[:, 0])
            return N, dNs, dNt
    else:
        x, w = np.polynomial.legendre.leggauss(3)
        pts = [((x[i], x[j]), w[i] * w[j]) for j in range(3) for i in range(3)]
        pp = np.array([a % 3 for a in range(9)])
        qq = np.array([a // 3 for a in range(9)])

        def fshape(s, t):
            ls, dls = lagrange3(s)
            lt, dlt = lagrange3(t)
            return ls[pp] * lt[qq], dls[pp] * lt[qq], ls[pp] * dlt[qq]
    for (s, t), wq in pts:
        N, dNs, dNt = fshape(s, t)
        a1 = np.einsum("a,fai->fi", dNs, Xf)
        a2 = np.einsum("a,fai->fi", dNt, Xf)
        dA = wq * np.linalg.norm(np.cross(a1, a2), axis=1)
        for c in range(3):
            np.add.at(P, 3 * faces.ravel() + c, (dA[:, None] * N[None, :] * t0[c]).ravel())
    return P


# ----------------------------------------------------------------------------
# element operators
# ----------------------------------------------------------------------------
def voigt_B(gradN_q, F=None):
    """Paper's 6x24 matrix B_{I,e} (Sec. 2.2, term 2) at one point; F = I gives the linear one.

    Rows: (11, 22, 33, 12, 23, 13) with engineering shears; columns: node A, comp i.
    """
    if F is None:
        F = I3
    n = gradN_q.shape[0]
    B = np.zeros((6, 3 * n))
    for A in range(n):
        d = gradN_q[A]
        for i in range(3):
            c = 3 * A + i
            B[0, c] = F[i, 0] * d[0]
            B[1, c] = F[i, 1] * d[1]
            B[2, c] = F[i, 2] * d[2]
            B[3, c] = F[i, 0] * d[1] + F[i, 1] * d[0]
            B[4, c] = F[i, 1] * d[2] + F[i, 2] * d[1]
            B[5, c] = F[i, 0] * d[2] + F[i, 2] * d[0]
    return B


def voigt_D(lam, mu):
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def element_stiffness(gradN_e, wdet_e, lam, mu):
    """Linear-elastic K_e = sum_q w detJ B^T D B (3n x 3n) of one element."""
    Dm = voigt_D(lam, mu)
    nd = 3 * gradN_e.shape[1]
    K = np.zeros((nd, nd))
    for q in range(gradN_e.shape[0]):
        B = voigt_B(gradN_e[q])
        K += wdet_e[q] * B.T @ Dm @ B
    return K


class Discretization:
    """Geometry, mass and load of one mesh, plus element-level operators."""

    def __init__(self, xyz, conn, material: Material, rho: float, n_gauss: int | None = None,
                 elem: str = "hex8"):
        self.xyz = np.asarray(xyz, dtype=np.float64)
        self.conn = np.asarray(conn, dtype=np.int64)
        self.n_nodes = self.xyz.shape[0]
        self.mat = material
        self.rho = rho
        self.elem = elem
        self.gradN, self.wdet = geometry(self.xyz, self.conn, n_gauss or ELEMENTS[elem][1], elem)
        self.M = lumped_mass(self.xyz, self.conn, rho, elem)
        self._K = None

    # nodal <-> element
    def gather(self, U):
        return np.asarray(U).reshape(-1, 3)[self.conn]            # (n_e, n, 3)

    def scatter(self, fe):
        out = np.zeros((self.n_nodes, 3))
        np.add.at(out, self.conn.ravel(), fe.reshape(-1, 3))
        return out.ravel()

    def grad(self, U):
        """D[e,q,i,k] = sum_A U_{A,i} dN_A/dX_k (gradient at the Gauss points)."""
        Ut = np.swapaxes(self.gather(U), 1, 2)[:, None]          # (n_e, 1, 3, n)
        return Ut @ self.gradN                                     # (n_e, Q, 3, 3)

    def integrate(self, S):
        """Nodal vector f_{A,i} = sum_e sum_q w detJ S[e,q,i,k] dN_A/dX_k."""
        fe = ((self.wdet[..., None, None] * self.gradN) @ np.swapaxes(S, -1, -2)).sum(axis=1)
        return self.scatter(fe)

    # operators
    def internal_force(self, U):
        """R(u) = sum_e int grad w : P(F) (weak-form term 2 written with P = F S)."""
        return self.integrate(self.mat.pk1(self.grad(U)))

    def internal_force_voigt(self, U):
        """R(u) in the paper's element form sum_e int B_{I,e}^T S_e (Sec. 2.2, term 2)."""
        D = self.grad(U)
        S = self.mat.pk2(D)
        R = np.zeros(3 * self.n_nodes)
        nd = 3 * self.conn.shape[1]
        for e in range(self.conn.shape[0]):
            fe = np.zeros(nd)
            for q in range(self.gradN.shape[1]):
                B = voigt_B(self.gradN[e, q], I3 + D[e, q])
                s = S[e, q]
                Sv = np.array([s[0, 0], s[1, 1], s[2, 2], s[0, 1], s[1, 2], s[0, 2]])
                fe += self.wdet[e, q] * B.T @ Sv
            idx = (3 * self.conn[e][:, None] + np.arange(3)).ravel()
            np.add.at(R, idx, fe)
        return R

    def H_apply(self, U, X):
        """H(u) x with the secant split: sum_e int grad w : secant(D(u), grad x)."""
        D = None if U is None else self.grad(U)      # linear: secant ignores D
        return self.integrate(self.mat.secant(D, self.grad(X)))

    def strain_energy(self, U):
        return float(np.einsum("eq,eq->", self.wdet, self.mat.psi(self.grad(U))))

    def stiffness(self):
        """Assembled linear-elastic K (sparse) with the small-strain Lame constants."""
        if self._K is None:
            lam, mu = self.mat.small_strain_lame()
            rows, cols, vals = [], [], []
            for e in range(self.conn.shape[0]):
                Ke = element_stiffness(self.gradN[e], self.wdet[e], lam, mu)
                idx = (3 * self.conn[e][:, None] + np.arange(3)).ravel()
                rows.append(np.repeat(idx, idx.size))
                cols.append(np.tile(idx, idx.size))
                vals.append(Ke.ravel())
            n = 3 * self.n_nodes
            self._K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                    shape=(n, n))
        return self._K
