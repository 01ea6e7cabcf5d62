"""Constitutive laws and the secant split of the internal force (ORACLE, test infrastructure).

Everything here acts on arrays of 3x3 displacement gradients D = grad_X u with
shape (..., 3, 3), D[..., i, k] = d u_i / d X_k, and F = I + D (Sec. 2.1,
constitutive equation).

The paper writes the internal force as R(u) = H(u) u (Sec. 2.3) and notes the
split is neither obvious nor unique; Appendix A builds it for St. Venant-Kirchhoff
and Yeoh solids by pulling one factor of the displacement gradient out of the
stress, using the matrix P_e with det F - 1 = P_e : D (App. A, the det F - 1
identity).  Here the same construction is written for the first Piola-Kirchhoff
stress P = F S:

    secant(D, X) is linear in X and secant(D, D) = P(F(D)),

so that (H(u) x)_A = sum_e sum_q w_q detJ_q secant(D_q, grad x_q) . grad N_A(q)
satisfies H(u) u = R(u) exactly.  For the Neo-Hookean and Yeoh solids it reads

    secant(D, X) = a (X + G X^T) + (W : X) G,      G = F^{-T},

with a, W scalar / matrix coefficients of the current D (given per model
below); it uses F - F^{-T} = D + G D^T, I_1 - 3 = (2 I + D) : D and
J - 1 = Q(D) : D.
"""
from __future__ import annotations

import numpy as np

I3 = np.eye(3)


def lame_from_E_nu(E: float, nu: float):
    """Lame constants (lambda, mu) of an isotropic solid."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def tr(A):
    return np.trace(A, axis1=-2, axis2=-1)


def ddot(A, B):
    """A : B = trace(A^T B) over the last two axes."""
    return np.einsum("...ij,...ij->...", A, B)


def T(A):
    return np.swapaxes(A, -1, -2)


def cof(D):
    """Cofactor matrix of D built from 2x2 minors (polynomial, defined at D = 0)."""
    c = np.empty(D.shape)
    c[..., 0, 0] = D[..., 1, 1] * D[..., 2, 2] - D[..., 1, 2] * D[..., 2, 1]
    c[..., 0, 1] = -(D[..., 1, 0] * D[..., 2, 2] - D[..., 1, 2] * D[..., 2, 0])
    c[..., 0, 2] = D[..., 1, 0] * D[..., 2, 1] - D[..., 1, 1] * D[..., 2, 0]
    c[..., 1, 0] = -(D[..., 0, 1] * D[..., 2, 2] - D[..., 0, 2] * D[..., 2, 1])
    c[..., 1, 1] = D[..., 0, 0] * D[..., 2, 2] - D[..., 0, 2] * D[..., 2, 0]
    c[..., 1, 2] = -(D[..., 0, 0] * D[..., 2, 1] - D[..., 0, 1] * D[..., 2, 0])
    c[..., 2, 0] = D[..., 0, 1] * D[..., 1, 2] - D[..., 0, 2] * D[..., 1, 1]
    c[..., 2, 1] = -(D[..., 0, 0] * D[..., 1, 2] - D[..., 0, 2] * D[..., 1, 0])
    c[..., 2, 2] = D[..., 0, 0] * D[..., 1, 1] - D[..., 0, 1] * D[..., 1, 0]
    return c


def Qmat(D):
    """The matrix called P_e in App. A: det(I + D) - 1 = Q(D) : D.

    Q = I + (tr D I - D^T) / 2 + cof(D) / 3: the three terms pick up the linear,
    quadratic (second invariant) and cubic (det D) parts of det(I + D) - 1.
    """
    return I3 + 0.5 * (tr(D)[..., None, None] * I3 - T(D)) + cof(D) / 3.0


def jm1(D):
    """J - 1 = det(I + D) - 1, evaluated as Q(D) : D (no cancellation near D = 0)."""
    return ddot(Qmat(D), D)


def log_ratio(x):
    """ln(1 + x) / x with its limit 1 at x = 0."""
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < 1e-8
    xs = np.where(small, 1.0, x)
    return np.where(small, 1.0 - 0.5 * x + x * x / 3.0, np.log1p(xs) / xs)


class Material:
    """model in {'linear', 'nh', 'yeoh', 'svk'}; params as in workloads."""

    def __init__(self, model: str, params):
        self.model = model
        self.params = tuple(float(p) for p in params)
        if model == "linear":
            self.lam, self.mu = lame_from_E_nu(*self.params)
        elif model == "nh":
            self.mu, self.lam = self.params
        elif model == "yeoh":
            self.C10, self.C20, self.C30, self.D1 = self.params
        elif model == "svk":
            self.lam, self.mu = self.params
        else:
            raise ValueError(model)

    # -- small-strain moduli of the linearisation at D = 0 ---------------------
    def small_strain_lame(self):
        """(lambda, mu) of the tangent at u = 0 (linear elasticity limit)."""
        if self.model in ("linear", "nh", "svk"):
            return self.lam, self.mu
        mu = 2.0 * self.C10
        kappa = 2.0 / self.D1
        return kappa - 2.0 * mu / 3.0, mu

    # -- strain energy density ------------------------------------------------
    def psi(self, D):
        if self.model == "linear":
            eps = 0.5 * (D + T(D))
            return 0.5 * self.lam * tr(eps) ** 2 + self.mu * ddot(eps, eps)
        F = I3 + D
        x = jm1(D)
        if self.model == "nh":
            # psi = mu/2 (I1 - 3) - mu ln J + lambda/2 (ln J)^2
            lnJ = np.log1p(x)
            I1 = ddot(F, F)
            return 0.5 * self.mu * (I1 - 3.0) - self.mu * lnJ + 0.5 * self.lam * lnJ ** 2
        if self.model == "yeoh":
            # App. A (Yeoh strain energy): C10 (I1b-3) + C20 (I1b-3)^2 + C30 (I1b-3)^3 + (J-1)^2 / D1
            J = 1.0 + x
            I1b = J ** (-2.0 / 3.0) * ddot(F, F)
            z = I1b - 3.0
            return self.C10 * z + self.C20 * z ** 2 + self.C30 * z ** 3 + x ** 2 / self.D1
        if self.model == "svk":
            E = 0.5 * (T(F) @ F - I3)
            return 0.5 * self.lam * tr(E) ** 2 + self.mu * ddot(E, E)
        raise ValueError(self.model)

    # -- second Piola-Kirchhoff stress (App. A) --------------------------------
    def pk2(self, D):
        F = I3 + D
        C = T(F) @ F
        if self.model == "svk":
            E = 0.5 * (C - I3)
            return self.lam * tr(E)[..., None, None] * I3 + 2.0 * self.mu * E
        if self.model == "yeoh":
            # App. A, Yeoh second Piola-Kirchhoff stress
            J = 1.0 + jm1(D)
            Jm23 = J ** (-2.0 / 3.0)
            trC = tr(C)
            z = trC * Jm23 - 3.0
            Cinv = np.linalg.inv(C)
            alpha = 2.0 * Jm23 * (self.C10 + 2.0 * self.C20 * z + 3.0 * self.C30 * z ** 2)
            return (alpha[..., None, None] * (I3 - Cinv * trC[..., None, None] / 3.0)
                    + (2.0 / self.D1 * J * (J - 1.0))[..., None, None] * Cinv)
        if self.model == "nh":
            J = 1.0 + jm1(D)
            Cinv = np.linalg.inv(C)
            return self.mu * (I3 - Cinv) + (self.lam * np.log(J))[..., None, None] * Cinv
        raise ValueError(self.model)

    # -- first Piola-Kirchhoff stress P = F S (or small-strain sigma) ----------
    def pk1(self, D):
        if self.model == "linear":
            eps = 0.5 * (D + T(D))
            return self.lam * tr(eps)[..., None, None] * I3 + 2.0 * self.mu * eps
        if self.model == "nh":
            F = I3 + D
            G = np.linalg.inv(T(F))
            lnJ = np.log1p(jm1(D))
            return self.mu * (F - G) + (self.lam * lnJ)[..., None, None] * G
        return (I3 + D) @ self.pk2(D)

    # -- secant split: secant(D, X) linear in X, secant(D, D) = pk1(D) ----------
    def secant_coeffs(self, D):
        """(a, G, W) with secant(D, X) = a (X + G X^T) + (W : X) G (NH / Yeoh)."""
        F = I3 + D
        G = np.linalg.inv(T(F))
        x = jm1(D)
        Q = Qmat(D)
        if self.model == "nh":
            a = np.full(D.shape[:-2], self.mu)
            W = (self.lam * log_ratio(x))[..., None, None] * Q
        elif self.model == "yeoh":
            J = 1.0 + x
            Jm23 = J ** (-2.0 / 3.0)
            z = ddot(F, F) * Jm23 - 3.0
            a = 2.0 * Jm23 * (self.C10 + 2.0 * self.C20 * z + 3.0 * self.C30 * z ** 2)
            beta = 2.0 / self.D1 * J
            W = -(a / 3.0)[..., None, None] * (2.0 * I3 + D) + beta[..., None, None] * Q
        else:
            raise ValueError("secant_coeffs is defined for 'nh' and 'yeoh'")
        return a, G, W

    def secant(self, D, X):
        if self.model == "linear":
            eps = 0.5 * (X + T(X))
            return self.lam * tr(eps)[..., None, None] * I3 + 2.0 * self.mu * eps
        if self.model == "svk":
            F = I3 + D
            c = ddot(I3 + 0.5 * D, X)
            return (self.lam * c)[..., None, None] * F + self.mu * F @ (X + T(X) @ F)
        a, G, W = self.secant_coeffs(D)
        return (a[..., None, None] * (X + G @ T(X))
                + ddot(W, X)[..., None, None] * G)
