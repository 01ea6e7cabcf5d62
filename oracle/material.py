"""Constitutive laws and the H-matrix split of the internal force (ORACLE, test infrastructure).

Everything here acts on arrays of 3x3 displacement gradients D = grad_X u with
shape (..., 3, 3), D[..., i, k] = d u_i / d X_k, and F = I + D (Sec. 2.1,
constitutive equation).

The paper writes the internal force as R(u) = H(u) u (Sec. 2.3) and builds H(u) in
App. A from the internal virtual work int dE : S dV = int grad w : (F S) dV,
with S the second Piola-Kirchhoff stress.  Its H-matrix blocks H_AB (the 3x3 block
between test node A and trial node B) are sums of terms of three shapes, which act
on a field x with nodal values x_B, X = grad_X x = sum_B x_B (x) grad N_B, as

    (grad N_B . M . grad N_A) I        ->  X M            (M a 3x3 matrix)
    L (grad N_B (x) grad N_A)          ->  L X^T
    L (grad N_A (x) grad N_B) R^T      ->  (R : X) L,

in the sense sum_B H_AB x_B = Phi(X) grad N_A summed over the quadrature.  So

    (H(u) x)_A = sum_e sum_q w_q detJ_q Phi(D_q, X_q) . grad N_A(q),

with Phi(D, X) = secant(D, X) below, term by term the printed H-matrix of App. A.
Every such Phi splits as S_lin(D, X) + X S(D): the geometric part X S(D) (the terms
that carry grad N_B . S . grad N_A) and the second Piola-Kirchhoff stress written
linearly in X, S_lin(D, D) = S(D), so that secant(D, D) = F S = P and H(u) u = R(u).
The matrix P_e of App. A (det F - 1 = P_e : D) is Qmat below.
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

    # -- the H-matrix of App. A written as an operator on X = grad x -----------
    def secant(self, D, X):
        """Phi(D, X): linear in X, Phi(D, D) = P(F); H(u) x integrates Phi(D(u), grad x).

        linear: sigma(X) (H = K, Sec. 5.2).
        svk:    App. A, St. Venant-Kirchhoff H-matrix (the 1/2 of dE included):
                  lambda/2 (dN_A (x) dN_B)(2I + D^T)  -> lambda ((I + D/2) : X) I
                  mu (dN_B . dN_A) I                  -> mu X
                  mu/2 (dN_B (x) dN_A)(2I + D^T)      -> mu (X^T + X^T D / 2)
                  mu/2 D^T (dN_A . dN_B)              -> mu D^T X / 2
                  (dN_B . S_SVK . dN_A) I             -> X S(D)
        yeoh:   App. A, Yeoh H-matrix with the 1/2 of dE (the internal virtual work of the
                Yeoh derivation) applied to each printed term; alpha = alpha_e,
                beta = beta_e = 2 J / D1, Ci = C^{-1} = F^{-1} F^{-T}:
                  2 alpha (dN_B . F^{-1} . dN_A) I          -> alpha X F^{-1}
                  2 alpha F^{-T} (dN_B (x) dN_A)            -> alpha F^{-T} X^T
                  -alpha (dN_B . Ci D^T . dN_A) I           -> -alpha/2 X Ci D^T
                  -alpha D Ci (dN_B (x) dN_A)               -> -alpha/2 D Ci X^T
                  -2/3 alpha Ci (dN_A (x) dN_B)(2I + D^T)   -> -alpha/3 ((2I + D) : X) Ci
                  2 alpha (dN_B . [I - Ci tr C / 3] . dN_A) I -> alpha X (I - Ci tr C / 3)
                  2 beta Ci (dN_A (x) dN_B) P_e^T           -> beta (P_e : X) Ci
                  2 beta (J - 1) (dN_A . Ci . dN_B) I       -> beta (J - 1) X Ci
                The first five terms and the P_e term give S_lin (at X = D they sum to
                alpha (I - Ci tr C / 3) + beta (J - 1) Ci = S, using J - 1 = P_e : D and
                D F^{-1} + F^{-T} D^T - D Ci D^T = I - Ci), the other two X S(D).
        nh:     the same construction for the compressible Neo-Hookean solid ("trivially
                extended", App. A): S = mu (I - Ci) + lambda ln J Ci, with mu in place of
                alpha in the first four Yeoh terms, ln J = l(J) (J - 1), l(J) = ln J / (J - 1),
                and lambda l(J) in place of beta in the P_e term, plus X S(D).
        """
        if self.model == "linear":
            eps = 0.5 * (X + T(X))
            return self.lam * tr(eps)[..., None, None] * I3 + 2.0 * self.mu * eps
        S = self.pk2(D)
        geo = X @ S                                         # (dN_B . S . dN_A) I terms
        if self.model == "svk":
            c = ddot(I3 + 0.5 * D, X)
            return ((self.lam * c)[..., None, None] * I3
                    + self.mu * (X + T(X) + 0.5 * (T(X) @ D + T(D) @ X)) + geo)
        F = I3 + D
        Finv = np.linalg.inv(F)
        FinvT = T(Finv)
        Ci = Finv @ FinvT
        x = jm1(D)
        PX = ddot(Qmat(D), X)                               # P_e : X
        if self.model == "nh":
            a = np.full(D.shape[:-2], self.mu)
            vol = self.lam * log_ratio(x)                   # lambda ln J / (J - 1)
            trterm = np.zeros(D.shape[:-2])
        elif self.model == "yeoh":
            J = 1.0 + x
            Jm23 = J ** (-2.0 / 3.0)
            z = ddot(F, F) * Jm23 - 3.0
            a = 2.0 * Jm23 * (self.C10 + 2.0 * self.C20 * z + 3.0 * self.C30 * z ** 2)   # alpha_e
            vol = 2.0 / self.D1 * J                                                       # beta_e
            trterm = -(a / 3.0) * ddot(2.0 * I3 + D, X)
        else:
            raise ValueError(self.model)
        a_ = a[..., None, None]
        Slin = (a_ * (X @ Finv + FinvT @ T(X) - 0.5 * (X @ Ci @ T(D)) - 0.5 * (D @ Ci @ T(X)))
                + (trterm + vol * PX)[..., None, None] * Ci)
        return Slin + geo
