"""Krylov evaluation of exp(tau A) w (ORACLE, test infrastructure).

Follows Sec. 4.3 of the paper (evaluation of exp(Omega) w):
  * Arnoldi builds an orthonormal basis V_m of the Krylov space of A and w and
    the upper Hessenberg H_m with A V_m = V_m H_m + h_{m+1,m} v_{m+1} e_m^T;
    the orthogonalisation is modified Gram-Schmidt (each projection uses the
    already-updated vector);
  * exp(A) w ~ ||w|| V_m exp(H_m) e_1;
  * exp(H_m) by a Taylor series when ||H_m|| <= 1, else by scaling and squaring
    (here with the degree-13 diagonal Pade approximant of Higham, "The scaling
    and squaring method for the matrix exponential revisited", SIAM J. Matrix
    Anal. Appl. 26 (2005)); no eigendecomposition;
  * the subspace error estimate eps_m = h_{m+1,m} ||w|| |[exp(H_m)]_{m,1}|
    (Sec. 4.3, subspace error estimate) chooses m.
Readings (the paper is silent): ||.|| of H_m is the 1-norm; the stopping rule is
eps_m <= tol * ||w||; eps is evaluated every `check_every` Arnoldi steps, but
not before m_hint - check_every (the size that sufficed last time); an
unconverged attempt at m_max is redone as k = 2, 4, ... substeps of tau/k on
the same frozen operator (exp(tau A) = exp(tau A / k)^k).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BREAKDOWN_TOL = 1e-14
THETA13 = 5.371920351148152      # Higham (2005), Table 2.3, degree 13


class KrylovError(RuntimeError):
    pass


def pade_coefficients(q: int = 13):
    """Coefficients c_j of the numerator of the [q/q] Pade approximant of e^x.

    c_j = (2q - j)! q! / ((2q)! j! (q - j)!); the denominator is the numerator at -x.
    """
    f = math.factorial
    return np.array([f(2 * q - j) * f(q) / (f(2 * q) * f(j) * f(q - j)) for j in range(q + 1)])


_C13 = pade_coefficients(13)


def norm1(A):
    return float(np.abs(A).sum(axis=0).max()) if A.size else 0.0


def expm_taylor(A, max_terms: int = 60):
    """Truncated Taylor series, stopped when the last term is below unit roundoff."""
    n = A.shape[0]
    E = np.eye(n)
    term = np.eye(n)
    for k in range(1, max_terms + 1):
        term = term @ A / k
        E = E + term
        if norm1(term) <= 2.0 ** -53 * norm1(E):
            break
    return E


def expm_pade13(A):
    """Scaling and squaring with the [13/13] Pade approximant."""
    n = A.shape[0]
    nrm = norm1(A)
    s = max(0, int(math.ceil(math.log2(nrm / THETA13)))) if nrm > 0 else 0
    A = A / 2.0 ** s
    c = _C13
    I = np.eye(n)
    A2 = A @ A
    A4 = A2 @ A2
    A6 = A4 @ A2
    U = A @ (A6 @ (c[13] * A6 + c[11] * A4 + c[9] * A2) + c[7] * A6 + c[5] * A4 + c[3] * A2 + c[1] * I)
    V = A6 @ (c[12] * A6 + c[10] * A4 + c[8] * A2) + c[6] * A6 + c[4] * A4 + c[2] * A2 + c[0] * I
    R = np.linalg.solve(V - U, V + U)
    for _ in range(s):
        R = R @ R
    return R


def expm(A):
    """exp(A) for a small dense matrix: Taylor if ||A||_1 <= 1, else scaling and squaring."""
    A = np.asarray(A, dtype=np.float64)
    if A.shape[0] == 0:
        return np.zeros((0, 0))
    return expm_taylor(A) if norm1(A) <= 1.0 else expm_pade13(A)


def arnoldi_mgs(apply, w, m: int):
    """m steps of Arnoldi with modified Gram-Schmidt.

    Returns (V (m+1, L), H (m+1, m), beta, steps) where steps < m on breakdown.
    """
    L = w.size
    V = np.zeros((m + 1, L))
    H = np.zeros((m + 1, m))
    beta = float(np.linalg.norm(w))
    if beta == 0.0:
        return V, H, beta, 0
    V[0] = w / beta
    hmax = 0.0
    for j in range(m):
        x = apply(V[j])
        for i in range(j + 1):
            H[i, j] = x @ V[i]
            x = x - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(x)
        hmax = max(hmax, float(np.abs(H[: j + 2, j]).max()))
        if H[j + 1, j] <= BREAKDOWN_TOL * hmax:
            return V, H, beta, j + 1
        V[j + 1] = x / H[j + 1, j]
    return V, H, beta, m


@dataclass
class ExpvInfo:
    m: int
    eps: float
    converged: bool
    breakdown: bool = False


def expv_once(apply, w, tol: float, m_max: int, check_every: int = 4,
              m_fixed: int = 0, m_hint: int = 0):
    """One Krylov projection of exp(Atilde) w with the a-posteriori choice of m.

    apply(v) returns Atilde v (the time-step factor already included).
    Returns (y or None, ExpvInfo).  y is None when eps stayed above tol*||w|| up to m_max.
    """
    L = w.size
    beta = float(np.linalg.norm(w))
    if beta == 0.0:
        return np.zeros(L), ExpvInfo(0, 0.0, True, True)
    m_cap = m_fixed if m_fixed else m_max
    V = np.zeros((m_cap + 1, L))
    H = np.zeros((m_cap + 1, m_cap))
    V[0] = w / beta
    hmax = 0.0
    for j in range(1, m_cap + 1):                    # j = subspace size after this step
        x = apply(V[j - 1])
        for i in range(j):                           # modified Gram-Schmidt
            H[i, j - 1] = x @ V[i]
            x = x - H[i, j - 1] * V[i]
        h = float(np.linalg.norm(x))
        H[j, j - 1] = h
        hmax = max(hmax, float(np.abs(H[: j + 1, j - 1]).max()))
        breakdown = h <= BREAKDOWN_TOL * hmax
        if m_fixed:
            check = breakdown or j == m_fixed
        else:
            check = (breakdown or j == m_max
                     or (j % check_every == 0 and j >= m_hint - check_every))
        if check:
            E = expm(H[:j, :j])
            eps = h * beta * abs(E[j - 1, 0])
            if breakdown or m_fixed or eps <= tol * beta:
                return beta * (V[:j].T @ E[:, 0]), ExpvInfo(j, eps, True, breakdown)
            if j == m_max:
                return None, ExpvInfo(j, eps, False)
        V[j] = x / h
    raise AssertionError("unreachable")


def expv(apply_tau, w, tau: float, tol: float, m_max: int = 64, check_every: int = 4,
         m_fixed: int = 0, k_fixed: int = 0, state: dict | None = None,
         max_substeps: int = 64):
    """exp(tau A) w with substepping.

    apply_tau(v, f) returns f * A v.  `state` carries the last converged m
    ("m_hint") and substep count ("k") between calls of the same kind; with
    k_fixed > 0 exactly k_fixed substeps are used.
    Returns (y, info dict with k, m list, eps list).
    """
    if state is None:
        state = {}
    k = k_fixed if k_fixed else state.get("k", 1)
    while True:
        x = w
        ms, epss = [], []
        hint = state.get("m_hint", 0)
        ok = True
        for _ in range(k):
            f = tau / k
            y, inf = expv_once(lambda v: apply_tau(v, f), x, tol, m_max, check_every,
                               m_fixed, hint)
            if y is None:
                ok = False
                break
            ms.append(inf.m)
            epss.append(inf.eps)
            if not inf.breakdown:
                hint = inf.m
            x = y
        if ok:
            state["k"] = k
            state["m_hint"] = hint
            return x, {"k": k, "m": ms, "eps": epss}
        if k_fixed or 2 * k > max_substeps:
            raise KrylovError(f"Krylov space not converged at m_max={m_max} with {k} substeps")
        k *= 2
        state["m_hint"] = 0
