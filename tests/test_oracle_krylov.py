"""Pins of the oracle's Krylov pieces: exp(H_m), Arnoldi-MGS and the subspace error estimate."""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import krylov
from tests.oracle_dense import dense_system

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _hessenberg(rng, m, scale):
    H = np.triu(rng.normal(size=(m, m)), -1)
    return scale * H / krylov.norm1(H)


@pytest.mark.parametrize("m,scale", [(1, 0.5), (5, 0.3), (12, 1.0), (12, 1.0001), (20, 7.0),
                                     (40, 60.0), (64, 400.0), (30, 1e-3)])
def test_expm_matches_scipy(m, scale):
    rng = np.random.default_rng(m)
    H = _hessenberg(rng, m, scale)
    E = krylov.expm(H)
    R = sla.expm(H)
    assert np.abs(E - R).max() <= 1e-13 * max(1.0, np.abs(R).max()) * max(1, scale)


def test_expm_branches_agree():
    rng = np.random.default_rng(9)
    H = _hessenberg(rng, 16, 0.9)
    assert np.allclose(krylov.expm_taylor(H), krylov.expm_pade13(H), rtol=0, atol=1e-15)


@pytest.mark.parametrize("a", [0.3, 2.0, 37.0])
def test_expm_rotation_closed_form(a):
    E = krylov.expm(np.array([[0.0, a], [-a, 0.0]]))
    R = np.array([[np.cos(a), np.sin(a)], [-np.sin(a), np.cos(a)]])
    assert np.abs(E - R).max() < 1e-13 * max(1.0, a)


def test_expm_det_is_exp_trace():
    rng = np.random.default_rng(10)
    H = _hessenberg(rng, 10, 3.0)
    assert math.isclose(np.linalg.det(krylov.expm(H)), math.exp(np.trace(H)), rel_tol=1e-12)


def test_pade13_coefficients_match_published_table():
    """[13/13] Pade numerator coefficients vs Higham (2005)'s printed integers (golden)."""
    b = np.loadtxt(os.path.join(GOLDEN, "pade13_higham2005.txt"))
    c = krylov.pade_coefficients(13)
    assert np.allclose(c, b / b[0], rtol=1e-15)


def test_arnoldi_relation_and_orthonormality():
    """A V_m = V_{m+1} Htilde (Sec. 4.3) and orthonormal columns, on the 10x2x2 beam."""
    A, w, _ = dense_system("c1", 1e-4)
    m = 30
    V, H, beta, steps = krylov.arnoldi_mgs(lambda v: A @ v, w, m)
    assert steps == m
    Vm = V[:m].T
    # MGS keeps ||I - V^T V|| at O(unit roundoff * condition of the Krylov basis)
    assert np.abs(V @ V.T - np.eye(m + 1)).max() < 1e-10
    resid = A @ Vm - V.T @ H
    assert np.abs(resid).max() <= 1e-13 * np.abs(A).max()
    assert np.allclose(np.triu(H, -1), H)


def test_full_dimension_krylov_is_exact():
    rng = np.random.default_rng(12)
    n = 12
    A = rng.normal(size=(n, n))
    w = rng.normal(size=n)
    y, info = krylov.expv_once(lambda v: A @ v, w, 1e-300, n, m_fixed=n)
    assert np.allclose(y, sla.expm(A) @ w, rtol=1e-12, atol=1e-12 * np.abs(y).max())
    # breakdown on an invariant subspace gives the exact result
    A2 = np.zeros((n, n)); A2[:3, :3] = rng.normal(size=(3, 3))
    w2 = np.zeros(n); w2[:3] = rng.normal(size=3)
    y2, info2 = krylov.expv_once(lambda v: A2 @ v, w2, 1e-12, 10)
    assert info2.breakdown and info2.m == 3
    assert np.allclose(y2, sla.expm(A2) @ w2, atol=1e-13)


@pytest.mark.parametrize("dt", [1e-5, 5e-5, 1e-4])
def test_error_estimate_traces_true_error(dt):
    """Sec. 6.1 (subspace error study): past a dt-dependent threshold the error drops
    exponentially and the estimate eps_m follows it.  The paper reads the estimate as an
    upper bound; on this beam it sits within a small factor of the true error (measured:
    a factor 1-5 below it), so the pin is a two-sided factor-10 band above round-off."""
    A, w, E = dense_system("c1", dt)
    exact = E @ w
    beta = np.linalg.norm(w)
    ms = list(range(2, 41, 2))
    errs, ests = [], []
    for m in ms:
        y, info = krylov.expv_once(lambda v: A @ v, w, 0.0, m, m_fixed=m)
        errs.append(np.linalg.norm(y - exact) / beta)
        ests.append(info.eps / beta)
    errs, ests = np.array(errs), np.array(ests)
    band = (errs < 1e-2) & (errs > 1e-11) & (ests > 1e-12)    # above the round-off floor
    assert band.sum() >= 3
    ratio = ests[band] / errs[band]
    assert np.all((ratio > 0.1) & (ratio < 10.0))
    # exponential drop in the band: every 2 more vectors gain at least a factor 5
    e = errs[band]
    assert np.all(e[1:] < e[:-1] / 5.0)


def test_threshold_grows_with_dt():
    ms_needed = []
    for dt in (1e-5, 5e-5, 2e-4):
        A, w, E = dense_system("c1", dt)
        st = {}
        y, info = krylov.expv(lambda v, f: f * (A @ v), w, 1.0, tol=1e-10, m_max=200, check_every=1,
                              state=st)
        ms_needed.append(info["m"][0])
        # tol 1e-10 on the estimate; round-off of the badly scaled A grows with m (~1e-9 at m~50)
        assert np.linalg.norm(y - E @ w) <= 1e-8 * np.linalg.norm(w)
    assert ms_needed[0] < ms_needed[1] < ms_needed[2]


def test_substeps_reproduce_unsplit_exponential():
    A, w, E = dense_system("c1", 4e-4)
    st = {}
    y, info = krylov.expv(lambda v, f: f * (A @ v), w, 1.0, tol=1e-10, m_max=24, state=st)
    assert info["k"] > 1
    assert np.linalg.norm(y - E @ w) <= 1e-9 * np.linalg.norm(w)
    with pytest.raises(krylov.KrylovError):
        krylov.expv(lambda v, f: f * (A @ v), w, 1.0, tol=1e-10, m_max=2, max_substeps=4, state={})
