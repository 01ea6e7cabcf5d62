"""Dense helpers for oracle pins on tiny meshes: the augmented first-order matrix A
(Sec. 2.3) built from the assembled sum B^T D B stiffness, and its exact exponential."""
import numpy as np
import scipy.linalg as sla

from workloads import config
from oracle.stepper import Propagator


def dense_parts(prob):
    """(Hbar dense, Pbar, Mh, free) on the free DOFs of a linear problem."""
    pr = Propagator(prob)
    K = pr.fem.stiffness().toarray()[np.ix_(pr.free, pr.free)]
    Hb = pr.Mih[:, None] * K * pr.Mih[None, :]
    return Hb, pr.P0bar, pr.Mh, pr.free, pr


def dense_system(name, dt, **over):
    """(dt*A, wbar0, exp(dt*A)) for a linear workload with a nonzero start state."""
    prob = config(name, **over)
    Hb, Pb, Mh, free, pr = dense_parts(prob)
    N = free.size
    A = np.zeros((2 * N + 1, 2 * N + 1))
    A[:N, N:2 * N] = np.eye(N)
    A[N:2 * N, :N] = -Hb
    A[N:2 * N, 2 * N] = Pb
    rng = np.random.default_rng(42)
    w = np.concatenate([Mh * rng.normal(0, 1e-6, N), Mh * rng.normal(0, 1e-3, N), [1.0]])
    A = dt * A
    return A, w, sla.expm(A)
