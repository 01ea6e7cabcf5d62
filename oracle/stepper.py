"""Exponential time propagator for the first-order elastodynamics system (ORACLE, test infrastructure).

Sec. 2.3 (proposed reformulation): with the diagonal mass M,
    ubar = M^{1/2} u,  Hbar(u) = M^{-1/2} H(u) M^{-1/2},  Pbar = M^{-1/2} P,
and wbar = [ubar; vbar; s] obeys d wbar/dt = A[u](t) wbar with the augmented
    A = [[0, I, 0], [-Hbar, 0, Pbar / s0], [0, 0, 0]]     (s = s0 = 1 in the paper).
Sec. 3.2-3.3 and 4.1: one step is wbar_n = exp(dt A(t_{n-1} + dt/2)) wbar_{n-1}
(Magnus expansion truncated after its first term, midpoint rule).
Sec. 4.2 (predictor-corrector): Hbar at the step midpoint is predicted by linear
extrapolation from the two previous midpoints to t_{n-1} + dt/4, wbar_{n-1} is
propagated by dt/2 with it, the half-step displacement defines Hbar(u_{n-1/2}),
and the step is redone from wbar_{n-1} over dt with that operator; H is formed
once per step.  Linear elasticity needs no predictor (H is constant).

Readings (paper silent): clamped DOFs are eliminated (vectors live on the free
DOFs); step 1 predicts with H(u_0) and step 2 with H(u_{1/2}); the load enters
through scale(t) evaluated where A is evaluated; after each propagation the
augmented entry (exactly constant in exact arithmetic) is reset to s0 and its
drift recorded.  When the load is identically zero the paper uses the 2N form
without the augmented row (Sec. 2.3, A for P = 0); that is s0 = 0 here (the
entry stays 0 and contributes nothing to norms).
"""
from __future__ import annotations

import numpy as np

from .fem import Discretization, traction_load
from .krylov import expv
from .material import Material


class Propagator:
    def __init__(self, prob, tol: float | None = None, m_max: int = 64, check_every: int = 4,
                 m_fixed: int = 0, k_fixed: int = 0, max_substeps: int = 64, s0: float | None = None):
        self.prob = prob
        self.mat = Material(prob.model, prob.params)
        self.fem = Discretization(prob.xyz, prob.conn, self.mat, prob.rho, elem=getattr(prob, "elem", "hex8"))
        n3 = 3 * prob.n_nodes
        self.n3 = n3
        self.free = np.setdiff1d(np.arange(n3), np.asarray(prob.clamped, dtype=np.int64))
        self.N = self.free.size
        M = self.fem.M[self.free]
        self.Mh = np.sqrt(M)
        self.Mih = 1.0 / np.sqrt(M)
        self.P0bar = self.Mih * traction_load(prob.xyz, prob.faces, prob.t0)[self.free]
        self.linear = prob.model == "linear"
        unloaded = (not np.any(self.P0bar)) or (not np.any(np.asarray(prob.knots_s)))
        # s0 = "scaled": the augmented entry at the problem's own scale (reading of the
        # augmented form, whose exact propagation does not depend on s0 while the stopping
        # rule eps <= tol ||wbar|| does), s0 = max(||[ubar; vbar]||, dt ||Pbar_0|| max |scale|),
        # fixed at the first step when dt is known
        self.s0_scaled = (s0 == "scaled") and not unloaded
        if s0 is None or s0 == "scaled":
            s0 = 0.0 if unloaded else 1.0
        self.kw = dict(tol=prob.tol if tol is None else tol, m_max=m_max, check_every=check_every,
                       m_fixed=m_fixed, k_fixed=k_fixed, max_substeps=max_substeps)
        self.s0 = float(s0)
        self.t = 0.0
        self.ubar = self.Mh * np.asarray(prob.u0)[self.free]
        self.vbar = self.Mh * np.asarray(prob.v0)[self.free]
        self.hist = []                      # midpoint displacements (full nodal), newest last
        self.hist4 = []                     # (t, u, v) of the previous step (fourth-order scheme)
        self.states = {"pred": {}, "corr": {}}
        self.log = []                       # per step: dict(k, m, eps, drift)
        self.matvecs = 0

    # ---------------------------------------------------------------- helpers
    def full(self, x_free):
        z = np.zeros(self.n3)
        z[self.free] = x_free
        return z

    def u(self):
        return self.full(self.Mih * self.ubar)

    def v(self):
        return self.full(self.Mih * self.vbar)

    def scale(self, t):
        return float(np.interp(t, self.prob.knots_t, self.prob.knots_s))

    def Hbar(self, hspec, x):
        """Hbar x on free DOFs; hspec = list of (weight, u_full) secant points (None: linear)."""
        X = self.full(self.Mih * x)
        if hspec is None:
            y = self.fem.H_apply(None, X)
        else:
            y = sum(wt * self.fem.H_apply(U, X) for (wt, U) in hspec)
        self.matvecs += 1
        return self.Mih * y[self.free]

    def A_apply(self, w, f, hspec, pbar):
        """f * A w for the augmented first-order system (Sec. 2.3, A for P != 0)."""
        N = self.N
        out = np.empty_like(w)
        out[:N] = f * w[N:2 * N]
        c = w[2 * N] / self.s0 if self.s0 != 0.0 else 0.0
        out[N:2 * N] = f * (-self.Hbar(hspec, w[:N]) + c * pbar)
        out[2 * N] = 0.0
        return out

    def propagate(self, w, tau, t_eval, hspec, kind):
        pbar = self.scale(t_eval) * self.P0bar
        return expv(lambda v, f: self.A_apply(v, f, hspec, pbar), w, tau,
                    state=self.states[kind], **self.kw)

    # ------------------------------------------------------------------- step
    def step(self, dt: float):
        N = self.N
        t = self.t
        if self.s0_scaled:
            self.s0_scaled = False
            smax = float(np.abs(np.asarray(self.prob.knots_s)).max())
            self.s0 = max(float(np.linalg.norm(np.concatenate([self.ubar, self.vbar]))),
                          dt * float(np.linalg.norm(self.P0bar)) * smax)
        w = np.concatenate([self.ubar, self.vbar, [self.s0]])
        rec = {}
        if self.linear:
            wn, info = self.propagate(w, dt, t + 0.5 * dt, None, "corr")
        else:
            if len(self.hist) == 0:
                pred = [(1.0, self.u())]
            elif len(self.hist) == 1:
                pred = [(1.0, self.hist[-1])]
            else:
                pred = [(1.75, self.hist[-1]), (-0.75, self.hist[-2])]
            wh, pinfo = self.propagate(w, 0.5 * dt, t + 0.25 * dt, pred, "pred")
            u_mid = self.full(self.Mih * wh[:N])
            wn, info = self.propagate(w, dt, t + 0.5 * dt, [(1.0, u_mid)], "corr")
            self.hist = (self.hist + [u_mid])[-2:]
            rec["pred"] = pinfo
        rec["corr"] = info
        rec["drift"] = abs(wn[2 * N] - self.s0)
        self.ubar = wn[:N].copy()
        self.vbar = wn[N:2 * N].copy()
        self.t = t + dt
        self.log.append(rec)
        return rec

    # ------------------------------------------------- fourth-order Magnus step
    def Hbar_u(self, U, x):
        """Hbar(U) x on free DOFs (U a full nodal displacement, None: linear)."""
        return self.Hbar(None if U is None else [(1.0, U)], x)

    def accel(self):
        """u'' = M^{-1} (P(t) - R(u)) at the current state (free DOFs, full nodal vector)."""
        u = self.u()
        R = self.fem.internal_force(u)
        P = self.scale(self.t) * traction_load(self.prob.xyz, self.prob.faces, self.prob.t0)
        return self.full((P - R)[self.free] * self.Mih ** 2)

    def u_at(self, tq):
        """Displacement predicted at a time tq inside the coming step: cubic Hermite
        extrapolation through (u, v) of the last two steps; on the first step the Taylor
        polynomial u + s v + s^2 / 2 u'' with u'' from the equation of motion."""
        t1, u1, v1 = self.t, self.u(), self.v()
        if not self.hist4:
            s = tq - t1
            return u1 + s * v1 + 0.5 * s * s * self.accel()
        t0, u0, v0 = self.hist4[-1]
        h = t1 - t0
        s = (tq - t0) / h
        h00 = 2 * s ** 3 - 3 * s ** 2 + 1
        h10 = s ** 3 - 2 * s ** 2 + s
        h01 = -2 * s ** 3 + 3 * s ** 2
        h11 = s ** 3 - s ** 2
        return h00 * u0 + h10 * h * v0 + h01 * u1 + h11 * h * v1

    def step4(self, dt: float):
        """One step of the fourth-order Magnus propagator: the Magnus series truncated after
        its two terms (Sec. 3.3, remark after the truncation-error bound), the two integrals
        evaluated by the two-point Gauss-Legendre rule at tau_{1,2} = t + (1/2 -+ sqrt(3)/6) dt
        (the fourth-order Magnus integrator of Blanes, Casas, Oteo and Ros, Phys. Rep. 470,
        2009):  Omega = dt/2 (A_1 + A_2) - sqrt(3) dt^2 / 12 [A_1, A_2],  A_i = A(tau_i).
        A_i = A[Hbar(u(tau_i)), Pbar(tau_i)], u(tau_i) predicted by u_at (reading: the paper
        gives no predictor for this scheme).  With A = [[0, I, 0], [-Hbar, 0, Pbar/s0], 0]:
            [A_1, A_2] x = [(Hbar_1 - Hbar_2) x_u + x_s (p_2 - p_1); (Hbar_2 - Hbar_1) x_v; 0],
        p_i = Pbar(tau_i) / s0, so Omega x needs Hbar_1 and Hbar_2 on x_u and x_v.  One Krylov
        projection of exp(Omega) w per step."""
        N = self.N
        t = self.t
        if self.s0_scaled:
            self.s0_scaled = False
            smax = float(np.abs(np.asarray(self.prob.knots_s)).max())
            self.s0 = max(float(np.linalg.norm(np.concatenate([self.ubar, self.vbar]))),
                          dt * float(np.linalg.norm(self.P0bar)) * smax)
        g = np.sqrt(3.0) / 6.0
        taus = (t + (0.5 - g) * dt, t + (0.5 + g) * dt)
        U = (None, None) if self.linear else tuple(self.u_at(tq) for tq in taus)
        inv_s0 = 1.0 / self.s0 if self.s0 != 0.0 else 0.0
        p1, p2 = (self.scale(tq) * self.P0bar * inv_s0 for tq in taus)
        c = np.sqrt(3.0) * dt * dt / 12.0

        def omega(w, f):
            xu, xv, xs = w[:N], w[N:2 * N], w[2 * N]
            H1u, H2u = self.Hbar_u(U[0], xu), self.Hbar_u(U[1], xu)
            H1v, H2v = self.Hbar_u(U[0], xv), self.Hbar_u(U[1], xv)
            out = np.empty_like(w)
            out[:N] = dt * xv - c * ((H1u - H2u) + xs * (p2 - p1))
            out[N:2 * N] = 0.5 * dt * (-(H1u + H2u) + xs * (p1 + p2)) - c * (H2v - H1v)
            out[2 * N] = 0.0
            return f * out

        w = np.concatenate([self.ubar, self.vbar, [self.s0]])
        u_prev, v_prev = self.u(), self.v()
        wn, info = expv(omega, w, 1.0, state=self.states["corr"], **self.kw)
        rec = {"corr": info, "drift": abs(wn[2 * N] - self.s0)}
        self.hist4 = [(t, u_prev, v_prev)]
        self.ubar = wn[:N].copy()
        self.vbar = wn[N:2 * N].copy()
        self.t = t + dt
        self.log.append(rec)
        return rec

    def run(self, dt: float, n_steps: int):
        for _ in range(n_steps):
            self.step(dt)

    # --------------------------------------------------------------- energies
    def energies(self):
        """(kinetic, strain, external work P(t)^T u) at the current state.

        Sec. 5.2 energy (1/2 vbar.vbar + strain energy), with the strain energy of the
        nonlinear models summed at the Gauss points and the work of the load reported
        separately so that E = kinetic + strain - external work.
        """
        ke = 0.5 * float(self.vbar @ self.vbar)
        u = self.u()
        se = self.fem.strain_energy(u)
        P = self.scale(self.t) * traction_load(self.prob.xyz, self.prob.faces, self.prob.t0)
        return ke, se, float(P @ u)
