"""The coupled macro/micro time step (oracle; test infrastructure).

System (a time-dependent two-field reduction of the paper's model,
Section 2.1, with its Robin exchange on the whole micro boundary):

    u_t - D Lap u = sigma * Fbar(x)            in Omega = [0,1]^2, u = 0 on dOmega
    v_t - d Lap_y v = 0                        in Y_x
    d grad_y v . n = kappa (p u(x) - v)        on dY_x
    Fbar(x) = mean over dY_x of kappa (p u(x) - v)

sigma = -1 is the paper's sign: the macro equation loses what enters the
cells (first line of the model system, the term -int (kappa1 u - kappa2 v)).

Discretisation: Q1 on B_H and on the reference cell Z (module fem); one
micro system per macro node, fed the nodal value u_i (Section 3.3, micro
system at the support point of the macro basis function); implicit Euler.
Unknowns of one step (u^{n+1}, v^{n+1}):

    S_i v_i - kappa p u_i b_i = M_i v_i^n / dt,   S_i = M_i/dt + d A_i + kappa B_i
    (M_H/dt + D K_H) u - sigma L F = M_H u^n/dt   on interior macro rows, u = 0 on dOmega
    F_i = kappa p u_i - (kappa/|dY_i|) b_i^T v_i

with L = diag(M_H 1) (the coupling source lumped at the support points).
The step is linear, so it has one solution (weak solvability theorem,
Section 2.2).  Three routes reach it:

* ``step``            exact Schur elimination: v_i = v0_i + u_i w_i with
                      w_i = kappa p S_i^{-1} b_i (time-invariant) and
                      v0_i = S_i^{-1} M_i v_i^n / dt, then one macro solve.
* ``step_fixed_point`` the paper's alternating coupling (Section 3.3):
                      macro solve with the previous micro data, micro solves
                      with the new macro data, until successive values of the
                      residual sum (macro residual plus mean micro residual,
                      the threshold of Section 3.5) stop changing.
* ``step_monolithic`` one dense solve of the whole block system (tiny cases).

Solves use banded Cholesky factorisations from LAPACK (scipy).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from . import fem


@dataclasses.dataclass
class Params:
    macro_cells: int
    dt: float
    D: float = 1.0
    d: float = 0.5
    kappa: float = 1.0
    p: float = 1.0
    sigma: int = -1


def _band_lower(A, bw):
    """Lower banded storage ab[k, j] = A[j+k, j] for k = 0..bw."""
    A = A.tocsr()
    n = A.shape[0]
    ab = np.zeros((bw + 1, n))
    for k in range(bw + 1):
        ab[k, : n - k] = A.diagonal(-k)
    return ab


class BandedSPD:
    """Cholesky factor of a sparse SPD matrix with known lower bandwidth."""

    def __init__(self, A, bw):
        self.cb = sla.cholesky_banded(_band_lower(A, bw), lower=True)

    def solve(self, rhs):
        return sla.cho_solve_banded((self.cb, True), rhs)


class Instance:
    """One micro system: time-invariant matrices and the affine response."""

    def __init__(self, N, a, theta, prm: Params, jacobians=None):
        self.N = int(N)
        if jacobians is None:
            self.a, self.theta = float(a), float(theta)
            self.M, self.A, self.B = fem.micro_matrices(self.N, self.a, self.theta)
        else:
            # a general map, given by its Jacobians at the quadrature points
            self.a = self.theta = None
            self.M, self.A, self.B = fem.micro_matrices_from_jacobians(self.N, *jacobians)
        self.S = (self.M / prm.dt + prm.d * self.A + prm.kappa * self.B).tocsr()
        self.b = np.asarray(self.B.sum(axis=1)).ravel()
        self.len = float(self.b.sum())
        self.chol = BandedSPD(self.S, self.N + 2)
        self.w = prm.kappa * prm.p * self.chol.solve(self.b)
        self.beta = prm.kappa * prm.p - prm.kappa / self.len * float(self.b @ self.w)

    @property
    def n(self):
        return (self.N + 1) ** 2


class TwoScale:
    """The full batch: one Instance per macro node plus the macro operator."""

    def __init__(self, prm: Params, levels, a, theta=None, jacobians=None):
        """jacobians: None (the deformation family with amplitudes a, angles
        theta) or one (Fc, Fb) pair per instance (fem.micro_matrices_from_jacobians)."""
        self.prm = prm
        n_inst = (prm.macro_cells + 1) ** 2
        levels = np.asarray(levels)
        assert levels.shape == (n_inst,)
        if jacobians is None:
            a = np.asarray(a, dtype=np.float64)
            theta = np.zeros(n_inst) if theta is None else np.asarray(theta, dtype=np.float64)
            assert a.shape == theta.shape == (n_inst,)
            self.inst = [Instance(levels[i], a[i], theta[i], prm) for i in range(n_inst)]
        else:
            assert len(jacobians) == n_inst
            self.inst = [Instance(levels[i], None, None, prm, jacobians[i]) for i in range(n_inst)]
        self.offsets = np.concatenate([[0], np.cumsum([I.n for I in self.inst])]).astype(np.int64)
        self.MH, self.KH, self.L = fem.macro_matrices(prm.macro_cells)
        self.bnd = fem.macro_boundary(prm.macro_cells)
        self.interior = np.flatnonzero(~self.bnd)
        self.beta = np.array([I.beta for I in self.inst])
        self.len = np.array([I.len for I in self.inst])
        # A_M = M_H/dt + D K_H - sigma L diag(beta), interior block
        AM = (self.MH / prm.dt + prm.D * self.KH).tolil()
        AM.setdiag(AM.diagonal() - prm.sigma * self.L * self.beta)
        self.AM = AM.tocsr()[self.interior][:, self.interior]
        self.AM_chol = BandedSPD(self.AM, max(prm.macro_cells - 1, 0) + 1)

    # -- ragged helpers ---------------------------------------------------
    def split(self, v):
        return [v[self.offsets[i]:self.offsets[i + 1]] for i in range(len(self.inst))]

    def zeros_micro(self):
        return np.zeros(int(self.offsets[-1]))

    # -- one step, exact Schur route ----------------------------------------
    def micro_free(self, v):
        """v0_i = S_i^{-1} M_i v_i^n / dt and alpha_i = -(kappa/|dY_i|) b_i^T v0_i."""
        prm = self.prm
        v0 = np.empty_like(v)
        alpha = np.empty(len(self.inst))
        for i, (I, vi) in enumerate(zip(self.inst, self.split(v))):
            x = I.chol.solve(I.M @ vi / prm.dt)
            v0[self.offsets[i]:self.offsets[i + 1]] = x
            alpha[i] = -prm.kappa / I.len * float(I.b @ x)
        return v0, alpha

    def macro_solve(self, u, alpha):
        """u^{n+1} from A_M u = M_H u^n/dt + sigma L alpha on interior rows."""
        prm = self.prm
        rhs = self.MH @ u / prm.dt + prm.sigma * self.L * alpha
        un = np.zeros_like(u)
        un[self.interior] = self.AM_chol.solve(rhs[self.interior])
        return un

    def step(self, u, v):
        """One implicit-Euler step.  Returns (u^{n+1}, v^{n+1}, F^{n+1})."""
        v0, alpha = self.micro_free(v)
        un = self.macro_solve(u, alpha)
        vn = v0.copy()
        for i, I in enumerate(self.inst):
            vn[self.offsets[i]:self.offsets[i + 1]] += un[i] * I.w
        F = self.beta * un + alpha
        return un, vn, F

    def flux(self, u, v):
        """F_i = kappa p u_i - (kappa/|dY_i|) b_i^T v_i (mean Robin flux)."""
        prm = self.prm
        bv = np.array([float(I.b @ vi) for I, vi in zip(self.inst, self.split(v))])
        return prm.kappa * prm.p * u - prm.kappa / self.len * bv

    # -- residuals of the coupled step equations ----------------------------
    def residuals(self, u, v, un, vn):
        """(macro residual on interior rows, per-instance micro residuals)."""
        prm = self.prm
        F = self.flux(un, vn)
        rm = (self.MH / prm.dt + prm.D * self.KH) @ un - prm.sigma * self.L * F - self.MH @ u / prm.dt
        rm = rm[self.interior]
        rv = [I.S @ x - prm.kappa * prm.p * un[i] * I.b - I.M @ xo / prm.dt
              for i, (I, x, xo) in enumerate(zip(self.inst, self.split(vn), self.split(v)))]
        return rm, rv

    # -- the paper's alternating coupling -------------------------------------
    def step_fixed_point(self, u, v, tol=1e-14, max_iter=500):
        """Alternate macro and micro solves (Section 3.3) until the residual
        sum (macro residual plus mean micro residual) changes by less than
        tol between iterations.  Returns (u, v, F, iterations)."""
        prm = self.prm
        kap, p, sg = prm.kappa, prm.p, prm.sigma
        # macro operator with the micro data lagged: the u-part of F moves left
        AMf = (self.MH / prm.dt + prm.D * self.KH).tolil()
        AMf.setdiag(AMf.diagonal() - sg * kap * p * self.L)
        AMf = AMf.tocsr()[self.interior][:, self.interior]
        solver = BandedSPD(AMf, max(prm.macro_cells - 1, 0) + 1)
        vk = v.copy()
        prev = None
        for it in range(1, max_iter + 1):
            bv = np.array([float(I.b @ x) for I, x in zip(self.inst, self.split(vk))])
            rhs = self.MH @ u / prm.dt - sg * self.L * (kap / self.len) * bv
            uk = np.zeros_like(u)
            uk[self.interior] = solver.solve(rhs[self.interior])
            vk = np.empty_like(v)
            for i, (I, xo) in enumerate(zip(self.inst, self.split(v))):
                vk[self.offsets[i]:self.offsets[i + 1]] = I.chol.solve(
                    I.M @ xo / prm.dt + kap * p * uk[i] * I.b)
            rm, rv = self.residuals(u, v, uk, vk)
            res = np.linalg.norm(rm) + np.mean([np.linalg.norm(r) for r in rv])
            if prev is not None and abs(res - prev) < tol:
                break
            prev = res
        return uk, vk, self.flux(uk, vk), it

    # -- dense monolithic solve (brute force, tiny cases only) -----------------
    def step_monolithic(self, u, v):
        prm = self.prm
        nm = len(u)
        nv = int(self.offsets[-1])
        Afull = np.zeros((nm + nv, nm + nv))
        rhs = np.zeros(nm + nv)
        Mu = (self.MH / prm.dt + prm.D * self.KH).toarray()
        for k in range(nm):
            if self.bnd[k]:
                Afull[k, k] = 1.0
                continue
            Afull[k, :nm] = Mu[k]
            # - sigma L_k F_k with F_k = kappa p u_k - (kappa/len_k) b_k^T v_k
            Afull[k, k] -= prm.sigma * self.L[k] * prm.kappa * prm.p
            o0, o1 = nm + self.offsets[k], nm + self.offsets[k + 1]
            Afull[k, o0:o1] += prm.sigma * self.L[k] * prm.kappa / self.len[k] * self.inst[k].b
            rhs[k] = (self.MH @ u)[k] / prm.dt
        for i, (I, xo) in enumerate(zip(self.inst, self.split(v))):
            o0, o1 = nm + self.offsets[i], nm + self.offsets[i + 1]
            Afull[o0:o1, o0:o1] = I.S.toarray()
            Afull[o0:o1, i] = -prm.kappa * prm.p * I.b
            rhs[o0:o1] = I.M @ xo / prm.dt
        z = np.linalg.solve(Afull, rhs)
        un, vn = z[:nm], z[nm:]
        return un, vn, self.flux(un, vn)

    # -- time loop ----------------------------------------------------------------
    def run(self, u0, v0, n_steps):
        """Returns dict(u=(n_steps+1, n_macro), F=(n_steps, n_inst), v=final v)."""
        us = [np.asarray(u0, dtype=np.float64).copy()]
        Fs = []
        u, v = us[0], np.asarray(v0, dtype=np.float64).copy()
        for _ in range(n_steps):
            u, v, F = self.step(u, v)
            us.append(u)
            Fs.append(F)
        return {"u": np.array(us), "F": np.array(Fs), "v": v}

    def observable(self, u):
        """J = u^T M_H u = int_Omega u_h^2 (exact for Q1)."""
        return float(u @ (self.MH @ u))
