"""Discrete adjoint of the time-stepped two-scale system (oracle; test
infrastructure).

The paper has no adjoint; this is the exact derivative of the discrete
forward map of module twoscale.  Observable: J = u^{N T} M_H u^N, the
integral of u_h(T)^2.  Parameters: the per-instance amplitudes a_i, which
enter S_i, M_i, b_i and |dY_i| through the pullback.

Step residuals (n = 0..N-1), as in twoscale:
    R_i^{n+1} = S_i v_i^{n+1} - kappa p u_i^{n+1} b_i - M_i v_i^n / dt
    Q^{n+1}   = (M_H/dt + D K_H) u^{n+1} - sigma L F^{n+1} - M_H u^n / dt   (interior rows)
Lagrangian: J - sum_n [ sum_i lam_i^{n+1 T} R_i^{n+1} + mu^{n+1 T} Q^{n+1} ].

Stationarity in v_i^{n+1} and u^{n+1} gives, backwards from n+1 = N with
lam^{N+1} = 0, mu^{N+1} = 0:
    S_i lam_i + sigma kappa L_ii mu_i / |dY_i| b_i = M_i lam_i^{n+2} / dt
    (M_H/dt + D K_H - sigma kappa p L) mu - kappa p (b_i^T lam_i)_i
          = delta_{n+1,N} 2 M_H u^N + M_H mu^{n+2} / dt           (interior rows)
Eliminating lam_i = lam0_i - sigma L_ii mu_i / (p |dY_i|) w_i with
lam0_i = S_i^{-1} M_i lam_i^{n+2}/dt leaves A_M mu = rhs + kappa p (b_i^T lam0_i)_i
with the forward macro matrix A_M (it is symmetric).

Gradient:
    dJ/da_i = - sum_n [ lam_i^{n+1 T} (dS_i v_i^{n+1} - kappa p u_i^{n+1} db_i
                                       - dM_i v_i^n / dt)
                        - sigma mu_i^{n+1} L_ii dF_i^{n+1} ]
    dF_i = -kappa [ db_i^T v_i / |dY_i| - (b_i^T v_i)(1^T db_i) / |dY_i|^2 ].
"""
from __future__ import annotations

import numpy as np

from . import fem
from .twoscale import TwoScale


def _derivative_data(ts: TwoScale):
    prm = ts.prm
    out = []
    for I in ts.inst:
        dM, dA, dB = fem.micro_matrices_da(I.N, I.a, I.theta)
        dS = (dM / prm.dt + prm.d * dA + prm.kappa * dB).tocsr()
        db = np.asarray(dB.sum(axis=1)).ravel()
        out.append((dM.tocsr(), dS, db, float(db.sum())))
    return out


def gradient(ts: TwoScale, u0, v0, n_steps):
    """Returns (J, dJ/da) for n_steps implicit-Euler steps from (u0, v0)."""
    prm = ts.prm
    kap, p, sg, dt = prm.kappa, prm.p, prm.sigma, prm.dt
    n_inst = len(ts.inst)
    us = [np.asarray(u0, dtype=np.float64).copy()]
    vs = [np.asarray(v0, dtype=np.float64).copy()]
    for _ in range(n_steps):
        u, v, _ = ts.step(us[-1], vs[-1])
        us.append(u)
        vs.append(v)
    J = ts.observable(us[-1])

    der = _derivative_data(ts)
    g = np.zeros(n_inst)
    lam_next = ts.zeros_micro()
    mu_next = np.zeros(len(us[0]))
    for m in range(n_steps, 0, -1):             # solve for lam^m, mu^m
        lam0 = ts.zeros_micro()
        blam0 = np.zeros(n_inst)
        for i, (I, ln) in enumerate(zip(ts.inst, ts.split(lam_next))):
            x = I.chol.solve(I.M @ ln / dt)
            lam0[ts.offsets[i]:ts.offsets[i + 1]] = x
            blam0[i] = float(I.b @ x)
        rhs = ts.MH @ mu_next / dt + kap * p * blam0
        if m == n_steps:
            rhs = rhs + 2.0 * (ts.MH @ us[-1])
        mu = np.zeros_like(mu_next)
        mu[ts.interior] = ts.AM_chol.solve(rhs[ts.interior])
        lam = lam0.copy()
        for i, I in enumerate(ts.inst):
            lam[ts.offsets[i]:ts.offsets[i + 1]] -= sg * ts.L[i] * mu[i] / (p * I.len) * I.w
        # gradient contributions of step m (states v^m, v^{m-1}, u^m)
        vm, vp, um = ts.split(vs[m]), ts.split(vs[m - 1]), us[m]
        for i, (I, li) in enumerate(zip(ts.inst, ts.split(lam))):
            dM, dS, db, dlen = der[i]
            dR = dS @ vm[i] - kap * p * um[i] * db - dM @ vp[i] / dt
            dF = -kap * (float(db @ vm[i]) / I.len
                         - float(I.b @ vm[i]) * dlen / I.len ** 2)
            g[i] -= float(li @ dR) - sg * mu[i] * ts.L[i] * dF
        lam_next, mu_next = lam, mu
    return J, g
