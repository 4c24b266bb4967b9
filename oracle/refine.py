"""Error-indicator-driven micro refinement (oracle; test infrastructure).

The paper's conclusions propose refining the microscopic computations from
an error indicator defined over all micro grids, to maximise the global
error reduction; they give no indicator.  Reading (the paper's
implementation is built on deal.II, whose standard indicator is the
gradient-jump estimator of Kelly et al.):

* per instance, the jump of the pulled-back flux d (C grad_z v) . nu across
  every interior edge of the reference mesh K_h (C = K K^T J, the
  coefficient of the pulled-back stiffness, Section 3.1), squared and
  integrated along the edge, weighted by h/12 (the cell-wise weight h/24 of
  that estimator, each interior edge seen from its two cells):
      eta_i^2 = sum_e (h/12) int_e [[ d (C grad_z v_i) . nu_e ]]^2 ds,
  with the 2-point Gauss rule on each edge and C at the edge's points;
  the tangential derivative of a Q1 function is continuous across an edge,
  so the jump is C11 [[d_z1 v]] across lines z1 = const and C22 [[d_z2 v]]
  across lines z2 = const;
* the global functional is sum_i eta_i^2; marking takes the fewest
  instances, largest eta first, whose indicators reach the fraction theta of
  it (bulk marking), among the instances that can still be refined;
* a marked instance goes from N to 2N cells per side; its micro field is
  carried over by Q1 interpolation, exact on the nested mesh.
"""
from __future__ import annotations

import numpy as np

from . import deformation as geo
from . import fem


def indicator(N, v, a, theta=0.0, d=0.5):
    """eta^2 of one instance with N x N cells, nodal values v ((N+1)^2),
    deformation amplitude a (and angle theta), micro diffusion d."""
    h = 2.0 / N
    V = np.asarray(v).reshape(N + 1, N + 1)       # [j2, j1]
    total = 0.0
    # lines z1 = -1 + j1 h, j1 = 1..N-1: edges between cells (j1-1, c2) and (j1, c2)
    for j1 in range(1, N):
        for c2 in range(N):
            for g, wg in zip(fem.GAUSS_X, fem.GAUSS_W):
                # d_z1 v of the left and right cells at the point (z1 fixed, z2 = -1 + (c2 + g) h)
                left = ((V[c2, j1] - V[c2, j1 - 1]) * (1 - g) + (V[c2 + 1, j1] - V[c2 + 1, j1 - 1]) * g) / h
                right = ((V[c2, j1 + 1] - V[c2, j1]) * (1 - g) + (V[c2 + 1, j1 + 1] - V[c2 + 1, j1]) * g) / h
                _, C = geo.pullback(-1.0 + j1 * h, -1.0 + (c2 + g) * h, a, theta)
                jump = d * C[0, 0] * (right - left)
                total += (h / 12.0) * wg * h * jump * jump
    # lines z2 = -1 + j2 h: edges between cells (c1, j2-1) and (c1, j2)
    for j2 in range(1, N):
        for c1 in range(N):
            for g, wg in zip(fem.GAUSS_X, fem.GAUSS_W):
                below = ((V[j2, c1] - V[j2 - 1, c1]) * (1 - g) + (V[j2, c1 + 1] - V[j2 - 1, c1 + 1]) * g) / h
                above = ((V[j2 + 1, c1] - V[j2, c1]) * (1 - g) + (V[j2 + 1, c1 + 1] - V[j2, c1 + 1]) * g) / h
                _, C = geo.pullback(-1.0 + (c1 + g) * h, -1.0 + j2 * h, a, theta)
                jump = d * C[1, 1] * (above - below)
                total += (h / 12.0) * wg * h * jump * jump
    return total


def mark(eta2, levels, theta, max_level=64):
    """Bulk marking over all instances: the fewest refinable instances,
    largest indicator first (ties: lower index first), whose indicators sum
    to at least theta times the global functional sum eta^2."""
    eta2 = np.asarray(eta2, dtype=np.float64)
    ok = np.asarray(levels) * 2 <= max_level
    total = float(eta2.sum())
    order = sorted(np.flatnonzero(ok).tolist(), key=lambda i: (-eta2[i], i))
    marked, acc = [], 0.0
    for i in order:
        if acc >= theta * total:
            break
        marked.append(i)
        acc += eta2[i]
    return np.array(sorted(marked), dtype=np.int64)


def prolong(N, v):
    """Q1 interpolation of nodal values on the N x N mesh onto the nested
    2N x 2N mesh of the same square."""
    V = np.asarray(v).reshape(N + 1, N + 1)
    F = np.empty((2 * N + 1, 2 * N + 1))
    for i2 in range(2 * N + 1):
        for i1 in range(2 * N + 1):
            a1, b1 = i1 // 2, i1 % 2
            a2, b2 = i2 // 2, i2 % 2
            # the fine node sits at the coarse cell's corner, edge midpoint or centre
            s = 0.0
            for q2 in range(b2 + 1):
                for q1 in range(b1 + 1):
                    s += V[a2 + q2, a1 + q1]
            F[i2, i1] = s / ((b1 + 1) * (b2 + 1))
    return F.ravel()
