"""Q1 finite elements on uniform square meshes (oracle; test infrastructure).

The paper builds one mesh B_H of the macro domain and one mesh K_h of the
reference cell Z, never a mesh of each Y_x (Section 3.1, first paragraph).
We use bilinear (Q1) elements on uniform quadrilateral meshes: the paper's
spaces are piecewise linear on deal.II cells, and the DoF counts it prints,
(N+1)^2, are those of Q1 on an N x N quad mesh.  Integrals use 2x2
Gauss-Legendre per cell and 2-point Gauss per boundary edge; the paper does
not state its rule, and the pulled-back integrands are not polynomial, so
the rule is part of the discrete problem and is fixed here.

Micro matrices on Z for one instance (discrete weak form on the reference
cell, Section 3.1; boundary weight from the change of variables):

    M_jk = int_Z  eta_j eta_k J                  (mass)
    A_jk = int_Z  grad eta_j . (K K^T J) grad eta_k   (stiffness)
    B_jk = int_dZ eta_j eta_k |cof(F) nu|        (boundary mass)
    b    = B 1,   |dY| = 1^T b

Node numbering: j = j2*(N+1) + j1 with reference coordinate
y = (-1 + j1 h, -1 + j2 h), h = 2/N.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import deformation as geo

# 2-point Gauss-Legendre rule on [0,1]
GAUSS_X = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
GAUSS_W = np.array([0.5, 0.5])

# local node l = l1 + 2*l2 sits at local corner (l1, l2)
LOCAL_CORNERS = np.array([[0, 0], [1, 0], [0, 1], [1, 1]])


def q1_shape(x1, x2):
    """Bilinear shape functions and their local gradients at (x1, x2) in
    [0,1]^2.  Returns (phi[4], dphi[4,2])."""
    phi = np.empty(4)
    dphi = np.empty((4, 2))
    for l, (l1, l2) in enumerate(LOCAL_CORNERS):
        f1 = x1 if l1 else 1.0 - x1
        f2 = x2 if l2 else 1.0 - x2
        d1 = 1.0 if l1 else -1.0
        d2 = 1.0 if l2 else -1.0
        phi[l] = f1 * f2
        dphi[l] = (d1 * f2, f1 * d2)
    return phi, dphi


def _cell_nodes(N):
    """Global node index of each local corner of every cell, shape (N*N, 4)."""
    c1, c2 = np.meshgrid(np.arange(N), np.arange(N), indexing="xy")
    c1, c2 = c1.ravel(), c2.ravel()
    idx = np.empty((N * N, 4), dtype=np.int64)
    for l, (l1, l2) in enumerate(LOCAL_CORNERS):
        idx[:, l] = (c2 + l2) * (N + 1) + (c1 + l1)
    return c1, c2, idx


def _quad_points(N, origin, h):
    """Physical coordinates and weights of the 2x2 rule in every cell.
    Returns y1, y2 of shape (N*N, 4), weight (4,), shape tables."""
    c1, c2, idx = _cell_nodes(N)
    y1 = np.empty((N * N, 4))
    y2 = np.empty((N * N, 4))
    wq = np.empty(4)
    phis = np.empty((4, 4))
    grads = np.empty((4, 4, 2))
    q = 0
    for g2 in range(2):
        for g1 in range(2):
            y1[:, q] = origin + (c1 + GAUSS_X[g1]) * h
            y2[:, q] = origin + (c2 + GAUSS_X[g2]) * h
            wq[q] = GAUSS_W[g1] * GAUSS_W[g2] * h * h
            phis[q], dl = q1_shape(GAUSS_X[g1], GAUSS_X[g2])
            grads[q] = dl / h
            q += 1
    return idx, y1, y2, wq, phis, grads


def _scatter(idx, Ke, n):
    rows = np.repeat(idx, 4, axis=1).ravel()
    cols = np.tile(idx, (1, 4)).ravel()
    return sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(n, n))


def assemble_cells(N, origin, h, J, C):
    """Mass and stiffness on a uniform N x N mesh with per-quadrature-point
    weights J (ncell, 4) and C (ncell, 4, 2, 2).  Returns (M, A) as CSR."""
    idx, _, _, wq, phis, grads = _quad_points(N, origin, h)
    n = (N + 1) ** 2
    Me = np.einsum("q,cq,ql,qm->clm", wq, J, phis, phis)
    Ae = np.einsum("q,qlr,cqrs,qms->clm", wq, grads, C, grads)
    return _scatter(idx, Me, n), _scatter(idx, Ae, n)


def boundary_edges(N):
    """The 4N boundary edges of Z: (node_a, node_b, y1(g), y2(g), tangent)
    with y of shape (N, 2) over the two Gauss points of each edge."""
    h = 2.0 / N
    e = np.arange(N)
    s = -1.0 + (e[:, None] + GAUSS_X[None, :]) * h       # coordinate along the edge
    edges = []
    # bottom y2 = -1 and top y2 = +1, tangent (1, 0)
    for row, yfix in ((0, -1.0), (N, 1.0)):
        na = row * (N + 1) + e
        edges.append((na, na + 1, s, np.full_like(s, yfix), (1.0, 0.0)))
    # left y1 = -1 and right y1 = +1, tangent (0, 1)
    for col, yfix in ((0, -1.0), (N, 1.0)):
        na = e * (N + 1) + col
        edges.append((na, na + N + 1, np.full_like(s, yfix), s, (0.0, 1.0)))
    return edges


def assemble_boundary(N, weight_fn):
    """B_jk = sum over boundary edges and 2 Gauss points of
    (h/2) * w(y) * eta_j eta_k, with w = weight_fn(y1, y2, tau)."""
    return assemble_boundary_weights(N, [weight_fn(y1, y2, tau) for _, _, y1, y2, tau in boundary_edges(N)])


def assemble_boundary_weights(N, weights):
    """B from the surface weights at the boundary Gauss points, one (N, 2)
    array per side in the order of boundary_edges (bottom, top, left, right)."""
    h = 2.0 / N
    n = (N + 1) ** 2
    rows, cols, vals = [], [], []
    basis = np.stack([1.0 - GAUSS_X, GAUSS_X], axis=1)     # (g, local)
    for (na, nb, _, _, _), w in zip(boundary_edges(N), weights):
        Be = np.einsum("g,eg,gl,gm->elm", GAUSS_W * h, w, basis, basis)
        loc = np.stack([na, nb], axis=1)
        rows.append(np.repeat(loc, 2, axis=1).ravel())
        cols.append(np.tile(loc, (1, 2)).ravel())
        vals.append(Be.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))



def micro_matrices(N, a, theta=0.0):
    """(M, A, B) of one instance with amplitude a and angle theta."""
    h = 2.0 / N
    _, y1, y2, _, _, _ = _quad_points(N, -1.0, h)
    J, C = geo.pullback(y1, y2, a, theta)
    M, A = assemble_cells(N, -1.0, h, J, C)
    B = assemble_boundary(N, lambda s1, s2, tau: geo.boundary_weight(s1, s2, tau, a, theta))
    return M, A, B


def quadrature_points(N):
    """Reference coordinates of the points where a map's Jacobian is needed:
    cells (N*N, 4) in cell order c2*N + c1 and point order g2*2 + g1, and
    boundary (4, N, 2) per side (bottom, top, left, right), edge, point."""
    h = 2.0 / N
    _, y1, y2, _, _, _ = _quad_points(N, -1.0, h)
    b1 = np.stack([e[2] for e in boundary_edges(N)])
    b2 = np.stack([e[3] for e in boundary_edges(N)])
    return (y1, y2), (b1, b2)


def micro_matrices_from_jacobians(N, Fc, Fb):
    """(M, A, B) of one instance whose map is known only through its
    Jacobians: Fc (N*N, 4, 2, 2) at the cell Gauss points and Fb (4, N, 2, 2, 2)
    at the boundary Gauss points (layout of quadrature_points)."""
    h = 2.0 / N
    J, C = geo.pullback_from_jacobian(Fc)
    M, A = assemble_cells(N, -1.0, h, J, C)
    W = [geo.boundary_weight_from_jacobian(Fb[k], tau) for k, (_, _, _, _, tau) in enumerate(boundary_edges(N))]
    return M, A, assemble_boundary_weights(N, W)


def micro_matrices_da(N, a, theta=0.0):
    """(dM/da, dA/da, dB/da) of one instance."""
    h = 2.0 / N
    _, y1, y2, _, _, _ = _quad_points(N, -1.0, h)
    dJ, dC = geo.pullback_da(y1, y2, a, theta)
    dM, dA = assemble_cells(N, -1.0, h, dJ, dC)
    dB = assemble_boundary(N, lambda s1, s2, tau: geo.boundary_weight_da(s1, s2, tau, a, theta))
    return dM, dA, dB


def macro_matrices(NM):
    """Q1 mass M_H and stiffness K_H on [0,1]^2 with NM x NM cells and the
    nodal coupling weights L = diag(M_H 1) (the integral of each hat)."""
    h = 1.0 / NM
    ncell = NM * NM
    J = np.ones((ncell, 4))
    C = np.broadcast_to(np.eye(2), (ncell, 4, 2, 2)).copy()
    MH, KH = assemble_cells(NM, 0.0, h, J, C)
    L = np.asarray(MH.sum(axis=1)).ravel()
    return MH, KH, L


def macro_boundary(NM):
    k = np.arange(NM + 1)
    k1, k2 = np.meshgrid(k, k, indexing="xy")
    return ((k1 == 0) | (k2 == 0) | (k1 == NM) | (k2 == NM)).ravel()
