"""The paper's stationary three-field system (oracle; test infrastructure).

Model (Section 2.1, the system with u, w on the macro domain and v in every
micro domain; Section 4 solves it on Omega = [-1,1]^2 and Z = [-1,1]^2):

    -Lap u            = f^u - int_{G^I} (k1 u - k2 v + g^v_1) dsigma_y   in Omega
     u = u_D on the Dirichlet part of dOmega,  grad u . n = g^u on the rest
    -Dv Lap_y v       = f^v                                             in Y_x
     Dv grad_y v . n  = k1 u - k2 v + g^v_1  on G^I_x
                        k3 w - k4 v + g^v_2  on G^O_x
                        g^v_3                on G^N_x
    -div(Dw grad w)   = f^w - int_{G^O} (k3 w - k4 v + g^v_2) dsigma_y   in Omega
     Dw grad w . n    = g^w on dOmega

The g terms are those of the manufactured form (Section 4.1); the model
itself has them zero.  Discretisation as for the time-dependent system
(modules fem and deformation): Q1 on the macro mesh and on the reference
cell Z, 2x2 Gauss per cell and 2-point Gauss per edge, the map entering
only through its Jacobian at those points (Section 3.1), one micro system
per macro node fed the nodal values u_k, w_k (Section 3.3), and the
exchange integral of each macro equation taken at the nodes with the
weights L = diag(M_H 1).  The parts G^I, G^O, G^N of dY_x are images of
whole sides of Z, one part per side (the text does not fix them).

The discrete unknowns (u, w, v_0 .. v_{n-1}) satisfy one sparse linear
system, written out here block by block:

    K_H u + L (k1 |G^I| u - k2 b_I^T v + G_I)       = F^u + N^u    (u not Dirichlet)
    Dw K_H w + L (k3 |G^O| w - k4 b_O^T v + G_O)    = F^w + N^w
    S_k v_k - k1 u_k b_I,k - k3 w_k b_O,k           = F^v_k
    S_k = Dv A_k + k2 B^I_k + k4 B^O_k

with b_I = B^I 1, |G^I| = 1^T b_I (b_O, |G^O| alike), G_I the G^I-integral
of g^v_1 at x_k, F the bulk loads, N the Neumann loads.  It is solved in
one sparse LU factorisation (scipy); nothing is eliminated by hand.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import deformation as geo
from . import fem

# side order of Z and of Omega, as in fem.boundary_edges: bottom, top, left, right
SIDE_NORMALS = ((0.0, -1.0), (0.0, 1.0), (-1.0, 0.0), (1.0, 0.0))
PART_N, PART_I, PART_O = 0, 1, 2


@dataclasses.dataclass
class StationaryParams:
    macro_cells: int
    Dv: float = 1.0
    Dw: float = 0.1
    kappa1: float = 0.5
    kappa2: float = 1.0
    kappa3: float = 0.25
    kappa4: float = 1.0
    # part of dY_x on each side of Z (bottom, top, left, right)
    parts: tuple = (PART_N, PART_N, PART_I, PART_O)
    # sides of Omega (same order) where u is prescribed
    dirichlet: tuple = (False, False, True, False)


@dataclasses.dataclass
class StationaryData:
    """Sources and boundary data.  x1, x2 are macro coordinates (arrays for
    macro quantities, scalars -- the node x_k -- for micro ones); z1, z2 are
    reference coordinates in Z."""
    fu: Callable = lambda x1, x2: 0.0 * x1
    fw: Callable = lambda x1, x2: 0.0 * x1
    fv: Callable = lambda x1, x2, z1, z2: 0.0 * z1
    # g^v of a part (PART_I: g^v_1, PART_O: g^v_2, PART_N: g^v_3)
    gv: Callable = lambda part, x1, x2, z1, z2: 0.0 * z1
    uD: Callable = lambda x1, x2: 0.0 * x1
    # Neumann fluxes grad u . n and Dw grad w . n on a side with outward normal n
    gu: Callable = lambda x1, x2, n: 0.0 * x1
    gw: Callable = lambda x1, x2, n: 0.0 * x1


def constant_data(fu=0.0, fv=0.0, fw=0.0, u_dirichlet=1.0) -> StationaryData:
    """Constant sources, zero Neumann data, constant Dirichlet value (the
    setting of the Case A/B experiments, Table 3: f^u = f^w = 0, u_0 = 1)."""
    return StationaryData(fu=lambda x1, x2: fu + 0.0 * x1, fw=lambda x1, x2: fw + 0.0 * x1,
                          fv=lambda x1, x2, z1, z2: fv + 0.0 * z1,
                          uD=lambda x1, x2: u_dirichlet + 0.0 * x1)


def macro_nodes(NM):
    """Node coordinates of the macro mesh of [-1,1]^2, node k = k2 (NM+1) + k1."""
    k = np.arange(NM + 1)
    k1, k2 = np.meshgrid(k, k, indexing="xy")
    H = 2.0 / NM
    return (-1.0 + k1 * H).ravel(), (-1.0 + k2 * H).ravel()


def _cell_load(N, origin, h, weight, fvals):
    """int f eta_j (weight) over the cells: weight and fvals (ncell, 4) at the
    2x2 Gauss points."""
    idx, _, _, wq, phis, _ = fem._quad_points(N, origin, h)
    n = (N + 1) ** 2
    le = np.einsum("q,cq,cq,ql->cl", wq, weight, fvals, phis)
    out = np.zeros(n)
    np.add.at(out, idx.ravel(), le.ravel())
    return out


def _side_load(N, side, vals):
    """int over one side of eta_j times vals (N, 2) at its Gauss points
    (vals includes the surface weight)."""
    h = 2.0 / N
    na, nb, _, _, _ = fem.boundary_edges(N)[side]
    basis = np.stack([1.0 - fem.GAUSS_X, fem.GAUSS_X], axis=1)     # (g, local)
    le = np.einsum("g,eg,gl->el", fem.GAUSS_W * h, vals, basis)
    out = np.zeros((N + 1) ** 2)
    np.add.at(out, na, le[:, 0])
    np.add.at(out, nb, le[:, 1])
    return out


def micro_system(prm: StationaryParams, N, Fc, Fb, x1, x2, data: StationaryData):
    """Operator and loads of the micro system at the macro node (x1, x2):
    S, b_I, b_O, |G^I|, |G^O|, F^v and the part integrals G_I, G_O of g^v."""
    h = 2.0 / N
    J, C = geo.pullback_from_jacobian(Fc)
    _, A = fem.assemble_cells(N, -1.0, h, J, C)
    edges = fem.boundary_edges(N)
    W = [geo.boundary_weight_from_jacobian(Fb[s], edges[s][4]) for s in range(4)]
    kap = {PART_N: 0.0, PART_I: prm.kappa2, PART_O: prm.kappa4}
    S = prm.Dv * A
    n = (N + 1) ** 2
    bI, bO = np.zeros(n), np.zeros(n)
    _, y1, y2, _, _, _ = fem._quad_points(N, -1.0, h)
    Fv = _cell_load(N, -1.0, h, J, data.fv(x1, x2, y1, y2))
    GI = GO = 0.0
    for s in range(4):
        Ws = [W[t] if t == s else np.zeros_like(W[t]) for t in range(4)]
        Bs = fem.assemble_boundary_weights(N, Ws)
        part = prm.parts[s]
        S = S + kap[part] * Bs
        ones = np.ones(n)
        _, _, z1, z2, _ = edges[s]
        g = data.gv(part, x1, x2, z1, z2) * W[s]
        Fv = Fv + _side_load(N, s, g)
        gint = float(np.sum(fem.GAUSS_W[None, :] * h * g))
        if part == PART_I:
            bI += Bs @ ones
            GI += gint
        elif part == PART_O:
            bO += Bs @ ones
            GO += gint
    return S.tocsr(), bI, bO, bI.sum(), bO.sum(), Fv, GI, GO


def macro_system(prm: StationaryParams, data: StationaryData):
    """K_H, L and the loads F^u + N^u, F^w + N^w on [-1,1]^2, and the mask
    and values of the Dirichlet nodes of u."""
    NM = prm.macro_cells
    H = 2.0 / NM
    ncell = NM * NM
    MH, KH = fem.assemble_cells(NM, -1.0, H, np.ones((ncell, 4)),
                                np.broadcast_to(np.eye(2), (ncell, 4, 2, 2)).copy())
    L = np.asarray(MH.sum(axis=1)).ravel()
    _, y1, y2, _, _, _ = fem._quad_points(NM, -1.0, H)
    ones = np.ones((ncell, 4))
    Fu = _cell_load(NM, -1.0, H, ones, data.fu(y1, y2))
    Fw = _cell_load(NM, -1.0, H, ones, data.fw(y1, y2))
    x1, x2 = macro_nodes(NM)
    dmask = np.zeros((NM + 1) ** 2, dtype=bool)
    for s, (na, nb, s1, s2, _) in enumerate(fem.boundary_edges(NM)):
        nrm = SIDE_NORMALS[s]
        Fw = Fw + _side_load(NM, s, data.gw(s1, s2, nrm))
        if prm.dirichlet[s]:
            dmask[na] = True
            dmask[nb] = True
        else:
            Fu = Fu + _side_load(NM, s, data.gu(s1, s2, nrm))
    uD = np.where(dmask, data.uD(x1, x2), 0.0)
    return KH.tocsr(), L, Fu, Fw, dmask, uD


def solve(prm: StationaryParams, levels, jacobians, data: Optional[StationaryData] = None):
    """Solve the discrete system.  levels[k] = N_k; jacobians[k] = (Fc, Fb),
    D zeta of instance k at the points of fem.quadrature_points(N_k).
    Returns dict(u, w, v (list of arrays), lenI, lenO)."""
    data = data or constant_data()
    NM = prm.macro_cells
    nM = (NM + 1) ** 2
    assert len(levels) == nM and len(jacobians) == nM
    KH, L, Fu, Fw, dmask, uD = macro_system(prm, data)
    x1, x2 = macro_nodes(NM)
    k1, k2, k3, k4 = prm.kappa1, prm.kappa2, prm.kappa3, prm.kappa4

    # blocks of the system, unknown order (u, w, v_0, ..., v_{nM-1})
    Suu = sp.lil_matrix(KH)
    Sww = sp.lil_matrix(prm.Dw * KH)
    Suv, Swv, Svu, Svw, Svv = [], [], [], [], []
    ru, rw, rv = Fu.copy(), Fw.copy(), []
    lenI, lenO = np.zeros(nM), np.zeros(nM)
    for k in range(nM):
        N = int(levels[k])
        Fc, Fb = jacobians[k]
        S, bI, bO, lI, lO, Fv, GI, GO = micro_system(prm, N, Fc, Fb, x1[k], x2[k], data)
        lenI[k], lenO[k] = lI, lO
        Suu[k, k] += L[k] * k1 * lI
        Sww[k, k] += L[k] * k3 * lO
        ru[k] -= L[k] * GI
        rw[k] -= L[k] * GO
        n = (N + 1) ** 2
        eu = sp.csr_matrix(([1.0], ([k], [0])), shape=(nM, 1))
        Suv.append(sp.csr_matrix(eu @ sp.csr_matrix(-L[k] * k2 * bI[None, :])))
        Swv.append(sp.csr_matrix(eu @ sp.csr_matrix(-L[k] * k4 * bO[None, :])))
        Svu.append(sp.csr_matrix((-k1 * bI, (np.arange(n), np.full(n, k))), shape=(n, nM)))
        Svw.append(sp.csr_matrix((-k3 * bO, (np.arange(n), np.full(n, k))), shape=(n, nM)))
        Svv.append(S)
        rv.append(Fv)
    Suu = Suu.tocsr()
    # Dirichlet rows of u: u_k = uD_k
    keep = sp.diags((~dmask).astype(float))
    Suu = (keep @ Suu + sp.diags(dmask.astype(float))).tocsr()
    ru = np.where(dmask, uD, ru)
    Suv = [keep @ B for B in Suv]
    blocks = [[Suu, None, sp.hstack(Suv)],
              [None, Sww.tocsr(), sp.hstack(Swv)],
              [sp.vstack(Svu), sp.vstack(Svw), sp.block_diag(Svv)]]
    Amat = sp.bmat(blocks, format="csc")
    rhs = np.concatenate([ru, rw] + rv)
    sol = spla.spsolve(Amat, rhs)
    u, w = sol[:nM], sol[nM:2 * nM]
    v, pos = [], 2 * nM
    for k in range(nM):
        n = (int(levels[k]) + 1) ** 2
        v.append(sol[pos:pos + n])
        pos += n
    return {"u": u, "w": w, "v": v, "lenI": lenI, "lenO": lenO}
