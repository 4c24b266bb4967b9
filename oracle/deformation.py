"""Pullback geometry of one micro instance (oracle; test infrastructure).

The micro domain Y_x is the image of the reference cell Z = [-1,1]^2 under a
map zeta(x, .) (Section 2, definition of Lambda and zeta).  Integrals over
Y_x are moved to Z with K = (D zeta)^{-1} and J = det D zeta (Section 3.1,
equations grad_map and det_map and the change-of-variables identities):

    int_{Y_x} grad v . grad psi dy = int_Z grad^ v^T (K K^T J) grad^ psi^ dy^
    int_{Y_x} v psi dy             = int_Z v^ psi^ J dy^
    int_{dY_x} v psi dsigma        = int_{dZ} |cof(F) nu| v^ psi^ dsigma^

with cof F = (det F) F^{-T}.  In 2D, |cof(F) nu| = |F tau| for the unit
tangent tau of the reference edge (Nanson's formula); the tests check this
identity independently.

Deformation family of the workloads: zeta(y) = R_theta (y + a phi(y)) with
phi(y) = (sin(pi y1) y2, sin(pi y2) y1) / 4, so F = R_theta (I + a G) with
G = D phi.  Everything here is evaluated literally, with the rotation kept.
"""
from __future__ import annotations

import numpy as np


def phi(y1, y2):
    """Displacement profile phi(y) (the a-independent part of the map)."""
    return 0.25 * np.sin(np.pi * y1) * y2, 0.25 * np.sin(np.pi * y2) * y1


def chi(y1, y2, a, theta=0.0):
    """The map zeta(y) = R_theta (y + a phi(y))."""
    p1, p2 = phi(y1, y2)
    z1 = y1 + a * p1
    z2 = y2 + a * p2
    c, s = np.cos(theta), np.sin(theta)
    return c * z1 - s * z2, s * z1 + c * z2


def grad_phi(y1, y2):
    """G = D phi as an array (..., 2, 2), G[r, c] = d phi_r / d y_c."""
    y1 = np.asarray(y1, dtype=np.float64)
    y2 = np.asarray(y2, dtype=np.float64)
    G = np.empty(np.broadcast(y1, y2).shape + (2, 2))
    G[..., 0, 0] = 0.25 * np.pi * np.cos(np.pi * y1) * y2
    G[..., 0, 1] = 0.25 * np.sin(np.pi * y1)
    G[..., 1, 0] = 0.25 * np.sin(np.pi * y2)
    G[..., 1, 1] = 0.25 * np.pi * np.cos(np.pi * y2) * y1
    return G


def rotation(theta):
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[c, -s], [s, c]])


def jacobian(y1, y2, a, theta=0.0):
    """F = D zeta = R_theta (I + a G), shape (..., 2, 2)."""
    G = grad_phi(y1, y2)
    M = np.eye(2) + a * G
    return np.einsum("ij,...jk->...ik", rotation(theta), M)


def pullback(y1, y2, a, theta=0.0):
    """J = det F and the stiffness weight C = K K^T J with K = F^{-1}.

    Returns (J, C) with C of shape (..., 2, 2)."""
    F = jacobian(y1, y2, a, theta)
    J = np.linalg.det(F)
    K = np.linalg.inv(F)
    C = np.einsum("...ij,...kj->...ik", K, K) * J[..., None, None]
    return J, C


def boundary_weight(y1, y2, tau, a, theta=0.0):
    """Surface measure |cof(F) nu| = |F tau| on a reference edge with unit
    tangent tau (a pair of floats)."""
    F = jacobian(y1, y2, a, theta)
    Ft = F @ np.asarray(tau, dtype=np.float64)
    return np.sqrt(np.sum(Ft * Ft, axis=-1))


def pullback_from_jacobian(F):
    """(J, C = K K^T J) from given Jacobians F = D zeta, shape (..., 2, 2):
    the same change of variables for a map known only through its Jacobian
    at the quadrature points."""
    F = np.asarray(F, dtype=np.float64)
    J = np.linalg.det(F)
    K = np.linalg.inv(F)
    C = np.einsum("...ij,...kj->...ik", K, K) * J[..., None, None]
    return J, C


def boundary_weight_from_jacobian(F, tau):
    """|F tau| for given Jacobians F (..., 2, 2) and a reference unit tangent."""
    Ft = np.asarray(F, dtype=np.float64) @ np.asarray(tau, dtype=np.float64)
    return np.sqrt(np.sum(Ft * Ft, axis=-1))


# ---------------------------------------------------------------------------
# a-derivatives (used by the discrete adjoint).  With M = I + a G and
# F = R M:  dF/da = R G;  dJ/da = J tr(F^{-1} dF/da);
# dC/da = [adj(dF) adj(F)^T + adj(F) adj(dF)^T] / J - C (dJ/da) / J, where
# adj is the 2x2 adjugate (linear in its argument);  d|F tau|/da =
# (F tau).(dF tau) / |F tau|.
# ---------------------------------------------------------------------------

def _adj(A):
    B = np.empty_like(A)
    B[..., 0, 0] = A[..., 1, 1]
    B[..., 0, 1] = -A[..., 0, 1]
    B[..., 1, 0] = -A[..., 1, 0]
    B[..., 1, 1] = A[..., 0, 0]
    return B


def pullback_da(y1, y2, a, theta=0.0):
    """(dJ/da, dC/da) at the given points."""
    G = grad_phi(y1, y2)
    R = rotation(theta)
    F = jacobian(y1, y2, a, theta)
    dF = np.einsum("ij,...jk->...ik", R, G)
    J = np.linalg.det(F)
    Finv = np.linalg.inv(F)
    dJ = J * np.einsum("...ij,...ji->...", Finv, dF)
    aF, adF = _adj(F), _adj(dF)
    C = np.einsum("...ij,...kj->...ik", aF, aF) / J[..., None, None]
    dC = (np.einsum("...ij,...kj->...ik", adF, aF)
          + np.einsum("...ij,...kj->...ik", aF, adF)) / J[..., None, None] \
        - C * (dJ / J)[..., None, None]
    return dJ, dC


def boundary_weight_da(y1, y2, tau, a, theta=0.0):
    G = grad_phi(y1, y2)
    R = rotation(theta)
    F = jacobian(y1, y2, a, theta)
    t = np.asarray(tau, dtype=np.float64)
    Ft = F @ t
    dFt = np.einsum("ij,...jk->...ik", R, G) @ t
    w = np.sqrt(np.sum(Ft * Ft, axis=-1))
    return np.sum(Ft * dFt, axis=-1) / w
