"""Seeded synthetic inputs for the two-scale micro batch.

This module holds only input generation: mesh sizes, deformation amplitudes,
rotation angles, per-instance refinement levels, initial data and finite
difference directions.  It contains none of the method's arithmetic, so both
the FP64 CPU oracle and the GPU path may import it.

Every workload is synthetic.  The paper (Section 4, Tables 1-3) measures on
manufactured problems and on two hand-picked deformation maps; it ships no
dataset.  The configurations below are the five batch workloads the GPU path
is measured on, each described by what it is and its sizes.

Random streams: ``SeedSequence(seed).spawn(4)`` gives independent streams for
(amplitudes, levels, rotation angles, FD directions), consumed with
``numpy.random.default_rng``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

STREAM_AMPLITUDE, STREAM_LEVEL, STREAM_THETA, STREAM_FD = range(4)


def _streams(seed: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(4)]


@dataclasses.dataclass(frozen=True)
class Workload:
    """One batch workload.  Instance i is macro node i, numbered
    lexicographically with x1 fastest: i = k2*(N_M+1) + k1."""

    name: str
    macro_cells: int           # N_M: macro Q1 cells per side on [0,1]^2
    micro_levels: tuple        # allowed micro cells per side
    level_probs: tuple         # probability of each level (uniform batch: (1.0,))
    amplitude: str             # "cfg1_analytic" or "uniform"
    amplitude_max: float       # bound of the uniform amplitude law
    smooth: bool               # one Jacobi sweep over the amplitudes
    rotate: bool               # random rotation angle in [0, pi/8]
    dt: float
    steps: int
    precision: str             # "fp64" or "fp32_refine"
    rtol: float                # relative residual target of every micro solve
    checkpoint_every: int = 0  # adjoint checkpoint spacing (0: no adjoint)
    grad_rtol: float = 0.0     # tolerance of the gradient's solves (0: rtol)
    fd_dirs: int = 0
    fd_h: float = 0.0
    # physical parameters of the two-scale system
    D: float = 1.0             # macro diffusion
    d: float = 0.5             # micro diffusion
    kappa: float = 1.0         # Robin transfer rate
    p: float = 1.0             # partition coefficient in kappa*(p*u - v)
    sigma: int = -1            # sign of the mean-flux source in the macro equation

    @property
    def n_inst(self) -> int:
        return (self.macro_cells + 1) ** 2


WORKLOADS = {
    # 81 instances of a 16x16 reference mesh, analytic amplitude, 10 steps.
    "small_fp64": Workload("small_fp64", 8, (16,), (1.0,), "cfg1_analytic", 0.2,
                           False, False, 0.01, 10, "fp64", 1e-12),
    # 4225 instances of 32x32, smoothed random amplitudes, 100 steps.
    "batched_fp64": Workload("batched_fp64", 64, (32,), (1.0,), "uniform", 0.3,
                             True, False, 0.005, 100, "fp64", 1e-12),
    # 4225 instances with 16x16 / 32x32 / 64x64 meshes mixed 0.5/0.3/0.2.
    "uneven_mixed": Workload("uneven_mixed", 64, (16, 32, 64), (0.5, 0.3, 0.2),
                             "uniform", 0.3, True, False, 0.005, 100,
                             "fp32_refine", 1e-10),
    # 1089 instances of 32x32, gradient of int u(T)^2 over 50 steps.
    "adjoint_fp64": Workload("adjoint_fp64", 32, (32,), (1.0,), "uniform", 0.2,
                             False, False, 0.01, 50, "fp64", 1e-12,
                             checkpoint_every=10, fd_dirs=16, fd_h=1e-6),
    # 16641 instances of 64x64 (70.3M micro DoFs), rotated, 200 steps + adjoint.
    # Solved to 1e-9: the outputs then agree with the FP64 oracle to 1e-8
    # after 200 steps (at 1e-8 the final micro state misses it, 4.6e-8:
    # the per-step errors accumulate); the gradient's solves to 1e-11.
    "large_mixed": Workload("large_mixed", 128, (64,), (1.0,), "uniform", 0.3,
                            False, True, 0.0025, 200, "fp32_refine", 1e-9,
                            checkpoint_every=20, grad_rtol=1e-11),
}


def macro_nodes(macro_cells: int) -> np.ndarray:
    """Macro node coordinates, shape (n_inst, 2), x1 fastest."""
    t = np.arange(macro_cells + 1, dtype=np.float64) / macro_cells
    x1, x2 = np.meshgrid(t, t, indexing="xy")
    return np.stack([x1.ravel(), x2.ravel()], axis=1)


def macro_boundary_mask(macro_cells: int) -> np.ndarray:
    k = np.arange(macro_cells + 1)
    k1, k2 = np.meshgrid(k, k, indexing="xy")
    return ((k1 == 0) | (k2 == 0) | (k1 == macro_cells) | (k2 == macro_cells)).ravel()


def _jacobi_sweep(a: np.ndarray, n_side: int) -> np.ndarray:
    """One Jacobi sweep of the 5-point Laplacian with a natural boundary:
    every value becomes the mean of its existing grid neighbours."""
    g = a.reshape(n_side, n_side)
    s = np.zeros_like(g)
    c = np.zeros_like(g)
    s[1:, :] += g[:-1, :]; c[1:, :] += 1
    s[:-1, :] += g[1:, :]; c[:-1, :] += 1
    s[:, 1:] += g[:, :-1]; c[:, 1:] += 1
    s[:, :-1] += g[:, 1:]; c[:, :-1] += 1
    return (s / c).ravel()


def amplitudes(w: Workload, seed: int = 0) -> np.ndarray:
    """Per-instance deformation amplitude a_i (float64[n_inst])."""
    x = macro_nodes(w.macro_cells)
    if w.amplitude == "cfg1_analytic":
        return w.amplitude_max * np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])
    rng = _streams(seed)[STREAM_AMPLITUDE]
    a = rng.uniform(-w.amplitude_max, w.amplitude_max, size=w.n_inst)
    if w.smooth:
        a = _jacobi_sweep(a, w.macro_cells + 1)
    return a


def thetas(w: Workload, seed: int = 0) -> Optional[np.ndarray]:
    """Per-instance rotation angle (float64[n_inst]) or None."""
    if not w.rotate:
        return None
    return _streams(seed)[STREAM_THETA].uniform(0.0, math.pi / 8, size=w.n_inst)


def levels(w: Workload, seed: int = 0) -> np.ndarray:
    """Micro cells per side of every instance (int32[n_inst])."""
    if len(w.micro_levels) == 1:
        return np.full(w.n_inst, w.micro_levels[0], dtype=np.int32)
    rng = _streams(seed)[STREAM_LEVEL]
    return rng.choice(np.asarray(w.micro_levels, dtype=np.int32), size=w.n_inst,
                      p=np.asarray(w.level_probs)).astype(np.int32)


def fd_directions(n_inst: int, count: int, seed: int = 0) -> np.ndarray:
    """Unit directions for finite-difference checks, shape (count, n_inst)."""
    rng = _streams(seed)[STREAM_FD]
    e = rng.standard_normal((count, n_inst))
    return e / np.linalg.norm(e, axis=1, keepdims=True)


def initial_macro(macro_cells: int) -> np.ndarray:
    """u^0 = sin(pi x1) sin(pi x2) at macro nodes, exactly 0 on the boundary."""
    x = macro_nodes(macro_cells)
    u = np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])
    u[macro_boundary_mask(macro_cells)] = 0.0
    return u


def offsets(levels_: np.ndarray) -> np.ndarray:
    """Start of every instance in the ragged micro vector (int64[n_inst+1])."""
    n = (np.asarray(levels_, dtype=np.int64) + 1) ** 2
    return np.concatenate([[0], np.cumsum(n)]).astype(np.int64)


def random_state(levels_: np.ndarray, macro_cells: int, seed: int = 0, scale: float = 1.0):
    """A seeded smooth-plus-noise (u, v) pair used as a mid-run state in
    single-step parity cases.  u is zero on the macro boundary."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 7919]))
    u = initial_macro(macro_cells) * (1.0 + 0.1 * rng.standard_normal((macro_cells + 1) ** 2))
    u[macro_boundary_mask(macro_cells)] = 0.0
    off = offsets(levels_)
    v = scale * rng.uniform(0.0, 1.0, size=int(off[-1]))
    return u, v


def make(name: str, seed: int = 0):
    """(workload, a, theta, levels) for a named workload."""
    w = WORKLOADS[name]
    return w, amplitudes(w, seed), thetas(w, seed), levels(w, seed)


# ---------------------------------------------------------------------------
# Maps given by their Jacobians (general-geometry input).  A user with any
# map zeta supplies D zeta at the points the interface lists: per instance,
# the 2x2 Gauss points of every reference cell (cells c2*N + c1, points
# g2*2 + g1) and the 2 Gauss points of every boundary edge (sides bottom,
# top, left, right; edges in increasing coordinate).  The generator below
# evaluates the derivative of a seeded test map there; it is input data.
# ---------------------------------------------------------------------------
_GAUSS01 = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))


def table_points(N: int):
    """Reference coordinates of the Jacobian table of one instance with N
    cells per side: cells (N*N, 4) and boundary (4, N, 2) arrays of (y1, y2)."""
    h = 2.0 / N
    g = np.array(_GAUSS01)
    c = np.arange(N)
    # cells: c2 slow, c1 fast; points: g2 slow, g1 fast
    y1 = (-1.0 + (c[None, :, None, None] + g[None, None, None, :]) * h) * np.ones((N, 1, 2, 1))
    y2 = (-1.0 + (c[:, None, None, None] + g[None, None, :, None]) * h) * np.ones((1, N, 1, 2))
    cell = (y1.reshape(N * N, 4), y2.reshape(N * N, 4))
    s = -1.0 + (c[:, None] + g[None, :]) * h              # (edge, point) along a side
    one = np.ones_like(s)
    b1 = np.stack([s, s, -one, one])
    b2 = np.stack([-one, one, s, s])
    return cell, (b1, b2)


def polynomial_map_jacobian(y1, y2, c, d, theta):
    """D zeta of the test map zeta(y) = R_theta (y1 + c y1 y2, y2 + d y1^2 y2),
    a map outside the sinusoidal family (the cell changes shape and size).
    det D zeta > 0 for |c|, |d| <= 0.25 on [-1,1]^2."""
    y1 = np.asarray(y1, dtype=np.float64)
    y2 = np.asarray(y2, dtype=np.float64)
    M = np.empty(y1.shape + (2, 2))
    M[..., 0, 0] = 1.0 + c * y2
    M[..., 0, 1] = c * y1
    M[..., 1, 0] = 2.0 * d * y1 * y2
    M[..., 1, 1] = 1.0 + d * y1 * y1
    R = np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]])
    return np.einsum("ij,...jk->...ik", R, M)


def scaling_map_jacobian(y1, y2, s):
    """D zeta of zeta(y) = s y: cells scaled by s, so the micro responses
    (and the coefficients of the macro system) vary with s."""
    y1 = np.asarray(y1, dtype=np.float64)
    M = np.zeros(y1.shape + (2, 2))
    M[..., 0, 0] = s
    M[..., 1, 1] = s
    return M


def sinusoidal_map_jacobian(y1, y2, a, theta):
    """D zeta of the workloads' family zeta(y) = R_theta (y + a phi(y)),
    phi = (sin(pi y1) y2, sin(pi y2) y1)/4 (for checking the table layout)."""
    y1 = np.asarray(y1, dtype=np.float64)
    y2 = np.asarray(y2, dtype=np.float64)
    M = np.empty(y1.shape + (2, 2))
    M[..., 0, 0] = 1.0 + a * 0.25 * math.pi * np.cos(math.pi * y1) * y2
    M[..., 0, 1] = a * 0.25 * np.sin(math.pi * y1)
    M[..., 1, 0] = a * 0.25 * np.sin(math.pi * y2)
    M[..., 1, 1] = 1.0 + a * 0.25 * math.pi * np.cos(math.pi * y2) * y1
    R = np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]])
    return np.einsum("ij,...jk->...ik", R, M)


def jacobian_tables(levels_: np.ndarray, jac_fn, params):
    """Tables of D zeta for every instance: jac_fn(y1, y2, *params[i]).
    Returns (per-instance list of (Fc (N*N,4,2,2), Fb (4,N,2,2,2)),
    flat cell table, flat boundary table) in the interface's layout."""
    per, flat_c, flat_b = [], [], []
    for i, N in enumerate(np.asarray(levels_).tolist()):
        (c1, c2), (b1, b2) = table_points(int(N))
        Fc = jac_fn(c1, c2, *params[i])
        Fb = jac_fn(b1, b2, *params[i])
        per.append((Fc, Fb))
        flat_c.append(Fc.ravel())
        flat_b.append(Fb.ravel())
    return per, np.concatenate(flat_c), np.concatenate(flat_b)


def polynomial_map_params(n_inst: int, seed: int = 0, strength: float = 0.25):
    """Seeded (c, d, theta) per instance for polynomial_map_jacobian."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 777]))
    c = rng.uniform(-strength, strength, n_inst)
    d = rng.uniform(-strength, strength, n_inst)
    th = rng.uniform(0.0, 2.0 * math.pi, n_inst)
    return list(zip(c.tolist(), d.tolist(), th.tolist()))


# ---------------------------------------------------------------------------
# The stationary three-field experiments (Section 4.4): macro domain
# [-1,1]^2, one micro system per macro node, the Table 3 parameters and two
# maps, zeta_0(x, y) = y (Case A) and the heterogeneous zeta_1 (Case B),
#   zeta_1(x, y) = ((2 x1 + 3) y1 / 4 - x2 y2 / 5,  (2 - x2) y2 / 4),
# both affine in y.  The paper's runs have 81 macro and 4225 micro DoFs.
# ---------------------------------------------------------------------------

def stationary_macro_nodes(macro_cells: int) -> np.ndarray:
    """Node coordinates of the macro mesh of [-1,1]^2, shape (n_inst, 2), x1 fastest."""
    t = -1.0 + 2.0 * np.arange(macro_cells + 1, dtype=np.float64) / macro_cells
    x1, x2 = np.meshgrid(t, t, indexing="xy")
    return np.stack([x1.ravel(), x2.ravel()], axis=1)


def stationary_case_jacobian(case: str):
    """D_y zeta of the Case A or Case B map as jac_fn(y1, y2, x1, x2) for
    jacobian_tables (params: the macro node of each instance)."""
    if case not in ("A", "B"):
        raise ValueError(case)

    def fn(y1, y2, x1, x2):
        F = np.eye(2) if case == "A" else np.array([[(2.0 * x1 + 3.0) / 4.0, -x2 / 5.0], [0.0, (2.0 - x2) / 4.0]])
        return np.broadcast_to(F, np.shape(y1) + (2, 2)).copy()
    return fn


def stationary_case(case: str, macro_cells: int = 8, micro_cells: int = 64):
    """(levels, per-instance tables, flat cell table, flat boundary table) of
    Case A or B at the given sizes (the paper's: 8 and 64)."""
    n = (macro_cells + 1) ** 2
    lv = np.full(n, micro_cells, dtype=np.int32)
    per, Fc, Fb = jacobian_tables(lv, stationary_case_jacobian(case),
                                  [tuple(x) for x in stationary_macro_nodes(macro_cells)])
    return lv, per, Fc, Fb
