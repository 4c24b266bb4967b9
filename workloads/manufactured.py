"""Manufactured solutions of the stationary three-field system: the method
of Section 4.1 (prescribe u, v, w and the map, derive the data), the data
evaluated at the quadrature points of the library's layouts, and the error
norms of Section 4.2.  Input generation and analysis only: no part of
either solver.

The data follow the manufactured form (eq. manu_pde_formulation): with exact
fields u(x), w(x), v(x, y) and the outward unit normal n of Y_x,
    f^v = -Dv Lap_y v,
    g^v = Dv grad_y v . n - (k1 u - k2 v)   on G^I,
          Dv grad_y v . n - (k3 w - k4 v)   on G^O,
          Dv grad_y v . n                   on G^N,
    f^u = -Lap u + int_{G^I} Dv grad_y v . n dsigma_y,
    f^w = -Dw Lap w + int_{G^O} Dv grad_y v . n dsigma_y,
    u_D = u,  g^u = grad u . n_Omega,  g^w = Dw grad w . n_Omega,
re-derived here with SymPy (the printed data, eq. manu_data, is garbled).
The normal of the image of a side of Z is cof(F) nu / |cof(F) nu|.
"""
from __future__ import annotations

import dataclasses
from typing import Callable

import numpy as np
import sympy as sy

from . import jacobian_tables, stationary_macro_nodes, table_points

X1, X2, Y1, Y2, Z1, Z2 = sy.symbols("x1 x2 y1 y2 z1 z2")
PART_N, PART_I, PART_O = 0, 1, 2
SIDE_NORMALS = ((0.0, -1.0), (0.0, 1.0), (-1.0, 0.0), (1.0, 0.0))   # bottom, top, left, right
_GL_S, _GL_W = np.polynomial.legendre.leggauss(12)

# the paper's manufactured solution and map (eq. manu_system)
ZETA_MANU = (sy.Rational(2, 5) * ((X1 + sy.Rational(13, 10)) + (sy.Rational(7, 5) * Z1 - sy.Rational(27, 50) * Z2)),
             sy.Rational(3, 10) * ((X2 + sy.Rational(6, 5)) + (-sy.Rational(2, 5) * Z1 + sy.Rational(4, 5) * Z2)))
U_MANU = X2 * sy.sin(X1)
V_MANU = X1 + X2 + Y1 * Y2 * (1 - Y2)
W_MANU = X1 * sy.cos(X2)


@dataclasses.dataclass
class Data:
    """Sources and boundary data as callables: x1, x2 macro coordinates,
    z1, z2 reference coordinates in Z (see the module docstring)."""
    fu: Callable
    fw: Callable
    fv: Callable
    gv: Callable      # gv(part, x1, x2, z1, z2)
    uD: Callable
    gu: Callable      # gu(x1, x2, n)
    gw: Callable


def _bc(f, like):
    return np.broadcast_to(np.asarray(f, dtype=float), np.shape(like))


def side_of(z1, z2):
    """The side of Z on which the points lie (bottom, top, left, right)."""
    z1, z2 = np.asarray(z1), np.asarray(z2)
    if np.all(z2 == -1.0):
        return 0
    if np.all(z2 == 1.0):
        return 1
    if np.all(z1 == -1.0):
        return 2
    if np.all(z1 == 1.0):
        return 3
    raise ValueError("points not on one side of Z")


def map_jacobian(zeta):
    """D_z zeta as a SymPy matrix."""
    return sy.Matrix([[sy.diff(zeta[r], zc) for zc in (Z1, Z2)] for r in range(2)])


def manufactured(prm, u, v, w, zeta) -> Data:
    """Data of the exact fields u(x), w(x), v(x, y) on the map y = zeta(x, z)
    (SymPy expressions in X1, X2, Y1, Y2, Z1, Z2).  prm gives Dv, Dw,
    kappa1..kappa4 and parts (the part of each side of Z)."""
    Dv, Dw = prm.Dv, prm.Dw
    F = map_jacobian(zeta)
    sub = {Y1: zeta[0], Y2: zeta[1]}
    gv_y = [sy.diff(v, s) for s in (Y1, Y2)]
    fv = (-Dv * (sy.diff(v, Y1, 2) + sy.diff(v, Y2, 2))).subs(sub)
    cof = F.det() * F.inv().T
    lam = lambda e: sy.lambdify((X1, X2, Z1, Z2), e, "numpy")
    fv_f = lam(fv)
    coupling = {PART_N: 0, PART_I: prm.kappa1 * u - prm.kappa2 * v, PART_O: prm.kappa3 * w - prm.kappa4 * v}
    g_f, flux_f = {}, {}
    for s, nu in enumerate(SIDE_NORMALS):
        cn = cof * sy.Matrix(nu)
        nrm = cn / sy.sqrt(cn[0] ** 2 + cn[1] ** 2)
        fl = Dv * (gv_y[0] * nrm[0] + gv_y[1] * nrm[1])
        g_f[s] = lam((fl - coupling[prm.parts[s]]).subs(sub))
        flux_f[s] = lam(fl.subs(sub))
    Fn = sy.lambdify((X1, X2, Z1, Z2), F, "numpy")

    def part_integral(part, x1, x2):
        tot = 0.0
        for s in range(4):
            if prm.parts[s] != part:
                continue
            if s < 2:
                z1, z2, tau = _GL_S, np.full_like(_GL_S, -1.0 if s == 0 else 1.0), (1.0, 0.0)
            else:
                z1, z2, tau = np.full_like(_GL_S, -1.0 if s == 2 else 1.0), _GL_S, (0.0, 1.0)
            Fv = np.stack([_bc(Fn(x1, x2, a, b), np.zeros((2, 2))) for a, b in zip(z1, z2)])
            om = np.linalg.norm(Fv @ np.asarray(tau), axis=-1)
            tot += np.sum(_GL_W * om * _bc(flux_f[s](x1, x2, z1, z2), z1))
        return tot

    lap = lambda e: sy.diff(e, X1, 2) + sy.diff(e, X2, 2)
    fu_base = sy.lambdify((X1, X2), -lap(u), "numpy")
    fw_base = sy.lambdify((X1, X2), -Dw * lap(w), "numpy")
    integ = {PART_I: np.vectorize(lambda a, b: part_integral(PART_I, a, b)),
             PART_O: np.vectorize(lambda a, b: part_integral(PART_O, a, b))}

    def fu(x1, x2):
        x1, x2 = np.asarray(x1, float), np.asarray(x2, float)
        return _bc(fu_base(x1, x2), x1) + integ[PART_I](x1, x2)

    def fw(x1, x2):
        x1, x2 = np.asarray(x1, float), np.asarray(x2, float)
        return _bc(fw_base(x1, x2), x1) + integ[PART_O](x1, x2)

    du = [sy.lambdify((X1, X2), sy.diff(u, s), "numpy") for s in (X1, X2)]
    dw = [sy.lambdify((X1, X2), Dw * sy.diff(w, s), "numpy") for s in (X1, X2)]
    uf = sy.lambdify((X1, X2), u, "numpy")
    return Data(
        fu=fu, fw=fw,
        fv=lambda x1, x2, z1, z2: _bc(fv_f(x1, x2, z1, z2), z1),
        gv=lambda part, x1, x2, z1, z2: _bc(g_f[side_of(z1, z2)](x1, x2, z1, z2), z1),
        uD=lambda x1, x2: _bc(uf(x1, x2), x1),
        gu=lambda x1, x2, n: _bc(du[0](x1, x2), x1) * n[0] + _bc(du[1](x1, x2), x1) * n[1],
        gw=lambda x1, x2, n: _bc(dw[0](x1, x2), x1) * n[0] + _bc(dw[1](x1, x2), x1) * n[1])


def constant_map_jacobian(zeta):
    """D_z zeta as a 2 x 2 float array when it is constant (in x and z),
    else None."""
    F = map_jacobian(zeta)
    if any(e.free_symbols for e in F):
        return None
    return np.array(F.evalf(), dtype=float)


def map_tables(NM, levels, zeta):
    """Jacobian tables of the map zeta(x, z) at every instance (jacobian_tables layout)."""
    Fn = sy.lambdify((X1, X2, Z1, Z2), map_jacobian(zeta), "numpy")

    def fn(z1, z2, x1, x2):
        out = np.empty(np.shape(z1) + (2, 2))
        for r in range(2):
            for c in range(2):
                out[..., r, c] = _bc(Fn(x1, x2, z1, z2)[r][c], z1)
        return out
    return jacobian_tables(np.asarray(levels), fn, [tuple(x) for x in stationary_macro_nodes(NM)])


def _micro_data(data: Data, xs, parts, ks, levels):
    """fv at the cell points and gv at the boundary points of instances ks."""
    fv, gv = [], []
    for k, N in zip(ks, levels):
        (c1, c2), (b1, b2) = table_points(int(N))
        x1, x2 = float(xs[k, 0]), float(xs[k, 1])
        fv.append(data.fv(x1, x2, c1, c2).ravel())
        gv.append(np.stack([data.gv(parts[s], x1, x2, b1[s], b2[s]) for s in range(4)]).ravel())
    return np.concatenate(fv), np.concatenate(gv)


def _macro_data(data: Data, NM, xs):
    (c1, c2), (b1, b2) = table_points(int(NM))     # the macro mesh is [-1,1]^2 as well
    return {"fu_cell": data.fu(c1, c2).ravel(), "fw_cell": data.fw(c1, c2).ravel(),
            "gu_bnd": np.stack([data.gu(b1[s], b2[s], SIDE_NORMALS[s]) for s in range(4)]).ravel(),
            "gw_bnd": np.stack([data.gw(b1[s], b2[s], SIDE_NORMALS[s]) for s in range(4)]).ravel(),
            "uD": data.uD(xs[:, 0], xs[:, 1]).ravel()}


def data_at_points(data: Data, NM, levels, parts):
    """The data at the quadrature points in the layouts of
    tsm_stationary_set_data: fv_cell, gv_bnd, fu_cell, fw_cell, gu_bnd,
    gw_bnd, uD (flat float64 arrays)."""
    xs = stationary_macro_nodes(NM)
    lv = np.asarray(levels).tolist()
    fv, gv = _micro_data(data, xs, parts, range(len(lv)), lv)
    out = {"fv_cell": fv, "gv_bnd": gv, **_macro_data(data, NM, xs)}
    return {k: np.array(v, dtype=np.float64) for k, v in out.items()}     # writable copies


# ---------------------------------------------------------------------------
# the same in worker processes (the finest rows of Section 4.2 have 16641
# instances of 16641 DoFs each): each worker derives the data once from the
# expressions and takes instances in chunks; results come back in order
# ---------------------------------------------------------------------------

_WORKER = {}


def _chunks(n, size):
    return [range(k, min(n, k + size)) for k in range(0, n, size)]


def _pool(workers, init, args):
    """Spawned worker processes (a worker that dies raises in the parent
    instead of leaving it waiting)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    return ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"), initializer=init, initargs=args)


def _init_data(phys, parts, exprs, NM):
    import types
    prm = types.SimpleNamespace(parts=tuple(parts), **phys)
    _WORKER["data"] = manufactured(prm, *exprs)
    _WORKER["xs"] = stationary_macro_nodes(NM)
    _WORKER["parts"] = tuple(parts)


def _data_job(job):
    ks, levels = job
    return _micro_data(_WORKER["data"], _WORKER["xs"], _WORKER["parts"], ks, levels)


def manufactured_data_at_points(phys, parts, NM, levels, workers=1, u=U_MANU, v=V_MANU, w=W_MANU, zeta=ZETA_MANU):
    """data_at_points of the manufactured data of (u, v, w, zeta) with the
    physical parameters phys (Dv, Dw, kappa1..kappa4), the micro part on
    `workers` processes."""
    import types
    prm = types.SimpleNamespace(parts=tuple(parts), **phys)
    data = manufactured(prm, u, v, w, zeta)
    xs = stationary_macro_nodes(NM)
    lv = np.asarray(levels).tolist()
    if workers <= 1:
        fv, gv = _micro_data(data, xs, parts, range(len(lv)), lv)
    else:
        jobs = [(list(r), [lv[k] for k in r]) for r in _chunks(len(lv), 64)]
        with _pool(workers, _init_data, (dict(phys), tuple(parts), (u, v, w, zeta), NM)) as pool:
            parts_out = list(pool.map(_data_job, jobs))
        fv = np.concatenate([a for a, _ in parts_out])
        gv = np.concatenate([b for _, b in parts_out])
        del parts_out
    out = {"fv_cell": fv, "gv_bnd": gv, **_macro_data(data, NM, xs)}
    return {k: np.ascontiguousarray(a, dtype=np.float64) for k, a in out.items()}


# ---------------------------------------------------------------------------
# error norms of Section 4.2 (3x3 Gauss per cell, vectorised over cells)
# ---------------------------------------------------------------------------

_G3 = 0.5 + 0.5 * np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
_W3 = np.array([5.0, 8.0, 5.0]) / 18.0


def q1_errors(N, nodal, exact, grad_exact, F=None):
    """(int e^2, int |grad e|^2) of the Q1 field `nodal` on the N x N mesh of
    [-1,1]^2 against exact(p1, p2) and grad_exact(p1, p2) -> (g1, g2);
    with a constant Jacobian F the integrals are over the image of the
    square (weight |det F|, gradients through F^-T)."""
    h = 2.0 / N
    U = np.asarray(nodal).reshape(N + 1, N + 1)
    c = np.arange(N)
    C1, C2 = np.meshgrid(c, c, indexing="xy")
    G1, G2 = np.meshgrid(_G3, _G3, indexing="xy")
    WW = np.outer(_W3, _W3)
    a = U[C2, C1][..., None, None]
    b = U[C2, C1 + 1][..., None, None]
    cc = U[C2 + 1, C1][..., None, None]
    d = U[C2 + 1, C1 + 1][..., None, None]
    val = a * (1 - G1) * (1 - G2) + b * G1 * (1 - G2) + cc * (1 - G1) * G2 + d * G1 * G2
    gz1 = ((b - a) * (1 - G2) + (d - cc) * G2) / h
    gz2 = ((cc - a) * (1 - G1) + (d - b) * G1) / h
    p1 = -1.0 + (C1[..., None, None] + G1) * h
    p2 = -1.0 + (C2[..., None, None] + G2) * h
    J = 1.0 if F is None else abs(np.linalg.det(F))
    Kt = np.eye(2) if F is None else np.linalg.inv(F).T
    g1 = Kt[0, 0] * gz1 + Kt[0, 1] * gz2
    g2 = Kt[1, 0] * gz1 + Kt[1, 1] * gz2
    e1, e2 = grad_exact(p1, p2)
    w = WW * h * h * J
    e0 = float(np.sum(w * (val - exact(p1, p2)) ** 2))
    eg = float(np.sum(w * ((g1 - e1) ** 2 + (g2 - e2) ** 2)))
    return e0, eg


def convergence_errors(NM, N, u_h, w_h, v_h, prm, u=U_MANU, v=V_MANU, w=W_MANU, zeta=ZETA_MANU, workers=1):
    """(e_uw, e_uw_grad, e_v, e_v_grad) of Section 4.2 for discrete u_h, w_h
    (nodal, (NM+1)^2) and v_h (one array per instance, all N x N) with a map
    whose D_z zeta is constant; the x-integral of the micro errors is taken
    at the nodes with the weights of the hats (int xi_k), over `workers`
    processes."""
    uf, wf = sy.lambdify((X1, X2), u, "numpy"), sy.lambdify((X1, X2), w, "numpy")
    gu = [sy.lambdify((X1, X2), sy.diff(u, s), "numpy") for s in (X1, X2)]
    gw = [sy.lambdify((X1, X2), sy.diff(w, s), "numpy") for s in (X1, X2)]
    a0, a1 = q1_errors(NM, u_h, lambda s, t: _bc(uf(s, t), s), lambda s, t: (_bc(gu[0](s, t), s), _bc(gu[1](s, t), s)))
    b0, b1 = q1_errors(NM, w_h, lambda s, t: _bc(wf(s, t), s), lambda s, t: (_bc(gw[0](s, t), s), _bc(gw[1](s, t), s)))
    if workers <= 1:
        _init_errors(NM, N, v, zeta)
        v0, v1 = _error_job((list(range(len(v_h))), v_h))
    else:
        jobs = [(list(r), [v_h[k] for k in r]) for r in _chunks(len(v_h), 64)]
        with _pool(workers, _init_errors, (NM, N, v, zeta)) as pool:
            sums = list(pool.map(_error_job, jobs))
        v0 = sum(a for a, _ in sums)
        v1 = sum(b for _, b in sums)
    return np.sqrt(a0) + np.sqrt(b0), np.sqrt(a1) + np.sqrt(b1), np.sqrt(v0), np.sqrt(v1)


def _init_errors(NM, N, v, zeta):
    k1 = np.arange(NM + 1)
    cells = ((k1 > 0).astype(int) + (k1 < NM))
    _WORKER.update(
        N=N, F=np.array(map_jacobian(zeta).evalf(), dtype=float),
        vy=sy.lambdify((X1, X2, Y1, Y2), v, "numpy"),
        gvy=[sy.lambdify((X1, X2, Y1, Y2), sy.diff(v, s), "numpy") for s in (Y1, Y2)],
        zm=sy.lambdify((X1, X2, Z1, Z2), zeta, "numpy"), xs=stationary_macro_nodes(NM),
        L=(0.25 * (2.0 / NM) ** 2) * np.outer(cells, cells).ravel())


def _error_job(job):
    """(sum_k L_k int e_k^2, sum_k L_k int |grad e_k|^2) over instances ks."""
    ks, v_h = job
    c = _WORKER
    vy, gvy, zm = c["vy"], c["gvy"], c["zm"]
    v0 = v1 = 0.0
    for k, vk in zip(ks, v_h):
        x1, x2 = float(c["xs"][k, 0]), float(c["xs"][k, 1])
        ex = lambda s, t: _bc(vy(x1, x2, *zm(x1, x2, s, t)), s)
        gex = lambda s, t: tuple(_bc(g(x1, x2, *zm(x1, x2, s, t)), s) for g in gvy)
        c0, c1 = q1_errors(c["N"], vk, ex, gex, F=c["F"])
        v0 += c["L"][k] * c0
        v1 += c["L"][k] * c1
    return v0, v1


def orders(dofs, errs):
    """The paper's observed orders ln(e_{k-1}/e_k) / ln(sqrt(DoF_k/DoF_{k-1}))."""
    return [float(np.log(errs[i - 1] / errs[i]) / np.log(np.sqrt(dofs[i] / dofs[i - 1]))) for i in range(1, len(errs))]
