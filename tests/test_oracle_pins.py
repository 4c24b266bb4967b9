"""Pins of the FP64 oracle against facts fixed by the paper and by the
mathematics (closed forms, identities, brute force, library routines).
None of these tests compares the oracle with itself."""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import adjoint, deformation as geo, fem, twoscale

HERE = os.path.dirname(os.path.abspath(__file__))


def _prm(NM, dt=0.01, **kw):
    return twoscale.Params(NM, dt, **kw)


# --------------------------------------------------------------------------
# Geometry: the pullback quantities of Section 3.1
# --------------------------------------------------------------------------

def test_jacobian_is_derivative_of_the_map():
    """F from its closed form equals a central difference of the map itself
    (pins G = D phi, the rotation and the amplitude scaling)."""
    rng = np.random.default_rng(0)
    y = rng.uniform(-1, 1, (50, 2))
    h = 1e-6
    for a, th in ((0.3, 0.0), (-0.25, 0.37)):
        F = geo.jacobian(y[:, 0], y[:, 1], a, th)
        for c in range(2):
            e = np.zeros(2); e[c] = h
            zp = np.stack(geo.chi(y[:, 0] + e[0], y[:, 1] + e[1], a, th), axis=1)
            zm = np.stack(geo.chi(y[:, 0] - e[0], y[:, 1] - e[1], a, th), axis=1)
            np.testing.assert_allclose(F[:, :, c], (zp - zm) / (2 * h), atol=1e-9)


def test_map_sends_square_onto_itself():
    """Every edge of [-1,1]^2 maps into itself (so Y_x = Y for the family)."""
    s = np.linspace(-1, 1, 101)
    for a in (-0.3, 0.3):
        z1, z2 = geo.chi(np.ones_like(s), s, a)
        assert np.allclose(z1, 1.0) and z2.min() >= -1 - 1e-15 and z2.max() <= 1 + 1e-15
        z1, z2 = geo.chi(s, -np.ones_like(s), a)
        assert np.allclose(z2, -1.0)
    y = np.random.default_rng(1).uniform(-1, 1, (20000, 2))
    J = np.linalg.det(geo.jacobian(y[:, 0], y[:, 1], 0.3))
    assert J.min() > 0.5


def test_stiffness_weight_is_KKtJ_and_invariant_under_rotation():
    rng = np.random.default_rng(2)
    y = rng.uniform(-1, 1, (40, 2))
    J0, C0 = geo.pullback(y[:, 0], y[:, 1], 0.27, 0.0)
    J1, C1 = geo.pullback(y[:, 0], y[:, 1], 0.27, 0.33)
    np.testing.assert_allclose(J0, J1, rtol=1e-14)
    np.testing.assert_allclose(C0, C1, rtol=1e-13, atol=1e-15)
    # C grad(v^) . grad(psi^) J-weighted == physical grad v . grad psi times J
    F = geo.jacobian(y[:, 0], y[:, 1], 0.27, 0.33)
    g1 = rng.standard_normal((40, 2)); g2 = rng.standard_normal((40, 2))
    phys1 = np.linalg.solve(np.transpose(F, (0, 2, 1)), g1[..., None])[..., 0]   # F^{-T} g
    phys2 = np.linalg.solve(np.transpose(F, (0, 2, 1)), g2[..., None])[..., 0]
    lhs = np.einsum("ni,nij,nj->n", g1, C1, g2)
    np.testing.assert_allclose(lhs, np.sum(phys1 * phys2, axis=1) * np.linalg.det(F), rtol=1e-12)


def test_boundary_weight_is_cofactor_normal_norm():
    """|F tau| equals |cof(F) nu| = |det F F^{-T} nu| (change of variables
    for boundary integrals, Section 3.1) on all four reference edges."""
    rng = np.random.default_rng(3)
    s = rng.uniform(-1, 1, 30)
    for (y1, y2, tau, nu) in ((s, -np.ones_like(s), (1, 0), (0, -1)),
                              (s, np.ones_like(s), (1, 0), (0, 1)),
                              (-np.ones_like(s), s, (0, 1), (-1, 0)),
                              (np.ones_like(s), s, (0, 1), (1, 0))):
        F = geo.jacobian(y1, y2, -0.29, 0.2)
        cof = np.linalg.det(F)[:, None, None] * np.linalg.inv(np.transpose(F, (0, 2, 1)))
        ref = np.linalg.norm(cof @ np.asarray(nu, float), axis=1)
        np.testing.assert_allclose(geo.boundary_weight(y1, y2, tau, -0.29, 0.2), ref, rtol=1e-13)


def test_amplitude_derivatives_match_finite_differences():
    rng = np.random.default_rng(4)
    y = rng.uniform(-1, 1, (30, 2))
    a, th, h = 0.21, 0.3, 1e-6
    dJ, dC = geo.pullback_da(y[:, 0], y[:, 1], a, th)
    Jp, Cp = geo.pullback(y[:, 0], y[:, 1], a + h, th)
    Jm, Cm = geo.pullback(y[:, 0], y[:, 1], a - h, th)
    np.testing.assert_allclose(dJ, (Jp - Jm) / (2 * h), atol=1e-8)
    np.testing.assert_allclose(dC, (Cp - Cm) / (2 * h), atol=1e-8)
    for tau in ((1.0, 0.0), (0.0, 1.0)):
        dw = geo.boundary_weight_da(y[:, 0], y[:, 1], tau, a, th)
        fd = (geo.boundary_weight(y[:, 0], y[:, 1], tau, a + h, th)
              - geo.boundary_weight(y[:, 0], y[:, 1], tau, a - h, th)) / (2 * h)
        np.testing.assert_allclose(dw, fd, atol=1e-8)


# --------------------------------------------------------------------------
# Q1 operators: textbook closed forms and structure
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N", [4, 7])
def test_q1_stencils_at_identity(N):
    """At a = 0: interior stiffness row (1/3)[-1 -1 -1; -1 8 -1; -1 -1 -1],
    mass row (h^2/36)[1 4 1; 4 16 4; 1 4 1], boundary edge row (h/6)[1 4 1]."""
    M, A, B = fem.micro_matrices(N, 0.0)
    h = 2.0 / N
    j1, j2 = 2, 2
    j = j2 * (N + 1) + j1
    stencil = lambda Mat: Mat.toarray()[j].reshape(N + 1, N + 1)[j2 - 1:j2 + 2, j1 - 1:j1 + 2]
    np.testing.assert_allclose(stencil(A), np.array([[-1, -1, -1], [-1, 8, -1], [-1, -1, -1]]) / 3, atol=1e-14)
    np.testing.assert_allclose(stencil(M), np.array([[1, 4, 1], [4, 16, 4], [1, 4, 1]]) * h * h / 36, atol=1e-15)
    row = B.toarray()[2][:5]            # bottom edge node j1 = 2
    np.testing.assert_allclose(row[1:4], np.array([1, 4, 1]) * h / 6, atol=1e-15)
    assert abs(B.toarray()[j].sum()) == 0.0


@pytest.mark.parametrize("a,theta", [(0.0, 0.0), (0.3, 0.0), (-0.3, 0.35)])
def test_micro_operator_structure(a, theta):
    """S symmetric, SPD; A 1 = 0; 1^T B = b^T; volume and boundary length."""
    N, dt, d, kap = 6, 0.01, 0.5, 1.0
    M, A, B = fem.micro_matrices(N, a, theta)
    S = (M / dt + d * A + kap * B).toarray()
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    sla.cholesky(S)                                           # raises if not SPD
    one = np.ones(S.shape[0])
    assert np.abs(A @ one).max() < 1e-13
    b = B @ one
    np.testing.assert_allclose(one @ B.toarray(), b, rtol=1e-14)
    if a == 0.0:
        assert abs(b.sum() - 8.0) < 1e-14 and abs(one @ (M @ one) - 4.0) < 1e-14


@pytest.mark.parametrize("N,a,theta", [(3, 0.0, 0.0), (5, 0.27, 0.4), (8, -0.3, 1.1)])
def test_mass_is_a_sum_of_kronecker_products(N, a, theta):
    """For the map family, J = det(I + aG) = 1 + a(c(y1) y2 + y1 c(y2))
    + a^2 (c(y1) y1 c(y2) y2 - s(y1) s(y2)) with s = sin(pi y)/4 and
    c = pi cos(pi y)/4, each term a product f(y1) g(y2); the 2x2 Gauss rule
    is a tensor rule, so the J-weighted Q1 mass is sum_T kappa_T (M1[g_T] x
    M1[f_T]) with 1D masses weighted at the 1D Gauss points (node order
    j = j2 (N+1) + j1).  Built here from the 1D rule alone and compared with
    the oracle's 2D assembly (R_theta leaves J unchanged)."""
    h = 2.0 / N
    gx = np.array([0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)])

    def m1(f):
        m = np.zeros((N + 1, N + 1))
        for e in range(N):
            for t in gx:
                y = -1.0 + (e + t) * h
                phi = np.array([1.0 - t, t])
                m[e:e + 2, e:e + 2] += 0.5 * h * f(y) * np.outer(phi, phi)
        return m

    s = lambda y: math.sin(math.pi * y) / 4
    c = lambda y: math.pi * math.cos(math.pi * y) / 4
    terms = [(1.0, lambda y: 1.0, lambda y: 1.0), (a, c, lambda y: y), (a, lambda y: y, c),
             (a * a, lambda y: c(y) * y, lambda y: c(y) * y), (-a * a, s, s)]
    Ms = sum(k * np.kron(m1(g), m1(f)) for k, f, g in terms)
    M = fem.micro_matrices(N, a, theta)[0].toarray()
    assert np.abs(M - Ms).max() <= 1e-14 * np.abs(M).max()


def test_geometry_totals_equal_square():
    """Y_x = Y = [-1,1]^2 for every amplitude, so the discrete volume
    1^T M 1 and boundary length 1^T B 1 equal 4 and 8.  The amplitude-linear
    and -quadratic parts of J and |F tau| are odd or periodic over the
    symmetric Gauss points, so the totals hold to rounding at every N."""
    for N in (3, 4, 8, 16):
        for a in (-0.3, 0.17, 0.3):
            M, A, B = fem.micro_matrices(N, a, 0.2)
            one = np.ones(M.shape[0])
            assert abs(one @ (M @ one) - 4.0) < 1e-13
            assert abs((B @ one).sum() - 8.0) < 1e-13


def test_affine_patch_test():
    """For an affine map (the paper's manufactured zeta, eq. manu_system) the
    2x2 rule is exact, so A v_h = 0 on interior nodes when v_h interpolates a
    function affine in the physical coordinate."""
    N = 6
    h = 2.0 / N
    x0, x1 = 0.3, -0.2
    F = np.array([[0.4 * 1.4, -0.4 * 0.54], [-0.3 * 0.4, 0.3 * 0.8]])
    zeta = lambda y1, y2: (0.4 * ((x0 + 1.3) + (1.4 * y1 - 0.54 * y2)),
                           0.3 * ((x1 + 1.2) + (-0.4 * y1 + 0.8 * y2)))
    ncell = N * N
    J = np.full((ncell, 4), np.linalg.det(F))
    K = np.linalg.inv(F)
    C = np.broadcast_to(K @ K.T * np.linalg.det(F), (ncell, 4, 2, 2)).copy()
    _, A = fem.assemble_cells(N, -1.0, h, J, C)
    t = -1.0 + h * np.arange(N + 1)
    Y1, Y2 = np.meshgrid(t, t, indexing="xy")
    z1, z2 = zeta(Y1.ravel(), Y2.ravel())
    v = 2.0 * z1 - 3.0 * z2 + 0.5
    r = (A @ v).reshape(N + 1, N + 1)[1:-1, 1:-1]
    assert np.abs(r).max() < 1e-13
    # energy: v^T A v = int_{Y_x} |grad v|^2 = |g|^2 * area(Y_x), g = (2, -3)
    area = 4.0 * abs(np.linalg.det(F))
    assert abs(v @ (A @ v) - 13.0 * area) < 1e-12 * 13.0 * area
    # a transposed weight K^T K J has the same patch property but the wrong energy
    Cw = np.broadcast_to(K.T @ K * np.linalg.det(F), (ncell, 4, 2, 2)).copy()
    _, Aw = fem.assemble_cells(N, -1.0, h, J, Cw)
    assert abs(v @ (Aw @ v) - 13.0 * area) > 1e-2


def test_banded_cholesky_matches_dense_solve():
    M, A, B = fem.micro_matrices(5, 0.2, 0.1)
    S = (M / 0.01 + 0.5 * A + B).tocsr()
    rhs = np.random.default_rng(5).standard_normal(S.shape[0])
    x = twoscale.BandedSPD(S, 5 + 2).solve(rhs)
    np.testing.assert_allclose(x, np.linalg.solve(S.toarray(), rhs), rtol=1e-12, atol=1e-14)


def test_macro_matrices_textbook():
    MH, KH, L = fem.macro_matrices(4)
    H = 0.25
    k = 2 * 5 + 2
    np.testing.assert_allclose(KH.toarray()[k].reshape(5, 5)[1:4, 1:4],
                               np.array([[-1, -1, -1], [-1, 8, -1], [-1, -1, -1]]) / 3, atol=1e-14)
    np.testing.assert_allclose(L[k], H * H, rtol=1e-14)
    assert abs(L.sum() - 1.0) < 1e-14


# --------------------------------------------------------------------------
# The coupled step
# --------------------------------------------------------------------------

def _tiny(NM=3, N=4, seed=1, ragged=False, kappa=1.0, sigma=-1):
    rng = np.random.default_rng(seed)
    n = (NM + 1) ** 2
    a = rng.uniform(-0.3, 0.3, n)
    th = rng.uniform(0, np.pi / 8, n)
    lv = rng.choice([2, 3, 4], n) if ragged else np.full(n, N)
    prm = _prm(NM, 0.01, kappa=kappa, sigma=sigma)
    ts = twoscale.TwoScale(prm, lv, a, th)
    u0 = W.initial_macro(NM) * (1 + 0.2 * rng.standard_normal(n))
    u0[ts.bnd] = 0.0
    v0 = rng.uniform(0, 1, int(ts.offsets[-1]))
    return ts, u0, v0


@pytest.mark.parametrize("NM,N,ragged,sigma", [(2, 2, False, -1), (3, 4, False, -1),
                                               (4, 3, True, -1), (3, 3, False, 1)])
def test_schur_equals_dense_monolithic_and_fixed_point(NM, N, ragged, sigma):
    ts, u0, v0 = _tiny(NM, N, ragged=ragged, sigma=sigma)
    u1, v1, F1 = ts.step(u0, v0)
    u2, v2, F2 = ts.step_monolithic(u0, v0)
    np.testing.assert_allclose(u1, u2, atol=1e-13)
    np.testing.assert_allclose(v1, v2, atol=1e-13)
    np.testing.assert_allclose(F1, F2, atol=1e-13)
    u3, v3, F3, it = ts.step_fixed_point(u0, v0)
    assert it < 500
    np.testing.assert_allclose(u1, u3, atol=1e-13)
    np.testing.assert_allclose(v1, v3, atol=1e-13)


def test_flux_bookkeeping_identity():
    """1^T M_i (v^{n+1} - v^n)/dt = |dY_i| F_i^{n+1} (A 1 = 0, 1^T B = b^T)."""
    ts, u0, v0 = _tiny(3, 4, ragged=True)
    u1, v1, F1 = ts.step(u0, v0)
    for i, I in enumerate(ts.inst):
        dv = ts.split(v1)[i] - ts.split(v0)[i]
        lhs = np.ones(I.n) @ (I.M @ dv) / ts.prm.dt
        assert abs(lhs - I.len * F1[i]) < 1e-11 * max(1.0, abs(lhs))


def _eig_1d(H):
    m1 = H / 6 * (4 + 2 * math.cos(math.pi * H))
    k1 = (2 - 2 * math.cos(math.pi * H)) / H
    return m1, k1


def test_kappa_zero_macro_closed_form():
    """kappa = 0 decouples the scales (Section 4.4, coupling limits): u^n =
    (1 + dt D lambda_h)^{-n} I_h(sin pi x1 sin pi x2), lambda_h =
    12 (1 - cos pi H) / (H^2 (2 + cos pi H)); at H = 1/8, dt = 0.01, n = 10
    this is lambda_h = 19.99416.., rho_10 = 0.161584.."""
    w = W.WORKLOADS["small_fp64"]
    prm = _prm(w.macro_cells, w.dt, kappa=0.0)
    a = W.amplitudes(w)
    ts = twoscale.TwoScale(prm, W.levels(w), a)
    u0 = W.initial_macro(w.macro_cells)
    out = ts.run(u0, np.zeros(int(ts.offsets[-1])), 10)
    H = 1.0 / w.macro_cells
    lam = 12 * (1 - math.cos(math.pi * H)) / (H * H * (2 + math.cos(math.pi * H)))
    assert abs(lam - 19.99416) < 1e-5
    rho = (1 + w.dt * lam) ** -10
    assert abs(rho - 0.161584) < 1e-6
    np.testing.assert_allclose(out["u"][-1], rho * u0, atol=1e-14)
    assert np.abs(out["F"]).max() == 0.0


def _integral_of_square_by_quadrature(NM, u):
    """int_Omega u_h^2 of the Q1 interpolant with nodal values u, by a 3x3
    Gauss rule on every macro cell (exact: u_h^2 has degree 2 per variable).
    Written from the bilinear interpolant itself, not from any mass matrix."""
    H = 1.0 / NM
    g, wg = np.polynomial.legendre.leggauss(3)
    t, wt = 0.5 * (g + 1.0), 0.5 * wg
    U = np.asarray(u).reshape(NM + 1, NM + 1)          # [k2, k1]
    total = 0.0
    for c2 in range(NM):
        for c1 in range(NM):
            u00, u10 = U[c2, c1], U[c2, c1 + 1]
            u01, u11 = U[c2 + 1, c1], U[c2 + 1, c1 + 1]
            for s, ws in zip(t, wt):
                for r, wr in zip(t, wt):
                    val = (u00 * (1 - s) * (1 - r) + u10 * s * (1 - r)
                           + u01 * (1 - s) * r + u11 * s * r)
                    total += ws * wr * H * H * val * val
    return total


@pytest.mark.parametrize("NM", [3, 8, 13])
def test_observable_is_integral_of_square(NM):
    """J = u^T M_H u is the integral of u_h^2 over Omega.  For
    u = I_h(sin pi x1 sin pi x2) it has the closed form
    J = m1^2 (NM/2)^2, m1 = H/6 (4 + 2 cos pi H) (the 1D Q1 mass eigenvalue
    of the sine mode, whose squared nodal norm is NM/2); at NM = 8 this is
    0.2374742089066.  A direct quadrature of u_h^2 agrees for any nodal
    values (here random ones, boundary included).  A lumped-mass J
    (L = diag(M_H 1) in place of M_H) differs from both, so this pin sees it."""
    prm = _prm(NM)
    ts = twoscale.TwoScale(prm, np.full((NM + 1) ** 2, 2), np.zeros((NM + 1) ** 2))
    u = W.initial_macro(NM)
    H = 1.0 / NM
    m1 = H / 6 * (4 + 2 * math.cos(math.pi * H))
    closed = m1 * m1 * (NM / 2.0) ** 2
    assert abs(ts.observable(u) - closed) <= 1e-14 * closed
    if NM == 8:
        assert abs(closed - 0.2374742089066) < 1e-12
    rng = np.random.default_rng(NM)
    ur = rng.standard_normal((NM + 1) ** 2)
    q = _integral_of_square_by_quadrature(NM, ur)
    assert abs(ts.observable(ur) - q) <= 1e-13 * q
    # a planted mistake: the lumped mass in place of M_H
    lumped = float(np.sum(ts.L * u * u))
    assert abs(lumped - closed) > 1e-3 * closed
    assert abs(float(np.sum(ts.L * ur * ur)) - q) > 1e-3 * q


def test_constant_amplitude_rank_one_reduction():
    """a = const, v^0 = 0, u^0 = I_h(sin sin): u^n = rho_n u^0 and
    v_i^n = u^0_i V^n, where (rho, V) solve a one-instance system with the
    eigenvalues of the 1D Q1 mass and stiffness matrices."""
    NM, N, dt, steps = 6, 5, 0.01, 4
    prm = _prm(NM, dt)
    n = (NM + 1) ** 2
    ts = twoscale.TwoScale(prm, np.full(n, N), np.full(n, 0.23))
    u0 = W.initial_macro(NM)
    out = ts.run(u0, np.zeros(int(ts.offsets[-1])), steps)
    # reduced system
    H = 1.0 / NM
    m1, k1 = _eig_1d(H)
    m, k = m1 * m1, 2 * k1 * m1
    M, A, B = fem.micro_matrices(N, 0.23)
    S = (M / dt + prm.d * A + prm.kappa * B).toarray()
    b = B @ np.ones(M.shape[0]); ln = b.sum()
    rho, V = 1.0, np.zeros(M.shape[0])
    for _ in range(steps):
        # S V' = M V/dt + kappa p rho' b ;  (m/dt + D k) rho' + H^2 F = m rho/dt
        # with F = kappa p rho' - kappa/len b^T V'   (sigma = -1)
        V0 = np.linalg.solve(S, M @ V / dt)
        Wv = np.linalg.solve(S, prm.kappa * prm.p * b)
        beta = prm.kappa * prm.p - prm.kappa / ln * b @ Wv
        alpha = -prm.kappa / ln * b @ V0
        rho_n = (m * rho / dt - H * H * alpha) / (m / dt + prm.D * k + H * H * beta)
        V = V0 + rho_n * Wv
        rho = rho_n
    np.testing.assert_allclose(out["u"][-1], rho * u0, atol=1e-14)
    vfin = np.stack(ts.split(out["v"]))
    np.testing.assert_allclose(vfin, np.outer(u0, V), atol=1e-13)


def test_boundary_instances_stay_zero():
    w = W.WORKLOADS["small_fp64"]
    ts = twoscale.TwoScale(_prm(w.macro_cells, w.dt), W.levels(w), W.amplitudes(w))
    out = ts.run(W.initial_macro(w.macro_cells), np.zeros(int(ts.offsets[-1])), 3)
    for i in np.flatnonzero(ts.bnd):
        assert np.abs(ts.split(out["v"])[i]).max() == 0.0
    assert np.abs(out["u"][:, ts.bnd]).max() == 0.0


def test_pullback_consistency_between_amplitudes():
    """Y_x = Y for every a, so a = 0.3 and a = 0 discretise the same
    continuum micro problem: under the same prescribed u-history their mean
    fluxes differ by O(h^2).  A wrong pullback weight breaks this."""
    dt, steps = 0.01, 5
    diffs = []
    for N in (8, 16, 32):
        Fs = []
        for a in (0.0, 0.3):
            prm = _prm(1, dt)
            I = twoscale.Instance(N, a, 0.0, prm)
            v = np.zeros(I.n)
            for n in range(1, steps + 1):
                un = math.exp(-n * dt)
                v = I.chol.solve(I.M @ v / dt + prm.kappa * prm.p * un * I.b)
            Fs.append(prm.kappa * prm.p * un - prm.kappa / I.len * I.b @ v)
        diffs.append(abs(Fs[1] - Fs[0]))
    rates = np.log2(np.array(diffs[:-1]) / np.array(diffs[1:]))
    assert (rates > 1.7).all(), (diffs, rates)


# --------------------------------------------------------------------------
# Adjoint
# --------------------------------------------------------------------------

def _J_of(prm, lv, a, th, u0, v0, steps):
    ts = twoscale.TwoScale(prm, lv, a, th)
    out = ts.run(u0, v0, steps)
    return ts.observable(out["u"][-1])


def test_adjoint_matches_central_differences():
    ts, u0, v0 = _tiny(3, 4, seed=3, ragged=True)
    a = np.array([I.a for I in ts.inst]); th = np.array([I.theta for I in ts.inst])
    lv = np.array([I.N for I in ts.inst])
    steps = 4
    J, g = adjoint.gradient(ts, u0, v0, steps)
    rng = np.random.default_rng(9)
    for _ in range(3):
        e = rng.standard_normal(len(a)); h = 1e-5
        fd = (_J_of(ts.prm, lv, a + h * e, th, u0, v0, steps)
              - _J_of(ts.prm, lv, a - h * e, th, u0, v0, steps)) / (2 * h)
        assert abs(g @ e - fd) <= 1e-7 * abs(fd) + 1e-13, (g @ e, fd)


def test_adjoint_exact_zeros():
    """g = 0 on macro-boundary instances started from v = 0; g = 0 for kappa = 0."""
    w = W.WORKLOADS["small_fp64"]
    ts = twoscale.TwoScale(_prm(w.macro_cells, w.dt), W.levels(w), W.amplitudes(w))
    J, g = adjoint.gradient(ts, W.initial_macro(w.macro_cells), np.zeros(int(ts.offsets[-1])), 3)
    assert np.abs(g[ts.bnd]).max() == 0.0 and np.abs(g[~ts.bnd]).max() > 0
    ts0 = twoscale.TwoScale(_prm(w.macro_cells, w.dt, kappa=0.0), W.levels(w), W.amplitudes(w))
    J0, g0 = adjoint.gradient(ts0, W.initial_macro(w.macro_cells), np.zeros(int(ts0.offsets[-1])), 3)
    assert np.abs(g0).max() == 0.0


# --------------------------------------------------------------------------
# The paper's convergence tables
# --------------------------------------------------------------------------

def _read_tables():
    rows, sec = {}, None
    with open(os.path.join(HERE, "golden", "paper_convergence_tables.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                sec = line[1:-1]; rows[sec] = []; continue
            rows[sec].append(line.split())
    return rows


def observed_rates(dofs, errs):
    """ln(e_{k-1}/e_k) / ln(sqrt(DoF_k/DoF_{k-1})): the paper's rate formula."""
    dofs = np.asarray(dofs, float); errs = np.asarray(errs, float)
    return np.log(errs[:-1] / errs[1:]) / np.log(np.sqrt(dofs[1:] / dofs[:-1]))


def test_paper_tables_rate_formula_after_unswapping_last_rows():
    t = _read_tables()
    t["macro"][-1], t["micro"][-1] = t["micro"][-1], t["macro"][-1]
    for sec in ("macro", "micro"):
        r = t[sec]
        d = [float(x[0]) for x in r]
        p = observed_rates(d, [float(x[2]) for x in r])
        q = observed_rates(d, [float(x[3]) for x in r])
        # printed rates live in the row of the finer mesh (swapped with the row)
        pp = [float(x[4]) for x in r[1:]]
        qq = [float(x[5]) for x in r[1:]]
        np.testing.assert_allclose(p, pp, atol=1.5e-3)
        np.testing.assert_allclose(q, qq, atol=1.5e-3)
    # as printed (not swapped back) the last rates are not reproduced
    t = _read_tables()
    r = t["macro"]
    q = observed_rates([float(x[0]) for x in r], [float(x[3]) for x in r])
    assert q[-1] < 0


# ------------------------------------------------------------ general maps
def test_jacobian_tables_reproduce_the_analytic_instance():
    """Tables of the family's own Jacobian (the workloads generator, its own
    layout) give the analytic instance's matrices: ties the table path, and
    the table layout, to the pinned analytic path."""
    from oracle import fem
    for N, a, th in ((4, 0.3, 0.0), (7, -0.25, 1.1)):
        per, _, _ = W.jacobian_tables(np.array([N]), W.sinusoidal_map_jacobian, [(a, th)])
        Mt, At, Bt = fem.micro_matrices_from_jacobians(N, *per[0])
        M, A, B = fem.micro_matrices(N, a, th)
        for X, Y in ((Mt, M), (At, A), (Bt, B)):
            assert abs(X - Y).max() <= 1e-14 * abs(Y).max()


def test_jacobian_tables_affine_map_closed_forms():
    """A constant Jacobian F (an affine map): area 4 det F, perimeter
    4(|F e1| + |F e2|), and the energy of the physically linear function
    v = g . zeta(y) is |g|^2 * area (Q1 reproduces it exactly)."""
    from oracle import fem
    F = np.array([[1.2, 0.3], [-0.1, 0.9]])
    g = np.array([0.7, -1.3])
    for N in (3, 8):
        per, _, _ = W.jacobian_tables(np.array([N]), lambda y1, y2: np.broadcast_to(F, np.shape(y1) + (2, 2)).copy(), [()])
        M, A, B = fem.micro_matrices_from_jacobians(N, *per[0])
        one = np.ones((N + 1) ** 2)
        area = 4.0 * np.linalg.det(F)
        assert abs(one @ M @ one - area) <= 1e-13 * area
        perim = 4.0 * (np.linalg.norm(F[:, 0]) + np.linalg.norm(F[:, 1]))
        assert abs(one @ B @ one - perim) <= 1e-13 * perim
        h = 2.0 / N
        j = np.arange((N + 1) ** 2)
        y1, y2 = -1.0 + (j % (N + 1)) * h, -1.0 + (j // (N + 1)) * h
        z = F @ np.stack([y1, y2])
        v = g @ z
        assert abs(v @ A @ v - g @ g * area) <= 1e-12 * g @ g * area


def test_polynomial_test_map_is_a_valid_deformation():
    """The general-map test family: Jacobian vs central differences of the
    map, det > 0 on the tables, and it really leaves the sinusoidal family
    (the cell's area changes)."""
    from oracle import fem
    c, d, th = 0.2, -0.25, 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    zeta = lambda y1, y2: R @ np.array([y1 + c * y1 * y2, y2 + d * y1 * y1 * y2])
    for y in ((0.3, -0.6), (-0.9, 0.8)):
        e = 1e-6
        Ffd = np.stack([(zeta(y[0] + e, y[1]) - zeta(y[0] - e, y[1])) / (2 * e),
                        (zeta(y[0], y[1] + e) - zeta(y[0], y[1] - e)) / (2 * e)], axis=1)
        assert np.allclose(W.polynomial_map_jacobian(y[0], y[1], c, d, th), Ffd, atol=1e-8)
    per, _, _ = W.jacobian_tables(np.array([6]), W.polynomial_map_jacobian, [(c, d, th)])
    assert np.linalg.det(per[0][0]).min() > 0.3
    M, _, _ = fem.micro_matrices_from_jacobians(6, *per[0])
    one = np.ones(49)
    # area of zeta(Z) = int (1 + c y2)(1 + d y1^2) - 2 c d y1^2 y2 = 4 (1 + d/3)
    assert abs(one @ M @ one - 4.0 * (1.0 + d / 3.0)) <= 1e-13 * 4.0   # Gauss is exact here
