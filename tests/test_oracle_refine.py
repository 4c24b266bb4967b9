"""Pins of the refinement oracle (indicator, bulk marking, nested
interpolation) against closed forms and exact special cases."""
import numpy as np
import pytest

from oracle import deformation as geo
from oracle import refine


def _nodes(N):
    t = -1.0 + 2.0 * np.arange(N + 1) / N
    z1, z2 = np.meshgrid(t, t, indexing="xy")
    return z1.ravel(), z2.ravel()


@pytest.mark.parametrize("N", [4, 8])
def test_affine_field_has_no_jumps(N):
    """An affine field on the undeformed cell (C = I) has a continuous
    flux: every jump vanishes."""
    z1, z2 = _nodes(N)
    assert refine.indicator(N, 1.0 + 0.3 * z1 - 0.7 * z2, 0.0) < 1e-28


@pytest.mark.parametrize("N", [4, 8, 16])
def test_kink_closed_form(N):
    """v = |z1| (+ |z2|) on the undeformed cell: the flux d dv/dz1 jumps by
    2d across the line z1 = 0 only, so eta^2 = (h/12) * (2d)^2 * 2 per
    kinked line (length 2)."""
    d = 0.5
    h = 2.0 / N
    z1, z2 = _nodes(N)
    one = (h / 12.0) * (2 * d) ** 2 * 2.0
    assert refine.indicator(N, np.abs(z1), 0.0, d=d) == pytest.approx(one, rel=1e-13)
    assert refine.indicator(N, np.abs(z1) + np.abs(z2), 0.0, d=d) == pytest.approx(2 * one, rel=1e-13)
    # a kink along the other family of lines, off-centre
    assert refine.indicator(N, np.abs(z2 - h), 0.0, d=d) == pytest.approx(one, rel=1e-13)


def test_kink_weighted_by_the_pulled_back_coefficient():
    """On a deformed cell the jump across z1 = 0 is weighted by C11 at the
    edge points: for v = |z1| the indicator is (h/12) sum over the line's
    Gauss points of (2 d C11)^2 times the point weights."""
    N, a, d = 8, 0.25, 0.5
    h = 2.0 / N
    z1, _ = _nodes(N)
    g = 0.5 + np.array([-0.5, 0.5]) / np.sqrt(3.0)
    s = (-1.0 + (np.arange(N)[:, None] + g[None, :]) * h).ravel()
    _, C = geo.pullback(np.zeros_like(s), s, a)
    expect = (h / 12.0) * np.sum(0.5 * h * (2 * d * C[:, 0, 0]) ** 2)
    assert refine.indicator(N, np.abs(z1), a, d=d) == pytest.approx(expect, rel=1e-13)
    assert abs(expect - refine.indicator(N, np.abs(z1), 0.0, d=d)) > 1e-3 * expect


@pytest.mark.parametrize("N", [2, 4, 16])
def test_prolongation_is_exact_for_bilinear_fields(N):
    f = lambda z1, z2: 1.0 + 2.0 * z1 - z2 + 0.5 * z1 * z2
    z1, z2 = _nodes(N)
    Z1, Z2 = _nodes(2 * N)
    assert np.max(np.abs(refine.prolong(N, f(z1, z2)) - f(Z1, Z2))) < 1e-14
    # a field that is not bilinear is interpolated, not reproduced
    g = lambda z1, z2: z1 * z1
    assert np.max(np.abs(refine.prolong(N, g(z1, z2)) - g(Z1, Z2))) > 1e-3


def test_bulk_marking():
    eta = np.array([0.1, 5.0, 0.0, 3.0, 1.0, 1.0])
    lv = np.array([16, 16, 16, 64, 32, 16])
    # refinable: all but the 64-cell instance; sum = 10.1; theta 0.5 -> 5.05
    assert refine.mark(eta, lv, 0.5).tolist() == [1, 4]
    assert refine.mark(eta, lv, 0.0).tolist() == []
    m = refine.mark(eta, lv, 0.9)            # 9.09: 5 + 1 + 1 + 0.1 = 7.1 never reaches it
    assert m.tolist() == [0, 1, 2, 4, 5]
    # minimal: the marked set reaches theta, without its smallest member it does not
    rng = np.random.default_rng(0)
    eta = rng.exponential(size=50)
    lv = np.full(50, 16)
    m = refine.mark(eta, lv, 0.6)
    s = eta[m].sum()
    assert s >= 0.6 * eta.sum() and s - eta[m].min() < 0.6 * eta.sum()
    assert set(np.argsort(-eta)[:len(m)].tolist()) == set(m.tolist())
