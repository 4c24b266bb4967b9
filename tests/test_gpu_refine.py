"""GPU parity of the refinement path (error indicator, nested
interpolation, a refined batch stepping on) against the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import refine, twoscale
from gpu_helpers import banner, rel

pytestmark = pytest.mark.gpu


def _case(NM=4, seed=3):
    n = (NM + 1) ** 2
    rng = np.random.default_rng(seed)
    lv = rng.choice(np.array([8, 16, 32, 12], np.int32), n)
    a = rng.uniform(-0.3, 0.3, n)
    return NM, lv, a


def test_indicator_on_a_given_state():
    """Same input state on both sides (set_state): the indicator per instance
    to 1e-12."""
    from paper_2103_17040_amd import TwoScaleBatch
    NM, lv, a = _case()
    u, v = W.random_state(lv, NM, seed=4)
    banner(f"indicator NM={NM} levels={sorted(set(lv.tolist()))}")
    g = TwoScaleBatch(NM, lv, a, d=0.5)
    try:
        g.set_state(u, v)
        eta = g.error_indicator().cpu().numpy()
    finally:
        g.close()
    off = W.offsets(lv)
    ref = np.array([refine.indicator(int(lv[i]), v[off[i]:off[i + 1]], a[i], d=0.5) for i in range(len(lv))])
    assert np.max(np.abs(eta - ref) / np.maximum(ref, 1e-300)) <= 1e-12


def test_prolong_is_bitwise():
    from paper_2103_17040_amd import tsm
    import torch
    NM, lv, _ = _case(seed=6)
    new = lv.copy()
    new[::3] = np.minimum(2 * lv[::3], 64)
    new[new > 2 * lv] = lv[new > 2 * lv]
    v = np.random.default_rng(7).standard_normal(int(W.offsets(lv)[-1]))
    banner("prolong")
    vo = torch.as_tensor(v, device="cuda:0")
    vn = torch.empty(int(W.offsets(new)[-1]), dtype=torch.float64, device="cuda:0")
    tsm.tsm_prolong(lv, new, vo, vn)
    out = vn.cpu().numpy()
    oo, on = W.offsets(lv), W.offsets(new)
    for i in range(len(lv)):
        x = v[oo[i]:oo[i + 1]]
        ref = refine.prolong(int(lv[i]), x) if new[i] != lv[i] else x
        assert np.array_equal(out[on[i]:on[i + 1]], ref), i


def test_refined_batch_steps_like_the_oracle():
    """Step, refine by the indicator (bulk marking, theta = 0.5), step on:
    the same marked instances and the same fields as the oracle doing the
    same with its own indicator, marking and interpolation."""
    from paper_2103_17040_amd import TwoScaleBatch
    NM, lv, a = _case(seed=8)
    dt, k1, k2 = 0.01, 3, 3
    u0 = W.initial_macro(NM)
    v0 = np.zeros(int(W.offsets(lv)[-1]))
    banner(f"refine NM={NM} levels={sorted(set(lv.tolist()))} steps {k1}+{k2}")
    # oracle
    ts = twoscale.TwoScale(twoscale.Params(NM, dt), lv, a)
    r1 = ts.run(u0, v0, k1)
    off = W.offsets(lv)
    eta_ref = np.array([refine.indicator(int(lv[i]), r1["v"][off[i]:off[i + 1]], a[i], d=0.5)
                        for i in range(len(lv))])
    m = refine.mark(eta_ref, lv, 0.5)
    # the decision must not hinge on rounding: a clear gap after the last marked
    srt = np.sort(eta_ref[lv * 2 <= 64])[::-1]
    assert len(m) < len(srt) and (srt[len(m) - 1] - srt[len(m)]) > 1e-6 * srt[0]
    new = lv.copy()
    new[m] *= 2
    offn = W.offsets(new)
    vn = np.concatenate([refine.prolong(int(lv[i]), r1["v"][off[i]:off[i + 1]]) if new[i] != lv[i]
                         else r1["v"][off[i]:off[i + 1]] for i in range(len(lv))])
    ts2 = twoscale.TwoScale(twoscale.Params(NM, dt), new, a)
    r2 = ts2.run(r1["u"][-1], vn, k2)
    # GPU
    g = TwoScaleBatch(NM, lv, a, dt=dt, rtol=1e-13)
    try:
        g.set_state(u0, v0)
        g.step(k1)
        g2, levels2, eta = g.refine(0.5)
    finally:
        g.close()
    try:
        assert np.array_equal(levels2, new)
        assert rel(eta, eta_ref) <= 1e-8
        g2.step(k2)
        u, v = g2.macro().cpu().numpy(), g2.micro().cpu().numpy()
    finally:
        g2.close()
    banner(f"  marked {len(m)} of {len(lv)}; rel u {rel(u, r2['u'][-1]):.2e} v {rel(v, r2['v']):.2e}")
    assert rel(u, r2["u"][-1]) <= 1e-10 and rel(v, r2["v"]) <= 1e-10


def test_two_refinements_step_like_the_oracle():
    """Two rounds of step and refine (theta = 0.6: meshes go up to twice
    refined), then steps on the final meshes, against the oracle."""
    from paper_2103_17040_amd import TwoScaleBatch
    NM, lv, a = _case(seed=12)
    dt, k = 0.01, 2
    u0 = W.initial_macro(NM)
    banner(f"two refinements NM={NM} levels={sorted(set(lv.tolist()))}")
    # oracle
    levels, u, v = lv.copy(), u0, np.zeros(int(W.offsets(lv)[-1]))
    marks = []
    for _ in range(2):
        ts = twoscale.TwoScale(twoscale.Params(NM, dt), levels, a)
        r = ts.run(u, v, k)
        u, v = r["u"][-1], r["v"]
        off = W.offsets(levels)
        eta = np.array([refine.indicator(int(levels[i]), v[off[i]:off[i + 1]], a[i], d=0.5)
                        for i in range(len(levels))])
        m = refine.mark(eta, levels, 0.6)
        srt = np.sort(eta[levels * 2 <= 64])[::-1]
        assert len(m) < len(srt) and (srt[len(m) - 1] - srt[len(m)]) > 1e-6 * srt[0]
        new = levels.copy()
        new[m] *= 2
        v = np.concatenate([refine.prolong(int(levels[i]), v[off[i]:off[i + 1]]) if new[i] != levels[i]
                            else v[off[i]:off[i + 1]] for i in range(len(levels))])
        levels = new
        marks.append(new)
    r = twoscale.TwoScale(twoscale.Params(NM, dt), levels, a).run(u, v, k)
    # GPU
    g = TwoScaleBatch(NM, lv, a, dt=dt, rtol=1e-13)
    try:
        g.set_state(u0, None)
        for rnd in range(2):
            g.step(k)
            g2, new, _ = g.refine(0.6)
            g.close()
            g = g2
            assert np.array_equal(new, marks[rnd]), rnd
        g.step(k)
        ug, vg = g.macro().cpu().numpy(), g.micro().cpu().numpy()
    finally:
        g.close()
    banner(f"  final levels {sorted(set(levels.tolist()))}; rel u {rel(ug, r['u'][-1]):.2e} v {rel(vg, r['v']):.2e}")
    assert rel(ug, r["u"][-1]) <= 1e-10 and rel(vg, r["v"]) <= 1e-10


def test_indicator_state_errors():
    from paper_2103_17040_amd import TwoScaleBatch, tsm
    NM, lv, a = _case(NM=2)
    banner("indicator errors")
    g = TwoScaleBatch(NM, lv, a)
    try:
        with pytest.raises(tsm.TsmError) as e:
            g.error_indicator()              # no state yet
        assert e.value.status == tsm.TSM_ESTATE
    finally:
        g.close()
    _, Fc, Fb = W.jacobian_tables(lv, W.sinusoidal_map_jacobian, [(x, 0.0) for x in a])
    g = TwoScaleBatch(NM, lv, jacobians=(Fc, Fb))
    try:
        g.set_state(W.initial_macro(NM))
        with pytest.raises(tsm.TsmError) as e:
            g.error_indicator()              # tables: C is not known off their points
        assert e.value.status == tsm.TSM_ESTATE
    finally:
        g.close()


def test_indicator_and_interpolation_above_64_cells():
    """Meshes of 65-256 cells per side: the indicator (read from global
    memory, coordinates evaluated where used) to 1e-12 and the nested
    interpolation up to 256 cells bitwise, against the oracle."""
    from paper_2103_17040_amd import TwoScaleBatch, tsm
    import torch
    NM = 2
    lv = np.array([91, 128, 65, 100, 256, 64, 128, 16, 97], np.int32)
    a = np.random.default_rng(12).uniform(-0.3, 0.3, lv.size)
    u, v = W.random_state(lv, NM, seed=13)
    banner(f"indicator and interpolation, levels {lv.tolist()}")
    g = TwoScaleBatch(NM, lv, a, d=0.5)
    try:
        g.set_state(u, v)
        eta = g.error_indicator().cpu().numpy()
    finally:
        g.close()
    off = W.offsets(lv)
    ref = np.array([refine.indicator(int(lv[i]), v[off[i]:off[i + 1]], a[i], d=0.5) for i in range(len(lv))])
    assert np.max(np.abs(eta - ref) / np.maximum(ref, 1e-300)) <= 1e-12
    new = np.where(lv <= 128, 2 * lv, lv).astype(np.int32)
    vo = torch.as_tensor(v, device="cuda:0")
    vn = torch.empty(int(W.offsets(new)[-1]), dtype=torch.float64, device="cuda:0")
    tsm.tsm_prolong(lv, new, vo, vn)
    out = vn.cpu().numpy()
    on = W.offsets(new)
    for i in range(len(lv)):
        x = v[off[i]:off[i + 1]]
        exp = refine.prolong(int(lv[i]), x) if new[i] != lv[i] else x
        assert np.array_equal(out[on[i]:on[i + 1]], exp), i


def test_refinement_into_large_meshes_steps_like_the_oracle():
    """Step, refine every interior instance with max_level 256 (64 -> 128,
    128 -> 256, 100 -> 200 cells per side), step on, against the oracle
    doing the same."""
    from paper_2103_17040_amd import TwoScaleBatch
    NM, dt, k1, k2 = 3, 0.01, 2, 2
    lv = np.full(16, 16, np.int32)
    lv[[5, 6, 9, 10]] = [64, 128, 32, 100]      # the interior nodes
    a = np.random.default_rng(21).uniform(-0.3, 0.3, lv.size)
    u0 = W.initial_macro(NM)
    v0 = np.zeros(int(W.offsets(lv)[-1]))
    banner(f"refine into large meshes, levels {lv.tolist()}")
    ts = twoscale.TwoScale(twoscale.Params(NM, dt), lv, a)
    r1 = ts.run(u0, v0, k1)
    off = W.offsets(lv)
    eta_ref = np.array([refine.indicator(int(lv[i]), r1["v"][off[i]:off[i + 1]], a[i], d=0.5)
                        for i in range(len(lv))])
    m = refine.mark(eta_ref, lv, 0.999, 256)
    srt = np.sort(eta_ref[lv * 2 <= 256])[::-1]
    assert len(m) < len(srt) and (srt[len(m) - 1] - srt[len(m)]) > 1e-6 * srt[0]
    new = lv.copy()
    new[m] *= 2
    assert new.max() > 128
    vn = np.concatenate([refine.prolong(int(lv[i]), r1["v"][off[i]:off[i + 1]]) if new[i] != lv[i]
                         else r1["v"][off[i]:off[i + 1]] for i in range(len(lv))])
    r2 = twoscale.TwoScale(twoscale.Params(NM, dt), new, a).run(r1["u"][-1], vn, k2)
    g = TwoScaleBatch(NM, lv, a, dt=dt, rtol=1e-13, max_iter=5000)
    try:
        g.set_state(u0, v0)
        g.step(k1)
        g2, levels2, eta = g.refine(0.999, max_level=256)
    finally:
        g.close()
    try:
        assert np.array_equal(levels2, new)
        assert rel(eta, eta_ref) <= 1e-8
        g2.step(k2)
        u, v = g2.macro().cpu().numpy(), g2.micro().cpu().numpy()
    finally:
        g2.close()
    banner(f"  marked {len(m)} of {len(lv)}; rel u {rel(u, r2['u'][-1]):.2e} v {rel(v, r2['v']):.2e}")
    assert rel(u, r2["u"][-1]) <= 1e-10 and rel(v, r2["v"]) <= 1e-10
