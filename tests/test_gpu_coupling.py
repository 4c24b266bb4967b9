"""The paper's alternating macro/micro coupling (Section 3.3) as a GPU step
mode: the macro solve with the micro data lagged, then every micro solve with
the new macro values, until the residual sum settles.  It must reach the
oracle's alternating step and the exact (Schur) step it converges to."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import banner, gpu_for, oracle_for, rel

pytestmark = pytest.mark.gpu


def _case(NM, levels, seed):
    rng = np.random.default_rng(seed)
    n = (NM + 1) ** 2
    lv = rng.choice(np.asarray(levels, np.int32), size=n)
    a = rng.uniform(-0.3, 0.3, n)
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    return lv, a, th


def _gpu_run(NM, lv, a, th, dt, steps, u0, v0, **kw):
    g = gpu_for(NM, lv, a, th, dt, **kw)
    try:
        g.set_state(u0, v0)
        us, Fs, its = [], [], []
        for _ in range(steps):
            g.step(1)
            us.append(g.macro().cpu().numpy())
            Fs.append(g.fluxes().cpu().numpy())
            its.append(g.stats()["fp_iters_last"])
        return np.array(us), np.array(Fs), g.micro().cpu().numpy(), its
    finally:
        g.close()


@pytest.mark.parametrize("levels", [[4, 8, 13], [16, 32, 64]])
def test_fixed_point_matches_oracle_alternating_and_exact(levels):
    NM, dt, steps = 4, 0.01, 3
    lv, a, th = _case(NM, levels, 21)
    u0 = W.initial_macro(NM)
    v0 = np.random.default_rng(5).uniform(0, 1, int(W.offsets(lv)[-1]))
    phys = dict(kappa=2.0, d=0.3)
    banner(f"fixed-point coupling vs oracle, levels {levels}")
    ts = oracle_for(NM, lv, a, th, dt, **phys)
    u, v = u0.copy(), v0.copy()
    ou, oF, o_it = [], [], []
    for _ in range(steps):
        u, v, F, it = ts.step_fixed_point(u, v)
        ou.append(u)
        oF.append(F)
        o_it.append(it)
    ex = ts.run(u0, v0, steps)
    gu, gF, gv, g_it = _gpu_run(NM, lv, a, th, dt, steps, u0, v0, rtol=1e-13, coupling="fixed_point",
                                fp_rtol=1e-13, **phys)
    banner(f"iterations per step: gpu {g_it}, oracle {o_it}")
    assert rel(gu, np.array(ou)) <= 1e-10
    assert rel(gF, np.array(oF)) <= 1e-10
    assert rel(gv, v) <= 1e-10
    # the exact step the alternation converges to
    assert rel(gu, ex["u"][1:]) <= 1e-10 and rel(gF, ex["F"]) <= 1e-10 and rel(gv, ex["v"]) <= 1e-10
    assert all(2 <= k < 50 for k in g_it)


def test_fixed_point_refine_matches_exact_coupling():
    NM, dt, steps = 6, 0.005, 3
    lv, a, th = _case(NM, [16, 32, 64, 20], 22)
    u0 = W.initial_macro(NM)
    v0 = np.zeros(int(W.offsets(lv)[-1]))
    banner("fixed-point coupling, FP32 + refinement, vs exact coupling")
    su, sF, sv, _ = _gpu_run(NM, lv, a, th, dt, steps, u0, v0, precision="fp32_refine", rtol=1e-11)
    fu, fF, fv, its = _gpu_run(NM, lv, a, th, dt, steps, u0, v0, precision="fp32_refine", rtol=1e-11,
                               coupling="fixed_point", fp_rtol=1e-11)
    assert rel(fu, su) <= 1e-8 and rel(fF, sF) <= 1e-8 and rel(fv, sv) <= 1e-8
    assert all(k >= 2 for k in its)
