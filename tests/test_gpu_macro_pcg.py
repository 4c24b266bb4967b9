"""Macro solve by PCG (sine-basis preconditioner) where the response
functionals are too heterogeneous for the tensor sweep: maps that change the
cell size by up to 20x, long steps and weak macro diffusion, against the
oracle's banded Cholesky of A_M (Section 3.3 coupling, Schur form)."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import banner, gpu_for, oracle_for, rel, workload_case
from oracle import adjoint, twoscale

pytestmark = pytest.mark.gpu


def _heterogeneous(NM, seed):
    n = (NM + 1) ** 2
    rng = np.random.default_rng(seed)
    lv = rng.choice(np.array([8, 16]), n).astype(np.int32)
    s = rng.uniform(0.2, 4.0, n)
    per, Fc, Fb = W.jacobian_tables(lv, W.scaling_map_jacobian, [(x,) for x in s])
    return lv, per, Fc, Fb


PHYS = dict(D=1e-4, d=0.5, kappa=5.0, p=1.0)


@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-12, 1e-10), ("fp32_refine", 1e-10, 1e-8)])
def test_heterogeneous_maps_use_pcg_and_match_oracle(precision, rtol, tol):
    NM, dt, steps = 6, 10.0, 3
    lv, per, Fc, Fb = _heterogeneous(NM, 3)
    u0 = W.initial_macro(NM)
    v0 = np.zeros(int(W.offsets(lv)[-1]))
    banner(f"macro PCG: scaled cells 0.2-4, dt={dt}, {precision}")
    ts = twoscale.TwoScale(twoscale.Params(NM, dt, **PHYS), lv, None, None, jacobians=per)
    ref = ts.run(u0, v0, steps)
    g = gpu_for(NM, lv, None, None, dt=dt, precision=precision, rtol=rtol, jacobians=(Fc, Fb), **PHYS)
    try:
        st0 = g.stats()
        g.set_state(u0, v0)
        us, Fs = [g.macro().cpu().numpy()], []
        for _ in range(steps):
            g.step(1)
            us.append(g.macro().cpu().numpy())
            Fs.append(g.fluxes().cpu().numpy())
        v = g.micro().cpu().numpy()
    finally:
        g.close()
    banner(f"  contraction bound {st0['macro_contraction']:.3f}, PCG iterations {st0['macro_pcg_iters']}")
    assert st0["macro_contraction"] >= 0.5 and st0["macro_pcg_iters"] > 0 and st0["macro_sweeps"] == 0
    eu, eF, ev = rel(np.array(us), ref["u"]), rel(np.array(Fs), ref["F"]), rel(v, ref["v"])
    banner(f"  rel u {eu:.2e} F {eF:.2e} v {ev:.2e}")
    assert eu <= tol and eF <= tol and ev <= tol


def test_forced_pcg_agrees_with_sweeps_and_adjoint():
    from paper_2103_17040_amd import tsm
    w, a, th, lv, u0, v0, phys = workload_case("small_fp64")
    outs = []
    for flags in (0, tsm.TSM_FLAG_MACRO_PCG):
        g = gpu_for(w.macro_cells, lv, a, th, dt=w.dt, rtol=1e-13, flags=flags, **phys)
        try:
            g.set_state(u0, v0)
            g.step(5)
            outs.append((g.macro().cpu().numpy(), g.micro().cpu().numpy(), g.stats()))
        finally:
            g.close()
    assert outs[0][2]["macro_pcg_iters"] == 0 and outs[1][2]["macro_pcg_iters"] > 0
    assert rel(outs[1][0], outs[0][0]) <= 1e-13 and rel(outs[1][1], outs[0][1]) <= 1e-13
    # the adjoint's macro solves go through the same PCG
    NM, steps = 3, 5
    rng = np.random.default_rng(12)
    n = (NM + 1) ** 2
    lv = rng.choice(np.array([4, 8, 16]), n).astype(np.int32)
    a = rng.uniform(-0.2, 0.2, n)
    u0 = W.initial_macro(NM)
    v0 = np.zeros(int(W.offsets(lv)[-1]))
    ts = oracle_for(NM, lv, a, None, dt=0.01)
    J_ref, g_ref = adjoint.gradient(ts, u0, v0, steps)
    g = gpu_for(NM, lv, a, None, dt=0.01, rtol=1e-13, checkpoint_every=2, flags=tsm.TSM_FLAG_MACRO_PCG)
    try:
        g.set_state(u0, v0)
        J, dJ = g.gradient(steps)
        dJ = dJ.cpu().numpy()
    finally:
        g.close()
    assert abs(J - J_ref) <= 1e-9 * abs(J_ref)
    assert rel(dJ, g_ref) <= 1e-9
