"""Extrapolated start of the forward refinement solves: the first inner FP32
solve of a time step starts from the increment extrapolated from the last
two steps.  The FP64 residual of the refinement takes the guess in exactly,
so the results meet the oracle with and without it (implicit Euler step of
the coupled system, Section 2.1 model problem, Schur form); the guess only
saves inner iterations.  The history restarts with the state."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import banner, gpu_for, oracle_for, rel

pytestmark = pytest.mark.gpu


def _case(NM, levels, seed):
    n = (NM + 1) ** 2
    rng = np.random.default_rng(seed)
    lv = rng.choice(np.asarray(levels), n).astype(np.int32)
    a = rng.uniform(-0.3, 0.3, n)
    th = rng.uniform(0.0, np.pi / 8, n)
    return lv, a, th


def _run(NM, lv, a, th, dt, steps, u0, v0, flags, precision="fp32_refine", rtol=1e-10):
    g = gpu_for(NM, lv, a, th, dt=dt, precision=precision, rtol=rtol, flags=flags)
    try:
        g.set_state(u0, v0)
        us, Fs, its = [g.macro().cpu().numpy()], [], []
        for _ in range(steps):
            g.step(1)
            us.append(g.macro().cpu().numpy())
            Fs.append(g.fluxes().cpu().numpy())
            its.append(g.stats()["iters_mean"])
        return {"u": np.array(us), "F": np.array(Fs), "v": g.micro().cpu().numpy(), "iters": np.array(its)}
    finally:
        g.close()


@pytest.mark.parametrize("precision,rtol,tol", [("fp32_refine", 1e-10, 1e-8), ("fp64", 1e-12, 1e-10)])
@pytest.mark.parametrize("plan", ["persistent", "per_size"])
def test_extrapolated_start_matches_oracle_and_saves_iterations(plan, precision, rtol, tol):
    from paper_2103_17040_amd import tsm
    NM, dt, steps = 4, 0.0025, 10
    lv, a, th = _case(NM, [16, 32, 64], 71)
    u0 = W.initial_macro(NM)
    v0 = np.zeros(int(W.offsets(lv)[-1]))
    base = tsm.TSM_FLAG_PERSISTENT if plan == "persistent" else 0
    banner(f"extrapolated start, {plan}, {precision}, NM={NM} levels 16/32/64, {steps} steps")
    ref = oracle_for(NM, lv, a, th, dt).run(u0, v0, steps)
    on = _run(NM, lv, a, th, dt, steps, u0, v0, base, precision, rtol)
    off = _run(NM, lv, a, th, dt, steps, u0, v0, base | tsm.TSM_FLAG_NO_EXTRAPOLATION, precision, rtol)
    for name, out in (("on", on), ("off", off)):
        eu, eF, ev = rel(out["u"], ref["u"]), rel(out["F"], ref["F"]), rel(out["v"], ref["v"])
        banner(f"  {name}: rel u {eu:.2e} F {eF:.2e} v {ev:.2e}; iterations {out['iters'].round(1).tolist()}")
        assert eu <= tol and eF <= tol and ev <= tol, name
    # the two runs differ only by rounding and the solver tolerance
    assert rel(on["v"], off["v"]) <= tol
    # the first step has no history (identical); from the third on the guess
    # is the linear extrapolation and must save iterations (refinement: inner
    # iterations)
    assert on["iters"][0] == off["iters"][0]
    # (the FP64 solves of these small, mass-dominated systems take ~6
    # iterations, so the guess saves less of them)
    assert on["iters"][3:].sum() < (0.9 if precision == "fp32_refine" else 0.95) * off["iters"][3:].sum()


def test_history_restarts_with_the_state():
    """After set_state the history is gone: a context that has stepped before
    continues exactly (bitwise) like a fresh context started from that state,
    and set_flags restarts it too."""
    from paper_2103_17040_amd import tsm
    NM, dt = 3, 0.0025
    lv, a, th = _case(NM, [16, 32, 64], 5)
    flags = tsm.TSM_FLAG_PERSISTENT
    u0 = W.initial_macro(NM)
    v0 = np.zeros(int(W.offsets(lv)[-1]))
    rng = np.random.default_rng(9)
    u1 = u0 * (1.0 + 0.05 * rng.standard_normal(u0.shape))
    v1 = rng.uniform(0.0, 0.2, v0.shape)
    banner("history restart at set_state / set_flags")
    g = gpu_for(NM, lv, a, th, dt=dt, precision="fp32_refine", rtol=1e-10, flags=flags)
    try:
        g.set_state(u0, v0)
        g.step(5)
        g.set_state(u1, v1)
        g.step(4)
        cont = (g.macro().cpu().numpy(), g.micro().cpu().numpy())
        g.set_state(u1, v1)
        g.step(2)
        g.set_flags(flags)
        g.step(2)
        reflag = (g.macro().cpu().numpy(), g.micro().cpu().numpy())
    finally:
        g.close()
    f = gpu_for(NM, lv, a, th, dt=dt, precision="fp32_refine", rtol=1e-10, flags=flags)
    try:
        f.set_state(u1, v1)
        f.step(4)
        fresh = (f.macro().cpu().numpy(), f.micro().cpu().numpy())
        f.set_state(u1, v1)
        f.step(2)
        f.set_flags(flags)
        f.step(2)
        fresh_reflag = (f.macro().cpu().numpy(), f.micro().cpu().numpy())
    finally:
        f.close()
    for x, y in zip(cont, fresh):
        assert np.array_equal(x, y)
    for x, y in zip(reflag, fresh_reflag):
        assert np.array_equal(x, y)
