"""Hand-written adjoint on the GPU: against the oracle's discrete adjoint,
against central finite differences of the GPU forward, invariance under the
checkpoint spacing (the segment recompute is bitwise equal to the forward),
and the autograd wrapper."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import banner, gpu_for, oracle_for, rel
from oracle import adjoint

pytestmark = pytest.mark.gpu


def _case(NM, levels, seed, steps):
    rng = np.random.default_rng(seed)
    n = (NM + 1) ** 2
    lv = rng.choice(np.asarray(levels), n).astype(np.int32)
    a = rng.uniform(-0.2, 0.2, n)
    u0 = W.initial_macro(NM)
    v0 = np.zeros(int(W.offsets(lv)[-1]))
    return lv, a, u0, v0


@pytest.mark.parametrize("precision,rtol,tol", [("fp64", 1e-13, 1e-9), ("fp32_refine", 1e-11, 1e-7)])
@pytest.mark.parametrize("NM,levels,steps,ck", [(3, [4, 8, 16], 6, 4), (4, [16, 32, 64], 5, 2)])
def test_gradient_matches_oracle_adjoint(NM, levels, steps, ck, precision, rtol, tol):
    lv, a, u0, v0 = _case(NM, levels, 7 + NM, steps)
    banner(f"adjoint NM={NM} levels={levels} steps={steps} ck={ck} {precision}")
    ts = oracle_for(NM, lv, a, None, dt=0.01)
    J_ref, g_ref = adjoint.gradient(ts, u0, v0, steps)
    g = gpu_for(NM, lv, a, None, dt=0.01, precision=precision, rtol=rtol, checkpoint_every=ck)
    try:
        g.set_state(u0, v0)
        J, dJ = g.gradient(steps)
        dJ = dJ.cpu().numpy()
    finally:
        g.close()
    assert abs(J - J_ref) <= tol * abs(J_ref)
    assert rel(dJ, g_ref) <= tol
    bnd = W.macro_boundary_mask(NM)
    assert np.abs(dJ[bnd]).max() == 0.0


def test_checkpoint_spacing_is_bitwise_invisible_and_state_restored():
    NM, steps = 4, 7
    lv, a, u0, v0 = _case(NM, [16, 32], 3, steps)
    outs = []
    for ck in (1, 3, 7, 10):
        banner(f"checkpoint_every={ck}")
        g = gpu_for(NM, lv, a, None, dt=0.01, checkpoint_every=ck)
        try:
            g.set_state(u0, v0)
            g.step(2)
            u_before = g.macro().cpu().numpy()
            v_before = g.micro().cpu().numpy()
            J, dJ = g.gradient(steps)
            assert np.array_equal(g.macro().cpu().numpy(), u_before)
            assert np.array_equal(g.micro().cpu().numpy(), v_before)
            outs.append((J, dJ.cpu().numpy()))
        finally:
            g.close()
    for J, dJ in outs[1:]:
        assert J == outs[0][0]
        assert np.array_equal(dJ, outs[0][1])


def test_refine_gradient_matches_oracle_adjoint_mid_size():
    """The gradient in the measured form (FP32 inner solves inside FP64
    refinement, the gradient's solves to 1e-11, dt = 0.0025, checkpoints
    every 20 steps, rotated cells, amplitudes U[-0.3, 0.3]) on 81 instances
    of 64 x 64 cells over 40 steps, against the oracle's FP64 discrete
    adjoint.  The cells keep their shape under this family, so dJ/da is
    ~3e-7 |J| here and its relative error is ~1e3 x the solver tolerance
    (measured: 2.3e-5 at 1e-8, 9.4e-7 at 1e-10, 1.0e-7 at 1e-11)."""
    NM, steps, ck, dt = 8, 40, 20, 0.0025
    n = (NM + 1) ** 2
    rng = np.random.default_rng(23)
    lv = np.full(n, 64, np.int32)
    a = rng.uniform(-0.3, 0.3, n)
    th = rng.uniform(0.0, np.pi / 8, n)
    u0 = W.initial_macro(NM)
    v0 = np.zeros(int(W.offsets(lv)[-1]))
    banner(f"adjoint mid-size NM={NM} 64^2 steps={steps} ck={ck} fp32_refine rtol 1e-8, gradient 1e-11")
    ts = oracle_for(NM, lv, a, th, dt=dt)
    J_ref, g_ref = adjoint.gradient(ts, u0, v0, steps)
    g = gpu_for(NM, lv, a, th, dt=dt, precision="fp32_refine", rtol=1e-8, grad_rtol=1e-11, checkpoint_every=ck)
    try:
        g.set_state(u0, v0)
        J, dJ = g.gradient(steps)
        dJ = dJ.cpu().numpy()
    finally:
        g.close()
    eJ, eg = abs(J - J_ref) / abs(J_ref), rel(dJ, g_ref)
    banner(f"J rel err {eJ:.2e}, dJ/da rel err {eg:.2e}")
    assert eJ <= 1e-8 and eg <= 1e-6, (eJ, eg)
    assert np.abs(dJ[W.macro_boundary_mask(NM)]).max() == 0.0


def test_gradient_matches_central_differences_of_gpu_forward():
    """Directional derivatives vs central differences of the GPU forward on
    16 seeded unit directions, forward solves at rtol 1e-15, to 1e-6.

    The difference quotient D(h) = (J(a+he) - J(a-he)) / 2h carries a
    truncation error c h^2 + O(h^4) and a rounding error ~ eps |J| / h.  At
    h = 1e-6 the rounding term dominates (|J| / |dJ.e| ~ 1e3 here, so about
    1e-7 .. 1e-5 relative); at h = 2e-3 and 1e-3 it is ~1e-10, and the
    Richardson combination (4 D(h/2) - D(h)) / 3 removes the h^2 term,
    leaving O(h^4) ~ 1e-11.

    The deformation family maps Y onto itself, so J depends on the
    amplitudes only through the discretisation error of the micro meshes:
    at 16x16-32x32 cells |dJ/da| ~ 1e-9 |J|, below what any difference
    quotient resolves in FP64.  The check therefore runs on coarse micro
    meshes with strong coupling, where dJ/da is resolvable."""
    NM, steps = 4, 6
    rng = np.random.default_rng(5)
    n = (NM + 1) ** 2
    lv = rng.choice(np.asarray([2, 3, 4]), n).astype(np.int32)
    a = rng.uniform(-0.3, 0.3, n)
    u0 = W.initial_macro(NM)
    v0 = np.zeros(int(W.offsets(lv)[-1]))
    phys = dict(kappa=3.0, d=0.2)
    dirs = W.fd_directions(n, 16, seed=1)
    g = gpu_for(NM, lv, a, None, dt=0.05, rtol=1e-15, max_iter=5000, **phys)
    errs = []
    try:
        g.set_state(u0, v0)
        J, dJ = g.gradient(steps)
        dJ = dJ.cpu().numpy()

        def quotient(e, h):
            vals = []
            for sgn in (1.0, -1.0):
                g.set_deformation(a + sgn * h * e)
                g.set_state(u0, v0)
                vals.append(g.gradient(steps)[0])
            return (vals[0] - vals[1]) / (2 * h)

        h = 2e-3
        for e in dirs:
            fd = (4.0 * quotient(e, h / 2) - quotient(e, h)) / 3.0
            errs.append(abs(dJ @ e - fd) / abs(fd))
    finally:
        g.close()
    banner(f"FD (Richardson) relative errors: max {max(errs):.2e} median {np.median(errs):.2e}")
    assert max(errs) <= 1e-6, errs


def test_autograd_function():
    import torch
    from paper_2103_17040_amd.autograd import objective
    NM, steps = 3, 4
    lv, a, u0, v0 = _case(NM, [8, 16], 11, steps)
    g = gpu_for(NM, lv, a, None, dt=0.01)
    try:
        at = torch.tensor(a, dtype=torch.float64, device="cuda", requires_grad=True)
        J = objective(at, g, u0, v0, steps)
        (2.5 * J).backward()
        J2, dJ = g.gradient(steps)
        assert float(J) == J2
        assert torch.equal(at.grad, 2.5 * dJ)
    finally:
        g.close()
