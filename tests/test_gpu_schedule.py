"""Launch plans and the autotuner.

The single persistent launch over every mesh size must give the per-size
launches' results bit for bit (same packs, same sums; only the workgroup that
takes a pack differs), also with more packs than workgroups so that
workgroups loop over the queue and the graph replays reset it.  The
autotuner must leave the state as it found it and keep a plan whose results
are those of the plans it chose from.
"""
import json

import numpy as np
import pytest

import workloads as W
from gpu_helpers import banner, gpu_for, rel

pytestmark = pytest.mark.gpu


def _case(NM, levels, seed):
    rng = np.random.default_rng(seed)
    n = (NM + 1) ** 2
    lv = rng.choice(np.asarray(levels, np.int32), size=n)
    a = rng.uniform(-0.3, 0.3, n)
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    return lv, a, th


def _run(NM, lv, a, th, prec, flags, steps, u0, v0, rtol):
    g = gpu_for(NM, lv, a, th, 0.005, precision=prec, rtol=rtol, flags=flags)
    try:
        g.set_state(u0, v0)
        g.step(steps)
        return g.macro().cpu().numpy(), g.micro().cpu().numpy(), g.fluxes().cpu().numpy()
    finally:
        g.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_persistent_matches_per_size_many_packs(prec):
    """NM=24 with 16/32/64 meshes: hundreds of packs over at most one
    workgroup per compute unit, replayed from a graph over several steps."""
    from paper_2103_17040_amd import tsm
    NM = 24
    lv, a, th = _case(NM, [16, 32, 64], 7)
    u0 = W.initial_macro(NM)
    v0 = np.random.default_rng(1).uniform(0, 1, int(W.offsets(lv)[-1]))
    rtol = 1e-12 if prec == "fp64" else 1e-10
    banner(f"persistent vs per-size {prec} NM={NM}")
    ref = _run(NM, lv, a, th, prec, 0, 5, u0, v0, rtol)
    out = _run(NM, lv, a, th, prec, tsm.TSM_FLAG_PERSISTENT, 5, u0, v0, rtol)
    for x, y in zip(ref, out):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("level", [16, 32, 64])
def test_persistent_single_size(level):
    """One packed mesh size: the persistent plan runs that size's own kernel
    with the work queue (more packs than compute units for 16 and 32)."""
    from paper_2103_17040_amd import tsm
    NM = {16: 80, 32: 40, 64: 18}[level]
    n = (NM + 1) ** 2
    rng = np.random.default_rng(level)
    lv = np.full(n, level, np.int32)
    a = rng.uniform(-0.3, 0.3, n)
    th = rng.uniform(0.0, 2.0 * np.pi, n)
    u0 = W.initial_macro(NM)
    v0 = np.random.default_rng(4).uniform(0, 1, int(W.offsets(lv)[-1]))
    banner(f"persistent single size {level}, NM={NM}")
    for prec, rtol in (("fp64", 1e-12), ("fp32_refine", 1e-10)):
        ref = _run(NM, lv, a, th, prec, 0, 3, u0, v0, rtol)
        out = _run(NM, lv, a, th, prec, tsm.TSM_FLAG_PERSISTENT, 3, u0, v0, rtol)
        for x, y in zip(ref, out):
            assert np.array_equal(x, y), prec


def test_persistent_with_generic_sizes():
    """Mesh sizes outside the packed kernels (odd sizes) still go to the
    one-instance-per-workgroup kernel next to the persistent launch."""
    from paper_2103_17040_amd import tsm
    NM = 6
    lv, a, th = _case(NM, [8, 13, 16, 33, 64], 11)
    u0 = W.initial_macro(NM)
    v0 = np.zeros(int(W.offsets(lv)[-1]))
    banner("persistent with generic sizes")
    ref = _run(NM, lv, a, th, "fp32_refine", 0, 3, u0, v0, 1e-10)
    out = _run(NM, lv, a, th, "fp32_refine", tsm.TSM_FLAG_PERSISTENT, 3, u0, v0, 1e-10)
    for x, y in zip(ref, out):
        assert np.array_equal(x, y)


def test_autotune_restores_state_and_keeps_results(tmp_path):
    from paper_2103_17040_amd import tsm
    NM = 12
    lv, a, th = _case(NM, [16, 32, 64], 5)
    u0 = W.initial_macro(NM)
    v0 = np.random.default_rng(3).uniform(0, 1, int(W.offsets(lv)[-1]))
    banner("autotune")
    ref = _run(NM, lv, a, th, "fp32_refine", 0, 4, u0, v0, 1e-10)
    g = gpu_for(NM, lv, a, th, 0.005, precision="fp32_refine", rtol=1e-10)
    try:
        g.set_state(u0, v0)
        before = (g.macro().cpu().numpy(), g.micro().cpu().numpy(), g.fluxes().cpu().numpy())
        cache = str(tmp_path / "plans.json")
        res = g.autotune(steps=2, cache=cache)
        after = (g.macro().cpu().numpy(), g.micro().cpu().numpy(), g.fluxes().cpu().numpy())
        for x, y in zip(before, after):
            assert np.array_equal(x, y)
        ms = res["ms_per_step"]
        timed = {k: v for k, v in ms.items() if v > 0}
        assert all(ms[k] > 0 for k in ("per_size", "persistent", "generic", "chosen"))
        assert res["flags"] & ~tsm.PLAN_BITS == 0
        assert res["plan"] == tsm.plan_name(res["flags"])
        # the chosen plan is at least as fast as every plan timed; the
        # matrix-free operator is not tried unless asked for
        assert ms["chosen"] == min(timed.values())
        assert ms["assembled_operator"] < 0 and not res["flags"] & tsm.TSM_FLAG_MATRIX_FREE
        assert g.stats()["steps_taken"] == 0
        g.step(4)
        out = (g.macro().cpu().numpy(), g.micro().cpu().numpy(), g.fluxes().cpu().numpy())
        # a second call reads the cached plan
        assert g.autotune(steps=2, cache=cache) == json.load(open(cache))[next(iter(json.load(open(cache))))]
    finally:
        g.close()
    for x, y in zip(ref, out):
        # the per-size plan is the reference's own; the persistent plan sums
        # in the same order, the generic kernels in another
        generic = tsm.TSM_FLAG_GENERIC | tsm.TSM_FLAG_GENERIC_16 | tsm.TSM_FLAG_GENERIC_32 | tsm.TSM_FLAG_GENERIC_64
        if not res["flags"] & generic:
            assert np.array_equal(x, y)
        else:
            assert rel(x, y) <= 1e-8


def test_per_size_generic_flags():
    """Moving every packed size to the one-instance-per-workgroup kernel is
    the generic plan bit for bit; a size flag for a size the batch lacks
    changes nothing; moving one size keeps results within the solver
    tolerance of the packed plan."""
    from paper_2103_17040_amd import tsm
    NM = 10
    lv, a, th = _case(NM, [16, 64], 9)
    u0 = W.initial_macro(NM)
    v0 = np.random.default_rng(2).uniform(0, 1, int(W.offsets(lv)[-1]))
    banner("per-size generic flags")
    all3 = tsm.TSM_FLAG_GENERIC_16 | tsm.TSM_FLAG_GENERIC_32 | tsm.TSM_FLAG_GENERIC_64
    for prec, rtol in (("fp64", 1e-12), ("fp32_refine", 1e-10)):
        gen = _run(NM, lv, a, th, prec, tsm.TSM_FLAG_GENERIC, 3, u0, v0, rtol)
        out = _run(NM, lv, a, th, prec, all3, 3, u0, v0, rtol)
        for x, y in zip(gen, out):
            assert np.array_equal(x, y), prec
        ref = _run(NM, lv, a, th, prec, tsm.TSM_FLAG_PERSISTENT, 3, u0, v0, rtol)
        out = _run(NM, lv, a, th, prec, tsm.TSM_FLAG_PERSISTENT | tsm.TSM_FLAG_GENERIC_32, 3, u0, v0, rtol)
        for x, y in zip(ref, out):
            assert np.array_equal(x, y), prec
        for bit in (tsm.TSM_FLAG_GENERIC_16, tsm.TSM_FLAG_GENERIC_64):
            out = _run(NM, lv, a, th, prec, tsm.TSM_FLAG_PERSISTENT | bit, 3, u0, v0, rtol)
            for x, y in zip(ref, out):
                assert rel(x, y) <= (1e-10 if prec == "fp64" else 1e-8), (prec, bit)
