"""Write the oracle's expected outputs for the full-size parity tests.

    python tests/golden/make_goldens.py [batched_fp64 uneven_mixed adjoint_fp64 stationary_caseB]

Calls only the FP64 oracle and the seeded input generators (seed 0).  Each
file stores a compact, sampled set of outputs (compressed .npz, no pickles):
macro fields at a few steps, all fluxes of the first and last step, the micro
field of a few sampled instances at the end, the response functionals, and
for the adjoint workload J and dJ/da; for the stationary Case B solve
(81 macro x 4225 micro DoFs, Table 3 parameters with a unit micro source)
u, w and v of nine instances spread over the macro mesh; for a 9409-node
macro mesh with 2 x 2 micro meshes u, w and v.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import adjoint, stationary, twoscale  # noqa: E402

SAMPLE_STEPS = (1, 2, 10)


def sampled_instances(w, lv, count=12, seed=0):
    """Interior instances spread over the batch, covering every mesh size."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 4242]))
    interior = np.flatnonzero(~W.macro_boundary_mask(w.macro_cells))
    picks = []
    for lvl in sorted(set(lv.tolist())):
        cand = interior[lv[interior] == lvl]
        picks += list(rng.choice(cand, size=min(len(cand), max(2, count // len(set(lv.tolist())))), replace=False))
    return np.array(sorted(set(int(i) for i in picks)), dtype=np.int64)


def forward_golden(name):
    w, a, th, lv = W.make(name, 0)
    prm = twoscale.Params(w.macro_cells, w.dt, w.D, w.d, w.kappa, w.p, w.sigma)
    t0 = time.time()
    ts = twoscale.TwoScale(prm, lv, a, th)
    print(f"{name}: setup {time.time() - t0:.1f} s", flush=True)
    u = W.initial_macro(w.macro_cells)
    v = np.zeros(int(ts.offsets[-1]))
    steps = sorted(set(SAMPLE_STEPS + (w.steps,)))
    us, F1 = {}, None
    t0 = time.time()
    for n in range(1, w.steps + 1):
        u, v, F = ts.step(u, v)
        if n == 1:
            F1 = F
        if n in steps:
            us[n] = u.copy()
    print(f"{name}: {w.steps} steps {time.time() - t0:.1f} s", flush=True)
    inst = sampled_instances(w, lv)
    vs = [v[ts.offsets[i]:ts.offsets[i + 1]] for i in inst]
    out = {
        "steps": np.array(steps, dtype=np.int64),
        "u": np.stack([us[n] for n in steps]),
        "F_first": F1, "F_last": F,
        "inst": inst,
        "v_len": np.array([len(x) for x in vs], dtype=np.int64),
        "v_last": np.concatenate(vs),
        "beta": ts.beta, "len": ts.len,
        "J": np.array(ts.observable(u)),
    }
    np.savez_compressed(os.path.join(HERE, f"{name}_seed0.npz"), **out)


def adjoint_golden(name="adjoint_fp64"):
    w, a, th, lv = W.make(name, 0)
    prm = twoscale.Params(w.macro_cells, w.dt, w.D, w.d, w.kappa, w.p, w.sigma)
    t0 = time.time()
    ts = twoscale.TwoScale(prm, lv, a, th)
    u0 = W.initial_macro(w.macro_cells)
    v0 = np.zeros(int(ts.offsets[-1]))
    J, g = adjoint.gradient(ts, u0, v0, w.steps)
    print(f"{name}: gradient {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, f"{name}_seed0.npz"), J=np.array(J), g=g)


def stationary_golden(name="stationary_caseB"):
    lv, per, _, _ = W.stationary_case("B", 8, 64)
    t0 = time.time()
    out = stationary.solve(stationary.StationaryParams(macro_cells=8), lv, per,
                           stationary.constant_data(fv=1.0))
    print(f"{name}: solve {time.time() - t0:.1f} s", flush=True)
    inst = np.array([0, 8, 20, 31, 40, 49, 60, 72, 80], dtype=np.int64)
    np.savez_compressed(os.path.join(HERE, f"{name}.npz"), u=out["u"], w=out["w"], inst=inst,
                        v=np.concatenate([out["v"][i] for i in inst]))


def stationary_large_macro_golden(name="stationary_large_macro"):
    """Case B map on a 97 x 97 macro mesh (9409 nodes) with 2 x 2 micro
    meshes, unit micro source and f^u = 0.2: u, w and v of every instance."""
    lv, per, _, _ = W.stationary_case("B", 96, 2)
    t0 = time.time()
    out = stationary.solve(stationary.StationaryParams(macro_cells=96), lv, per,
                           stationary.constant_data(fv=1.0, fu=0.2))
    print(f"{name}: solve {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, f"{name}.npz"), u=out["u"], w=out["w"], v=np.concatenate(out["v"]))


if __name__ == "__main__":
    names = sys.argv[1:] or ["batched_fp64", "uneven_mixed", "adjoint_fp64", "stationary_caseB",
                             "stationary_large_macro"]
    for nm in names:
        if nm == "adjoint_fp64":
            adjoint_golden(nm)
        elif nm == "stationary_caseB":
            stationary_golden(nm)
        elif nm == "stationary_large_macro":
            stationary_large_macro_golden(nm)
        else:
            forward_golden(nm)
