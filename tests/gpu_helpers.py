"""Shared helpers of the GPU parity tests: run the same seeded case through
the HIP library and through the FP64 oracle."""
import sys

import numpy as np

import workloads as W
from oracle import twoscale


def banner(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def rel(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (den if den > 0 else 1.0))


def oracle_for(NM, levels, a, theta=None, dt=0.01, **kw):
    prm = twoscale.Params(NM, dt, **kw)
    return twoscale.TwoScale(prm, levels, a, theta)


def gpu_for(NM, levels, a, theta=None, dt=0.01, precision="fp64", **kw):
    from paper_2103_17040_amd import TwoScaleBatch
    return TwoScaleBatch(NM, levels, a, theta, dt=dt, precision=precision, **kw)


def run_both(NM, levels, a, theta, dt, steps, u0, v0, precision="fp64", rtol=1e-12, gpu_kw=None, **phys):
    """Returns (oracle dict, gpu dict) with u (steps+1, n), F (steps, n), v final."""
    banner(f"NM={NM} levels={sorted(set(np.asarray(levels).tolist()))} steps={steps} {precision} rtol={rtol}")
    ts = oracle_for(NM, levels, a, theta, dt, **phys)
    ref = ts.run(u0, v0, steps)
    g = gpu_for(NM, levels, a, theta, dt, precision=precision, rtol=rtol, **phys, **(gpu_kw or {}))
    try:
        g.set_state(u0, v0)
        us, Fs = [g.macro().cpu().numpy()], []
        for _ in range(steps):
            g.step(1)
            us.append(g.macro().cpu().numpy())
            Fs.append(g.fluxes().cpu().numpy())
        out = {"u": np.array(us), "F": np.array(Fs), "v": g.micro().cpu().numpy(), "stats": g.stats()}
    finally:
        g.close()
    return ref, out, ts


def workload_case(name, seed=0):
    w, a, th, lv = W.make(name, seed)
    u0 = W.initial_macro(w.macro_cells)
    v0 = np.zeros(int(W.offsets(lv)[-1]))
    phys = dict(D=w.D, d=w.d, kappa=w.kappa, p=w.p, sigma=w.sigma)
    return w, a, th, lv, u0, v0, phys
