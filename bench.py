"""Benchmark of the two-scale micro batch on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one implicit-Euler time step of the whole hot path: every micro
solve of the batch (FP32 PCG inside FP64 refinement, or plain FP64), the
Robin flux averages, the macro coupling solve and the state update, replayed
as one captured hipGraph.  Inputs are synthetic and seeded (module
workloads); they are resident in HBM before the timed region starts.

Prints one JSON line.  `value` is micro DoF-updates/s of the FP32+refinement
form (sum over instances of (N_i+1)^2 per step); the plain FP64 form on the
same workload and tolerance is timed beside it, the dominant kernel's
duration is measured with HIP events on the library's stream for the
roofline, and the FP64 oracle is timed on a bounded sample on the host.
Side legs: the gradient (checkpointed forward + adjoint) and the paper's
alternating macro/micro coupling timed against the exact coupling step, on
the same workload; a general map given by Jacobian tables on the uneven
4225-instance batch; every output's error against the oracle's stored
outputs for three other workloads (tests/golden).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

PEAK_HBM_GBS = 8000.0
# FP64 FMA and non-packed FP32 FMA issue at 64 lanes per clock per CU on
# gfx950: 256 CUs * 2.4 GHz * 64 FMA * 2 flop = 78.6 TFLOP/s for either type
# (packed FP32, which would double FP32, is not used).  The published FP32
# vector figure (157.3 TFLOP/s) counts packed FP32; both are reported.
PEAK_ALU_TFLOPS = 78.6
PEAK_FP32_PUBLISHED_TFLOPS = 157.3
# The state floor of one micro DoF-update: read v0 and M w, write v (FP64).
# Everything else a solve touches can stay on chip for a whole instance.
B_FLOOR = 24.0

# Algorithmic work per micro DoF-update of the micro kernel.
# Flops: per PCG iteration 9-point stencil (9 FMA), p.q, x/d update, r update,
# z = D^{-1} r, r.z, r.r, p update = 15 FMA + 1 MUL = 31 flops; per FP64
# residual update of the refinement S d with S = S32 + Slo (9 ADD + 9 FMA),
# r -= ||r|| S d, r.r, x += ||r|| d = 33 flops; per solve x0 = X0 + u w,
# K x0, M x0 (9 FMA each), ||b||^2 and ||r||^2 = 43 flops.
FLOP_ITER, FLOP_SWEEP, FLOP_SOLVE = 31.0, 33.0, 43.0   # (refine: S x0 replaces M x0 in the solve term)
# The matrix-free operator of a refinement solve, per DoF (one cell per
# DoF): at each of 4 Gauss points M = I + aG (2 FMA), J (MUL + FMA), 1/J
# (reciprocal + 2 Newton steps, 4 FMA), C = adj adj^T / J (3 x (MUL, FMA,
# MUL)) and the moments of C and J (19 FMA) = 69 flops; 10 element
# entries (3 ADD + 1 FMA); K x0 on the 4 corners (16 FMA); the node sums
# (~10 ADD): 4 * 69 + 50 + 32 + 10 = 368 flops.
FLOP_OPERATOR_MF = 368.0
# The extrapolated start of the first inner solve, per DoF: e1 = X0 - hx and
# the extrapolation 3 (e1 - e2) + e3 (3), the guess's residual r - S d0 (9 FMA
# + 1 ADD) and the two dot products of the guessed and plain residuals (2 x
# (MUL + FMA)) = 24 flops.
FLOP_GUESS = 24.0
# The separable mass of the start residual (default for the analytic family),
# per DoF: the column pass along R+2 rows for R nodes (5 x 3 FMA a row, ~20
# FMA a node at R = 6), the row pass (15 FMA) and the 1/dt scale (1 FMA) = 72
# flops in place of K x0 (18); the refinement adds the low part Slo x0 at
# its first update (9 FMA = 18 flops).
FLOP_MASS, FLOP_LOW0 = 72.0 - 18.0, 18.0
# Bytes the instance-resident micro kernel must move per DoF per step
# (algorithmic: the vectors of the iterations stay on chip; operators are read
# from their symmetric upper-half planes, 5 coefficients per node):
#   both forms: x0 = v0 + u w (read v0, w: 16), r = -K x0 (FP64 K, 40; none
#               with the separable mass, which comes from per-level tables),
#               write x (8); b^T x for the flux average is a separate pass
#               over the 4N boundary nodes (b and x: 16 B each, below 1 B
#               per node of the mesh)
#   refine:     the FP32 stencil once (20; it also gives ||b|| = ||S x0 + r||)
#               and the FP32 low part of the stencil, copied to LDS once per
#               solve for the FP64 residual updates (20)
#   FP64:       the FP64 stencil once, into registers for the whole solve
#               (40; it also gives ||b|| = ||S x0 + r|| and diag^{-1})
B_START, B_K, B_END = 16.0, 40.0, 8.0
B_S64, B_S32, B_SLO = 40.0, 20.0, 20.0
#   extrapolated start (packed kernels on the assembled operator): the
#   previous X0 and the two increments before it read and written in FP32
#   (12 + 12)
B_HIST = 24.0


PACKED_LEVELS = (16, 32, 64)
GENERIC_SLOTS = (1, 2, 3, 5, 9, 17)      # nodes per lane of the generic kernel (256 lanes)


def packed_under(N, flags):
    """Whether the launch plan `flags` solves N x N instances with a packed kernel."""
    per_size = {16: 1 << 6, 32: 1 << 7, 64: 1 << 8}
    return N in PACKED_LEVELS and not (flags & (1 << 3)) and not (flags & per_size[N])


def matrix_free(N, flags, refine):
    """Whether the packed refinement kernel evaluates the operator from the
    amplitudes (the matrix-free flag on a per-size plan) instead of reading
    the assembled planes."""
    return refine and packed_under(N, flags) and bool(flags & (1 << 9)) and not (flags & (1 << 4))


def extrapolated(N, flags, refine):
    """Whether the packed kernel starts its solve (refinement: its first inner
    solve) from the extrapolated increment (assembled operator, unless
    switched off)."""
    return packed_under(N, flags) and not matrix_free(N, flags, refine) and not (flags & (1 << 13))


def mass_free(N, flags, refine):
    """Whether the packed kernel on the assembled operator forms its start
    residual with the separable mass instead of reading K (analytic family;
    unless the assembled-start flag is set)."""
    return packed_under(N, flags) and not matrix_free(N, flags, refine) and not (flags & (1 << 14))


def micro_bytes_per_dof(N, flags, refine, iters, sweeps):
    """Algorithmic HBM bytes per DoF-update of the micro kernel that solves an
    N x N instance under the launch plan `flags` (packed kernels: symmetric
    planes as above, or none when the operator is evaluated matrix-free;
    generic kernel: full 9-coefficient rows, FP64 M for b, its stencil held
    in registers when the instance fits, else streamed)."""
    if packed_under(N, flags):
        bdot = 16.0 * 4 * N / (N + 1) ** 2      # the boundary pass for b^T x
        if matrix_free(N, flags, refine):
            return B_START + B_END + bdot
        hist = B_HIST if extrapolated(N, flags, refine) else 0.0
        kb = 0.0 if mass_free(N, flags, refine) else B_K
        if refine:
            return B_START + kb + B_S32 + B_SLO + B_END + hist + bdot
        return B_START + kb + B_S64 + B_END + hist + bdot
    slots = next(s for s in GENERIC_SLOTS if s * 256 >= (N + 1) ** 2)
    if refine:   # FP32 stencil once (resident) or per inner iteration; FP64 rows per residual
        return 16 + 72 + 72 * sweeps + (36 if slots <= 9 else 36 * iters) + 16
    return 16 + 72 + 72 + (0 if slots <= 5 else 72 * iters) + 16


def streaming_bytes(refine, iters, sweeps):
    """Bytes per DoF-update of a PCG that streams its vectors through HBM
    every iteration (10 words per iteration for a two-pass fused PCG, the FP64
    residual sweeps at 6 words, 3 state words): the reference bandwidth model
    the resident kernel is compared with."""
    if refine:
        return iters * 10 * 4 + max(sweeps - 1, 1) * 6 * 8 + 3 * 8
    return iters * 10 * 8 + 3 * 8


KERNEL_SOURCES = ("micro_packed.hip", "device_common.h", "tsm_internal.h")
COUNTERS = os.path.join(ROOT, "profiles", "micro_kernel_counters.json")


def code_text(src):
    """C++ source without its comments and blank lines (what the counters
    depend on)."""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(line.rstrip() for line in src.splitlines() if line.strip())


def kernel_source_hash():
    """sha256 of the micro kernels' code (comments excluded)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2103_17040_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
    return h.hexdigest()


def measured_traffic(workload, form):
    """Counter-measured HBM bytes per launch of the micro kernel (scaled
    FETCH_SIZE + WRITE_SIZE) from the committed profile, or None when the
    kernel sources changed since the counters were taken."""
    try:
        with open(COUNTERS) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    ent = rec.get("launches", {}).get(f"{workload}/{form}")
    return None if ent is None else ent["fetch_bytes"] + ent["write_bytes"]


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


PLAN_FLAGS = {"per_size": 0, "persistent": 1 << 4, "generic": 1 << 3,
              "persistent+generic16": (1 << 4) | (1 << 6)}


def run_form(w, a, th, lv, precision, steps, warmup, rtol, adjoint_steps=0, plan="auto", fp_steps=0):
    import torch
    from paper_2103_17040_amd import TwoScaleBatch, tsm
    g = TwoScaleBatch(w.macro_cells, lv, a, th, D=w.D, d=w.d, kappa=w.kappa, p=w.p, dt=w.dt,
                      sigma=w.sigma, precision=precision, rtol=rtol, grad_rtol=w.grad_rtol,
                      checkpoint_every=max(w.checkpoint_every, 1))
    try:
        setup_ms = g.stats()["setup_ms"]
        u0 = W.initial_macro(w.macro_cells)
        g.set_state(u0, None)
        g.step(warmup)
        # launch plan: per-size launches, one persistent launch, or the
        # one-instance-per-workgroup kernels, timed on this state (restored)
        if plan == "auto":
            plan = g.autotune(steps=3)
        else:
            g.set_flags(PLAN_FLAGS[plan])
            plan = {"flags": PLAN_FLAGS[plan], "ms_per_step": None}
        # the state the timed steps start from, so that the roofline pass
        # times the same steps
        u_start, v_start = g.macro().clone(), g.micro().clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        st = g.stats()
        # roofline pass: the same steps again, direct launches bracketed by
        # HIP events, one call per step so that the inner iterations and
        # sweeps of every step enter the work model (they fall over the run
        # as the extrapolated start improves)
        g.set_flags(tsm.TSM_FLAG_TIMING | plan["flags"])
        g.set_state(u_start, v_start)
        acc = {"micro_ms": 0.0, "macro_ms": 0.0, "iters_mean": 0.0, "sweeps_mean": 0.0}
        for _ in range(steps):
            g.step(1)
            s1 = g.stats()
            for k in acc:
                acc[k] += s1[k]
        tst = dict(s1)
        tst.update(micro_ms=acc["micro_ms"], macro_ms=acc["macro_ms"], timed_steps=steps,
                   iters_mean_run=acc["iters_mean"] / steps, sweeps_mean_run=acc["sweeps_mean"] / steps)
        g.set_flags(plan["flags"])
        fp = None
        if fp_steps > 0:
            # the paper's alternating coupling on the same workload: every
            # iteration is a full batch of micro solves
            g.set_flags(plan["flags"] | tsm.TSM_FLAG_FIXED_POINT)
            g.set_state(u0, None)
            g.step(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            iters = []
            for _ in range(fp_steps):
                g.step(1)
                iters.append(g.stats()["fp_iters_last"])
            torch.cuda.synchronize()
            tf = time.perf_counter() - t0
            g.set_flags(plan["flags"])
            fp = {"steps": fp_steps, "ms_per_step": tf / fp_steps * 1e3, "iterations": iters}
        adj = None
        if adjoint_steps > 0:
            # gradient of int u(T)^2 from the initial state: checkpointed
            # forward, then segment recompute + adjoint + gradient
            g.set_state(u0, None)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            J, dJ = g.gradient(adjoint_steps)
            torch.cuda.synchronize()
            tg = time.perf_counter() - t0
            gs = g.stats()
            adj = {"steps": adjoint_steps, "checkpoint_every": max(w.checkpoint_every, 1),
                   "grad_rtol": w.grad_rtol if w.grad_rtol > 0 else rtol,
                   "J": J, "grad_norm": float(dJ.norm()), "wall_s": tg,
                   "forward_ms": gs["grad_forward_ms"], "backward_ms": gs["grad_backward_ms"]}
        plan = {"plan": tsm.plan_name(plan["flags"]), "flags": plan["flags"], "ms_per_step": plan["ms_per_step"]}
        return {"t": t, "setup_ms": setup_ms, "stats": st, "timing": tst, "n_dofs": g.n_micro, "adjoint": adj,
                "plan": plan, "fixed_point": fp}
    finally:
        g.close()


def general_map_leg(steps, precision="fp32_refine", rtol=1e-10):
    """A map outside the sinusoidal family, given by its Jacobian tables, on
    the uneven 4225-instance batch (16/32/64 cells): setup from the tables
    against setup from amplitudes on the same meshes, and the step time."""
    import torch
    from paper_2103_17040_amd import TwoScaleBatch
    w, a, th, lv = W.make("uneven_mixed", 0)
    per, Fc, Fb = W.jacobian_tables(lv, W.polynomial_map_jacobian, W.polynomial_map_params(len(lv), seed=2))
    del per
    u0 = W.initial_macro(w.macro_cells)
    kw = dict(D=w.D, d=w.d, kappa=w.kappa, p=w.p, dt=w.dt, sigma=w.sigma, precision=precision, rtol=rtol)
    g = TwoScaleBatch(w.macro_cells, lv, a, th, **kw)
    setup_analytic = g.stats()["setup_ms"]
    g.close()
    g = TwoScaleBatch(w.macro_cells, lv, jacobians=(Fc, Fb), **kw)
    try:
        setup_tables = g.stats()["setup_ms"]
        g.set_state(u0, None)
        g.step(1)
        plan = g.autotune(steps=2)      # the launch plan a user's autotune call picks (state restored)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        st = g.stats()
    finally:
        g.close()
    return {"workload": f"{len(lv)} instances, 16/32/64 cells (uneven batch), polynomial map from Jacobian tables",
            "table_bytes": 8 * (Fc.size + Fb.size), "setup_ms_tables": setup_tables,
            "setup_ms_analytic": setup_analytic, "steps": steps, "ms_per_step": t * 1e3, "plan": plan["plan"],
            "micro_dofs": int(W.offsets(lv)[-1]), "iters_mean": st["iters_mean"], "precision": precision}


def macro_pcg_leg(steps=5):
    """The macro solve of a heterogeneous batch: 4225 instances of 16/32
    cells scaled by s ~ U[0.1, 8] (so the micro responses beta_i spread over
    a factor of 50), dt = 30, kappa = 10 and D = 1e-6, where the sweep's
    contraction bound exceeds 0.5 and the library solves A_M by PCG with the
    sine-basis preconditioner; per-phase times from TSM_FLAG_TIMING."""
    from paper_2103_17040_amd import TwoScaleBatch, tsm
    NM = 64
    n = (NM + 1) ** 2
    rng = np.random.default_rng(3)
    lv = rng.choice(np.array([16, 32], np.int32), n)
    sc = rng.uniform(0.1, 8.0, n)
    _, Fc, Fb = W.jacobian_tables(lv, W.scaling_map_jacobian, [(x,) for x in sc])
    g = TwoScaleBatch(NM, lv, jacobians=(Fc, Fb), dt=30.0, D=1e-6, d=0.5, kappa=10.0, p=1.0, precision="fp64",
                      rtol=1e-10, max_iter=20000, flags=tsm.TSM_FLAG_TIMING)
    try:
        g.set_state(W.initial_macro(NM), None)
        g.step(1)
        g.step(steps)
        st = g.stats()
    finally:
        g.close()
    ts = max(st["timed_steps"], 1)
    return {"workload": f"{n} instances, 16/32 cells, cells scaled by U[0.1, 8], dt 30, kappa 10, D 1e-6",
            "macro_contraction_bound": st["macro_contraction"], "macro_pcg_iters": st["macro_pcg_iters"],
            "macro_ms_per_step": st["macro_ms"] / ts, "micro_ms_per_step": st["micro_ms"] / ts,
            "steps": steps, "unconverged": st["unconverged"]}


GOLD = os.path.join(ROOT, "tests", "golden")


def _rel(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.linalg.norm(ref))
    return float(np.linalg.norm(x - ref) / (den if den > 0 else 1.0))


def stationary_leg(reps, parity=True, flags=0):
    """The paper's stationary three-field system (Section 2.1 model) on the
    Case B map with the Table 3 parameters and a unit micro source (the
    Table 3 data alone give the constant state), at the paper's size (81
    macro x 4225 micro DoFs, checked against the oracle's solution stored in
    tests/golden) and on a 4225-node macro mesh (17.8M micro DoFs).  Each
    solve: three batched FP64 micro PCG solves per instance, the macro PCG,
    the micro fields; times from HIP events around the solve, median of
    `reps` solves after one warm-up."""
    import statistics
    from paper_2103_17040_amd import StationarySystem
    res = {}
    for name, NM in (("case_B_81x4225", 8), ("case_B_4225x4225", 64)):
        lv, _, Fc, Fb = W.stationary_case("B", NM, 64)
        g = StationarySystem(NM, lv, jacobians=(Fc, Fb), fv=1.0, flags=flags)
        try:
            g.solve()
            ms, micro = [], []
            for _ in range(reps):
                u, w, v = g.solve()
                st = g.stats()
                ms.append(st["solve_ms"])
                micro.append(st["micro_ms"])
            u, w, v = (t.cpu().numpy() for t in (u, w, v))
        finally:
            g.close()
        n_micro = int(W.offsets(lv)[-1])
        t_micro = statistics.median(micro) * 1e-3
        dof_iters = n_micro * sum(st["micro_iters_mean"])
        ent = {"macro_nodes": len(lv), "micro_dofs": n_micro, "solve_ms": statistics.median(ms),
               "micro_ms": statistics.median(micro), "micro_iters_mean": st["micro_iters_mean"],
               "micro_iters_max": st["micro_iters_max"], "macro_iters": st["macro_iters"],
               "micro_dof_iterations_per_s": dof_iters / t_micro,
               # a PCG streaming its FP64 vectors: 10 words per DoF and iteration
               "streaming_model_GBs": dof_iters * 80.0 / t_micro / 1e9}
        if flags == 0:
            # the multigrid V-cycle on every mesh size (by default only above
            # 64 cells per side, where it replaces one-workgroup Jacobi CG)
            from paper_2103_17040_amd import tsm
            mg = StationarySystem(NM, lv, jacobians=(Fc, Fb), fv=1.0, flags=tsm.TSM_FLAG_MULTIGRID)
            try:
                mg.solve()
                mms = []
                for _ in range(reps):
                    mg.solve()
                    mst = mg.stats()
                    mms.append(mst["solve_ms"])
            finally:
                mg.close()
            ent["multigrid_all_sizes"] = {"solve_ms": statistics.median(mms),
                                          "micro_iters_mean": mst["micro_iters_mean"],
                                          "micro_iters_max": mst["micro_iters_max"]}
        if parity and NM == 8:
            ref = np.load(os.path.join(GOLD, "stationary_caseB.npz"), allow_pickle=False)
            off = W.offsets(lv)
            vs = np.concatenate([v[off[i]:off[i + 1]] for i in ref["inst"]])
            ent["parity_vs_oracle"] = {"u": _rel(u, ref["u"]), "w": _rel(w, ref["w"]), "v_sampled": _rel(vs, ref["v"])}
        res[name] = ent
    return res


def stationary_oracle_time():
    """The oracle (test infrastructure) on the same Case B problem at the
    paper's size: one monolithic sparse LU solve (scipy), timed on the host."""
    from oracle import stationary as ost
    lv, per, _, _ = W.stationary_case("B", 8, 64)
    t0 = time.perf_counter()
    ost.solve(ost.StationaryParams(macro_cells=8), lv, per, ost.constant_data(fv=1.0))
    return {"solve_s": time.perf_counter() - t0, "kind": "oracle", "cores": 1,
            "sample": "the whole Case B problem at 81 x 4225 DoFs: one sparse LU of the monolithic system"}


def refinement_oracle_time(theta=0.3, sample=12):
    """The oracle's indicator, marking and interpolation (test
    infrastructure) on a sample of the refinement leg's instances, scaled to
    the batch by DoFs; the marking on the whole batch."""
    from oracle import refine as orf
    w, a, th, lv = W.make("uneven_mixed", 0)
    rng = np.random.default_rng(1)
    pick = rng.choice(len(lv), size=sample, replace=False)
    n_b = float(((lv.astype(np.int64) + 1) ** 2).sum())
    n_s = float(((lv[pick].astype(np.int64) + 1) ** 2).sum())
    t0 = time.perf_counter()
    for i in pick:
        N = int(lv[i])
        z = np.linspace(-1.0, 1.0, N + 1)
        v = np.add.outer(z ** 2, np.abs(z)).ravel()
        orf.indicator(N, v, a[i], th[i] if th is not None else 0.0)
    t_ind = time.perf_counter() - t0
    eta = rng.exponential(size=len(lv))
    t0 = time.perf_counter()
    orf.mark(eta, lv, theta)
    t_mark = time.perf_counter() - t0
    t0 = time.perf_counter()
    for i in pick:
        N = int(lv[i])
        if 2 * N <= 64:
            orf.prolong(N, np.zeros((N + 1) ** 2))
    t_pro = time.perf_counter() - t0
    return {"indicator_ms": t_ind * n_b / n_s * 1e3, "marking_ms": t_mark * 1e3,
            "prolong_ms": t_pro * n_b / n_s * 1e3, "kind": "oracle", "cores": 1,
            "sample": f"indicator and interpolation on {sample} sampled instances, scaled to the batch by DoFs; "
                      "marking on the whole batch"}


def refinement_leg(steps=5, theta=0.3):
    """Error-indicator-driven micro refinement on the uneven 4225-instance
    batch (16/32/64 cells, FP32+refinement): step, indicator of every micro
    field, bulk marking over the global functional, nested interpolation
    into the refined batch (new context: setup), and the step time before
    and after.  Times: HIP-synchronised wall clock, median of 5 (indicator,
    marking, interpolation)."""
    import statistics
    import torch
    from paper_2103_17040_amd import TwoScaleBatch, tsm
    w, a, th, lv = W.make("uneven_mixed", 0)
    g = TwoScaleBatch(w.macro_cells, lv, a, th, D=w.D, d=w.d, kappa=w.kappa, p=w.p, dt=w.dt, sigma=w.sigma,
                      precision="fp32_refine", rtol=w.rtol)

    def timed(fn, reps=5):
        ts, out = [], None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return statistics.median(ts), out

    plans = []

    def step_ms(b):
        b.step(1)
        plans.append(b.autotune(steps=2)["plan"])     # state restored
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3

    try:
        g.set_state(W.initial_macro(w.macro_cells), None)
        before = step_ms(g)
        ms_ind, eta = timed(lambda: g.error_indicator())
        eta = eta.cpu().numpy()
        ms_mark, (new, n_marked) = timed(lambda: tsm.tsm_mark_refine(eta, lv, theta, 64))
        v = g.micro()
        vn = torch.empty(int(W.offsets(new)[-1]), dtype=torch.float64, device="cuda:0")
        ms_pro, _ = timed(lambda: tsm.tsm_prolong(lv, new, v, vn))
        t0 = time.perf_counter()
        g2, new2, _ = g.refine(theta)
        t_refine = (time.perf_counter() - t0) * 1e3
    finally:
        g.close()
    try:
        after = step_ms(g2)
        setup2 = g2.stats()["setup_ms"]
    finally:
        g2.close()
    lv_b, c_b = np.unique(lv, return_counts=True)
    lv_a, c_a = np.unique(new2, return_counts=True)
    return {"workload": "4225 instances, 16/32/64 cells (uneven batch), FP32+refinement, theta %.2f" % theta,
            "levels_before": dict(zip(map(str, lv_b.tolist()), c_b.tolist())),
            "levels_after": dict(zip(map(str, lv_a.tolist()), c_a.tolist())), "marked": int(n_marked),
            "micro_dofs_before": int(W.offsets(lv)[-1]), "micro_dofs_after": int(W.offsets(new2)[-1]),
            "indicator_ms": ms_ind, "marking_ms": ms_mark, "prolong_ms": ms_pro,
            "refine_total_ms": t_refine, "setup_ms_refined": setup2,
            "ms_per_step_before": before, "ms_per_step_after": after, "plans": plans}


def _paper_table_rows():
    """Rows of Tables 1 and 2 from tests/golden/paper_convergence_tables.txt,
    the last rows un-swapped: {DoFs: (e_uw, e_uw_grad, e_v, e_v_grad)}."""
    tab, cur = {"macro": [], "micro": []}, None
    with open(os.path.join(GOLD, "paper_convergence_tables.txt")) as fh:
        for ln in fh:
            ln = ln.strip()
            if not ln or ln.startswith("#"):
                continue
            if ln.startswith("["):
                cur = ln.strip("[]")
                continue
            f = ln.split()
            tab[cur].append((int(f[0]), float(f[2]), float(f[3])))
    tab["macro"][-1], tab["micro"][-1] = tab["micro"][-1], tab["macro"][-1]
    return {m[0]: (m[1], m[2], v[1], v[2]) for m, v in zip(tab["macro"], tab["micro"])}


PAPER_CONVERGENCE_ROWS = (8, 11, 16, 23, 32, 45, 64, 91, 128)   # cells per side, Tables 1-2


def _constant_tables(levels, F, device):
    """Jacobian tables (cell and boundary, the interface's flat layouts) of a
    map whose Jacobian is the constant F, built on the device."""
    import torch
    lv = np.asarray(levels, dtype=np.int64)
    n_cell_pts = int((4 * lv * lv).sum())      # 2x2 Gauss points per cell
    n_bnd_pts = int((8 * lv).sum())            # 4 sides x N edges x 2 points
    f = torch.as_tensor(np.asarray(F, dtype=np.float64).reshape(1, 4), device=device)
    return f.expand(n_cell_pts, 4).contiguous().view(-1), f.expand(n_bnd_pts, 4).contiguous().view(-1)


def stationary_convergence_leg(sizes=PAPER_CONVERGENCE_ROWS, workers=None, flags=0):
    """The convergence benchmark of Section 4.2 on the GPU: the paper's
    manufactured solution and map (eq. manu_system; data re-derived), N_M = N
    cells per side on both scales -- the rows of Tables 1-2, 81 to 16641
    DoFs per scale -- errors e_uw, e_uw_grad, e_v, e_v_grad and the observed
    orders; the paper's printed errors at the same DoF counts beside them
    (its parameters are not given, so only the orders compare).  The map's
    Jacobian is constant, so its tables are built on the device; data and
    error integrals run on `workers` host processes."""
    import torch
    from paper_2103_17040_amd import StationarySystem
    from workloads import manufactured as MF
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    phys = dict(Dv=1.0, Dw=0.5, kappa1=0.5, kappa2=1.0, kappa3=0.25, kappa4=1.0)
    parts = (0, 0, 1, 2)

    class P:
        pass
    prm = P()
    prm.parts = parts
    for k, v in phys.items():
        setattr(prm, k, v)
    F = MF.constant_map_jacobian(MF.ZETA_MANU)
    paper = _paper_table_rows()
    rows, dofs, errs = [], [], []
    for N in sizes:
        t0 = time.perf_counter()
        levels = np.full((N + 1) ** 2, N, dtype=np.int32)
        pts = MF.manufactured_data_at_points(phys, parts, N, levels, workers)
        t1 = time.perf_counter()
        Fc, Fb = _constant_tables(levels, F, "cuda")
        g = StationarySystem(N, levels, jacobians=(Fc, Fb), rtol=1e-13, flags=flags, **phys)
        del Fc, Fb
        torch.cuda.empty_cache()
        try:
            g.set_data(**pts)
            del pts
            u, w, v = g.solve()
            st = g.stats()
            u, w, v = (t.cpu().numpy() for t in (u, w, v))
        finally:
            g.close()
        t2 = time.perf_counter()
        off = W.offsets(levels)
        e = MF.convergence_errors(N, N, u, w, [v[off[k]:off[k + 1]] for k in range(len(levels))], prm,
                                  workers=workers)
        del v
        t3 = time.perf_counter()
        n = (N + 1) ** 2
        dofs.append(n)
        errs.append(e)
        rows.append({"macro_dofs": n, "micro_dofs_each": n, "micro_dofs_total": n * n, "e_uw": e[0],
                     "e_uw_grad": e[1], "e_v": e[2], "e_v_grad": e[3], "solve_ms": st["solve_ms"],
                     "micro_iters_max": st["micro_iters_max"], "macro_iters": st["macro_iters"],
                     "host_data_s": t1 - t0, "gpu_context_s": t2 - t1, "host_errors_s": t3 - t2,
                     "paper_e_uw_e_uw_grad_e_v_e_v_grad": paper.get(n)})
        _log(f"  convergence N={N}: {n} x {n} DoFs, e = {', '.join(f'{x:.3e}' for x in e)}, "
             f"solve {st['solve_ms']:.1f} ms, micro iters {st['micro_iters_max']}, "
             f"host {t1 - t0:.1f} + {t3 - t2:.1f} s")
    E = np.array(errs)
    return {"rows": rows, "orders": {"p_M": MF.orders(dofs, E[:, 0]), "q_M": MF.orders(dofs, E[:, 1]),
                                     "p_v": MF.orders(dofs, E[:, 2]), "q_v": MF.orders(dofs, E[:, 3])},
            "paper_orders_printed": "p 1.94-2.31, q 1.01-1.20 (Tables 1-2)", "host_workers": workers}


def parity_leg():
    """Relative discrete l2 errors of every output against the FP64 oracle's
    outputs stored in tests/golden (written by tests/golden/make_goldens.py,
    which calls only the oracle) for the 4225 x 32^2 FP64 workload, the
    uneven 4225-instance FP32+refinement workload and the 1089 x 32^2
    gradient workload."""
    from paper_2103_17040_amd import TwoScaleBatch
    res = {}
    for name, prec, rtol in (("batched_fp64", "fp64", 1e-12), ("uneven_mixed", "fp32_refine", 1e-10)):
        ref = np.load(os.path.join(GOLD, f"{name}_seed0.npz"), allow_pickle=False)
        w, a, th, lv = W.make(name, 0)
        g = TwoScaleBatch(w.macro_cells, lv, a, th, D=w.D, d=w.d, kappa=w.kappa, p=w.p, dt=w.dt,
                          sigma=w.sigma, precision=prec, rtol=rtol)
        try:
            beta, ln, _ = (t.cpu().numpy() for t in g.setup())
            g.set_state(W.initial_macro(w.macro_cells), None)
            us, done, F_first = [], 0, None
            for n in ref["steps"]:
                g.step(int(n) - done)
                done = int(n)
                us.append(g.macro().cpu().numpy())
                if done == 1:
                    F_first = g.fluxes().cpu().numpy()
            F_last = g.fluxes().cpu().numpy()
            v = g.micro().cpu().numpy()
        finally:
            g.close()
        off = W.offsets(lv)
        v_s = np.concatenate([v[off[i]:off[i + 1]] for i in ref["inst"]])
        res[name] = {"precision": prec, "rtol": rtol, "steps": int(done), "u": _rel(np.stack(us), ref["u"]),
                     "F_first": _rel(F_first, ref["F_first"]), "F_last": _rel(F_last, ref["F_last"]),
                     "v_last_sampled": _rel(v_s, ref["v_last"]), "beta": _rel(beta, ref["beta"]),
                     "len": _rel(ln, ref["len"])}
    ref = np.load(os.path.join(GOLD, "adjoint_fp64_seed0.npz"), allow_pickle=False)
    w, a, th, lv = W.make("adjoint_fp64", 0)
    g = TwoScaleBatch(w.macro_cells, lv, a, th, D=w.D, d=w.d, kappa=w.kappa, p=w.p, dt=w.dt,
                      sigma=w.sigma, rtol=1e-12, checkpoint_every=w.checkpoint_every)
    try:
        g.set_state(W.initial_macro(w.macro_cells), None)
        J, dJ = g.gradient(w.steps)
        dJ = dJ.cpu().numpy()
    finally:
        g.close()
    res["adjoint_fp64"] = {"steps": w.steps, "J": abs(J - float(ref["J"])) / abs(float(ref["J"])),
                           "dJda": _rel(dJ, ref["g"])}
    return res


def host_info():
    """CPU model, logical cores usable by this process and RAM of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ram = 0
    try:
        with open("/proc/meminfo") as fh:
            for ln in fh:
                if ln.startswith("MemTotal"):
                    ram = int(ln.split()[1]) * 1024
                    break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0))
    # a box's CPU share is what OMP_NUM_THREADS states there, whatever the
    # affinity mask shows
    share = os.environ.get("OMP_NUM_THREADS")
    if share and share.isdigit() and int(share) > 0:
        cores = min(cores, int(share))
    return {"cpu_model": model, "cores": cores, "ram_bytes": ram}


def _oracle_worker(job):
    """One process of the CPU baseline: the FP64 oracle's exact step, as it
    stands, on its own (S+1)^2-instance batch, one BLAS thread; setup first,
    then steps until `seconds` have passed."""
    S, lvl, a, th, prm, seconds = job
    from threadpoolctl import threadpool_limits
    from oracle import twoscale
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ts = twoscale.TwoScale(twoscale.Params(S, *prm), lvl, a, th)
        t_setup = time.perf_counter() - t0
        u = W.initial_macro(S)
        v = np.zeros(int(ts.offsets[-1]))
        K = 0
        t0 = time.perf_counter()
        while True:
            u, v, _ = ts.step(u, v)
            K += 1
            if time.perf_counter() - t0 > seconds or K >= 400:
                break
        t = time.perf_counter() - t0
    return int(ts.offsets[-1]), K, t, t_setup


def cpu_baseline(w, a, th, lv, seconds_hint=12.0):
    """The FP64 oracle, as it stands, on every host core: one process per
    core (spawned, one BLAS thread each), each stepping its own bounded
    sample of the workload -- a macro mesh of S cells per side, so (S+1)^2
    instances, with the workload's micro meshes, dt and amplitudes (process
    q takes the next (S+1)^2 of them).  The rate is the sum of the
    processes' micro DoF-updates per second; they run at the same time."""
    import multiprocessing as mp
    info = host_info()
    P = info["cores"]
    S = 3
    n = (S + 1) ** 2
    prm = (w.dt, w.D, w.d, w.kappa, w.p, w.sigma)
    jobs = []
    for q in range(P):
        idx = (np.arange(n) + q * n) % len(lv)
        jobs.append((S, lv[idx], a[idx], None if th is None else th[idx], prm, seconds_hint))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(P) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    rate = sum(d * K / t for d, K, t, _ in res)
    Ks = [K for _, K, _, _ in res]
    return {"value": rate, "unit": "micro DoF-updates/s", "cores": P, "kind": "oracle",
            "cpu_model": info["cpu_model"], "ram_bytes": info["ram_bytes"],
            "sample": f"{P} processes at once (one per core, one BLAS thread each), each the oracle's exact "
                      f"step on its own {n} instances ({S}x{S} macro cells) of the workload's micro meshes "
                      f"and amplitudes, {min(Ks)}-{max(Ks)} implicit-Euler steps of ~{seconds_hint:.0f} s, "
                      f"banded-Cholesky micro solves factored once (setup "
                      f"{max(r[3] for r in res):.1f} s excluded, as for the GPU value); "
                      f"{wall:.0f} s wall clock in all"}


def oracle_rate(w, lv, a, th, jacobians=None, fixed_point=False, S=3, seconds=4.0):
    """The oracle (as it stands, one core) on (S+1)^2 instances with the
    given micro meshes and geometry: micro DoF-updates per second of its
    exact step, or of the paper's alternating step (fixed_point)."""
    from threadpoolctl import threadpool_limits
    from oracle import twoscale
    n = (S + 1) ** 2
    with threadpool_limits(limits=1):
        ts = twoscale.TwoScale(twoscale.Params(S, w.dt, w.D, w.d, w.kappa, w.p, w.sigma), np.resize(lv, n)[:n],
                               a[:n], None if th is None else th[:n],
                               jacobians=None if jacobians is None else jacobians[:n])
        u, v = W.initial_macro(S), np.zeros(int(ts.offsets[-1]))
        K, t0 = 0, time.perf_counter()
        while K < 1 or time.perf_counter() - t0 < seconds:
            u, v = (ts.step_fixed_point(u, v)[:2] if fixed_point else ts.step(u, v)[:2])
            K += 1
        t = time.perf_counter() - t0
    return {"value": int(ts.offsets[-1]) * K / t, "unit": "micro DoF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} instances ({S}x{S} macro cells), {K} steps"
                      + (", the alternating coupling" if fixed_point else "")
                      + (", geometry from the Jacobian tables" if jacobians is not None else "")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0,
                    help="timed steps (0: the workload's own step count, 200 for the large batch)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large_mixed", choices=sorted(W.WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--plan", default="auto", choices=["auto"] + sorted(PLAN_FLAGS),
                    help="launch plan of the micro solves (auto: the autotuner picks on the live state)")
    ap.add_argument("--no-parity", action="store_true",
                    help="skip the parity leg (errors against the oracle's stored outputs)")
    ap.add_argument("--st-reps", type=int, default=3,
                    help="stationary three-field solves timed per size (0: skip that leg)")
    ap.add_argument("--st-conv-sizes", type=lambda t: [int(x) for x in t.split(",") if x],
                    default=list(PAPER_CONVERGENCE_ROWS),
                    help="cells per side (both scales) of the stationary convergence rows, comma-separated")
    ap.add_argument("--gm-steps", type=int, default=5,
                    help="steps of the general-map leg (Jacobian tables, uneven batch; 0: skip)")
    ap.add_argument("--fp-steps", type=int, default=3,
                    help="steps of the alternating-coupling leg (0: skip), timed against the exact step")
    ap.add_argument("--adjoint-steps", type=int, default=-1,
                    help="steps of the gradient leg (-1: the workload's step count; 0: skip); "
                         "checkpoint spacing from the workload")
    ap.add_argument("--calib-bytes", type=int, default=0,
                    help="first run a plain device copy of this many bytes (3 times), the reference "
                         "for scaling HBM counters (FETCH_SIZE, WRITE_SIZE) in profiles")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the batch shards by instance "
              "with one allgather of per-instance scalars per step, which is not built here.", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calib_bytes > 0:
        src = torch.ones(args.calib_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        _log(f"calibration copy: {args.calib_bytes} bytes read + written, 3 times")
        del src, dst
    w, a, th, lv = W.make(args.workload, args.seed)
    if args.steps <= 0:
        args.steps = w.steps
    if args.adjoint_steps < 0:
        args.adjoint_steps = w.steps if w.checkpoint_every > 0 else 0
    refine = w.precision == "fp32_refine"
    _log(f"workload {w.name}: {w.n_inst} instances, levels {sorted(set(lv.tolist()))}, "
         f"{int(W.offsets(lv)[-1])} micro DoFs, precision {w.precision}, rtol {w.rtol}")

    main_form = run_form(w, a, th, lv, w.precision, args.steps, args.warmup, w.rtol, args.adjoint_steps, args.plan,
                         args.fp_steps)
    _log(f"main form done: {main_form['t']:.3f} s for {args.steps} steps; stats {main_form['stats']}")
    fp64 = None
    if refine and not args.no_fp64:
        fp64 = run_form(w, a, th, lv, "fp64", args.steps, args.warmup, w.rtol, plan=args.plan)
        _log(f"fp64 form done: {fp64['t']:.3f} s; stats {fp64['stats']}")

    n_dofs = main_form["n_dofs"]
    K = args.steps
    value = n_dofs * K / main_form["t"]

    # roofline of the dominant kernel (the micro solve), per launch
    tst = main_form["timing"]
    launches = tst["timed_steps"] * tst["micro_launches"]
    micro_ms_per_launch = tst["micro_ms"] / max(launches, 1)
    st = main_form["stats"]
    # inner iterations and sweeps per solve, means over the timed steps
    iters = tst["iters_mean_run"]
    sweeps = tst["sweeps_mean_run"] if refine else 0
    dofs_per_launch = n_dofs / max(tst["micro_launches"], 1)
    plan_flags = main_form["plan"]["flags"]
    mf_dofs = sum((N + 1) ** 2 for N in lv.tolist() if matrix_free(int(N), plan_flags, refine))
    ex_dofs = sum((N + 1) ** 2 for N in lv.tolist() if extrapolated(int(N), plan_flags, refine))
    sm_dofs = sum((N + 1) ** 2 for N in lv.tolist() if mass_free(int(N), plan_flags, refine))
    flop_sm = FLOP_MASS + (FLOP_LOW0 if refine else 0.0)
    flops = (dofs_per_launch * (FLOP_ITER * iters + FLOP_SWEEP * sweeps + FLOP_SOLVE)
             + (mf_dofs * FLOP_OPERATOR_MF + ex_dofs * FLOP_GUESS + sm_dofs * flop_sm)
             / max(tst["micro_launches"], 1))
    step_bytes = sum((N + 1) ** 2 * micro_bytes_per_dof(int(N), plan_flags, refine, iters, sweeps)
                     for N in lv.tolist())
    nbytes = step_bytes / max(tst["micro_launches"], 1)
    t_launch = micro_ms_per_launch * 1e-3
    alu = flops / t_launch / 1e12
    hbm = nbytes / t_launch / 1e9
    traffic = measured_traffic(w.name, w.precision)
    n_packed = len({N for N in lv.tolist() if packed_under(int(N), plan_flags)})
    if n_packed == 0:
        kname = "micro_kernel (micro PCG)"
    elif plan_flags & (1 << 4):
        kname = ("packed_kernel, persistent" if n_packed == 1 else "packed_mixed_kernel") + " (micro PCG)"
    else:
        kname = "packed_kernel (micro PCG)"
    if 0 < n_packed and any(not packed_under(int(N), plan_flags) for N in set(lv.tolist())):
        kname += " + micro_kernel"
    # The roofline object of the dominant kernel.  Algorithmic bytes: the
    # state floor (24 B per DoF-update: v0 and M w read, v written; the
    # vectors of every iteration stay on chip) plus the boundary pass of the
    # flux average; algorithmic flops: the arithmetic of the kernel's own
    # work model (FLOP_*).  The bound is the roof with the larger fraction.
    # The counter-measured traffic and its ratio to the algorithmic bytes,
    # the bytes of the kernel's current data flow (resident model) and the
    # bytes a PCG streaming its vectors through HBM would need are reported
    # beside it.
    floor_units = dofs_per_launch
    bdot_bytes = sum(16.0 * 4 * int(N) for N in lv.tolist() if packed_under(int(N), plan_flags)) / max(
        tst["micro_launches"], 1)
    alg_bytes = B_FLOOR * floor_units + bdot_bytes
    hbm_alg = alg_bytes / t_launch / 1e9
    hbm_frac = hbm_alg / PEAK_HBM_GBS
    alu_frac = alu / PEAK_ALU_TFLOPS
    if alu_frac >= hbm_frac:
        roof = {"bound": "alu", "achieved": alu, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s", "frac": alu_frac,
                "traffic": traffic}
    else:
        roof = {"bound": "hbm", "achieved": hbm_alg, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": hbm_frac,
                "traffic": traffic}
    per_unit = streaming_bytes(refine, iters, sweeps)
    roof.update({
        "kernel": kname, "launch_ms": micro_ms_per_launch, "units_per_launch": dofs_per_launch,
        "unit_of_work": "one micro DoF-update (one DoF of one instance, one time step)",
        "peak_note": "alu peak: FP64 and non-packed FP32 FMA at 64 lanes/clock/CU, 256 CUs, 2.4 GHz "
                     "(packed FP32 is off in this build); hbm peak 8 TB/s",
        "alu_achieved_TFLOPs": alu, "alu_frac": alu_frac,
        "alu_frac_of_published_fp32_157_3": alu / PEAK_FP32_PUBLISHED_TFLOPS,
        "algorithmic_flops_per_launch": flops,
        "hbm_algorithmic_bytes_per_unit": alg_bytes / max(floor_units, 1),
        "hbm_algorithmic_GBs": hbm_alg, "hbm_frac": hbm_frac,
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated); "
                        "null when the kernel code (comments aside) changed since the counters were taken",
        "traffic_over_algorithmic": (traffic / alg_bytes) if traffic else None,
        "traffic_frac_of_hbm_peak": (traffic / t_launch / 1e9 / PEAK_HBM_GBS) if traffic else None,
        "resident_model_bytes_per_unit": nbytes / max(dofs_per_launch, 1),
        "resident_model_frac": hbm / PEAK_HBM_GBS,
        "streaming_model": {"bytes_per_unit": per_unit,
                            "GBs_equivalent": dofs_per_launch * per_unit / t_launch / 1e9,
                            "what": "a PCG streaming its vectors through HBM: 10 words per inner iteration "
                                    "(FP32 in refinement), 6 FP64 words per refinement sweep, 3 FP64 state "
                                    "words; the resident kernel moves far fewer bytes"},
    })

    out = {
        "metric": "micro DoF-updates/s (batched FP32+refine vs plain FP64) at 1e-8 rel; adjoint/fwd",
        "value": value,
        "unit": "micro DoF-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": main_form["t"] / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if refine else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "instances": w.n_inst, "micro_levels": sorted(set(lv.tolist())),
                   "micro_dofs": n_dofs, "dt": w.dt, "rtol": w.rtol, "precision": w.precision,
                   "seed": args.seed},
        "iters_mean": iters, "iters_mean_last_step": st["iters_mean"], "iters_max": st["iters_max"],
        "sweeps_max": st["sweeps_max"], "sweeps_mean": tst["sweeps_mean_run"] if refine else st["sweeps_mean"],
        "setup_ms": main_form["setup_ms"],
        "macro_ms_per_step": tst["macro_ms"] / max(tst["timed_steps"], 1),
        "launch_plan": main_form["plan"],
        "roofline": roof,
    }
    if fp64 is not None:
        v64 = n_dofs * K / fp64["t"]
        out["fp64_value"] = v64
        out["fp32_refine_speedup_vs_fp64"] = value / v64
        out["fp64_iters_mean"] = fp64["timing"]["iters_mean_run"]
    adj = main_form["adjoint"]
    if adj is not None:
        plain_fwd_ms = main_form["t"] / K * 1e3 * adj["steps"]
        adj["plain_forward_ms"] = plain_fwd_ms
        adj["backward_over_forward"] = adj["backward_ms"] / adj["forward_ms"]
        adj["total_over_plain_forward"] = (adj["forward_ms"] + adj["backward_ms"]) / plain_fwd_ms
        out["adjoint"] = adj
        out["adjoint_over_forward"] = adj["backward_over_forward"]
    fpl = main_form["fixed_point"]
    if fpl is not None:
        fpl["over_exact_step"] = fpl["ms_per_step"] / out["ms_per_step"]
        fpl["value"] = n_dofs / (fpl["ms_per_step"] * 1e-3)
        if not args.no_cpu_baseline:
            fpl["cpu_oracle"] = oracle_rate(w, lv, a, th, fixed_point=True)
        out["fixed_point_coupling"] = fpl
    if not args.no_parity:
        _log("parity leg ...")
        out["parity_vs_oracle"] = parity_leg()
    if args.gm_steps > 0:
        _log("general-map leg ...")
        out["general_map"] = general_map_leg(args.gm_steps)
        gm = out["general_map"]
        gm["value"] = gm["micro_dofs"] / (gm["ms_per_step"] * 1e-3)
        if not args.no_cpu_baseline:
            wu, au, thu, lvu = W.make("uneven_mixed", 0)
            per, _, _ = W.jacobian_tables(lvu[:16], W.polynomial_map_jacobian,
                                          W.polynomial_map_params(len(lvu), seed=2)[:16])
            gm["cpu_oracle"] = oracle_rate(wu, lvu[:16], au, thu, jacobians=per)
    if args.gm_steps > 0:
        _log("heterogeneous macro leg ...")
        out["general_map"]["heterogeneous_macro_pcg"] = macro_pcg_leg()
        _log("refinement leg ...")
        out["refinement"] = refinement_leg()
        if not args.no_cpu_baseline:
            out["refinement"]["cpu_oracle"] = refinement_oracle_time()
    if args.st_reps > 0:
        _log("stationary three-field leg ...")
        out["stationary"] = stationary_leg(args.st_reps, parity=not args.no_parity)
        if not args.no_cpu_baseline:
            out["stationary"]["case_B_81x4225"]["cpu_oracle"] = stationary_oracle_time()
        _log("stationary convergence leg ...")
        out["stationary"]["convergence"] = stationary_convergence_leg(tuple(args.st_conv_sizes))
    if not args.no_cpu_baseline:
        _log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, a, th, lv)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
