"""Two-scale micro-batch FEM (arXiv 2103.17040) on MI355X.

``tsm``            ctypes binding of libtsm.so (same names as include/tsm.h)
``TwoScaleBatch``  owner of one library context plus torch-allocated device
                   buffers for its inputs and outputs
``StationarySystem`` the same for the stationary three-field system
"""
from __future__ import annotations

__all__ = ["TwoScaleBatch", "StationarySystem"]


class TwoScaleBatch:
    """One batch of micro problems (one per macro node) and the macro field.

    All arithmetic happens in libtsm; this class only moves arguments.
    Inputs may be numpy arrays or torch tensors; outputs are torch CUDA
    tensors (float64)."""

    def __init__(self, macro_cells, micro_cells, a=None, theta=None, *, jacobians=None, D=1.0, d=0.5, kappa=1.0, p=1.0,
                 dt=0.01, sigma=-1, precision="fp64", rtol=1e-12, inner_rtol=1e-2, setup_rtol=1e-14,
                 max_iter=1000, max_refine=12, checkpoint_every=10, flags=0, coupling="schur",
                 fp_rtol=1e-10, fp_max_iter=50, grad_rtol=0.0, device="cuda:0"):
        import numpy as np
        import torch
        global tsm
        from . import tsm
        self.torch = torch
        self.device = torch.device(device)
        self._ctor = dict(D=D, d=d, kappa=kappa, p=p, dt=dt, sigma=sigma, precision=precision, rtol=rtol,
                          inner_rtol=inner_rtol, setup_rtol=setup_rtol, max_iter=max_iter, max_refine=max_refine,
                          checkpoint_every=checkpoint_every, flags=flags, coupling=coupling, fp_rtol=fp_rtol,
                          fp_max_iter=fp_max_iter, grad_rtol=grad_rtol, device=device)
        prm = tsm.tsm_default_params()
        prm.macro_cells = int(macro_cells)
        prm.D, prm.d, prm.kappa, prm.p, prm.dt = float(D), float(d), float(kappa), float(p), float(dt)
        prm.source_sign = int(sigma)
        prm.precision = {"fp64": tsm.TSM_FP64, "fp32_refine": tsm.TSM_FP32_REFINE}[precision]
        prm.rtol, prm.inner_rtol, prm.setup_rtol = float(rtol), float(inner_rtol), float(setup_rtol)
        prm.max_iter, prm.max_refine, prm.checkpoint_every = int(max_iter), int(max_refine), int(checkpoint_every)
        prm.flags = int(flags) | {"schur": 0, "fixed_point": tsm.TSM_FLAG_FIXED_POINT}[coupling]
        prm.fp_rtol, prm.fp_max_iter = float(fp_rtol), int(fp_max_iter)
        prm.grad_rtol = float(grad_rtol)
        self.params = prm
        self._flags = int(prm.flags)
        self.n_inst = (int(macro_cells) + 1) ** 2
        with torch.cuda.device(self.device):
            self.ctx = tsm.tsm_create(prm, None)
        try:
            self._levels = np.asarray(micro_cells, dtype=np.int32)
            tsm.tsm_set_reference_mesh(self.ctx, self._levels)
            self.offsets = tsm.tsm_get_offsets(self.ctx, self.n_inst)
            self.n_micro = int(self.offsets[-1])
            if jacobians is not None:
                self.set_jacobians(*jacobians)
            else:
                self.set_deformation(a, theta)
        except Exception:
            self.close()
            raise

    def _dev(self, x):
        if x is None:
            return None
        t = self.torch.as_tensor(x, dtype=self.torch.float64, device=self.device).contiguous()
        return t

    def _empty(self, n):
        return self.torch.empty(n, dtype=self.torch.float64, device=self.device)

    def set_deformation(self, a, theta=None):
        self._a = self._dev(a)
        self._theta = self._dev(theta)
        tsm.tsm_set_deformation(self.ctx, self._a, self._theta, self.n_inst)

    def set_jacobians(self, Fcell, Fbnd):
        """Geometry of a general map from its Jacobians at the quadrature
        points (layout of tsm_set_jacobians in include/tsm.h)."""
        self._Fc, self._Fb = self._dev(Fcell), self._dev(Fbnd)
        tsm.tsm_set_jacobians(self.ctx, self._Fc, self._Fc.numel(), self._Fb, self._Fb.numel())
        self._Fc = self._Fb = None   # read during the call only

    def set_state(self, u, v=None):
        tu, tv = self._dev(u), self._dev(v)
        tsm.tsm_set_state(self.ctx, tu, tv)

    def step(self, n_steps=1, allow_noconv=False):
        return tsm.tsm_step(self.ctx, n_steps, allow_noconv)

    def macro(self):
        out = self._empty(self.n_inst)
        tsm.tsm_get_macro(self.ctx, out)
        return out

    def fluxes(self):
        out = self._empty(self.n_inst)
        tsm.tsm_get_fluxes(self.ctx, out)
        return out

    def micro(self):
        out = self._empty(self.n_micro)
        tsm.tsm_get_micro(self.ctx, out)
        return out

    def setup(self):
        beta, ln, w = self._empty(self.n_inst), self._empty(self.n_inst), self._empty(self.n_micro)
        tsm.tsm_get_setup(self.ctx, beta, ln, w)
        return beta, ln, w

    def apply(self, x):
        tx = self._dev(x)
        y = self._empty(self.n_micro)
        tsm.tsm_apply_operator(self.ctx, tx, y)
        return y

    def gradient(self, n_steps):
        g = self._empty(self.n_inst)
        J = tsm.tsm_gradient(self.ctx, n_steps, g)
        return J, g

    def set_flags(self, flags):
        tsm.tsm_set_flags(self.ctx, flags)
        self._flags = int(flags)

    def error_indicator(self):
        """eta_i^2 of the current micro state (tsm_error_indicator)."""
        out = self._empty(self.n_inst)
        tsm.tsm_error_indicator(self.ctx, out)
        return out

    def refine(self, theta=0.5, max_level=64):
        """Refine the micro meshes from the indicator: bulk marking over all
        instances (tsm_mark_refine), marked instances get twice the cells per
        side, and a new batch with the same parameters, deformation and state
        (micro fields carried over by tsm_prolong) is returned with the new
        levels and the indicator.  This batch is left unchanged."""
        import numpy as np
        eta2 = self.error_indicator().cpu().numpy()
        levels = np.asarray(self._levels, dtype=np.int32)
        new_levels, _ = tsm.tsm_mark_refine(eta2, levels, theta, max_level)
        u, v = self.macro(), self.micro()
        n_new = int(((new_levels.astype(np.int64) + 1) ** 2).sum())
        v_new = self._empty(n_new)
        self.torch.cuda.synchronize(self.device)
        tsm.tsm_prolong(levels, new_levels, v, v_new)
        kw = dict(self._ctor)
        kw["flags"] = self._flags          # keep a plan chosen since construction
        g = TwoScaleBatch(self.params.macro_cells, new_levels, self._a, self._theta, **kw)
        g.set_state(u, v_new)
        return g, new_levels, eta2

    def autotune(self, steps=2, cache=None):
        """Pick the fastest launch plan on the current state (which is left
        unchanged).  With `cache` (a JSON path), a plan measured before for
        the same device, precision and mesh-size histogram is reused."""
        import json
        import os
        import numpy as np
        key = None
        if cache is not None:
            levels, counts = np.unique(np.asarray(self._levels), return_counts=True)
            key = "|".join([self.torch.cuda.get_device_name(self.device), str(self.params.precision),
                            str(self.params.macro_cells),
                            ",".join(f"{l}x{c}" for l, c in zip(levels.tolist(), counts.tolist()))])
            if os.path.exists(cache):
                with open(cache) as fh:
                    rec = json.load(fh)
                if key in rec:
                    self.set_flags((self._flags & ~tsm.PLAN_BITS) | int(rec[key]["flags"]))
                    return rec[key]
        ms, flags = tsm.tsm_autotune(self.ctx, steps)
        self._flags = (self._flags & ~tsm.PLAN_BITS) | flags
        res = {"flags": flags, "plan": tsm.plan_name(flags),
               "ms_per_step": {"per_size": ms[0], "persistent": ms[1], "generic": ms[2], "chosen": ms[3],
                               "assembled_operator": ms[4]}}
        if cache is not None:
            rec = {}
            if os.path.exists(cache):
                with open(cache) as fh:
                    rec = json.load(fh)
            rec[key] = res
            with open(cache, "w") as fh:
                json.dump(rec, fh, indent=1)
        return res

    def stats(self):
        return tsm.tsm_get_stats(self.ctx)

    def close(self):
        from . import tsm
        if getattr(self, "ctx", None):
            tsm.tsm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StationarySystem:
    """The stationary three-field system (u, w macro; v per macro node) on
    [-1,1]^2: one library context.  Geometry from amplitudes a (the
    sinusoidal family) or from Jacobian tables (any map).  All arithmetic
    happens in libtsm; outputs are torch CUDA tensors (float64)."""

    _NAMES = ("Dv", "Dw", "kappa1", "kappa2", "kappa3", "kappa4", "fu", "fv", "fw", "u_dirichlet", "rtol",
              "macro_rtol", "max_iter", "macro_max_iter")

    def __init__(self, macro_cells, micro_cells, a=None, theta=None, *, jacobians=None, parts=None,
                 dirichlet=None, flags=0, device="cuda:0", **kw):
        import numpy as np
        import torch
        global tsm
        from . import tsm
        self.torch = torch
        self.device = torch.device(device)
        prm = tsm.tsm_stationary_default_params()
        prm.macro_cells = int(macro_cells)
        for k, v in kw.items():
            if k not in self._NAMES:
                raise TypeError(f"unknown parameter {k}")
            setattr(prm, k, type(getattr(prm, k))(v))
        if parts is not None:
            for s, v in enumerate(parts):
                prm.parts[s] = int(v)
        if dirichlet is not None:
            for s, v in enumerate(dirichlet):
                prm.dirichlet[s] = int(bool(v))
        prm.flags = int(flags)
        self.params = prm
        self.n_inst = (int(macro_cells) + 1) ** 2
        with torch.cuda.device(self.device):
            self.ctx = tsm.tsm_stationary_create(prm, None)
        try:
            self._levels = np.asarray(micro_cells, dtype=np.int32)
            tsm.tsm_set_reference_mesh(self.ctx, self._levels)
            self.offsets = tsm.tsm_get_offsets(self.ctx, self.n_inst)
            self.n_micro = int(self.offsets[-1])
            if jacobians is not None:
                Fc = torch.as_tensor(jacobians[0], dtype=torch.float64, device=self.device).contiguous()
                Fb = torch.as_tensor(jacobians[1], dtype=torch.float64, device=self.device).contiguous()
                tsm.tsm_set_jacobians(self.ctx, Fc, Fc.numel(), Fb, Fb.numel())
            else:
                ta = torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()
                tt = None if theta is None else torch.as_tensor(theta, dtype=torch.float64,
                                                               device=self.device).contiguous()
                tsm.tsm_set_deformation(self.ctx, ta, tt, self.n_inst)
        except Exception:
            self.close()
            raise

    def set_data(self, fv_cell=None, gv_bnd=None, fu_cell=None, fw_cell=None, gu_bnd=None, gw_bnd=None, uD=None):
        """Sources and boundary data at the quadrature points (layouts of
        tsm_stationary_set_data in include/tsm.h); None keeps the constant."""
        t = self.torch
        dev = [None if x is None else t.as_tensor(x, dtype=t.float64, device=self.device).contiguous()
               for x in (fv_cell, gv_bnd, fu_cell, fw_cell, gu_bnd, gw_bnd, uD)]
        tsm.tsm_stationary_set_data(self.ctx, *dev)

    def solve(self, with_micro=True):
        """Returns (u, w, v) (v None unless with_micro)."""
        t = self.torch
        u = t.empty(self.n_inst, dtype=t.float64, device=self.device)
        w = t.empty_like(u)
        v = t.empty(self.n_micro, dtype=t.float64, device=self.device) if with_micro else None
        tsm.tsm_stationary_solve(self.ctx, u, w, v)
        return u, w, v

    def apply(self, x):
        t = self.torch
        tx = t.as_tensor(x, dtype=t.float64, device=self.device).contiguous()
        y = t.empty(self.n_micro, dtype=t.float64, device=self.device)
        tsm.tsm_apply_operator(self.ctx, tx, y)
        return y

    def set_flags(self, flags):
        tsm.tsm_set_flags(self.ctx, flags)

    def stats(self):
        return tsm.tsm_stationary_get_stats(self.ctx)

    def close(self):
        from . import tsm
        if getattr(self, "ctx", None):
            tsm.tsm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
