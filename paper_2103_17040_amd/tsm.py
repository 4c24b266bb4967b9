"""ctypes binding of libtsm.so: the C ABI of include/tsm.h with the same
names.  Argument marshalling only: every step of the path runs in the HIP
library.  Device pointers are passed as integers (e.g. ``tensor.data_ptr()``
of a torch CUDA tensor); PyTorch is only a convenient owner of device memory.

If the shared library is missing the import of this module fails loudly:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch ships its own HIP runtime.  Loading torch first makes libtsm bind to
# that same runtime (same soname); a second copy loaded from the ROCm tree
# would not see the device once torch's copy owns it.
import torch  # noqa: F401

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtsm.so")

TSM_OK, TSM_EINVAL, TSM_EGEOM, TSM_ENOCONV, TSM_EHIP, TSM_ENOMEM, TSM_ESTATE = 0, -1, -2, -3, -4, -5, -6
TSM_FP64, TSM_FP32_REFINE = 0, 1
TSM_FLAG_NO_GRAPH = 1 << 0
TSM_FLAG_STENCIL_STREAM = 1 << 1
TSM_FLAG_TIMING = 1 << 2
TSM_FLAG_GENERIC = 1 << 3
TSM_FLAG_PERSISTENT = 1 << 4
TSM_FLAG_FIXED_POINT = 1 << 5
TSM_FLAG_GENERIC_16 = 1 << 6
TSM_FLAG_GENERIC_32 = 1 << 7
TSM_FLAG_GENERIC_64 = 1 << 8
TSM_FLAG_MATRIX_FREE = 1 << 9
TSM_FLAG_MACRO_PCG = 1 << 10
TSM_FLAG_MULTIGRID = 1 << 11
TSM_FLAG_NO_MULTIGRID = 1 << 12
TSM_FLAG_NO_EXTRAPOLATION = 1 << 13
TSM_FLAG_ASSEMBLED_START = 1 << 14
TSM_PART_N, TSM_PART_I, TSM_PART_O = 0, 1, 2

STATUS_NAMES = {0: "TSM_OK", -1: "TSM_EINVAL", -2: "TSM_EGEOM", -3: "TSM_ENOCONV",
                -4: "TSM_EHIP", -5: "TSM_ENOMEM", -6: "TSM_ESTATE"}

EXPORTED = ["tsm_default_params", "tsm_create", "tsm_set_reference_mesh", "tsm_get_offsets",
            "tsm_set_deformation", "tsm_set_jacobians", "tsm_set_state", "tsm_step", "tsm_get_macro", "tsm_get_fluxes",
            "tsm_get_micro", "tsm_get_setup", "tsm_apply_operator", "tsm_gradient", "tsm_set_flags", "tsm_autotune", "tsm_get_stats",
            "tsm_last_error", "tsm_destroy", "tsm_stationary_default_params", "tsm_stationary_create",
            "tsm_stationary_solve", "tsm_stationary_set_data", "tsm_stationary_get_stats",
            "tsm_error_indicator", "tsm_mark_refine", "tsm_prolong", "tsm_prolong_noalloc"]


class tsm_params(ctypes.Structure):
    _fields_ = [("macro_cells", ctypes.c_int32), ("D", ctypes.c_double), ("d", ctypes.c_double),
                ("kappa", ctypes.c_double), ("p", ctypes.c_double), ("dt", ctypes.c_double),
                ("source_sign", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double), ("setup_rtol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("checkpoint_every", ctypes.c_int32), ("flags", ctypes.c_uint64),
                ("fp_rtol", ctypes.c_double), ("fp_max_iter", ctypes.c_int32), ("grad_rtol", ctypes.c_double)]


class tsm_stats(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int64), ("n_micro_dofs", ctypes.c_int64), ("steps_taken", ctypes.c_int64),
                ("iters_min", ctypes.c_int32), ("iters_max", ctypes.c_int32), ("iters_mean", ctypes.c_double),
                ("sweeps_max", ctypes.c_int32), ("unconverged", ctypes.c_int32),
                ("macro_sweeps", ctypes.c_int32), ("macro_contraction", ctypes.c_double),
                ("setup_ms", ctypes.c_double), ("step_ms", ctypes.c_double),
                ("micro_ms", ctypes.c_double), ("macro_ms", ctypes.c_double),
                ("timed_steps", ctypes.c_int32), ("micro_launches", ctypes.c_int32),
                ("grad_forward_ms", ctypes.c_double), ("grad_backward_ms", ctypes.c_double),
                ("sweeps_mean", ctypes.c_double),
                ("fp_iters_last", ctypes.c_int32), ("fp_iters_max", ctypes.c_int32),
                ("macro_pcg_iters", ctypes.c_int32), ("fp64_fallbacks", ctypes.c_int32)]


class tsm_stationary_params(ctypes.Structure):
    _fields_ = [("macro_cells", ctypes.c_int32), ("Dv", ctypes.c_double), ("Dw", ctypes.c_double),
                ("kappa1", ctypes.c_double), ("kappa2", ctypes.c_double), ("kappa3", ctypes.c_double),
                ("kappa4", ctypes.c_double), ("fu", ctypes.c_double), ("fv", ctypes.c_double),
                ("fw", ctypes.c_double), ("u_dirichlet", ctypes.c_double), ("parts", ctypes.c_int32 * 4),
                ("dirichlet", ctypes.c_int32 * 4), ("rtol", ctypes.c_double), ("macro_rtol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("macro_max_iter", ctypes.c_int32), ("flags", ctypes.c_uint64)]


class tsm_stationary_stats(ctypes.Structure):
    _fields_ = [("micro_iters_max", ctypes.c_int32 * 3), ("micro_iters_mean", ctypes.c_double * 3),
                ("unconverged", ctypes.c_int32), ("macro_iters", ctypes.c_int32),
                ("macro_rel_residual", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("micro_ms", ctypes.c_double)]


class TsmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_17040_amd.build` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D, VP = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    sig = {
        "tsm_default_params": (None, [ctypes.POINTER(tsm_params)]),
        "tsm_create": (I32, [ctypes.POINTER(tsm_params), VP, ctypes.POINTER(P)]),
        "tsm_set_reference_mesh": (I32, [P, ctypes.POINTER(I32), I64]),
        "tsm_get_offsets": (I32, [P, ctypes.POINTER(I64)]),
        "tsm_set_deformation": (I32, [P, VP, VP, I64]),
        "tsm_set_jacobians": (I32, [P, VP, I64, VP, I64]),
        "tsm_set_state": (I32, [P, VP, I64, VP, I64]),
        "tsm_step": (I32, [P, I32]),
        "tsm_get_macro": (I32, [P, VP, I64]),
        "tsm_get_fluxes": (I32, [P, VP, I64]),
        "tsm_get_micro": (I32, [P, VP, I64]),
        "tsm_get_setup": (I32, [P, VP, VP, I64, VP, I64]),
        "tsm_apply_operator": (I32, [P, VP, VP, I64]),
        "tsm_gradient": (I32, [P, I32, ctypes.POINTER(D), VP, I64]),
        "tsm_set_flags": (I32, [P, ctypes.c_uint64]),
        "tsm_autotune": (I32, [P, I32, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_uint64)]),
        "tsm_get_stats": (I32, [P, ctypes.POINTER(tsm_stats)]),
        "tsm_last_error": (ctypes.c_char_p, [P]),
        "tsm_destroy": (None, [P]),
        "tsm_stationary_default_params": (None, [ctypes.POINTER(tsm_stationary_params)]),
        "tsm_stationary_create": (I32, [ctypes.POINTER(tsm_stationary_params), VP, ctypes.POINTER(P)]),
        "tsm_stationary_solve": (I32, [P, VP, VP, I64, VP, I64]),
        "tsm_stationary_set_data": (I32, [P, VP, I64, VP, I64, VP, I64, VP, I64, VP, I64, VP, I64, VP, I64]),
        "tsm_error_indicator": (I32, [P, VP, I64]),
        "tsm_mark_refine": (I32, [I64, ctypes.POINTER(D), ctypes.POINTER(I32), D, I32, ctypes.POINTER(I32),
                                  ctypes.POINTER(I64)]),
        "tsm_prolong": (I32, [I64, ctypes.POINTER(I32), ctypes.POINTER(I32), VP, I64, VP, I64, VP]),
        "tsm_prolong_noalloc": (I32, [I64, ctypes.POINTER(I32), ctypes.POINTER(I32), VP, I64, VP, I64, VP]),
        "tsm_stationary_get_stats": (I32, [P, ctypes.POINTER(tsm_stationary_stats)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def _check(ctx, status):
    if status != TSM_OK:
        msg = _lib.tsm_last_error(ctx).decode() if ctx else ""
        raise TsmError(status, msg)


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _n(x, n=None):
    """Entry count passed beside a device pointer: the tensor's numel, or n
    for a raw integer pointer (which carries no size of its own)."""
    if x is None:
        return 0
    if isinstance(x, int):
        if n is None:
            raise ValueError("a raw device pointer needs an explicit entry count")
        return int(n)
    return int(x.numel())


def tsm_default_params() -> tsm_params:
    p = tsm_params()
    _lib.tsm_default_params(ctypes.byref(p))
    return p


def tsm_create(params: tsm_params, stream=None):
    out = ctypes.c_void_p()
    st = _lib.tsm_create(ctypes.byref(params), stream, ctypes.byref(out))
    if st != TSM_OK:
        raise TsmError(st, "tsm_create: " + _lib.tsm_last_error(None).decode())
    return out.value


def tsm_set_reference_mesh(ctx, micro_cells) -> None:
    mc = np.ascontiguousarray(micro_cells, dtype=np.int32)
    _check(ctx, _lib.tsm_set_reference_mesh(ctx, mc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), mc.size))


def tsm_get_offsets(ctx, n_inst: int) -> np.ndarray:
    out = np.zeros(n_inst + 1, dtype=np.int64)
    _check(ctx, _lib.tsm_get_offsets(ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return out


def tsm_set_deformation(ctx, a, theta, n_inst: int) -> None:
    _check(ctx, _lib.tsm_set_deformation(ctx, _ptr(a), _ptr(theta), n_inst))


def tsm_set_jacobians(ctx, Fcell, n_cell: int, Fbnd, n_bnd: int) -> None:
    _check(ctx, _lib.tsm_set_jacobians(ctx, _ptr(Fcell), int(n_cell), _ptr(Fbnd), int(n_bnd)))


def tsm_set_state(ctx, u, v, n_u=None, n_v=None) -> None:
    _check(ctx, _lib.tsm_set_state(ctx, _ptr(u), _n(u, n_u), _ptr(v), _n(v, n_v)))


def tsm_step(ctx, n_steps: int, allow_noconv: bool = False) -> int:
    st = _lib.tsm_step(ctx, int(n_steps))
    if st == TSM_ENOCONV and allow_noconv:
        return st
    _check(ctx, st)
    return st


def tsm_get_macro(ctx, u_out, n=None) -> None:
    _check(ctx, _lib.tsm_get_macro(ctx, _ptr(u_out), _n(u_out, n)))


def tsm_get_fluxes(ctx, F_out, n=None) -> None:
    _check(ctx, _lib.tsm_get_fluxes(ctx, _ptr(F_out), _n(F_out, n)))


def tsm_get_micro(ctx, v_out, n=None) -> None:
    _check(ctx, _lib.tsm_get_micro(ctx, _ptr(v_out), _n(v_out, n)))


def tsm_get_setup(ctx, beta_out=None, len_out=None, w_out=None) -> None:
    n_inst = _n(beta_out) if beta_out is not None else _n(len_out)
    if beta_out is not None and len_out is not None and _n(len_out) != n_inst:
        raise ValueError("beta_out and len_out differ in size")
    _check(ctx, _lib.tsm_get_setup(ctx, _ptr(beta_out), _ptr(len_out), n_inst, _ptr(w_out), _n(w_out)))


def tsm_apply_operator(ctx, x, y) -> None:
    if _n(x) != _n(y):
        raise ValueError("x and y differ in size")
    _check(ctx, _lib.tsm_apply_operator(ctx, _ptr(x), _ptr(y), _n(x)))


def tsm_gradient(ctx, n_steps: int, dJda_out) -> float:
    J = ctypes.c_double()
    _check(ctx, _lib.tsm_gradient(ctx, int(n_steps), ctypes.byref(J), _ptr(dJda_out), _n(dJda_out)))
    return J.value


def tsm_set_flags(ctx, flags: int) -> None:
    _check(ctx, _lib.tsm_set_flags(ctx, int(flags)))


PLAN_BITS = (TSM_FLAG_PERSISTENT | TSM_FLAG_GENERIC | TSM_FLAG_GENERIC_16 | TSM_FLAG_GENERIC_32
             | TSM_FLAG_GENERIC_64 | TSM_FLAG_MATRIX_FREE)


def plan_name(flags: int) -> str:
    """Readable name of the launch-plan bits of a flag word."""
    if flags & TSM_FLAG_GENERIC:
        return "generic"
    name = "persistent" if flags & TSM_FLAG_PERSISTENT else "per_size"
    for bit, lvl in ((TSM_FLAG_GENERIC_16, 16), (TSM_FLAG_GENERIC_32, 32), (TSM_FLAG_GENERIC_64, 64)):
        if flags & bit:
            name += f"+generic{lvl}"
    if flags & TSM_FLAG_MATRIX_FREE:
        name += "+matrix_free"
    return name


def tsm_autotune(ctx, steps: int):
    """Returns (ms per step [per-size, persistent, generic, chosen, chosen plan
    with the assembled operator when the matrix-free one was asked for], chosen
    plan flags)."""
    ms = (ctypes.c_double * 5)()
    fl = ctypes.c_uint64()
    _check(ctx, _lib.tsm_autotune(ctx, int(steps), ms, ctypes.byref(fl)))
    return list(ms), fl.value


def tsm_get_stats(ctx) -> dict:
    s = tsm_stats()
    _check(ctx, _lib.tsm_get_stats(ctx, ctypes.byref(s)))
    return {name: getattr(s, name) for name, _ in tsm_stats._fields_}


def tsm_last_error(ctx) -> str:
    return _lib.tsm_last_error(ctx).decode()


def tsm_destroy(ctx) -> None:
    _lib.tsm_destroy(ctx)


def tsm_stationary_default_params() -> tsm_stationary_params:
    p = tsm_stationary_params()
    _lib.tsm_stationary_default_params(ctypes.byref(p))
    return p


def tsm_stationary_create(params: tsm_stationary_params, stream=None):
    out = ctypes.c_void_p()
    st = _lib.tsm_stationary_create(ctypes.byref(params), stream, ctypes.byref(out))
    if st != TSM_OK:
        raise TsmError(st, "tsm_stationary_create: " + _lib.tsm_last_error(None).decode())
    return out.value


def tsm_stationary_solve(ctx, u_out, w_out, v_out=None) -> None:
    if _n(u_out) != _n(w_out):
        raise ValueError("u_out and w_out differ in size")
    _check(ctx, _lib.tsm_stationary_solve(ctx, _ptr(u_out), _ptr(w_out), _n(u_out), _ptr(v_out), _n(v_out)))


def tsm_stationary_set_data(ctx, fv_cell=None, gv_bnd=None, fu_cell=None, fw_cell=None, gu_bnd=None, gw_bnd=None,
                            uD=None) -> None:
    args = []
    for x in (fv_cell, gv_bnd, fu_cell, fw_cell, gu_bnd, gw_bnd, uD):
        args += [_ptr(x), _n(x)]
    _check(ctx, _lib.tsm_stationary_set_data(ctx, *args))


def tsm_error_indicator(ctx, eta2_out) -> None:
    _check(ctx, _lib.tsm_error_indicator(ctx, _ptr(eta2_out), _n(eta2_out)))


def tsm_mark_refine(eta2, level, theta: float, max_level: int = 64):
    """Returns (new levels, number marked)."""
    e = np.ascontiguousarray(eta2, dtype=np.float64)
    lv = np.ascontiguousarray(level, dtype=np.int32)
    out = np.empty_like(lv)
    nm = ctypes.c_int64()
    st = _lib.tsm_mark_refine(lv.size, e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              lv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), float(theta), int(max_level),
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(nm))
    if st != TSM_OK:
        raise TsmError(st, _lib.tsm_last_error(None).decode())
    return out, nm.value


def tsm_prolong(level_old, level_new, v_old, v_new, stream=None, n_old=None, n_new=None) -> None:
    lo = np.ascontiguousarray(level_old, dtype=np.int32)
    ln = np.ascontiguousarray(level_new, dtype=np.int32)
    st = _lib.tsm_prolong(lo.size, lo.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          ln.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(v_old), _n(v_old, n_old),
                          _ptr(v_new), _n(v_new, n_new), stream)
    if st != TSM_OK:
        raise TsmError(st, _lib.tsm_last_error(None).decode())


def tsm_prolong_noalloc(level_old, level_new, v_old, v_new, stream=None, n_old=None, n_new=None) -> None:
    """tsm_prolong without device allocation (static workspace, at most
    131072 instances)."""
    lo = np.ascontiguousarray(level_old, dtype=np.int32)
    ln = np.ascontiguousarray(level_new, dtype=np.int32)
    st = _lib.tsm_prolong_noalloc(lo.size, lo.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  ln.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(v_old), _n(v_old, n_old),
                                  _ptr(v_new), _n(v_new, n_new), stream)
    if st != TSM_OK:
        raise TsmError(st, _lib.tsm_last_error(None).decode())


def tsm_stationary_get_stats(ctx) -> dict:
    s = tsm_stationary_stats()
    _check(ctx, _lib.tsm_stationary_get_stats(ctx, ctypes.byref(s)))
    out = {}
    for name, _ in tsm_stationary_stats._fields_:
        v = getattr(s, name)
        out[name] = list(v) if hasattr(v, "__len__") else v
    return out
