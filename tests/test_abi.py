"""The C ABI library loads without a GPU and exports every entry point the
header declares; parameter validation runs on the host."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsm.h")
LIB = os.path.join(ROOT, "paper_2103_17040_amd", "libtsm.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tsm_[a-z_]+)\s*\(", src)))


def _exported():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    return sorted({line.split()[-1] for line in out.splitlines() if " T " in line and line.split()[-1].startswith("tsm_")})


@pytest.fixture(scope="module")
def lib_built():
    if not os.path.exists(LIB):
        pytest.fail("libtsm.so is not built: run `python -m paper_2103_17040_amd.build`")
    return LIB


def test_every_declared_symbol_is_exported(lib_built):
    decl = _declared()
    assert len(decl) >= 15
    assert decl == _exported()


def test_binding_names_match_header(lib_built):
    from paper_2103_17040_amd import tsm
    assert sorted(tsm.EXPORTED) == _declared()


def test_params_struct_layout_and_validation(lib_built):
    from paper_2103_17040_amd import tsm
    p = tsm.tsm_default_params()
    assert p.macro_cells == 8 and p.kappa == 1.0 and p.source_sign == -1 and p.rtol == 1e-12
    bad = []
    for field, value in (("D", 0.0), ("dt", -1.0), ("source_sign", 0), ("precision", 7), ("macro_cells", 1),
                         ("inner_rtol", 1.5), ("p", float("nan")), ("fp_rtol", 0.0), ("fp_max_iter", 1)):
        q = tsm.tsm_default_params()
        setattr(q, field, value)
        bad.append(q)
    for q in bad:
        with pytest.raises(tsm.TsmError) as e:
            tsm.tsm_create(q, None)
        assert e.value.status == tsm.TSM_EINVAL
        # the reason of a rejected create is kept per thread under the NULL context
        assert tsm._lib.tsm_last_error(None) == b"parameter out of range"
        assert "parameter out of range" in str(e.value)


def test_null_safety(lib_built):
    from paper_2103_17040_amd import tsm
    tsm._lib.tsm_destroy(None)
    assert isinstance(tsm._lib.tsm_last_error(None), bytes)


def STRUCTS(tsm):
    return (("tsm_params", tsm.tsm_params), ("tsm_stats", tsm.tsm_stats),
            ("tsm_stationary_params", tsm.tsm_stationary_params),
            ("tsm_stationary_stats", tsm.tsm_stationary_stats))


def test_stationary_params_defaults_and_validation(lib_built):
    """Defaults are the Table 3 parameters; bad values are rejected on the
    host before any device call."""
    from paper_2103_17040_amd import tsm
    p = tsm.tsm_stationary_default_params()
    assert (p.Dv, p.Dw, p.kappa1, p.kappa2, p.kappa3, p.kappa4, p.u_dirichlet) == (1.0, 0.1, 0.5, 1.0, 0.25, 1.0, 1.0)
    assert list(p.parts) == [tsm.TSM_PART_N, tsm.TSM_PART_N, tsm.TSM_PART_I, tsm.TSM_PART_O]
    assert list(p.dirichlet) == [0, 0, 1, 0] and p.macro_cells == 8
    cases = [("Dv", 0.0), ("Dw", -1.0), ("kappa3", 0.0), ("kappa2", float("inf")), ("fv", float("nan")),
             ("macro_cells", 1), ("macro_cells", 257), ("max_iter", 0), ("macro_rtol", 0.0), ("flags", 1 << 5)]
    for field, value in cases:
        q = tsm.tsm_stationary_default_params()
        setattr(q, field, value)
        with pytest.raises(tsm.TsmError) as e:
            tsm.tsm_stationary_create(q, None)
        assert e.value.status == tsm.TSM_EINVAL, field
    for parts, dirichlet in (((0, 0, 1, 1), (0, 0, 1, 0)), ((0, 0, 2, 2), (0, 0, 1, 0)),
                             ((0, 0, 1, 3), (0, 0, 1, 0)), ((0, 0, 1, 2), (0, 0, 0, 0))):
        q = tsm.tsm_stationary_default_params()
        for s in range(4):
            q.parts[s], q.dirichlet[s] = parts[s], dirichlet[s]
        with pytest.raises(tsm.TsmError) as e:
            tsm.tsm_stationary_create(q, None)
        assert e.value.status == tsm.TSM_EINVAL, (parts, dirichlet)


def test_struct_layouts_match_header(tmp_path):
    """The ctypes structs have the size and field offsets that a C compiler
    gives the header's structs."""
    from paper_2103_17040_amd import tsm
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tsm.h"', 'int main(void) {']
    for cname, py in STRUCTS(tsm):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    want = {}
    for ln in out:
        if ln:
            c, f, v = ln.split()
            want[(c, f)] = int(v)
    for cname, py in STRUCTS(tsm):
        assert ctypes.sizeof(py) == want[(cname, "size")], cname
        for f, _ in py._fields_:
            assert getattr(py, f).offset == want[(cname, f)], (cname, f)


def test_binding_constants_match_header():
    """Every TSM_ flag, status and precision the header defines has the same
    value in the binding."""
    from paper_2103_17040_amd import tsm
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    defs = re.findall(r"#define\s+(TSM_[A-Z0-9_]+)\s+\(?\s*(\d+)(?:ull)?\s*(?:<<\s*(\d+))?\s*\)?", src)
    assert len(defs) >= 9, defs
    for name, base, shift in defs:
        value = int(base) << int(shift or 0)
        assert getattr(tsm, name) == value, name


def test_mark_refine_matches_the_oracle(lib_built):
    """Bulk marking is host code in the library: the same decisions as the
    oracle's marking on seeded indicators (with ties), and its errors."""
    import numpy as np
    from oracle import refine
    from paper_2103_17040_amd import tsm
    rng = np.random.default_rng(5)
    for trial in range(20):
        n = int(rng.integers(1, 200))
        eta = rng.exponential(size=n)
        eta[rng.integers(0, n, size=n // 4)] = eta[0]          # ties
        lv = rng.choice(np.array([8, 16, 32, 64], np.int32), n)
        theta = float(rng.uniform(0, 1))
        new, nm = tsm.tsm_mark_refine(eta, lv, theta, 64)
        m = refine.mark(eta, lv, theta, 64)
        expect = lv.copy()
        expect[m] *= 2
        assert np.array_equal(new, expect) and nm == len(m), trial
    # meshes above 64 cells per side refine up to 256
    for trial in range(10):
        n = int(rng.integers(1, 100))
        eta = rng.exponential(size=n)
        lv = rng.choice(np.array([16, 64, 91, 128, 256], np.int32), n)
        new, nm = tsm.tsm_mark_refine(eta, lv, 0.6, 256)
        m = refine.mark(eta, lv, 0.6, 256)
        expect = lv.copy()
        expect[m] *= 2
        assert np.array_equal(new, expect) and nm == len(m) and new.max() <= 256, trial
    for eta, lv, th in (([1.0, -1.0], [8, 8], 0.5), ([1.0, np.nan], [8, 8], 0.5), ([1.0], [8], 1.5),
                        ([1.0], [1], 0.5), ([1.0], [257], 0.5)):
        with pytest.raises(tsm.TsmError) as e:
            tsm.tsm_mark_refine(np.array(eta), np.array(lv, np.int32), th)
        assert e.value.status == tsm.TSM_EINVAL
    for lo, ln in ((8, 12), (129, 258)):     # bad levels are refused before any device call
        with pytest.raises(tsm.TsmError) as e:
            tsm.tsm_prolong(np.array([lo], np.int32), np.array([ln], np.int32), 0, 0, n_old=(lo + 1) ** 2,
                            n_new=(ln + 1) ** 2)
        assert e.value.status == tsm.TSM_EINVAL
    # so are vectors whose entry counts do not match the levels (81 and 289
    # here); the pointers are never touched, the counts are checked first
    for n_old, n_new in ((80, 289), (81, 288), (0, 0)):
        with pytest.raises(tsm.TsmError) as e:
            tsm.tsm_prolong(np.array([8], np.int32), np.array([16], np.int32), 256, 512, n_old=n_old, n_new=n_new)
        assert e.value.status == tsm.TSM_EINVAL and "must hold" in str(e.value), (n_old, n_new)


def _declared_arity():
    """Parameter count of every function the header declares."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for name, params in re.findall(r"\b(tsm_[a-z_]+)\s*\(([^)]*)\)\s*;", src):
        params = params.strip()
        out[name] = 0 if params in ("", "void") else len(params.split(","))
    return out


def test_binding_signatures_match_header(lib_built):
    """Every ctypes prototype of the binding has as many arguments as the
    header's declaration (a count passed beside each caller array included)."""
    from paper_2103_17040_amd import tsm
    arity = _declared_arity()
    assert sorted(arity) == _declared()
    for name, n in arity.items():
        assert len(getattr(tsm._lib, name).argtypes) == n, name
