"""CPU checks of the boundary: the library loads and exports every symbol
the headers under include/ declare (no compute call without a GPU)."""
import ctypes
import os
import re

import paper_1405_7487_amd as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    return sorted(set(re.findall(r"FMM_API\s+[\w\s\*]*?\b(fmm_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("fmm_build", "fmm_evaluate", "fmm_evaluate_plan", "fmm_adjoint", "fmm_destroy"):
        assert s in syms
    assert set(syms) == set(F.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = F.load()
    for s in declared_symbols():
        assert hasattr(lib, s), s
        assert ctypes.cast(getattr(lib, s), ctypes.c_void_p).value


def test_params_default_and_last_error_without_gpu():
    lib = F.load()
    p = F._binding._Params()
    lib.fmm_params_default(ctypes.byref(p))
    assert (p.p, p.theta, p.ncrit, p.precision, p.coarse_fp64_levels, p.kahan, p.tight, p.m2l_sparse,
            p.m2l_rotation, p.mutual) == (8, 0.4, 64, 1, 3, 1, 0, -1, 0, 0)
    assert lib.fmm_last_error() == b""
    # argument validation happens before any device call
    out = ctypes.c_void_p()
    assert lib.fmm_build(None, 0, -1, None, None, None, ctypes.byref(out)) == 1
    assert lib.fmm_build(None, 0, 10, None, None, None, ctypes.byref(out)) == 1
    assert b"NULL" in lib.fmm_last_error()
    assert lib.fmm_build(None, 0, 10, None, None, None, None) == 1
    assert lib.fmm_evaluate_plan(None, None, None, None, None) == 1
    assert lib.fmm_adjoint(None, None, None, None, None, None, None) == 1
    assert lib.fmm_list_digest(None, None) == 1
    assert lib.fmm_count_body_pairs(None, None) == 1


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1405_7487_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "liboracle" not in txt, f


def test_entry_build_calls_both_compilers(monkeypatch):
    """__graft_entry__.build() reaches the oracle's and the library's build
    functions (stubbed here; the real compile runs outside the unit tests)."""
    import importlib
    import sys

    sys.path.insert(0, ROOT)
    try:
        entry = importlib.import_module("__graft_entry__")
    finally:
        sys.path.remove(ROOT)
    called = []
    for mod in ("oracle.build", "paper_1405_7487_amd.build"):
        m = importlib.import_module(mod)
        monkeypatch.setattr(m, "build", lambda *a, _m=mod, **k: called.append(_m))
    entry.build()
    assert called == ["oracle.build", "paper_1405_7487_amd.build"]
