"""The C-ABI library loads, exports every symbol include/mspcg.h declares, and
validates arguments on the host (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_1804_08593_amd import mspcg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mspcg.h")).read()
    return sorted(set(re.findall(r"\b(mspcg_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = mspcg.load()
    names = _declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert set(mspcg.EXPORTS) == set(names)
    assert lib.mspcg_version() == 1


def test_strerror_texts():
    codes = (mspcg.OK, mspcg.EINVAL, mspcg.ENOMEM, mspcg.EHIP, mspcg.ENOGAUGE, mspcg.ENOCONV,
             mspcg.EBREAKDOWN, mspcg.EUNSUPPORTED, mspcg.ESCRATCH, mspcg.EINTERNAL)
    for code in codes:
        assert mspcg.strerror(code) != "unknown error"
    assert len(set(codes)) == len(codes)
    assert mspcg.strerror(-99) == "unknown error"


def test_no_exception_leaves_an_entry_point():
    """Every entry point that does more than return a constant is a
    function-try-block closed by the catch clauses that map C++ exceptions to
    error codes."""
    csrc = os.path.join(ROOT, "paper_1804_08593_amd", "csrc")
    seen = set()
    for fn in sorted(os.listdir(csrc)):
        if not fn.endswith(".hip"):
            continue
        lines = open(os.path.join(csrc, fn)).read().split("\n")
        for i, ln in enumerate(lines):
            if not ln.startswith('extern "C"'):
                continue
            name = re.search(r"(mspcg_\w+)\(", ln).group(1)
            seen.add(name)
            if name in ("mspcg_version", "mspcg_strerror"):
                continue
            j = i
            while not lines[j].rstrip().endswith("{"):
                j += 1
            assert lines[j].rstrip().endswith(") try {"), name
            k = j + 1
            while lines[k] != "}" and not lines[k].startswith("} catch"):
                k += 1
            closing = lines[k] + lines[k + 1]
            assert "MSPCG_ABI_CATCH" in closing or lines[k].startswith("} catch (...)"), name
    assert seen == set(_declared())


@pytest.mark.parametrize("dims,Ls,err", [
    ((3, 4, 4, 4), 8, mspcg.EINVAL),      # odd extent
    ((4, 4, 4, 0), 8, mspcg.EINVAL),      # empty lattice
    ((4, 4, 4, 4), 1, mspcg.EINVAL),      # Ls < 2
    ((4, 4, 4, 4), 7, mspcg.EUNSUPPORTED),  # Ls not compiled in
])
def test_create_rejects_bad_actions(dims, Ls, err):
    lib = mspcg.load()
    a = mspcg.Action()
    for i in range(4):
        a.dims[i] = dims[i]
    a.Ls, a.M5, a.mf, a.b, a.c, a.antiperiodic_t = Ls, 1.8, 0.1, 1.0, 0.0, 1
    h = ctypes.c_void_p()
    assert lib.mspcg_create(ctypes.byref(a), 0, ctypes.byref(h)) == err
    assert not h.value


def test_create_rejects_bad_parameters():
    lib = mspcg.load()
    for b, c, mf in [(0.0, 0.5, 0.1), (float("nan"), 0.0, 0.1), (1.0, 0.0, float("inf"))]:
        a = mspcg.Action()
        for i in range(4):
            a.dims[i] = 4
        a.Ls, a.M5, a.mf, a.b, a.c, a.antiperiodic_t = 8, 1.8, mf, b, c, 1
        h = ctypes.c_void_p()
        assert lib.mspcg_create(ctypes.byref(a), 0, ctypes.byref(h)) == mspcg.EINVAL


def test_null_pointers_rejected():
    lib = mspcg.load()
    assert lib.mspcg_create(None, 0, None) == mspcg.EINVAL
    assert lib.mspcg_apply(None, 0, 0, None, None, None) == mspcg.EINVAL
    assert lib.mspcg_solve(None, None, None, None, None, None) == mspcg.EINVAL
    assert lib.mspcg_force(None, None, None, None, None, None) == mspcg.EINVAL
    assert lib.mspcg_autotune(None, None, None, None) == mspcg.EINVAL
    assert lib.mspcg_get_tuning(None, None) == mspcg.EINVAL
    assert lib.mspcg_load_gauge(None, None, None) == mspcg.EINVAL
    lib.mspcg_destroy(None)
