"""The C-ABI library loads on the host and exports every symbol that
include/krs.h declares; workspace sizes respect the paper's storage
formulas (no GPU needed: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "krs.h")
LIB = os.path.join(ROOT, "paper_1501_03358_amd", "libkrs.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(krs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libkrs.so not built")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_binding_names_match_header():
    from paper_1501_03358_amd import krs
    assert sorted(krs.EXPORTS) == declared_functions()


def _ws(lib, solver, n, m, k, dt):
    out = ctypes.c_size_t()
    fn = lib.krs_workspace_size
    fn.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                   ctypes.POINTER(ctypes.c_size_t)]
    rc = fn(solver, n, m, k, dt, ctypes.byref(out))
    assert rc == 0
    return out.value


FIXED = 32 << 20  # partial sums and the scalar area, independent of N


@pytest.mark.parametrize("n", [13824, 2097152])
def test_workspace_within_paper_storage(lib, n):
    """GMRES(m): the paper counts (m+1)N + 4N; the library keeps V (m+1
    columns) and two temporaries (one vector of the iterate lives in x).
    rGCROT adds U, C (2kN, owned by the caller).  BiCGStab: 8N."""
    ld = (n + 63) // 64 * 64 + 1088  # rounded up to 64, plus the column pad
    for m in (20, 30, 50):
        w = _ws(lib, 1, n, m, 20, 0)
        assert w <= 8 * ld * (m + 5) + FIXED
    w = _ws(lib, 2, n, 30, 20, 0)
    assert w <= 8 * ld * 8 + FIXED
    w32 = _ws(lib, 2, n, 30, 20, 1)
    assert w32 <= 4 * ld * 8 + FIXED
    # rGCROT with the GCROT rule: m more vectors (the previous selection space)
    for m, dt, wb in ((30, 0, 8), (10, 1, 4)):
        extra = _ws(lib, 4, n, m, 20, dt) - _ws(lib, 1, n, m, 20, dt)
        assert wb * ld * m <= extra <= wb * ld * m + 4096


def test_invalid_arguments_are_rejected(lib):
    fn = lib.krs_workspace_size
    fn.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                   ctypes.POINTER(ctypes.c_size_t)]
    out = ctypes.c_size_t()
    assert fn(1, 0, 30, 20, 0, ctypes.byref(out)) == -1
    assert fn(1, 100, 300, 20, 0, ctypes.byref(out)) == -1
    assert fn(9, 100, 30, 20, 0, ctypes.byref(out)) == -1
    assert fn(1, 100, 30, 20, 7, ctypes.byref(out)) == -1


def test_timing_classes_rejects_null_context(lib):
    fn = lib.krs_timing_classes
    fn.argtypes = [ctypes.c_void_p, ctypes.c_uint]
    fn.restype = ctypes.c_int
    assert fn(None, 1) == -1
