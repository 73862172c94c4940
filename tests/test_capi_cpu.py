"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/csrad.h, and the binding covers them;
argument errors come back as status codes without touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2212_05159_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "csrad.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(csr_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(capi.LIB_PATH):
        pytest.skip("libcsrad.so not built")
    return capi.load()


def test_every_declared_symbol_is_exported_and_bound(lib):
    names = _declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), f"{n} missing from libcsrad.so"
    assert sorted(capi.exported_symbols()) == names


def _param_counts():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(csr_[a-z0-9_]+)\s*\(([^)]*)\)\s*;", txt):
        params = [p for p in m.group(2).split(",") if p.strip() and p.strip() != "void"]
        out[m.group(1)] = len(params)
    return out


def test_binding_argument_counts_match_header():
    # A ctypes signature with the wrong arity shifts every later argument.
    counts = _param_counts()
    for name, (_, args) in capi._SIGS.items():
        assert len(args) == counts[name], f"{name}: binding has {len(args)} args, header {counts[name]}"


def test_status_strings(lib):
    for st in range(-7, 1):
        s = lib.csr_status_string(st).decode()
        assert s and s != "unknown status"
    assert lib.csr_status_string(-99).decode() == "unknown status"


def test_argument_errors_return_codes(lib):
    # Null descriptors / bad shapes are rejected on the host before any launch.
    assert lib.csr_spmv_fwd(None, None, None, None) == -1
    d = capi.csrad_csr(4, 4, 3, 7, 1, 1, 1)  # bogus dtype
    assert lib.csr_spmv_fwd(C.byref(d), 1, 1, None) == -2
    d = capi.csrad_csr(-1, 4, 0, 0, 1, None, None)
    assert lib.csr_spmv_fwd(C.byref(d), 1, 1, None) == -1
    d = capi.csrad_csr(4, 4, 4, 0, 1, 1, 1)
    assert lib.csr_spmm_fwd(C.byref(d), 0, 1, 1, 1, 1, None, None) == -1      # k <= 0
    assert lib.csr_spmm_fwd(C.byref(d), 8, 1, 4, 1, 8, None, None) == -1      # ldb < k
    bad_plan = capi.csrad_plan(5, 0)  # stride without a tile
    assert lib.csr_spmm_fwd(C.byref(d), 8, 1, 8, 1, 8, C.byref(bad_plan), None) == -1
    big_plan = capi.csrad_plan(99, 16)  # stride beyond the row count
    assert lib.csr_spmm_fwd(C.byref(d), 8, 1, 8, 1, 8, C.byref(big_plan), None) == -1
    sz = C.c_size_t(0)
    assert lib.csr_transpose_workspace(C.byref(d), C.byref(sz)) == 0 and sz.value > 0
    # too-small workspace is reported, not overrun
    assert lib.csr_transpose(C.byref(d), 1, 1, 1, 1, 8, None) == -5
    e = capi.csrad_csr(4, 5, 4, 0, 1, 1, 1)
    assert lib.csr_spgemm_workspace(C.byref(d), C.byref(e), C.byref(sz)) == 0
    f = capi.csrad_csr(5, 4, 4, 0, 1, 1, 1)  # inner dimensions disagree
    nnz = C.c_int64(0)
    assert lib.csr_spgemm_symbolic(C.byref(d), C.byref(f), 1, C.byref(nnz), None, 1, 1 << 30,
                                   None) == -1
    g = capi.csrad_csr(4, 4, 4, 1, 1, 1, 1)  # dtype mismatch between A and B
    assert lib.csr_spgemm_symbolic(C.byref(d), C.byref(g), 1, C.byref(nnz), None, 1, 1 << 30,
                                   None) == -2
    # non-square triangular operand
    assert lib.csr_trisolve_fwd(C.byref(e), 1, 1, None, None, None, 1, 1, None) == -1


def test_sparse_add_and_inverse_factor_argument_errors(lib):
    # sparse + sparse: operands of different shapes, missing outputs, dtype mismatch
    d = capi.csrad_csr(4, 4, 4, 0, 1, 1, 1)
    e = capi.csrad_csr(4, 5, 4, 0, 1, 1, 1)
    sz = C.c_size_t(0)
    assert lib.csr_spadd_workspace(C.byref(d), C.byref(d), C.byref(sz)) == 0 and sz.value > 0
    assert lib.csr_spadd_workspace(C.byref(d), C.byref(e), C.byref(sz)) == -1
    nnz = C.c_int64(0)
    assert lib.csr_spadd_symbolic(C.byref(d), C.byref(d), None, C.byref(nnz), 1, 1 << 30,
                                  None) == -1
    assert lib.csr_spadd_symbolic(C.byref(d), C.byref(d), 1, C.byref(nnz), 1, 8, None) == -5
    g = capi.csrad_csr(4, 4, 4, 1, 1, 1, 1)
    assert lib.csr_spadd_fwd(C.byref(d), C.byref(g), 1.0, 1.0, 1, 1, 1, None) == -2
    assert lib.csr_spadd_fwd(C.byref(d), C.byref(d), 1.0, 1.0, 1, 1, None, None) == -1
    assert lib.csr_spadd_bwd(C.byref(d), C.byref(d), C.byref(e), 1.0, 1.0, 1, 1, 1, None) == -1
    # PCG kind 3 (inverse factor): L and its transpose are required, shapes must agree
    assert lib.csr_pcg_step(C.byref(d), 3, None, None, None, None, 0, None, None, None,
                            1, 1, 1, 1, 1, 1, None, 0, 1, 1 << 30, None) == -1
    Lt = capi.csrad_csr(4, 4, 3, 0, 1, 1, None)  # nnz differs from L's
    assert lib.csr_pcg_step(C.byref(d), 3, None, C.byref(d), C.byref(Lt), 1, 0, None, None,
                            None, 1, 1, 1, 1, 1, 1, None, 0, 1, 1 << 30, None) == -1


def test_split_spmv_bwd_argument_errors(lib):
    # the paired split backward needs A^T (of A's transposed shape), perm and
    # both outputs; every refusal comes back before any launch
    d = capi.csrad_csr(4, 5, 4, 0, 1, 1, 1)
    t = capi.csrad_csr(5, 4, 4, 0, 1, 1, None)
    assert lib.csr_spmv_bwd_split(C.byref(d), None, 1, 1, 1, 1, 1, None) == -1
    assert lib.csr_spmv_bwd_split(C.byref(d), C.byref(t), None, 1, 1, 1, 1, None) == -1
    assert lib.csr_spmv_bwd_split(C.byref(d), C.byref(t), 1, 1, 1, None, 1, None) == -1
    assert lib.csr_spmv_bwd_split(C.byref(d), C.byref(t), 1, 1, 1, 1, None, None) == -1
    same = capi.csrad_csr(4, 5, 4, 0, 1, 1, None)  # A's own shape, not A^T's
    assert lib.csr_spmv_bwd_split(C.byref(d), C.byref(same), 1, 1, 1, 1, 1, None) == -1
    bad = capi.csrad_csr(4, 5, 4, 7, 1, 1, 1)  # unknown value type
    assert lib.csr_spmv_bwd_split(C.byref(bad), C.byref(t), 1, 1, 1, 1, 1, None) == -2
