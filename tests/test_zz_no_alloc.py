"""The workspace-free transpose (csr_transpose_noalloc) against the
workspace form (csr_transpose) through the C ABI: two calls in a row on one
stream, the second with a smaller input, each bit-identical to the
workspace form on the same pattern; a pattern whose transpose needs more
than the static scratch is refused on the host."""
import numpy as np
import pytest
import torch

from paper_2212_05159_amd import capi, gen

pytestmark = pytest.mark.gpu


def _dev_pattern(A):
    rp = torch.as_tensor(A.rowptr.astype(np.int32)).cuda()
    ci = torch.as_tensor(A.colind.astype(np.int32)).cuda()
    return rp, ci


def _with_workspace(A, rp, ci):
    d = capi.desc(A.nrows, A.ncols, rp, ci, dtype=torch.float32)
    ws = torch.empty(capi.csr_transpose_workspace(d), dtype=torch.uint8, device="cuda")
    rpT = torch.empty(A.ncols + 1, dtype=torch.int32, device="cuda")
    ciT = torch.empty(max(A.nnz, 1), dtype=torch.int32, device="cuda")
    perm = torch.empty(max(A.nnz, 1), dtype=torch.int32, device="cuda")
    capi.csr_transpose(d, rpT, ciT, perm, ws)
    return rpT, ciT[:A.nnz], perm[:A.nnz]


def _noalloc(A, rp, ci):
    d = capi.desc(A.nrows, A.ncols, rp, ci, dtype=torch.float32)
    rpT = torch.full((A.ncols + 1,), -7, dtype=torch.int32, device="cuda")
    ciT = torch.full((max(A.nnz, 1),), -7, dtype=torch.int32, device="cuda")
    perm = torch.full((max(A.nnz, 1),), -7, dtype=torch.int32, device="cuda")
    capi.csr_transpose_noalloc(d, rpT, ciT, perm)
    return rpT, ciT[:A.nnz], perm[:A.nnz]


# general path (random rows, heavy-tailed rows), then smaller inputs of each
# path the transpose has: symmetric square pattern, general, column-sorted
CASES = [
    ("random_large", gen.random_rows(60000, 50000, 10, seed=[7, 1])),
    ("power_law", gen.power_law_rows(20000, seed=[7, 3], max_len=3000, empty=0.05)),
    ("poisson3d", gen.poisson3d(24)),
    ("random_small", gen.random_csr(3000, 2000, 0.004, seed=[7, 2], empty_rows=0.1)),
    ("aggregation", gen.aggregation(4097, 8)),
]


def test_noalloc_transpose_matches_workspace_form_on_calls_in_a_row():
    torch.cuda.synchronize()
    for name, A in CASES:
        rp, ci = _dev_pattern(A)
        want = _with_workspace(A, rp, ci)
        got = _noalloc(A, rp, ci)
        torch.cuda.synchronize()
        for w, g, what in zip(want, got, ("rowptrT", "colindT", "perm")):
            assert torch.equal(w, g), f"{name}: {what} differs from csr_transpose"


def test_noalloc_transpose_refuses_patterns_beyond_the_scratch():
    cap = capi.csr_noalloc_scratch_bytes()
    assert cap == 64 << 20
    # a descriptor whose transpose would need about 2*nnz*4 bytes > cap;
    # refused on the host before any launch (pointers are never read)
    nnz = cap // 8 + 1
    rp = torch.zeros(2, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    d = capi.csrad_csr(1, 1, nnz, 0, rp.data_ptr(), ci.data_ptr(), None)
    out = torch.empty(2, dtype=torch.int32, device="cuda")
    st = capi.load().csr_transpose_noalloc(capi.C.byref(d), out.data_ptr(), out.data_ptr(),
                                           out.data_ptr(), None)
    assert st == -5
