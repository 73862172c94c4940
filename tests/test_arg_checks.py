"""Host-side argument checks of the functional forms: a tensor on the wrong
device, of another value type or of the wrong length raises before any
kernel launch (the C ABI sees only bare pointers).  The CPU tests drive
the checks with host tensors; the GPU tests call the real forms."""
import numpy as np
import pytest
import torch

from paper_2212_05159_amd import gen
from paper_2212_05159_amd import sparse as sp


def _cpu_pattern(m):
    return sp.Pattern(m.nrows, m.ncols, torch.as_tensor(m.rowptr.astype(np.int32)),
                      torch.as_tensor(m.colind.astype(np.int32)))


def test_host_values_rejected_before_launch():
    A = gen.poisson2d(4, 4)
    P = _cpu_pattern(A)
    v = torch.as_tensor(A.vals)
    x = torch.zeros(A.ncols, dtype=torch.float64)
    for call in (lambda: sp.spmv(P, v, x),
                 lambda: sp.spmv_bwd(P, v, x, x),
                 lambda: sp.spmm(P, v, torch.zeros(A.ncols, 4, dtype=torch.float64)),
                 lambda: sp.transpose_vals(P, v)):
        with pytest.raises(TypeError, match="CUDA"):
            call()


def test_dense_checks_on_host_tensors():
    ref = torch.zeros(5, dtype=torch.float32)
    sp._check_dense(torch.zeros(7, dtype=torch.float32), ref, (7,), "x")
    with pytest.raises(TypeError, match="dtype"):
        sp._check_dense(torch.zeros(7, dtype=torch.float64), ref, (7,), "x")
    with pytest.raises(ValueError, match="shape"):
        sp._check_dense(torch.zeros(6, dtype=torch.float32), ref, (7,), "x")
    with pytest.raises(ValueError, match="contiguous"):
        sp._check_dense(torch.zeros(14, dtype=torch.float32)[::2], ref, (7,), "x")
    with pytest.raises(ValueError, match="unit-stride"):
        sp._check_dense(torch.zeros(4, 7, dtype=torch.float32).t(), ref, (7, 4), "B")
    with pytest.raises(TypeError, match="tensor"):
        sp._check_dense(np.zeros(7, np.float32), ref, (7,), "x")


def test_value_array_checks_on_host_tensors():
    A = gen.poisson2d(3, 3)
    P = _cpu_pattern(A)
    with pytest.raises(TypeError, match="float32 or float64"):
        sp._check_vals(P, torch.zeros(A.nnz, dtype=torch.int32))
    with pytest.raises(TypeError, match="tensor"):
        sp._check_vals(P, A.vals)


@pytest.mark.gpu
def test_gpu_forms_reject_bad_operands():
    A = gen.poisson2d(8, 8)
    At = sp.CsrTensor.from_host(A, dtype=torch.float32)
    P, v = At.pattern, At.vals
    n = A.nrows
    good = torch.zeros(n, dtype=torch.float32, device="cuda")
    with pytest.raises(TypeError, match="cuda"):
        sp.spmv(P, v, torch.zeros(n, dtype=torch.float32))           # host x
    with pytest.raises(TypeError, match="dtype"):
        sp.spmv(P, v, torch.zeros(n, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="shape"):
        sp.spmv(P, v, torch.zeros(n - 1, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError, match="shape"):
        sp.spmv_bwd(P, v, good, good[:-1])
    with pytest.raises(ValueError, match="shape"):
        sp.spmm(P, v, torch.zeros(n - 3, 8, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError, match="shape"):
        sp.spmm_bwd(P, v, torch.zeros(n, 8, dtype=torch.float32, device="cuda"),
                    torch.zeros(n, 4, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError, match="nnz"):
        sp.spmv(P, v[:-1], good)
    L = sp.CsrTensor.from_host(gen.tril(A), dtype=torch.float32)
    with pytest.raises(ValueError, match="shape"):
        sp.trisolve(L.pattern, L.vals, good[:-2])
    with pytest.raises(TypeError, match="dtype"):
        sp.trisolve(L.pattern, L.vals, good.double())
    # the valid call still works after the rejected ones
    y = sp.spmv(P, v, torch.ones(n, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    assert torch.isfinite(y).all()
