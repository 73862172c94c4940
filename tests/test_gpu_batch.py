"""Batched block-diagonal execution: one launch per op over uneven blocks
must give, block by block, what each block gives alone, and match the FP64
oracle.  Integer structure (level sets) and every result whose reduction
shape does not depend on the matrix's mean row length (SpMM and its
backward, value gradients of SpMV) are bit-identical; row sums whose lane
count follows the mean row length (SpMV, A^T products of SpMV,
tri-solves) may round differently and are held to 1e-6."""
import numpy as np
import pytest
import torch

import oracle
from paper_2212_05159_amd import batch as bt
from paper_2212_05159_amd import gen
from paper_2212_05159_amd import sparse as sp

from _util import assert_close, to_dev, upcast

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def blocks():
    # uneven random geometric-graph Laplacians (the batched workload's recipe,
    # smaller sizes)
    return bt.geometric_batch(12, n_range=(300, 5000), k_range=(6, 14))


def test_batched_spmv_spmm_equal_per_block(blocks):
    B = bt.Batch(blocks)
    n = B.A.pattern.nrows
    x = to_dev(gen.normal(n, 1), torch.float32)
    X = to_dev(gen.normal((n, 64), 2), torch.float32)
    G = to_dev(gen.normal((n, 64), 3), torch.float32)
    gy = to_dev(gen.normal(n, 4), torch.float32)
    y = sp.spmv(B.pattern, B.A.vals, x)
    gx, gv = sp.spmv_bwd(B.pattern, B.A.vals, x, gy)
    Cm = sp.spmm(B.pattern, B.A.vals, X)
    gX, gvm = sp.spmm_bwd(B.pattern, B.A.vals, X, G)
    nnz_off = np.concatenate([[0], np.cumsum([b.nnz for b in blocks])])
    for i, blk in enumerate(blocks):
        a, c = int(B.block_rowptr[i]), int(B.block_rowptr[i + 1])
        Ab = sp.CsrTensor.from_host(blk, dtype=torch.float32)
        sl = slice(int(nnz_off[i]), int(nnz_off[i + 1]))
        y1 = sp.spmv(Ab.pattern, Ab.vals, x[a:c].contiguous())
        assert torch.allclose(y[a:c], y1, rtol=1e-6, atol=1e-6 * float(y1.abs().max()))
        gxb, gvb = sp.spmv_bwd(Ab.pattern, Ab.vals, x[a:c].contiguous(), gy[a:c].contiguous())
        assert torch.allclose(gx[a:c], gxb, rtol=1e-6, atol=1e-6 * float(gxb.abs().max()))
        assert torch.equal(gv[sl], gvb)
        assert torch.equal(Cm[a:c], sp.spmm(Ab.pattern, Ab.vals, X[a:c].contiguous()))
        gXb, gvmb = sp.spmm_bwd(Ab.pattern, Ab.vals, X[a:c].contiguous(), G[a:c].contiguous())
        assert torch.equal(gX[a:c], gXb) and torch.equal(gvm[sl], gvmb)
    Ao = upcast(B.host, torch.float32)
    assert_close(Cm, oracle.spmm(Ao, X.double().cpu().numpy()), torch.float32, "C")


def test_batched_trisolve_levels_and_values(blocks):
    Ls = [gen.tril(b) for b in blocks]
    B = bt.Batch(Ls)
    n = B.A.pattern.nrows
    b = to_dev(gen.normal(n, 5), torch.float32)
    g = to_dev(gen.normal(n, 6), torch.float32)
    nl, lph, lp, lr, lor = B.pattern.levels(True)
    xb = sp.trisolve(B.pattern, B.A.vals, b, True)
    gbb, gvb = sp.trisolve_bwd(B.pattern, B.A.vals, xb, g, True)
    lo, lpo, lro = oracle.levels(B.host, True)
    assert np.array_equal(lor.cpu().numpy(), lo) and np.array_equal(lr.cpu().numpy(), lro)
    levels_per_block = []
    nnz_off = np.concatenate([[0], np.cumsum([m.nnz for m in Ls])])
    for i, blk in enumerate(Ls):
        a, c = int(B.block_rowptr[i]), int(B.block_rowptr[i + 1])
        Tb = sp.CsrTensor.from_host(blk, dtype=torch.float32)
        nlb, _, _, _, lorb = Tb.pattern.levels(True)
        levels_per_block.append(nlb)
        assert torch.equal(lor[a:c], lorb)  # a row keeps its level
        x1 = sp.trisolve(Tb.pattern, Tb.vals, b[a:c].contiguous(), True)
        close = lambda u, v: torch.allclose(u, v, rtol=1e-6, atol=1e-6 * float(v.abs().max()))
        assert close(xb[a:c], x1)
        gb1, gv1 = sp.trisolve_bwd(Tb.pattern, Tb.vals, x1, g[a:c].contiguous(), True)
        assert close(gbb[a:c], gb1)
        assert close(gvb[int(nnz_off[i]):int(nnz_off[i + 1])], gv1)
    assert nl == max(levels_per_block)
    To = upcast(B.host, torch.float32)
    xo = oracle.trisolve(To, b.double().cpu().numpy(), True)
    assert_close(xb, xo, torch.float32, "x")
