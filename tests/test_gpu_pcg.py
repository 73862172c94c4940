"""GPU parity of PCG (Section 4.3) against the FP64 oracle.

Float64 runs (float64 vectors and dots) reproduce the oracle's residual
history entry by entry within 10x the oracle's own rounding band plus
1e-12 (how far the oracle's history moves when b is perturbed at the level
of float64 rounding: the GPU takes every sum in another order, which is a
perturbation of that size at every step), and stop within one step of it; exact factors converge in one step; float32
values with float64 vectors reach ||b - A x||/||b|| <= 1e-6 (checked on the
host in float64); breakdowns are reported and fall back to Jacobi."""
import numpy as np
import pytest
import torch

import oracle
from paper_2212_05159_amd import gen
from paper_2212_05159_amd import pcg as pcgmod
from paper_2212_05159_amd import sparse as sp

from _util import assert_pcg_f64_parity, pcg_rounding_band, rel_err, to_dev, true_residual, upcast

pytestmark = pytest.mark.gpu


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    M = (rng.random((n, n)) < 0.03) * rng.standard_normal((n, n))
    S = np.triu(M, 1)
    S = S + S.T
    S += np.diag(np.abs(S).sum(1) * 0.6 + 0.05 + rng.random(n))
    r, c = np.nonzero(S)
    return gen._from_coo(n, n, r, c, S[r, c])


@pytest.mark.parametrize("precond", ["jacobi", "none"])
@pytest.mark.parametrize("name,mk", [("spd400", lambda: _spd(400, 1)),
                                     ("q1_aniso40", lambda: gen.anisotropic_q1(40, 1e-2, 0.4))],
                         ids=["spd400", "q1_aniso40"])
def test_pcg_fp64_matches_oracle(precond, name, mk):
    A = mk()
    b = gen.normal(A.nrows, 2)
    Ad = sp.CsrTensor.from_host(A, dtype=torch.float64)
    x, info = pcgmod.pcg(Ad, to_dev(b), precond=precond, tol=1e-8, record=True)
    ref = pcg_rounding_band(A, b, precond, tol=1e-8)
    assert info["converged"] and ref["iters"] > 0
    assert_pcg_f64_parity(info, x, ref, f"{name}/{precond}")
    assert true_residual(A, x, b) < 2e-8


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_pcg_arrow_matrix_reads_csr_rows(dtype):
    # one dense row and column: A's ELL copy would need n slots per row, far
    # beyond twice nnz(A), so the product reads A's CSR rows instead
    n = 3000
    r = np.concatenate([np.arange(n), np.zeros(n - 1, int), np.arange(1, n)])
    c = np.concatenate([np.arange(n), np.arange(1, n), np.zeros(n - 1, int)])
    v = np.concatenate([[float(n)], np.full(n - 1, 2.0), np.full(2 * (n - 1), -0.5)])
    A = gen._from_coo(n, n, r, c, v)
    b = gen.normal(n, 8)
    Ad = sp.CsrTensor.from_host(A, dtype=dtype)
    x, info = pcgmod.pcg(Ad, to_dev(b), precond="jacobi", tol=1e-8, record=True)
    Ao = upcast(A, dtype)
    ref = pcg_rounding_band(Ao, b, "jacobi", tol=1e-8)
    assert info["converged"]
    assert_pcg_f64_parity(info, x, ref, "arrow")
    assert true_residual(Ao, x, b) < 2e-8


def test_pcg_exact_factor_converges_in_one_step():
    A = gen.poisson1d(500)
    Lp = gen.tril(A)
    L = gen.Csr(500, 500, Lp.rowptr, Lp.colind, oracle.ic0(A, Lp))
    b = gen.normal(500, 3)
    Ad = sp.CsrTensor.from_host(A, dtype=torch.float64)
    Ld = sp.CsrTensor.from_host(L, dtype=torch.float64)
    x, info = pcgmod.pcg(Ad, to_dev(b), precond="factor", L=Ld, tol=1e-10)
    assert info["converged"] and info["iters"] == 1
    assert true_residual(A, x, b) < 1e-10


@pytest.mark.parametrize("graph", [False, True])
def test_pcg_fp32_values_reach_1e6(graph):
    A = gen.anisotropic_q1(96, 1e-3, np.pi / 4)
    b = gen.normal(A.nrows, 4)
    Ad = sp.CsrTensor.from_host(A, dtype=torch.float32)
    x, info = pcgmod.pcg(Ad, to_dev(b), precond="jacobi", tol=1e-6, graph=graph)
    assert info["converged"]
    # the system solved is the float32-rounded matrix
    assert true_residual(upcast(A, torch.float32), x, b) <= 1.05e-6
    _, ito, _ = oracle.pcg(upcast(A, torch.float32), b, "jacobi", tol=1e-6)
    assert abs(info["iters"] - ito) <= 2


def test_pcg_factor_matches_oracle_factor():
    # a non-exact factor: L = (D + tril) D^{-1/2} (symmetric Gauss-Seidel)
    A = gen.anisotropic_q1(48, 1e-2, 1.1)
    T = gen.tril(A)
    rows = T.row_of_entry()
    d = np.zeros(A.nrows)
    d[rows[T.colind == rows]] = T.vals[T.colind == rows]
    L = gen.Csr(A.nrows, A.ncols, T.rowptr, T.colind, T.vals / np.sqrt(d[T.colind]))
    b = gen.normal(A.nrows, 5)
    Ad = sp.CsrTensor.from_host(A, dtype=torch.float64)
    Ld = sp.CsrTensor.from_host(L, dtype=torch.float64)
    x, info = pcgmod.pcg(Ad, to_dev(b), precond="factor", L=Ld, tol=1e-8, record=True)
    ref = pcg_rounding_band(A, b, "factor", L=L, tol=1e-8)
    assert info["converged"]
    assert_pcg_f64_parity(info, x, ref, "sgs-factor")
    _, itj, _ = oracle.pcg(A, b, "jacobi", tol=1e-8)
    assert ref["iters"] < itj  # the factor helps


def _sgs_factor(A):
    T = gen.tril(A)
    rows = T.row_of_entry()
    d = np.zeros(A.nrows)
    d[rows[T.colind == rows]] = T.vals[T.colind == rows]
    return gen.Csr(A.nrows, A.ncols, T.rowptr, T.colind, T.vals / np.sqrt(d[T.colind]))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("graph", [False, True])
def test_pcg_level_ordered_factor_matches_oracle(dtype, graph):
    # four-coloured Q1 on 96^2: 4 levels of 2304 rows, so the steps solve
    # over the level-ordered copies of L and L^T
    N = 96
    A = gen.permute_sym(gen.anisotropic_q1(N, 3e-3, 0.7), gen.four_color_2d(N))
    L = _sgs_factor(A)
    Ad = sp.CsrTensor.from_host(A, dtype=dtype)
    Ld = sp.CsrTensor.from_host(L, dtype=dtype)
    nl, lph, _, _, _ = Ld.pattern.levels(True)
    assert nl == 4 and np.diff(lph).min() >= 1024
    Lh = Ld.pattern.desc(Ld.vals)
    from paper_2212_05159_amd import capi
    assert capi.csr_pcg_workspace(Ad.pattern.desc(Ad.vals), Lh, nl, lph) > \
        capi.csr_pcg_workspace(Ad.pattern.desc(Ad.vals))
    b = gen.normal(A.nrows, 7)
    Ao, Lo = upcast(A, dtype), upcast(L, dtype)
    x, info = pcgmod.pcg(Ad, to_dev(b), precond="factor", L=Ld, tol=1e-8, graph=graph,
                         record=not graph)
    ref = pcg_rounding_band(Ao, b, "factor", L=Lo, tol=1e-8)
    assert info["converged"]
    if graph:
        info["hist"] = ref["hist"][1:]  # no history under capture: x and the count only
    assert_pcg_f64_parity(info, x, ref, f"level-ordered/{dtype}/graph={graph}")
    assert true_residual(Ao, x, b) < 2e-8


def test_pcg_ell_factor_interleaved_levels():
    # L with even rows on level 0 and odd rows on level 1 (levels interleave
    # in the row order, each with 2048 rows): the solves go through the
    # level-row lists
    A = gen.poisson2d(64, 64)
    n = A.nrows
    r, c, v = list(range(n)), list(range(n)), [2.0] * n
    for i in range(1, n, 2):
        for d, w in ((1, -0.5), (3, -0.25)):
            if i - d >= 0:
                r.append(i), c.append(i - d), v.append(w)
    L = gen._from_coo(n, n, np.array(r), np.array(c), np.array(v))
    Ad = sp.CsrTensor.from_host(A, dtype=torch.float64)
    Ld = sp.CsrTensor.from_host(L, dtype=torch.float64)
    nl, lph, _, lr, _ = Ld.pattern.levels(True)
    assert nl == 2 and np.diff(lph).min() >= 1024
    assert not np.array_equal(lr.cpu().numpy(), np.arange(n))
    b = gen.normal(n, 9)
    x, info = pcgmod.pcg(Ad, to_dev(b), precond="factor", L=Ld, tol=1e-8, record=True)
    ref = pcg_rounding_band(A, b, "factor", L=L, tol=1e-8)
    assert info["converged"]
    assert_pcg_f64_parity(info, x, ref, "interleaved")
    assert true_residual(A, x, b) < 2e-8


def test_pcg_breakdown_falls_back_to_jacobi():
    A = gen.poisson2d(20, 20)
    T = gen.tril(A)
    bad = gen.Csr(A.nrows, A.ncols, T.rowptr, T.colind,
                  np.where(T.colind == T.row_of_entry(), 0.0, T.vals))  # zero diagonal
    b = gen.normal(A.nrows, 6)
    Ad = sp.CsrTensor.from_host(A, dtype=torch.float64)
    Ld = sp.CsrTensor.from_host(bad, dtype=torch.float64)
    x, info = pcgmod.pcg(Ad, to_dev(b), precond="factor", L=Ld, tol=1e-8, fallback=False)
    assert info["breakdown"] and not info["converged"]
    x, info = pcgmod.pcg(Ad, to_dev(b), precond="factor", L=Ld, tol=1e-8, fallback=True)
    assert info["fallback"] and info["converged"]
    assert true_residual(A, x, b) < 2e-8
