"""Pins for the reference of the sparse approximate inverse by direct
minimisation (Section 4.6).

Independent checks: the sparse composition's loss equals the row-wise sum
of least-squares residuals the section states; its gradient matches
central differences; the row-wise least-squares optimum has zero
gradient and beats perturbations of itself; a diagonal A gives M = A^{-1}
with zero loss; the paper's start M = mask(A) on the 8x8 Poisson matrix
gives the dense product's loss (3032)."""
import numpy as np

from oracle import spai_ref
from paper_2212_05159_amd import gen


def _rowwise_loss(A, Mv):
    n = A.nrows
    Ad = A.todense()
    total = 0.0
    for i in range(n):
        S = A.colind[A.rowptr[i]:A.rowptr[i + 1]]
        e = np.zeros(n)
        e[i] = 1.0
        total += np.sum((e - Ad[S, :].T @ Mv[A.rowptr[i]:A.rowptr[i + 1]]) ** 2)
    return total


def test_loss_equals_rowwise_least_squares_residuals(orc):
    A = gen.random_csr(30, 30, 0.15, seed=1, empty_rows=0.1)
    Mv = gen.normal(A.nnz, seed=2)
    loss, _ = spai_ref.loss_and_grad(A, Mv)
    assert abs(loss - _rowwise_loss(A, Mv)) <= 1e-11 * loss


def test_gradient_matches_central_differences(orc):
    A = gen.poisson2d(5, 4)
    Mv = 0.3 * gen.normal(A.nnz, seed=3)
    _, g = spai_ref.loss_and_grad(A, Mv)
    h = 1e-6
    for e in (0, 7, 30, A.nnz - 1):
        p, m = Mv.copy(), Mv.copy()
        p[e] += h
        m[e] -= h
        fd = (spai_ref.loss_and_grad(A, p)[0] - spai_ref.loss_and_grad(A, m)[0]) / (2 * h)
        assert abs(fd - g[e]) < 1e-6 * max(1.0, abs(fd))


def test_optimum_is_stationary_and_minimal(orc):
    A = gen.poisson2d(6, 6)
    Mo = spai_ref.optimum(A)
    lo, g = spai_ref.loss_and_grad(A, Mo)
    assert np.linalg.norm(g) < 1e-10
    rng = np.random.default_rng(4)
    for _ in range(3):
        assert spai_ref.loss_and_grad(A, Mo + 1e-3 * rng.standard_normal(A.nnz))[0] > lo


def test_diagonal_system_is_inverted_exactly(orc):
    d = np.linspace(1.0, 3.0, 9)
    A = gen.Csr(9, 9, np.arange(10, dtype=np.int32), np.arange(9, dtype=np.int32), d)
    Mo = spai_ref.optimum(A)
    np.testing.assert_allclose(Mo, 1.0 / d, rtol=1e-14)
    assert spai_ref.loss_and_grad(A, Mo)[0] < 1e-28


def test_paper_start_loss_8x8(orc):
    """M = mask(A), the paper's starting point: the sparse composition gives
    the dense product's loss, 3032."""
    A = gen.poisson2d(8, 8)
    loss, _ = spai_ref.loss_and_grad(A, np.ones(A.nnz))
    Ad = A.todense()
    M = (Ad != 0).astype(float)
    assert loss == np.sum((np.eye(64) - M @ Ad) ** 2) == 3032.0
