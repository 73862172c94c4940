"""Pins for the oracle's PCG with the approximate-inverse preconditioner
M = L L^T of Section 4.3 (z = L (L^T r)).

Independent checks: a diagonal L = D^{-1/2} gives Jacobi's iterates and
L = I gives plain CG's (other branches of the oracle), an exact inverse
factor (L L^T = A^{-1}, dense Cholesky of the inverse) converges in one
step, and the first residual matches dense NumPy arithmetic with M = L L^T
(so a transposed product M = L^T L would fail it).  The reference loss of
the learned form: a diagonal L gives the same loss as the factor form with
the reciprocal diagonal (the same M, through triangular solves), and its
gradient matches central differences."""
import numpy as np
import torch

from oracle import mpnn_ref
from paper_2212_05159_amd import gen


def _diag_csr(d):
    n = len(d)
    return gen.Csr(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                   np.asarray(d, np.float64))


def _dense_lower(Ld):
    rows, cols = np.nonzero(np.tril(np.ones_like(Ld, dtype=bool)))
    return gen._from_coo(Ld.shape[0], Ld.shape[1], rows, cols, Ld[rows, cols])


def test_diagonal_factor_is_jacobi(orc):
    A = gen.anisotropic_q1(12, 1e-2, 0.7)
    b = gen.normal(A.nrows, seed=1)
    L = _diag_csr(1.0 / np.sqrt(np.diag(A.todense())))
    _, it_f, h_f = orc.pcg(A, b, "fsai", L=L, tol=1e-8)
    _, it_j, h_j = orc.pcg(A, b, "jacobi", tol=1e-8)
    assert it_f == it_j > 5
    np.testing.assert_allclose(h_f, h_j, rtol=1e-9, atol=0)


def test_identity_factor_is_plain_cg(orc):
    A = gen.poisson2d(9, 7)
    b = gen.normal(A.nrows, seed=2)
    _, it_f, h_f = orc.pcg(A, b, "fsai", L=_diag_csr(np.ones(A.nrows)), tol=1e-10)
    _, it_n, h_n = orc.pcg(A, b, "none", tol=1e-10)
    assert it_f == it_n
    np.testing.assert_array_equal(h_f, h_n)


def test_exact_inverse_factor_converges_in_one_step(orc):
    A = gen.poisson2d(6, 5)
    Ainv = np.linalg.inv(A.todense())
    L = _dense_lower(np.linalg.cholesky(Ainv))
    b = gen.normal(A.nrows, seed=3)
    _, it, h = orc.pcg(A, b, "fsai", L=L, tol=1e-10)
    assert it == 1 and h[1] < 1e-12


def test_first_residual_matches_dense_m_equals_l_lt(orc):
    A = gen.poisson2d(8, 8)
    Ad = A.todense()
    rng = np.random.default_rng(4)
    Ld = np.tril(rng.standard_normal((64, 64)) * (rng.random((64, 64)) < 0.15), -1)
    Ld += np.diag(0.5 + rng.random(64))
    L = _dense_lower(Ld)
    L = gen.Csr(L.nrows, L.ncols, L.rowptr, L.colind, L.vals)
    b = gen.normal(64, seed=5)
    M = Ld @ Ld.T
    z = M @ b
    alpha = (b @ z) / (z @ Ad @ z)
    r1 = b - alpha * (Ad @ z)
    _, _, h = orc.pcg(A, b, "fsai", L=L, tol=0.0, maxit=1)
    assert abs(h[1] - np.linalg.norm(r1) / np.linalg.norm(b)) < 1e-13
    # the transposed form would differ
    Mt = Ld.T @ Ld
    zt = Mt @ b
    rt = b - (b @ zt) / (zt @ Ad @ zt) * (Ad @ zt)
    assert abs(np.linalg.norm(rt) - np.linalg.norm(r1)) / np.linalg.norm(b) > 1e-6


def test_loss_diagonal_fsai_equals_factor_form():
    A = gen.poisson2d(8, 8)
    Lp = gen.tril(A)
    d = np.diag(A.todense())
    diag = Lp.rowptr[1:] - 1  # the diagonal is last in each row of tril(A)
    v_inv = np.zeros(Lp.nnz)
    v_inv[diag] = 1.0 / np.sqrt(d)
    v_fac = np.zeros(Lp.nnz)
    v_fac[diag] = np.sqrt(d)
    b = gen.normal(64, seed=6)
    l_inv = mpnn_ref.pcg_loss(A, Lp, torch.as_tensor(v_inv), b, form="fsai")
    l_fac = mpnn_ref.pcg_loss(A, Lp, torch.as_tensor(v_fac), b, form="factor")
    assert abs(float(l_inv) - float(l_fac)) < 1e-13 * float(l_fac)


def test_loss_fsai_gradient_matches_central_differences():
    A = gen.poisson2d(8, 8)
    rows = np.arange(64)
    P = gen._from_coo(64, 64, np.concatenate([rows, rows[1:]]),
                      np.concatenate([rows, rows[:-1]]), np.ones(127))  # bidiagonal
    rng = np.random.default_rng(7)
    v = 0.5 + 0.1 * rng.standard_normal(P.nnz)
    b = gen.normal(64, seed=8)
    t = torch.as_tensor(v).requires_grad_(True)
    mpnn_ref.pcg_loss(A, P, t, b, form="fsai").backward()
    h = 1e-6
    for e in (0, 5, 40, 100):
        vp, vm = v.copy(), v.copy()
        vp[e] += h
        vm[e] -= h
        fd = (float(mpnn_ref.pcg_loss(A, P, torch.as_tensor(vp), b, form="fsai")) -
              float(mpnn_ref.pcg_loss(A, P, torch.as_tensor(vm), b, form="fsai"))) / (2 * h)
        assert abs(fd - float(t.grad[e])) < 1e-6 * max(1.0, abs(fd)), (e, fd, float(t.grad[e]))
