"""Pins for the oracle's CG, its reverse mode, PCG and the residual-history
loss of Section 4.3.

Independent checks: CG in exact-enough arithmetic reaches A^{-1} b after n
steps (NumPy dense solve); torch float64 autograd through the unrolled
iteration; central differences; the SpSolve VJP of Table 1 as the limit of
the CG gradient; Jacobi-PCG equals CG for a constant diagonal; an exact
Cholesky factor converges in one step."""
import numpy as np
import pytest
import torch

from paper_2212_05159_amd import gen


def _spd(n, seed):
    # Symmetric, diagonally dominant, with a random sparse pattern.
    rng = np.random.default_rng(seed)
    M = (rng.random((n, n)) < 0.2) * rng.standard_normal((n, n))
    S = np.triu(M, 1)
    S = S + S.T
    S += np.diag(np.abs(S).sum(1) + 1.0 + rng.random(n))
    r, c = np.nonzero(S)
    return gen._from_coo(n, n, r, c, S[r, c])


def _torch_cg(Ad, b, K):
    x = torch.zeros_like(b)
    r = b.clone()
    p = r.clone()
    rho = r @ r
    rs = []
    for _ in range(K):
        q = Ad @ p
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        rho1 = r @ r
        p = r + (rho1 / rho) * p
        rho = rho1
        rs.append(r)
    return x, rs


def test_cg_reaches_solution_in_n_steps(orc):
    A = _spd(24, 1)
    b = gen.normal(24, 2)
    x = orc.cg(A, b, 24)
    np.testing.assert_allclose(x, np.linalg.solve(A.todense(), b), rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("K", [1, 3, 10])
def test_cg_bwd_vs_torch_autograd(orc, K):
    A = _spd(20, 3)
    b = gen.normal(20, 4)
    t = gen.normal(20, 5)
    x = orc.cg(A, b, K)
    gv, gb = orc.cg_bwd(A, b, K, gx=x - t)
    Ad = torch.tensor(A.todense(), requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    xt, _ = _torch_cg(Ad, bt, K)
    np.testing.assert_allclose(xt.detach().numpy(), x, rtol=1e-12, atol=1e-12)
    (0.5 * ((xt - torch.tensor(t)) ** 2).sum()).backward()
    np.testing.assert_allclose(gb, bt.grad.numpy(), rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(gv, Ad.grad.numpy()[A.row_of_entry(), A.colind], rtol=1e-9, atol=1e-11)


def test_cg_bwd_residual_history_vs_torch_autograd(orc):
    A = _spd(16, 6)
    b = gen.normal(16, 7)
    K = 4
    _, R = orc.cg(A, b, K, want_history=True)
    wts = gen.normal(K, 8)
    # loss = sum_i w_i ||r_i||  -> gR_i = w_i r_i / ||r_i||
    gR = wts[:, None] * R / np.linalg.norm(R, axis=1)[:, None]
    gv, gb = orc.cg_bwd(A, b, K, gR=gR)
    Ad = torch.tensor(A.todense(), requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    _, rs = _torch_cg(Ad, bt, K)
    sum(float(w) * torch.linalg.norm(r) for w, r in zip(wts, rs)).backward()
    np.testing.assert_allclose(gb, bt.grad.numpy(), rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(gv, Ad.grad.numpy()[A.row_of_entry(), A.colind], rtol=1e-9, atol=1e-11)


def test_cg_bwd_central_differences(orc):
    A = _spd(10, 9)
    b = gen.normal(10, 10)
    t = gen.normal(10, 11)
    K = 5

    def loss(vals, bb):
        x = orc.cg(gen.Csr(10, 10, A.rowptr, A.colind, vals), bb, K)
        return 0.5 * np.sum((x - t) ** 2)

    x = orc.cg(A, b, K)
    gv, gb = orc.cg_bwd(A, b, K, gx=x - t)
    h = 1e-6
    for e in range(0, A.nnz, 2):
        d = np.zeros(A.nnz); d[e] = h
        fd = (loss(A.vals + d, b) - loss(A.vals - d, b)) / (2 * h)
        assert abs(fd - gv[e]) < 1e-6 * (1 + abs(fd))
    for j in range(10):
        d = np.zeros(10); d[j] = h
        fd = (loss(A.vals, b + d) - loss(A.vals, b - d)) / (2 * h)
        assert abs(fd - gb[j]) < 1e-6 * (1 + abs(fd))


def test_cg_gradient_limit_is_solve_vjp(orc):
    # After n steps CG computes A^{-1} b, so for symmetric perturbations the
    # CG gradient must agree with Table 1's SpSolve VJP:
    #   grad_b = A^{-T} v, grad_A = -(A^{-T} v) x^T on the pattern.
    # Only the symmetric part g_ij + g_ji is comparable, because CG's output
    # depends on A only through its action on the Krylov space.
    n = 12
    A = _spd(n, 12)
    b = gen.normal(n, 13)
    v = gen.normal(n, 14)
    gv, gb = orc.cg_bwd(A, b, n, gx=v)
    Ad = A.todense()
    x = np.linalg.solve(Ad, b)
    w = np.linalg.solve(Ad.T, v)
    np.testing.assert_allclose(gb, w, rtol=1e-6, atol=1e-8)
    G = np.zeros((n, n))
    G[A.row_of_entry(), A.colind] = gv
    ref = -np.outer(w, x)
    mask = Ad != 0
    np.testing.assert_allclose((G + G.T)[mask], (ref + ref.T)[mask], rtol=1e-6, atol=1e-8)


def test_jacobi_pcg_equals_cg_for_constant_diagonal(orc):
    A = gen.poisson2d(12, 12)  # diagonal is 4 everywhere
    b = gen.normal(144, 15)
    xj, itj, hj = orc.pcg(A, b, "jacobi", tol=1e-8)
    xn, itn, hn = orc.pcg(A, b, "none", tol=1e-8)
    assert itj == itn
    np.testing.assert_allclose(hj, hn, rtol=1e-9)
    np.testing.assert_allclose(xj, xn, rtol=1e-9, atol=1e-12)


def test_pcg_exact_factor_one_iteration(orc):
    # Full lower pattern: IC(0) is the exact Cholesky factor, M = A^{-1}.
    A = _spd(15, 16)
    r, c = np.nonzero(np.ones((15, 15)))
    Ad = A.todense()
    Af = gen._from_coo(15, 15, r, c, Ad[r, c])
    Lp = gen.tril(Af)
    L = gen.Csr(15, 15, Lp.rowptr, Lp.colind, orc.ic0(Af, Lp))
    b = gen.normal(15, 17)
    x, it, _ = orc.pcg(A, b, "factor", L=L, tol=1e-10)
    assert it == 1
    np.testing.assert_allclose(Ad @ x, b, rtol=1e-9, atol=1e-9)
    # 1D Poisson: tril pattern has no fill, IC(0) is exact.
    A1 = gen.poisson1d(64)
    L1p = gen.tril(A1)
    L1 = gen.Csr(64, 64, L1p.rowptr, L1p.colind, orc.ic0(A1, L1p))
    _, it1, _ = orc.pcg(A1, gen.normal(64, 18), "factor", L=L1, tol=1e-10)
    assert it1 == 1


def test_pcg_breakdown_reported(orc):
    A = gen.poisson1d(8)
    Lp = gen.tril(A)
    bad = gen.Csr(8, 8, Lp.rowptr, Lp.colind, np.where(Lp.colind == Lp.row_of_entry(), 0.0, -1.0))
    _, it, _ = orc.pcg(A, np.ones(8), "factor", L=bad)
    assert it == -1


def test_paper_loss_weights(orc):
    # weights gamma^(Nit-i) / sum_j gamma^(Nit-j): sum to one and grow with i
    val, w = orc.paper_loss([0.5, 0.25, 0.125, 0.0625], 1.0, gamma=0.6)
    assert abs(w.sum() - 1) < 1e-15
    np.testing.assert_allclose(w, np.array([0.216, 0.36, 0.6, 1.0]) / 2.176, rtol=1e-14)
    assert abs(val - w @ [0.5, 0.25, 0.125, 0.0625]) < 1e-15
    v1, w1 = orc.paper_loss([1.0, 3.0], 2.0, gamma=1.0)
    assert np.allclose(w1, 0.5) and abs(v1 - 1.0) < 1e-15
    v0, _ = orc.paper_loss([0.0] * 4, 1.0)
    assert v0 == 0.0
