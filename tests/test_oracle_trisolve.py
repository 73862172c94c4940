"""Pins for the oracle's level sets, triangular solve and its VJP
(Section 3.1.5; Table 1, SpSolve row), and IC(0).

Independent checks: closed-form level counts of natural and coloured grid
orderings, the longest-path characterisation of levels, SciPy dense
triangular solves, the closed-form Cholesky factor of the 1D Poisson
matrix A_N (Eq. mat_1d_fd), NumPy's dense Cholesky, torch float64 dense
autograd, the adjoint identity and central differences."""
import numpy as np
import pytest
import scipy.linalg as sla
import torch

from paper_2212_05159_amd import gen


def _check_longest_path(T, lor, lower):
    # level(i) > level(j) for every dependency j of i, and a row above level
    # 0 has some dependency exactly one level below: this characterises the
    # longest-path levels uniquely.
    rows = T.row_of_entry()
    dep = (T.colind < rows) if lower else (T.colind > rows)
    r, c = rows[dep], T.colind[dep]
    assert np.all(lor[r] > lor[c])
    tight = np.zeros(T.nrows, bool)
    tight[r[lor[r] == lor[c] + 1]] = True
    assert np.all(tight | (lor == 0))


def _check_grouping(lor, lptr, lrows):
    n = len(lor)
    assert lptr[0] == 0 and lptr[-1] == n
    for l in range(len(lptr) - 1):
        seg = lrows[lptr[l]:lptr[l + 1]]
        assert np.all(np.diff(seg) > 0) and np.all(lor[seg] == l)


@pytest.mark.parametrize("n", [1, 2, 17])
def test_levels_1d_chain(orc, n):
    T = gen.tril(gen.poisson1d(n))
    lor, lptr, lrows = orc.levels(T)
    assert len(lptr) - 1 == n
    assert np.array_equal(lor, np.arange(n))


@pytest.mark.parametrize("nx,ny", [(4, 7), (32, 32)])
def test_levels_2d_5pt(orc, nx, ny):
    T = gen.tril(gen.poisson2d(nx, ny))
    lor, lptr, lrows = orc.levels(T)
    assert len(lptr) - 1 == nx + ny - 1
    _check_longest_path(T, lor, True)
    _check_grouping(lor, lptr, lrows)
    # upper solve: same count by symmetry of the grid
    lu, lpu, lru = orc.levels(gen.triu(gen.poisson2d(nx, ny)), lower=False)
    assert len(lpu) - 1 == nx + ny - 1
    _check_longest_path(gen.triu(gen.poisson2d(nx, ny)), lu, False)


def test_levels_3d_7pt(orc):
    N = 12
    lor, lptr, _ = orc.levels(gen.tril(gen.poisson3d(N)))
    assert len(lptr) - 1 == 3 * N - 2


def test_levels_9pt_natural_and_four_coloured(orc):
    N = 32
    A = gen.anisotropic_q1(N, 1e-3, np.pi / 4)
    lor, lptr, _ = orc.levels(gen.tril(A))
    assert len(lptr) - 1 == 3 * N - 2  # level(ix, iy) = ix + 2 iy
    iy, ix = np.divmod(np.arange(N * N), N)
    assert np.array_equal(lor, ix + 2 * iy)
    Ac = gen.permute_sym(A, gen.four_color_2d(N))
    Tc = gen.tril(Ac)
    lc, lpc, lrc = orc.levels(Tc)
    assert len(lpc) - 1 == 4
    assert np.array_equal(np.diff(lpc), [N * N // 4] * 4)
    _check_longest_path(Tc, lc, True)


def test_levels_random_lower(orc):
    T = gen.random_lower(60, 0.08, seed=3)
    lor, lptr, lrows = orc.levels(T)
    _check_longest_path(T, lor, True)
    _check_grouping(lor, lptr, lrows)


@pytest.mark.parametrize("lower", [True, False])
def test_trisolve_matches_scipy(orc, lower):
    L = gen.random_lower(50, 0.2, seed=5)
    T = L if lower else gen.Csr(50, 50, *orc.transpose(L)[:2], L.vals[orc.transpose(L)[2]])
    b = gen.normal(50, 6)
    x = orc.trisolve(T, b, lower=lower)
    ref = sla.solve_triangular(T.todense(), b, lower=lower)
    np.testing.assert_allclose(x, ref, rtol=1e-11, atol=1e-12)


def test_trisolve_missing_diagonal_reported(orc):
    T = gen.tril(gen.poisson1d(5), -1)  # strictly lower: no diagonal
    with pytest.raises(ZeroDivisionError):
        orc.trisolve(T, np.ones(5))


def test_poisson1d_cholesky_closed_form(orc):
    # A_N = L L^T with L_ii = sqrt((i+1)/i), L_{i+1,i} = -sqrt(i/(i+1))
    # (1-based).  A tridiagonal matrix has no fill, so IC(0) is exact.
    N = 40
    A = gen.poisson1d(N)
    Lp = gen.tril(A)
    lv = orc.ic0(A, Lp)
    rows = Lp.row_of_entry() + 1
    cols = Lp.colind + 1
    want = np.where(rows == cols, np.sqrt((rows + 1) / rows), -np.sqrt(cols / (cols + 1.0)))
    np.testing.assert_allclose(lv, want, rtol=1e-14)
    L = gen.Csr(N, N, Lp.rowptr, Lp.colind, lv)
    b = gen.normal(N, 7)
    y = orc.trisolve(L, b)
    Lt = orc.transpose(L)
    U = gen.Csr(N, N, Lt[0], Lt[1], lv[Lt[2]])
    x = orc.trisolve(U, y, lower=False)
    np.testing.assert_allclose(A.todense() @ x, b, rtol=1e-12, atol=1e-12)


def test_ic0_full_pattern_is_cholesky(orc):
    rng = np.random.default_rng(8)
    M = rng.standard_normal((12, 12))
    S = M @ M.T + 12 * np.eye(12)
    r, c = np.nonzero(np.ones((12, 12)))
    A = gen._from_coo(12, 12, r, c, S[r, c])
    Lp = gen.tril(A)
    lv = orc.ic0(A, Lp)
    Ld = np.linalg.cholesky(S)
    np.testing.assert_allclose(lv, Ld[Lp.row_of_entry(), Lp.colind], rtol=1e-12)


@pytest.mark.parametrize("lower", [True, False])
def test_trisolve_vjp_vs_torch_dense_autograd(orc, lower):
    L = gen.random_lower(30, 0.25, seed=9)
    if lower:
        T = L
    else:
        rpT, ciT, perm = orc.transpose(L)
        T = gen.Csr(30, 30, rpT, ciT, L.vals[perm])
    b = gen.normal(30, 10)
    g = gen.normal(30, 11)
    x = orc.trisolve(T, b, lower=lower)
    gb, gv = orc.trisolve_bwd(T, x, g, lower=lower)
    Td = torch.tensor(T.todense(), requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    xt = torch.linalg.solve_triangular(Td, bt[:, None], upper=not lower)[:, 0]
    (xt * torch.tensor(g)).sum().backward()
    np.testing.assert_allclose(gb, bt.grad.numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(gv, Td.grad.numpy()[T.row_of_entry(), T.colind], rtol=1e-10, atol=1e-12)
    # Table 1: grad_b = T^{-T} v, grad_T = -(T^{-T} v) x^T on the pattern
    w = sla.solve_triangular(T.todense().T, g, lower=not lower)
    np.testing.assert_allclose(gb, w, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(gv, -w[T.row_of_entry()] * x[T.colind], rtol=1e-10, atol=1e-12)


def test_trisolve_adjoint_identity_and_fd(orc):
    L = gen.random_lower(20, 0.3, seed=12)
    b, y = gen.normal(20, 13), gen.normal(20, 14)
    x = orc.trisolve(L, b)
    w, gv = orc.trisolve_bwd(L, x, y)
    assert abs(x @ y - b @ w) < 1e-11 * (1 + abs(x @ y))
    h = 1e-6
    for e in range(0, L.nnz, 3):
        d = np.zeros(L.nnz); d[e] = h
        fp = orc.trisolve(gen.Csr(20, 20, L.rowptr, L.colind, L.vals + d), b) @ y
        fm = orc.trisolve(gen.Csr(20, 20, L.rowptr, L.colind, L.vals - d), b) @ y
        assert abs((fp - fm) / (2 * h) - gv[e]) < 1e-6 * (1 + abs(gv[e]))
