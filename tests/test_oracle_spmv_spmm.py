"""Pins for the oracle's SpMV and SpDMM (Section 3.1.1, 3.1.3; Table 1).

Each check is independent of the oracle's own loops: dense NumPy products,
torch float64 dense autograd, central finite differences, the adjoint
identity and closed forms of the Poisson matrices (Section 4, Eqs.
mat_1d_fd / mat_2d_fd)."""
import numpy as np
import pytest
import torch

from paper_2212_05159_amd import gen


def _cases():
    yield gen.poisson2d(32, 32)  # the n = 1024 Poisson operand
    yield gen.random_csr(37, 53, 0.1, seed=1, empty_rows=0.2)
    yield gen.random_csr(64, 17, 0.3, seed=2, long_rows=2, long_len=17)
    yield gen.random_csr(1, 1, 1.0, seed=3)
    yield gen.random_csr(5, 9, 0.0, seed=4)  # no stored entries at all


@pytest.mark.parametrize("A", list(_cases()), ids=lambda a: f"{a.nrows}x{a.ncols}nnz{a.nnz}")
def test_spmv_matches_dense(orc, A):
    x = gen.normal(A.ncols, 10)
    np.testing.assert_allclose(orc.spmv(A, x), A.todense() @ x, rtol=1e-13, atol=1e-13)


def test_poisson_times_ones_counts_missing_neighbours(orc):
    # Each row sums to the number of grid neighbours cut off by the
    # Dirichlet boundary: 0 inside, 1 on a face, 2 at a 2D corner, 3 at a
    # 3D corner.  Exact in float64 (small integers).
    n = 32
    A = gen.poisson2d(n, n)
    y = orc.spmv(A, np.ones(A.ncols))
    ix, iy = np.divmod(np.arange(n * n), n)
    missing = ((ix == 0) | (ix == n - 1)).astype(int) + ((iy == 0) | (iy == n - 1)).astype(int)
    assert np.array_equal(y, missing.astype(float))
    m = 8
    A3 = gen.poisson3d(m)
    y3 = orc.spmv(A3, np.ones(A3.ncols))
    c = np.unravel_index(np.arange(m ** 3), (m, m, m))
    miss3 = sum(((ci == 0) | (ci == m - 1)).astype(int) for ci in c)
    assert np.array_equal(y3, miss3.astype(float))
    assert set(np.unique(y3)) == {0.0, 1.0, 2.0, 3.0}


def test_poisson_generators_match_kronecker_form():
    # Eq. mat_2d_fd written with scipy's Kronecker product.
    import scipy.sparse as sps
    a1 = lambda n: sps.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    nx, ny = 5, 7
    ref = sps.kron(a1(nx), sps.eye(ny)) + sps.kron(sps.eye(nx), a1(ny))
    assert np.array_equal(gen.poisson2d(nx, ny).todense(), ref.toarray())
    n = 4
    I = sps.eye(n)
    ref3 = sps.kron(sps.kron(a1(n), I), I) + sps.kron(sps.kron(I, a1(n)), I) + sps.kron(sps.kron(I, I), a1(n))
    assert np.array_equal(gen.poisson3d(n).todense(), ref3.toarray())
    assert np.array_equal(gen.poisson1d(6).todense(), a1(6).toarray())


def test_spmv_vjp_config_small_vs_torch_dense_autograd(orc):
    # 2D Poisson 32x32, x and t ~ N(0,1) from seed 0, loss = 0.5||Ax - t||^2.
    A = gen.poisson2d(32, 32)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(1024)
    t = rng.standard_normal(1024)
    g = orc.spmv(A, x) - t
    gx, gv = orc.spmv_bwd(A, x, g)

    Ad = torch.tensor(A.todense(), requires_grad=True)
    xt = torch.tensor(x, requires_grad=True)
    loss = 0.5 * ((Ad @ xt - torch.tensor(t)) ** 2).sum()
    loss.backward()
    np.testing.assert_allclose(gx, xt.grad.numpy(), rtol=1e-12, atol=1e-12)
    rows = A.row_of_entry()
    dense_gA = Ad.grad.numpy()
    np.testing.assert_allclose(gv, dense_gA[rows, A.colind], rtol=1e-12, atol=1e-12)
    # The dense gradient is nonzero off the pattern: keeping only the stored
    # entries is the sparse-gradient convention, not a property of the math.
    off = np.ones_like(dense_gA, dtype=bool)
    off[rows, A.colind] = False
    assert np.abs(dense_gA[off]).max() > 1e-3


def test_spmv_vjp_central_differences(orc):
    A = gen.random_csr(12, 9, 0.4, seed=5)
    x = gen.normal(9, 6)
    t = gen.normal(12, 7)

    def loss(vals, xx):
        B = gen.Csr(A.nrows, A.ncols, A.rowptr, A.colind, vals)
        return 0.5 * np.sum((orc.spmv(B, xx) - t) ** 2)

    g = orc.spmv(A, x) - t
    gx, gv = orc.spmv_bwd(A, x, g)
    h = 1e-6
    for e in range(A.nnz):
        d = np.zeros(A.nnz); d[e] = h
        fd = (loss(A.vals + d, x) - loss(A.vals - d, x)) / (2 * h)
        assert abs(fd - gv[e]) < 1e-6 * max(1, abs(fd))
    for j in range(9):
        d = np.zeros(9); d[j] = h
        fd = (loss(A.vals, x + d) - loss(A.vals, x - d)) / (2 * h)
        assert abs(fd - gx[j]) < 1e-6 * max(1, abs(fd))


def test_spmv_adjoint_identity(orc):
    A = gen.random_csr(40, 31, 0.15, seed=8, empty_rows=0.1)
    x = gen.normal(31, 1)
    y = gen.normal(40, 2)
    aty, _ = orc.spmv_bwd(A, x, y, want_vals=False)
    assert abs(orc.spmv(A, x) @ y - x @ aty) < 1e-12 * np.abs(x).sum() * np.abs(y).sum()


def test_spmv_bwd_pattern_invariant(orc):
    # g_vals has one entry per stored value, and a stored explicit zero
    # still receives its gradient (structural mask).
    A = gen.random_csr(10, 10, 0.3, seed=9)
    A.vals[::3] = 0.0
    x, g = gen.normal(10, 1), gen.normal(10, 2)
    _, gv = orc.spmv_bwd(A, x, g)
    assert gv.shape == (A.nnz,)
    rows = A.row_of_entry()
    np.testing.assert_allclose(gv, g[rows] * x[A.colind], rtol=0, atol=0)


@pytest.mark.parametrize("k", [1, 5, 64])
def test_spmm_matches_dense_and_columnwise_spmv(orc, k):
    A = gen.random_csr(30, 22, 0.2, seed=11, empty_rows=0.1)
    B = gen.normal((22, k), 12)
    Cm = orc.spmm(A, B)
    np.testing.assert_allclose(Cm, A.todense() @ B, rtol=1e-13, atol=1e-13)
    for c in range(k):
        np.testing.assert_allclose(Cm[:, c], orc.spmv(A, B[:, c]), rtol=1e-14, atol=1e-14)


def test_spmm_vjp_vs_torch_dense_autograd(orc):
    A = gen.random_csr(25, 19, 0.25, seed=13)
    B = gen.normal((19, 8), 14)
    G = gen.normal((25, 8), 15)
    gB, gv = orc.spmm_bwd(A, B, G)
    Ad = torch.tensor(A.todense(), requires_grad=True)
    Bt = torch.tensor(B, requires_grad=True)
    (Ad @ Bt * torch.tensor(G)).sum().backward()
    np.testing.assert_allclose(gB, Bt.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gv, Ad.grad.numpy()[A.row_of_entry(), A.colind], rtol=1e-12, atol=1e-12)


def test_spmm_adjoint_identity_frobenius(orc):
    A = gen.random_csr(33, 27, 0.1, seed=16)
    B = gen.normal((27, 6), 17)
    Y = gen.normal((33, 6), 18)
    atY, _ = orc.spmm_bwd(A, B, Y, want_vals=False)
    lhs = np.sum(orc.spmm(A, B) * Y)
    rhs = np.sum(B * atY)
    assert abs(lhs - rhs) < 1e-11 * (1 + abs(lhs))


def test_transpose_matches_library_and_involution(orc):
    import scipy.sparse as sps
    for A in [gen.random_csr(23, 41, 0.1, seed=19, empty_rows=0.3), gen.poisson2d(4, 6),
              gen.aggregation(20, 8), gen.random_csr(4, 4, 0.0, seed=0)]:
        rpT, ciT, perm = orc.transpose(A)
        ref = sps.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.nrows, A.ncols)).T.tocsr()
        ref.sort_indices()
        assert np.array_equal(rpT, ref.indptr) and np.array_equal(ciT, ref.indices)
        assert np.array_equal(A.vals[perm], ref.data)
        At = gen.Csr(A.ncols, A.nrows, rpT, ciT, A.vals[perm])
        rp2, ci2, perm2 = orc.transpose(At)
        assert np.array_equal(rp2, A.rowptr) and np.array_equal(ci2, A.colind)
        assert np.array_equal(perm[perm2], np.arange(A.nnz))


def test_openmp_build_returns_the_same_bits():
    # The all-cores build only splits independent rows among threads; every
    # output must equal the single-threaded build's bit for bit.
    import oracle

    oracle.build()
    A = gen.random_csr(700, 500, 0.02, 41, empty_rows=0.1, long_rows=3, long_len=300)
    rng = np.random.default_rng(42)
    x, gy = rng.standard_normal(500), rng.standard_normal(700)
    B, G = rng.standard_normal((500, 24)), rng.standard_normal((700, 24))
    outs = []
    for th in (False, True):
        oracle.use_threads(th)
        try:
            outs.append([oracle.spmv(A, x), *oracle.spmv_bwd(A, x, gy), oracle.spmm(A, B),
                         *oracle.spmm_bwd(A, B, G)])
            assert oracle.threads() >= 1
        finally:
            oracle.use_threads(False)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
