"""Pins for the oracle's sparse + sparse (Section 3.1.4; Table 1, Sp + Sp rows).

Independent checks: the union pattern from Python sets of stored
coordinates, values against dense NumPy arithmetic, the same sum written
as a sparse-sparse product [A | B] [alpha I; beta I] through the oracle's
(separately pinned) SpSpMM and its VJP, the adjoint identity of the
linear map (vals_A, vals_B) -> vals_C, structural cancellation, empty
operands, and the tridiagonal matrix that the Jacobi example of
Section 4.1 assembles from shifted identities."""
import numpy as np
import pytest

from paper_2212_05159_amd import gen


def _coords(A):
    rows = np.repeat(np.arange(A.nrows), np.diff(A.rowptr))
    return set(zip(rows.tolist(), np.asarray(A.colind).tolist()))


def _csr(m, n, rp, ci, v):
    return gen.Csr(m, n, np.asarray(rp, np.int32), np.asarray(ci, np.int32), np.asarray(v))


def _with_stored_zeros(A, seed):
    """Same pattern, some values set to exactly zero (still stored)."""
    v = A.vals.copy()
    rng = np.random.default_rng(seed)
    v[rng.random(len(v)) < 0.2] = 0.0
    return gen.Csr(A.nrows, A.ncols, A.rowptr, A.colind, v)


CASES = [
    (7, 9, 0.3, 0.4, 1.0, 1.0),
    (13, 11, 0.2, 0.5, 0.5, -2.0),
    (20, 20, 0.1, 0.1, -1.0, 3.0),
    (5, 30, 0.6, 0.05, 2.0, 0.0),
]


@pytest.mark.parametrize("m,n,da,db,alpha,beta", CASES)
def test_pattern_is_union_and_values_match_dense(orc, m, n, da, db, alpha, beta):
    A = _with_stored_zeros(gen.random_csr(m, n, da, seed=m, empty_rows=0.2), 1)
    B = _with_stored_zeros(gen.random_csr(m, n, db, seed=m + 100, empty_rows=0.2), 2)
    rp, ci, v = orc.spadd(A, B, alpha, beta)
    C = _csr(m, n, rp, ci, v)
    assert _coords(C) == _coords(A) | _coords(B)
    for i in range(m):
        assert np.all(np.diff(ci[rp[i]:rp[i + 1]]) > 0)
    dense = alpha * A.todense() + beta * B.todense()
    np.testing.assert_allclose(C.todense(), dense, rtol=0, atol=1e-14)


@pytest.mark.parametrize("m,n,da,db,alpha,beta", CASES)
def test_equals_spgemm_with_stacked_identities(orc, m, n, da, db, alpha, beta):
    """alpha A + beta B = [A | B] [alpha I; beta I], pattern included."""
    A = gen.random_csr(m, n, da, seed=3 * m, empty_rows=0.1)
    B = gen.random_csr(m, n, db, seed=3 * m + 1, empty_rows=0.1)
    rows_a = np.repeat(np.arange(m), np.diff(A.rowptr))
    rows_b = np.repeat(np.arange(m), np.diff(B.rowptr))
    H = gen._from_coo(m, 2 * n, np.concatenate([rows_a, rows_b]),
                      np.concatenate([A.colind, B.colind + n]),
                      np.concatenate([A.vals, B.vals]))
    S = gen._from_coo(2 * n, n, np.arange(2 * n), np.concatenate([np.arange(n)] * 2),
                      np.concatenate([np.full(n, alpha), np.full(n, beta)]))
    rp_g, ci_g, v_g = orc.spgemm(H, S)
    rp, ci, v = orc.spadd(A, B, alpha, beta)
    np.testing.assert_array_equal(rp, rp_g)
    np.testing.assert_array_equal(ci, ci_g)
    np.testing.assert_allclose(v, v_g, rtol=1e-15, atol=1e-15)

    gC = gen.normal(len(ci), seed=m)
    gH, _ = orc.spgemm_bwd(H, S, rp_g, ci_g, gC, want_B=False)
    # H's entries of row i are A's row then B's row (columns n.. follow 0..n-1).
    gA_ref = np.empty(A.nnz)
    gB_ref = np.empty(B.nnz)
    for i in range(m):
        la = A.rowptr[i + 1] - A.rowptr[i]
        seg = gH[H.rowptr[i]:H.rowptr[i + 1]]
        gA_ref[A.rowptr[i]:A.rowptr[i + 1]] = seg[:la]
        gB_ref[B.rowptr[i]:B.rowptr[i + 1]] = seg[la:]
    gA, gB = orc.spadd_bwd(A, B, rp, ci, gC, alpha, beta)
    np.testing.assert_allclose(gA, gA_ref, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(gB, gB_ref, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_adjoint_identity(orc, seed):
    """<gC, C(dA, dB)> = <gA, dA> + <gB, dB>: the VJP is the adjoint of the
    linear map from the input values to the output values."""
    m, n = 17, 23
    A = gen.random_csr(m, n, 0.25, seed=seed)
    B = gen.random_csr(m, n, 0.3, seed=seed + 50)
    alpha, beta = 0.75, -1.25
    rp, ci, _ = orc.spadd(A, B, alpha, beta)
    dA = gen.Csr(m, n, A.rowptr, A.colind, gen.normal(A.nnz, seed + 1))
    dB = gen.Csr(m, n, B.rowptr, B.colind, gen.normal(B.nnz, seed + 2))
    _, _, dC = orc.spadd(dA, dB, alpha, beta)
    gC = gen.normal(len(ci), seed + 3)
    gA, gB = orc.spadd_bwd(A, B, rp, ci, gC, alpha, beta)
    lhs = float(gC @ dC)
    rhs = float(gA @ dA.vals + gB @ dB.vals)
    assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs))


def test_cancellation_keeps_the_pattern(orc):
    A = gen.random_csr(12, 12, 0.3, seed=7)
    rp, ci, v = orc.spadd(A, A, 1.0, -1.0)
    np.testing.assert_array_equal(rp, A.rowptr)
    np.testing.assert_array_equal(ci, A.colind)
    assert np.all(v == 0.0)


def test_empty_operands(orc):
    B = gen.random_csr(6, 8, 0.4, seed=3)
    E = gen.Csr(6, 8, np.zeros(7, np.int32), np.zeros(0, np.int32), np.zeros(0))
    rp, ci, v = orc.spadd(E, B, 2.0, -0.5)
    np.testing.assert_array_equal(rp, B.rowptr)
    np.testing.assert_array_equal(ci, B.colind)
    np.testing.assert_array_equal(v, -0.5 * B.vals)
    gA, gB = orc.spadd_bwd(E, B, rp, ci, np.ones(len(ci)), 2.0, -0.5)
    assert gA.size == 0
    np.testing.assert_array_equal(gB, np.full(B.nnz, -0.5))
    rp, ci, v = orc.spadd(E, E)
    assert rp.tolist() == [0] * 7 and ci.size == 0
    Z = gen.Csr(0, 4, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    rp, ci, v = orc.spadd(Z, Z)
    assert rp.tolist() == [0]


def test_jacobi_example_tridiagonal(orc):
    """2 I - I_{+1} - I_{-1} is the 1D Poisson matrix [-1, 2, -1]."""
    N = 16

    def shifted_eye(k):
        i = np.arange(max(0, -k), min(N, N - k))
        return gen._from_coo(N, N, i, i + k, np.ones(len(i)))

    rp, ci, v = orc.spadd(shifted_eye(0), shifted_eye(1), 2.0, -1.0)
    T1 = _csr(N, N, rp, ci, v)
    rp, ci, v = orc.spadd(T1, shifted_eye(-1), 1.0, -1.0)
    ref = gen.poisson1d(N)
    np.testing.assert_array_equal(rp, ref.rowptr)
    np.testing.assert_array_equal(ci, ref.colind)
    np.testing.assert_array_equal(v, ref.vals)
