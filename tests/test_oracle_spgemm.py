"""Pins for the oracle's SpSpMM (Section 3.1.2; Table 1; Fig. 2).

Independent checks: the pattern and gradient flow drawn in Fig. 2 (golden
file), boolean dense products for the structural pattern, dense NumPy
products and torch float64 autograd for values and gradients, A I = A,
bilinearity, and closed forms of the Galerkin product P^T A P for the 3D
Poisson matrix with an aggregation prolongator."""
import os

import numpy as np
import pytest
import torch

from paper_2212_05159_amd import gen

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig2_spgemm.txt")


def _read_fig2():
    pats, arrows, cur = {}, [], None
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] in ("A", "B", "C"):
            cur = tok[0]
            pats[cur] = (int(tok[1]), int(tok[2]), [])
        elif tok[0] == "ARROW":
            ci, cj = int(tok[1]) - 1, int(tok[2]) - 1
            refs = [(tok[t], int(tok[t + 1]) - 1, int(tok[t + 2]) - 1) for t in range(3, len(tok), 3)]
            arrows.append(((ci, cj), refs))
        else:
            r = int(tok[0].rstrip(":")) - 1
            pats[cur][2].extend((r, int(c) - 1) for c in tok[1:])
    return pats, arrows


def _pattern(rp, ci):
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return set(zip(rows.tolist(), np.asarray(ci).tolist()))


def _csr(m, n, rp, ci, v):
    return gen.Csr(m, n, np.asarray(rp, np.int32), np.asarray(ci, np.int32), np.asarray(v, float))


def test_fig2_pattern(orc):
    pats, _ = _read_fig2()
    A, B = gen.fig2_pair()
    assert _pattern(A.rowptr, A.colind) == set(pats["A"][2])
    assert _pattern(B.rowptr, B.colind) == set(pats["B"][2])
    rpC, ciC, _ = orc.spgemm(A, B)
    assert len(ciC) == 19
    assert _pattern(rpC, ciC) == set(pats["C"][2])
    for i in range(9):  # ascending, unique columns within each row
        row = ciC[rpC[i]:rpC[i + 1]]
        assert np.all(np.diff(row) > 0)


def test_fig2_gradient_flow(orc):
    # One-hot upstream gradient on a product entry reaches exactly the
    # entries of A and B the figure's arrows point at (generic values).
    pats, arrows = _read_fig2()
    A, B = gen.fig2_pair()
    rng = np.random.default_rng(21)
    A = _csr(9, 9, A.rowptr, A.colind, rng.uniform(1, 2, A.nnz))
    B = _csr(9, 3, B.rowptr, B.colind, rng.uniform(1, 2, B.nnz))
    rpC, ciC, _ = orc.spgemm(A, B)
    Apos = {(r, c): e for e, (r, c) in enumerate(zip(A.row_of_entry(), A.colind))}
    Bpos = {(r, c): e for e, (r, c) in enumerate(zip(B.row_of_entry(), B.colind))}
    Cpos = {(r, c): e for e, (r, c) in enumerate(zip(np.repeat(np.arange(9), np.diff(rpC)), ciC))}
    for (ci, cj), refs in arrows:
        gC = np.zeros(len(ciC))
        gC[Cpos[(ci, cj)]] = 1.0
        gA, gB = orc.spgemm_bwd(A, B, rpC, ciC, gC)
        wantA = {Apos[(r, c)] for (w, r, c) in refs if w == "A"}
        wantB = {Bpos[(r, c)] for (w, r, c) in refs if w == "B"}
        assert set(np.nonzero(gA)[0].tolist()) == wantA
        assert set(np.nonzero(gB)[0].tolist()) == wantB


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_spgemm_vs_dense(orc, seed):
    rng = np.random.default_rng(seed)
    m, n, p = rng.integers(1, 40, size=3)
    A = gen.random_csr(int(m), int(n), 0.15, seed=[seed, 1], empty_rows=0.2)
    B = gen.random_csr(int(n), int(p), 0.2, seed=[seed, 2], empty_rows=0.2)
    rpC, ciC, vC = orc.spgemm(A, B)
    Ad, Bd = A.todense(), B.todense()
    struct = ((Ad != 0).astype(int) @ (Bd != 0).astype(int)) > 0
    assert _pattern(rpC, ciC) == set(zip(*np.nonzero(struct)))
    Cd = Ad @ Bd
    rows = np.repeat(np.arange(A.nrows), np.diff(rpC))
    np.testing.assert_allclose(vC, Cd[rows, ciC], rtol=1e-13, atol=1e-13)


def test_spgemm_keeps_cancelled_entries(orc):
    # (1 1) (1; -1) = 0: the structural pattern keeps the entry.
    A = _csr(1, 2, [0, 2], [0, 1], [1.0, 1.0])
    B = _csr(2, 1, [0, 1, 2], [0, 0], [1.0, -1.0])
    rpC, ciC, vC = orc.spgemm(A, B)
    assert list(rpC) == [0, 1] and list(ciC) == [0] and vC[0] == 0.0


def test_spgemm_identity(orc):
    A = gen.random_csr(19, 19, 0.2, seed=4)
    I = _csr(19, 19, np.arange(20), np.arange(19), np.ones(19))
    for L, R in [(A, I), (I, A)]:
        rpC, ciC, vC = orc.spgemm(L, R)
        assert np.array_equal(rpC, A.rowptr) and np.array_equal(ciC, A.colind)
        assert np.array_equal(vC, A.vals)


def test_spgemm_bwd_vs_torch_dense_autograd(orc):
    A = gen.random_csr(21, 17, 0.2, seed=31, empty_rows=0.1)
    B = gen.random_csr(17, 13, 0.25, seed=32)
    rpC, ciC, vC = orc.spgemm(A, B)
    V = gen.normal(len(ciC), 33)
    gA, gB = orc.spgemm_bwd(A, B, rpC, ciC, V)
    Vd = np.zeros((21, 13))
    Vd[np.repeat(np.arange(21), np.diff(rpC)), ciC] = V
    Ad = torch.tensor(A.todense(), requires_grad=True)
    Bd = torch.tensor(B.todense(), requires_grad=True)
    ((Ad @ Bd) * torch.tensor(Vd)).sum().backward()
    np.testing.assert_allclose(gA, Ad.grad.numpy()[A.row_of_entry(), A.colind], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gB, Bd.grad.numpy()[B.row_of_entry(), B.colind], rtol=1e-12, atol=1e-12)
    # bilinearity: <gA, A> = <V, C> = <gB, B>
    vc = V @ vC
    assert abs(gA @ A.vals - vc) < 1e-11 * (1 + abs(vc))
    assert abs(gB @ B.vals - vc) < 1e-11 * (1 + abs(vc))


def test_spgemm_bwd_central_differences(orc):
    A = gen.random_csr(6, 5, 0.5, seed=41)
    B = gen.random_csr(5, 4, 0.5, seed=42)
    rpC, ciC, _ = orc.spgemm(A, B)
    V = gen.normal(len(ciC), 43)

    def loss(va, vb):
        return V @ orc.spgemm(_csr(6, 5, A.rowptr, A.colind, va), _csr(5, 4, B.rowptr, B.colind, vb))[2]

    gA, gB = orc.spgemm_bwd(A, B, rpC, ciC, V)
    h = 1e-6
    for e in range(A.nnz):
        d = np.zeros(A.nnz); d[e] = h
        assert abs((loss(A.vals + d, B.vals) - loss(A.vals - d, B.vals)) / (2 * h) - gA[e]) < 1e-7
    for e in range(B.nnz):
        d = np.zeros(B.nnz); d[e] = h
        assert abs((loss(A.vals, B.vals + d) - loss(A.vals, B.vals - d)) / (2 * h) - gB[e]) < 1e-7


@pytest.mark.parametrize("N", [16, 32])
def test_galerkin_closed_forms(orc, N):
    # 3D 7-point Poisson on N^3 (last index fastest) and P[i, i // 8] = 1.
    # Counting neighbours by direction gives
    #   nnz(A P)     = n (1 + 4 (1 - 1/N) + 2 (N/8 - 1)/N)
    #   nnz(P^T A P) = n/8 + 2 (N/8 - 1) N^2 + 4 (N/8) (N - 1) N
    # and P^T A P is the 7-point stencil on the (N, N, N/8) coarse grid with
    # 34 on the diagonal (8*6 - 2*7), -8 to x/y neighbours and -1 along z.
    A = gen.poisson3d(N)
    P = gen.aggregation(N ** 3, 8)
    n = N ** 3
    rpAP, ciAP, vAP = orc.spgemm(A, P)
    assert len(ciAP) == round(n * (1 + 4 * (1 - 1 / N) + 2 * (N / 8 - 1) / N))
    rpT, ciT, perm = orc.transpose(P)
    Pt = gen.Csr(P.ncols, P.nrows, rpT, ciT, P.vals[perm])
    AP = gen.Csr(n, P.ncols, rpAP, ciAP, vAP)
    rpC, ciC, vC = orc.spgemm(Pt, AP)
    assert len(ciC) == n // 8 + 2 * (N // 8 - 1) * N * N + 4 * (N // 8) * (N - 1) * N
    coarse = gen._stencil((N, N, N // 8),
                          [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)],
                          [-8.0, -8.0, -1.0, 34.0, -1.0, -8.0, -8.0])
    assert np.array_equal(rpC, coarse.rowptr) and np.array_equal(ciC, coarse.colind)
    assert np.array_equal(vC, coarse.vals)
