"""GPU parity: every HIP op against the FP64 oracle on the same inputs.

Integer outputs (transpose, SpGEMM pattern, level sets) must match bit for
bit; float32 values within infinity-norm relative error 1e-5, float64
within 1e-12 (tests/_util.py).  Sizes span several workgroups and ragged
tails; the edge cases are empty matrices and rows, single entries, long
rows/columns (every length class of the transpose and SpGEMM kernels) and
deep, narrow level structures."""
import numpy as np
import pytest
import torch

import oracle
from paper_2212_05159_amd import gen
from paper_2212_05159_amd import sparse as sp

from _util import assert_close, rounded, to_dev, upcast

pytestmark = pytest.mark.gpu
DTYPES = [torch.float32, torch.float64]


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build()


def _dev(m, dtype):
    return sp.CsrTensor.from_host(m, dtype=dtype)


def _matrices():
    yield "poisson32", gen.poisson2d(32, 32)
    yield "rand_ragged", gen.random_csr(777, 523, 0.01, seed=1, empty_rows=0.2)
    yield "rand_long_rows", gen.random_csr(300, 4000, 0.002, seed=2, long_rows=3, long_len=3000)
    yield "one", gen.random_csr(1, 1, 1.0, seed=3)
    yield "empty", gen.random_csr(9, 7, 0.0, seed=4)
    yield "wide_rows", gen.random_csr(64, 200, 0.5, seed=5)


MATS = list(_matrices())


# ---------------------------------------------------------------- SpMV
@pytest.mark.parametrize("dtype", DTYPES)
def test_spmv_poisson_config_small(dtype):
    # 2D Poisson 32x32, x and t ~ N(0,1) from seed 0, loss 0.5||Ax - t||^2
    A = gen.poisson2d(32, 32)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(1024)
    t = rng.standard_normal(1024)
    Ad = _dev(A, dtype)
    Ad.vals.requires_grad_(True)
    xd = to_dev(x, dtype).requires_grad_(True)
    y = Ad @ xd
    loss = 0.5 * ((y - to_dev(t, dtype)) ** 2).sum()
    loss.backward()
    Ao, xo = upcast(A, dtype), rounded(x, dtype)
    yo = oracle.spmv(Ao, xo)
    assert_close(y, yo, dtype, "y")
    g = rounded(y.detach().cpu().numpy(), dtype) - rounded(t, dtype)
    gxo, gvo = oracle.spmv_bwd(Ao, xo, g)
    assert_close(xd.grad, gxo, dtype, "grad x")
    assert_close(Ad.vals.grad, gvo, dtype, "grad vals")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("name,A", MATS, ids=[n for n, _ in MATS])
@pytest.mark.parametrize("use_t", [True, False], ids=["gather", "atomic"])
def test_spmv_fwd_bwd(dtype, name, A, use_t):
    x = gen.normal(A.ncols, 11)
    gy = gen.normal(A.nrows, 12)
    Ad = _dev(A, dtype)
    y = sp.spmv(Ad.pattern, Ad.vals, to_dev(x, dtype))
    gx, gv = sp.spmv_bwd(Ad.pattern, Ad.vals, to_dev(x, dtype), to_dev(gy, dtype),
                         use_transpose=use_t)
    Ao = upcast(A, dtype)
    assert_close(y, oracle.spmv(Ao, rounded(x, dtype)), dtype, "y")
    gxo, gvo = oracle.spmv_bwd(Ao, rounded(x, dtype), rounded(gy, dtype))
    assert_close(gx, gxo, dtype, "gx")
    assert_close(gv, gvo, dtype, "gvals")
    # one-sided requests
    gx2, _ = sp.spmv_bwd(Ad.pattern, Ad.vals, to_dev(x, dtype), to_dev(gy, dtype),
                         need_vals=False, use_transpose=use_t)
    _, gv2 = sp.spmv_bwd(Ad.pattern, Ad.vals, to_dev(x, dtype), to_dev(gy, dtype),
                         need_x=False, use_transpose=use_t)
    assert_close(gx2, gxo, dtype, "gx only")
    assert_close(gv2, gvo, dtype, "gvals only")


# ---------------------------------------------------------------- SpMM
@pytest.mark.parametrize("dtype", DTYPES)
# 16-lane cooperative kernels: k = 32 in float64 (16 lanes of 2 values), 48 in
# float32 (12 of the 16 lanes active) and 64 in float32 (all 16)
@pytest.mark.parametrize("k", [1, 3, 8, 32, 48, 64, 100])
@pytest.mark.parametrize("name", ["poisson32", "rand_ragged", "rand_long_rows", "empty"])
def test_spmm_fwd_bwd(dtype, k, name):
    A = dict(MATS)[name]
    B = gen.normal((A.ncols, k), 21)
    G = gen.normal((A.nrows, k), 22)
    Ad = _dev(A, dtype)
    Bd, Gd = to_dev(B, dtype), to_dev(G, dtype)
    Cd = sp.spmm(Ad.pattern, Ad.vals, Bd)
    gB, gv = sp.spmm_bwd(Ad.pattern, Ad.vals, Bd, Gd)
    _, gv_only = sp.spmm_bwd(Ad.pattern, Ad.vals, Bd, Gd, need_B=False)
    gB_only, _ = sp.spmm_bwd(Ad.pattern, Ad.vals, Bd, Gd, need_vals=False)
    Ao, Bo, Go = upcast(A, dtype), rounded(B, dtype), rounded(G, dtype)
    assert_close(Cd, oracle.spmm(Ao, Bo), dtype, "C")
    gBo, gvo = oracle.spmm_bwd(Ao, Bo, Go)
    assert_close(gB, gBo, dtype, "gB")
    assert_close(gv, gvo, dtype, "gvals")
    assert_close(gv_only, gvo, dtype, "gvals only")
    assert_close(gB_only, gBo, dtype, "gB only")
    # the row-wise value-gradient pass and the fused pass over A^T form the
    # same dots with the same reduction: the same bits
    assert torch.equal(gv_only, gv)


@pytest.mark.parametrize("dtype", DTYPES)
def test_spmm_strided_operands(dtype):
    # Leading dimensions larger than k (column slices of wider buffers).
    A = gen.random_csr(500, 300, 0.02, seed=7, empty_rows=0.1)
    k = 64
    Bw = to_dev(gen.normal((300, 80), 23), dtype)
    Gw = to_dev(gen.normal((500, 72), 24), dtype)
    B, G = Bw[:, 4:4 + k], Gw[:, 8:8 + k]
    Ad = _dev(A, dtype)
    out = torch.empty(500, 96, dtype=dtype, device="cuda")[:, :k]
    from paper_2212_05159_amd import capi
    capi.csr_spmm_fwd(Ad.pattern.desc(Ad.vals), k, B, B.stride(0), out, out.stride(0))
    Pt, perm = Ad.pattern.transpose()
    gB = torch.empty(300, 70, dtype=dtype, device="cuda")[:, 2:2 + k]
    gv = torch.empty(A.nnz, dtype=dtype, device="cuda")
    capi.csr_spmm_bwd(Ad.pattern.desc(Ad.vals), Pt.desc(dtype=dtype), perm, k, B, B.stride(0),
                      G, G.stride(0), gB, gB.stride(0), gv)
    Ao = upcast(A, dtype)
    Bo, Go = B.double().cpu().numpy(), G.double().cpu().numpy()
    assert_close(out, oracle.spmm(Ao, Bo), dtype, "C")
    gBo, gvo = oracle.spmm_bwd(Ao, Bo, Go)
    assert_close(gB, gBo, dtype, "gB")
    assert_close(gv, gvo, dtype, "gvals")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("case", ["grid", "random"])
def test_spmm_plans_do_not_change_results(dtype, case):
    # A traversal plan only reorders rows: results must be bit-identical.
    from paper_2212_05159_amd import capi
    if case == "grid":
        A = gen.poisson3d(16)
        plans = [(256, 64), (256, 100), (256, 300), (4096, 16), (1, 1)]
    else:
        A = gen.random_csr(1000, 900, 0.01, seed=81, empty_rows=0.1)
        plans = [(37, 5), (1000, 64), (333, 1000), (1, 7)]
    k = 64
    Ad = _dev(A, dtype)
    Bd = to_dev(gen.normal((A.ncols, k), 82), dtype)
    Gd = to_dev(gen.normal((A.nrows, k), 83), dtype)
    nat = capi.csrad_plan(0, 0)
    C0 = sp.spmm(Ad.pattern, Ad.vals, Bd, plan=nat)
    gB0, gv0 = sp.spmm_bwd(Ad.pattern, Ad.vals, Bd, Gd, plan=nat)
    _, sv0 = sp.spmm_bwd(Ad.pattern, Ad.vals, Bd, Gd, need_B=False, plan=nat)
    for st, tl in plans:
        pl = capi.csrad_plan(min(st, A.nrows), tl)
        C1 = sp.spmm(Ad.pattern, Ad.vals, Bd, plan=pl)
        assert torch.equal(C0, C1), (st, tl)
        pl_t = capi.csrad_plan(min(st, A.ncols), tl)
        gB1, gv1 = sp.spmm_bwd(Ad.pattern, Ad.vals, Bd, Gd, plan=pl_t)
        assert torch.equal(gB0, gB1) and torch.equal(gv0, gv1), (st, tl)
        _, sv1 = sp.spmm_bwd(Ad.pattern, Ad.vals, Bd, Gd, need_B=False, plan=pl)
        assert torch.equal(sv0, sv1)
    Ao = upcast(A, dtype)
    assert_close(C0, oracle.spmm(Ao, Bd.double().cpu().numpy()), dtype, "C")


def test_autotuner_picks_a_valid_plan():
    from paper_2212_05159_amd import autotune
    A = gen.poisson3d(24)
    Ad = _dev(A, torch.float32)
    Bd = to_dev(gen.normal((A.ncols, 64), 84), torch.float32)
    Gd = to_dev(gen.normal((A.nrows, 64), 85), torch.float32)
    maxrow, bw, nonempty, nnz = Ad.pattern.stats()
    assert (maxrow, bw, nonempty, nnz) == (7, 24 * 24, A.nrows, A.nnz)
    res = autotune.tune_spmm(Ad.pattern, Ad.vals, Bd, Gd, reps=1, use_cache=False)
    assert set(res) == {"spmm_fwd", "spmm_bwd"}
    C1 = sp.spmm(Ad.pattern, Ad.vals, Bd)  # uses the tuned plan
    assert_close(C1, oracle.spmm(upcast(A, torch.float32), Bd.double().cpu().numpy()),
                 torch.float32, "C tuned")


@pytest.mark.parametrize("m", [1, 1000, 300_001])
def test_pattern_stats_match_host(m):
    # 300_001 rows: more rows than the stats kernel's capped grid covers in
    # one sweep, so blocks stride; a fifth of the rows are empty
    rng = np.random.default_rng(91)
    k = np.where(rng.random(m) < 0.2, 0, rng.integers(1, 10, m))
    r = np.repeat(np.arange(m), k)
    A = gen._from_coo(m, m, r, rng.integers(0, m, r.size), np.ones(r.size))
    lens = np.diff(A.rowptr)
    rows = A.row_of_entry()
    want = (int(lens.max(initial=0)), int(np.abs(A.colind - rows).max(initial=0)),
            int((lens > 0).sum()), A.nnz)
    assert tuple(sp.Pattern.from_host(A).stats()) == want


# ---------------------------------------------------------------- transpose
def _with_long_columns():
    # columns of length ~50 (workgroup sort) and 9000 (chunked sort)
    rng = np.random.default_rng(31)
    m, n = 12000, 400
    rows, cols = [], []
    base = gen.random_csr(m, n, 0.003, seed=32)
    r0 = base.row_of_entry()
    rows.append(r0)
    cols.append(base.colind)
    rows.append(rng.choice(m, 50, replace=False)); cols.append(np.full(50, 7))
    rows.append(rng.choice(m, 9000, replace=False)); cols.append(np.full(9000, 13))
    rows.append(np.arange(m)); cols.append(np.full(m, n - 1))  # a full column
    r = np.concatenate(rows); c = np.concatenate(cols)
    key = np.unique(r.astype(np.int64) * n + c)
    return gen._from_coo(m, n, key // n, key % n, rng.standard_normal(len(key)))


def _few_cols():
    # 100000 x 3, nearly dense: every wave hits the same few counters
    rng = np.random.default_rng(33)
    mask = rng.random((100000, 3)) < 0.9
    r, c = np.nonzero(mask)
    return gen._from_coo(100000, 3, r, c, rng.standard_normal(len(r)))


def _col_sorted_cases():
    # column indices never decreasing over the entry array (the column-sorted
    # path), with empty leading, inner and trailing columns and one column
    # spanning many rows; and the same with one decrease near the end, which
    # must take the general path
    rng = np.random.default_rng(34)
    m, n = 30000, 9000
    cols = np.sort(rng.choice(np.arange(5, n - 7), 40000))
    cols[(cols > 3000) & (cols < 3400)] = 3200
    rows = np.sort(rng.integers(0, m, cols.size))
    key = np.unique(rows.astype(np.int64) * n + cols)
    r, c = key // n, key % n
    sorted_ = gen._from_coo(m, n, r, c, np.ones(len(r)))
    assert np.all(np.diff(sorted_.colind) >= 0)
    c2 = c.copy()
    c2[-3] = 1
    broken = gen._from_coo(m, n, r, c2, np.ones(len(r)))
    agg = gen.aggregation(10001, 8)
    aggT = gen._from_coo(agg.ncols, agg.nrows, agg.colind, agg.row_of_entry(), agg.vals)
    one_col = gen._from_coo(5000, 7, np.arange(5000), np.zeros(5000, int), np.ones(5000))
    eye = gen._from_coo(777, 777, np.arange(777), np.arange(777), np.ones(777))
    return [("col_sorted", sorted_), ("col_sorted_broken", broken), ("agg_T", aggT),
            ("one_col", one_col), ("identity", eye)]


def _skewed_blocks():
    # every row takes one column in [0, 4096) and two anywhere in [0, 200000):
    # the column blocks over [0, 4096) hold more entries than fit in LDS
    # (grouped in the scratch pairs), with columns of about 20 entries
    rng = np.random.default_rng(35)
    m, n = 80000, 200000
    r = np.repeat(np.arange(m), 3)
    c = np.stack([rng.integers(0, 4096, m), rng.integers(0, n, m), rng.integers(0, n, m)], 1)
    key = np.unique(r.astype(np.int64) * n + c.reshape(-1))
    return gen._from_coo(m, n, key // n, key % n, rng.standard_normal(len(key)))


def _nearly_symmetric():
    # a structurally symmetric pattern with one extra entry below the
    # diagonal (every entry above still finds its mirror: only the
    # above/below count tells), and the same with one extra entry above
    s = gen.poisson2d(60, 50)
    r, c = s.row_of_entry(), s.colind
    rng = np.random.default_rng(36)
    out = []
    for name, (i, j) in (("sym_extra_lower", (2000, 3)), ("sym_extra_upper", (3, 2000))):
        key = np.unique(np.concatenate([r.astype(np.int64) * s.ncols + c, [i * s.ncols + j]]))
        out.append((name, gen._from_coo(s.nrows, s.ncols, key // s.ncols, key % s.ncols,
                                        rng.standard_normal(len(key)))))
    return out


TRANSPOSE_CASES = MATS + [("long_cols", _with_long_columns()), ("agg", gen.aggregation(10001, 8)),
                          ("few_cols", _few_cols()), ("skewed_blocks", _skewed_blocks())] \
    + _col_sorted_cases() + _nearly_symmetric() + [("poisson2d_sym", gen.poisson2d(60, 50))]


@pytest.mark.parametrize("name,A", TRANSPOSE_CASES, ids=[n for n, _ in TRANSPOSE_CASES])
def test_transpose_bit_exact(name, A):
    P = sp.Pattern.from_host(A)
    Pt, perm = P.transpose()
    rpT, ciT, permo = oracle.transpose(A)
    assert np.array_equal(Pt.rowptr.cpu().numpy(), rpT)
    assert np.array_equal(Pt.colind.cpu().numpy(), ciT)
    assert np.array_equal(perm.cpu().numpy(), permo)


# ---------------------------------------------------------------- SpGEMM
def _spgemm_cases():
    a, b = gen.fig2_pair()
    yield "fig2", a, b
    for s in range(3):
        yield f"rand{s}", gen.random_csr(300, 200, 0.03, seed=[s, 1], empty_rows=0.1), \
            gen.random_csr(200, 250, 0.03, seed=[s, 2], empty_rows=0.1)
    # product counts in every bin: up to 16, 64, 512, 4096 and beyond
    yield "bins", gen.random_csr(400, 300, 0.02, seed=9, long_rows=6, long_len=250), \
        gen.random_csr(300, 5000, 0.004, seed=10, long_rows=10, long_len=600)
    yield "dense_row", gen.random_csr(20, 150, 0.05, seed=11, long_rows=2, long_len=150), \
        gen.random_csr(150, 9000, 0.003, seed=12, long_rows=40, long_len=200)
    A3 = gen.poisson3d(16)
    yield "galerkin_AP", A3, gen.aggregation(16 ** 3, 8)
    yield "empty", gen.random_csr(5, 6, 0.0, seed=0), gen.random_csr(6, 4, 0.5, seed=1)


SPG = list(_spgemm_cases())


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("name,A,B", SPG, ids=[c[0] for c in SPG])
def test_spgemm_fwd_bwd(dtype, name, A, B):
    Ad, Bd = _dev(A, dtype), _dev(B, dtype)
    PC, vC = sp.spgemm(Ad.pattern, Ad.vals, Bd.pattern, Bd.vals)
    Ao, Bo = upcast(A, dtype), upcast(B, dtype)
    rpo, cio, vo = oracle.spgemm(Ao, Bo)
    assert np.array_equal(PC.rowptr.cpu().numpy(), rpo)
    assert np.array_equal(PC.colind.cpu().numpy(), cio)
    assert_close(vC, vo, dtype, "C vals")
    # the numeric call without the symbolic call's row classes classifies
    # the rows again and launches every class: same result bit for bit
    from paper_2212_05159_amd import capi
    dA, dB = Ad.pattern.desc(Ad.vals), Bd.pattern.desc(Bd.vals)
    ws = capi._ws(capi.csr_spgemm_workspace(dA, dB), Ad.vals.device)
    rp2 = torch.empty_like(PC.rowptr)
    assert capi.csr_spgemm_symbolic(dA, dB, rp2, ws) == PC.nnz
    ci2, v2 = torch.empty_like(PC.colind), torch.empty_like(vC)
    capi.csr_spgemm_fwd(dA, dB, rp2, ci2, v2, ws)
    assert torch.equal(rp2, PC.rowptr) and torch.equal(ci2, PC.colind) and torch.equal(v2, vC)
    V = gen.normal(len(cio), 13)
    gA, gB = sp.spgemm_bwd(Ad.pattern, Ad.vals, Bd.pattern, Bd.vals, PC, to_dev(V, dtype))
    gAo, gBo = oracle.spgemm_bwd(Ao, Bo, rpo, cio, rounded(V, dtype))
    assert_close(gA, gAo, dtype, "gA")
    assert_close(gB, gBo, dtype, "gB")


@pytest.mark.parametrize("N", [16, 32])
def test_galerkin_pattern_and_values(N):
    # P^T (A P) for the 3D Poisson matrix and 8-aggregation: exact pattern,
    # and the coarse values 34 / -1 / -8 are exact in float32.
    A = _dev(gen.poisson3d(N), torch.float32)
    P = gen.aggregation(N ** 3, 8)
    rpT, ciT, perm = oracle.transpose(P)
    Pt = _dev(gen.Csr(P.ncols, P.nrows, rpT, ciT, P.vals[perm]), torch.float32)
    Pd = _dev(P, torch.float32)
    PAP, vAP = sp.spgemm(A.pattern, A.vals, Pd.pattern, Pd.vals)
    PC, vC = sp.spgemm(Pt.pattern, Pt.vals, PAP, vAP)
    coarse = gen._stencil((N, N, N // 8),
                          [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)],
                          [-8.0, -8.0, -1.0, 34.0, -1.0, -8.0, -8.0])
    assert np.array_equal(PC.rowptr.cpu().numpy(), coarse.rowptr)
    assert np.array_equal(PC.colind.cpu().numpy(), coarse.colind)
    assert np.array_equal(vC.cpu().numpy().astype(np.float64), coarse.vals)


# ---------------------------------------------------------------- levels / tri-solve
def _tri_cases():
    yield "poisson2d_lower", gen.tril(gen.poisson2d(40, 23)), True
    yield "poisson2d_upper", gen.triu(gen.poisson2d(40, 23)), False
    yield "rand_lower", gen.random_lower(3000, 0.002, seed=41), True
    yield "chain", gen.tril(gen.poisson1d(5000)), True
    yield "q1_four_colour", gen.tril(gen.permute_sym(gen.anisotropic_q1(64, 1e-3, np.pi / 4),
                                                     gen.four_color_2d(64))), True
    yield "q1_natural", gen.tril(gen.anisotropic_q1(48, 1e-2, 0.3)), True
    yield "rb3d", gen.tril(gen.permute_sym(gen.poisson3d(40), gen.red_black_3d(40))), True
    yield "rb3d_upper", gen.triu(gen.permute_sym(gen.poisson3d(24), gen.red_black_3d(24))), False
    yield "diag_only", gen._from_coo(3000, 3000, np.arange(3000), np.arange(3000),
                                     np.linspace(1, 2, 3000)), True
    yield "one", gen._from_coo(1, 1, [0], [0], [2.0]), True


TRI = list(_tri_cases())
# Few levels over many rows: the grouping by level runs as a multi-split
# over many tiles and chunks (regression cover for its per-chunk counts).
LEVELS_WIDE = [
    ("q1_four_colour_400", gen.tril(gen.permute_sym(gen.anisotropic_q1(400, 1e-2, 0.7),
                                                    gen.four_color_2d(400))), True),
    ("geometric_29", gen.tril(gen.block_diag([gen.geometric_graph_laplacian(
        b, n_range=(300, 5000), k_range=(6, 14)) for b in range(12)])[0]), True),
]


@pytest.mark.parametrize("name,T,lower", TRI + LEVELS_WIDE, ids=[c[0] for c in TRI + LEVELS_WIDE])
def test_levels_bit_exact(name, T, lower):
    P = sp.Pattern.from_host(T)
    nl, lph, lp, lr, lor = P.levels(lower)
    lo, lpo, lro = oracle.levels(T, lower)
    assert nl == len(lpo) - 1
    assert np.array_equal(lor.cpu().numpy(), lo)
    assert np.array_equal(lph, lpo)
    assert np.array_equal(lp.cpu().numpy(), lpo)
    assert np.array_equal(lr.cpu().numpy(), lro)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("name,T,lower", TRI + LEVELS_WIDE, ids=[c[0] for c in TRI + LEVELS_WIDE])
def test_trisolve_fwd_bwd(dtype, name, T, lower):
    # the wide-level cases run their levels as grid launches with 4 lanes of
    # 4 entries per row past the first level, over rows of uneven length
    if name.startswith(("q1", "poisson", "geometric")):
        # make the factor diagonally dominant so the solve is well conditioned
        T = gen.Csr(T.nrows, T.ncols, T.rowptr, T.colind,
                    np.where(T.colind == T.row_of_entry(), 3.0 + np.abs(T.vals), T.vals))
    b = gen.normal(T.nrows, 51)
    g = gen.normal(T.nrows, 52)
    Td = _dev(T, dtype)
    Td.vals.requires_grad_(True)
    bd = to_dev(b, dtype).requires_grad_(True)
    x = Td.solve_triangular(bd, lower=lower)
    (x * to_dev(g, dtype)).sum().backward()
    To = upcast(T, dtype)
    xo = oracle.trisolve(To, rounded(b, dtype), lower)
    assert_close(x, xo, dtype, "x")
    gbo, gvo = oracle.trisolve_bwd(To, xo, rounded(g, dtype), lower)
    assert_close(bd.grad, gbo, dtype, "gb")
    assert_close(Td.vals.grad, gvo, dtype, "gvals")


def test_trisolve_missing_diagonal_is_reported():
    from paper_2212_05159_amd import capi
    T = gen.tril(gen.poisson1d(50), -1)
    P = sp.Pattern.from_host(T)
    with pytest.raises(capi.CsradError) as ei:
        P.levels(True)
    assert ei.value.status == -4


# ---------------------------------------------------------------- determinism
def test_run_twice_bit_identical():
    A = gen.random_csr(2000, 1500, 0.01, seed=61, empty_rows=0.05)
    B = gen.random_csr(1500, 1800, 0.01, seed=62)
    Ad, Bd = _dev(A, torch.float32), _dev(B, torch.float32)
    x = to_dev(gen.normal(1500, 63), torch.float32)
    Xd = to_dev(gen.normal((1500, 64), 64), torch.float32)
    Gd = to_dev(gen.normal((2000, 64), 65), torch.float32)
    outs = []
    for _ in range(2):
        P = sp.Pattern.from_host(A)  # fresh transpose each time
        y = sp.spmv(P, Ad.vals, x)
        Cm = sp.spmm(P, Ad.vals, Xd)
        gB, gv = sp.spmm_bwd(P, Ad.vals, Xd, Gd)
        PC, vC = sp.spgemm(P, Ad.vals, Bd.pattern, Bd.vals)
        Pt, perm = P.transpose()
        outs.append([t.cpu().numpy() for t in (y, Cm, gB, gv, PC.rowptr, PC.colind, vC,
                                               Pt.rowptr, Pt.colind, perm)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_validate():
    from paper_2212_05159_amd import capi
    A = gen.random_csr(100, 80, 0.05, seed=71)
    P = sp.Pattern.from_host(A)
    ws = torch.empty(8, dtype=torch.uint8, device="cuda")
    st, bad = capi.csr_validate(P.desc(dtype=torch.float32), ws)
    assert st == 0 and bad == -1
    ci = A.colind.copy()
    r = int(np.nonzero(np.diff(A.rowptr) >= 2)[0][3])
    s = A.rowptr[r]
    ci[s], ci[s + 1] = ci[s + 1], ci[s]  # unsorted row
    Pbad = sp.Pattern(A.nrows, A.ncols, P.rowptr, to_dev(ci))
    st, bad = capi.csr_validate(Pbad.desc(dtype=torch.float32), ws)
    assert st == -3 and bad == r


@pytest.mark.parametrize("dtype", DTYPES)
def test_spmv_bwd_split_equals_fused(dtype):
    # the two ways of forming the SpMV backward give the same bits; the
    # autotuner picks one of them
    from paper_2212_05159_amd import autotune
    for seed, A in enumerate([gen.random_csr(2000, 1500, 0.01, seed=91, empty_rows=0.1),
                              gen.poisson2d(40, 40)]):
        Ad = _dev(A, dtype)
        x = to_dev(gen.normal(A.ncols, 92 + seed), dtype)
        gy = to_dev(gen.normal(A.nrows, 94 + seed), dtype)
        gx1, gv1 = sp.spmv_bwd(Ad.pattern, Ad.vals, x, gy, mode="fused")
        gx2, gv2 = sp.spmv_bwd(Ad.pattern, Ad.vals, x, gy, mode="split")
        assert torch.equal(gx1, gx2) and torch.equal(gv1, gv2)
        choice, _ = autotune.tune_spmv_bwd(Ad.pattern, Ad.vals, x, gy, reps=1, use_cache=False)
        assert choice in ("fused", "split")
        gx3, gv3 = sp.spmv_bwd(Ad.pattern, Ad.vals, x, gy)
        assert torch.equal(gx1, gx3) and torch.equal(gv1, gv3)
