"""Batched block-diagonal execution (one persistent launch per op over a
work queue) against the FP64 oracle, forward and backward.

Blocks: uneven random geometric-graph Laplacians (the batched workload's
recipe at smaller sizes), heavy-tailed row-length blocks (a few rows with
thousands of entries: the merge-path case), a block with one row spanning
every piece of its task, empty rows, and 1- and 2-row blocks.  Every
variant assignment (automatic, all row-split widths, staged, merge-path,
a random mix per block) must match the oracle on every output (float32
within infinity-norm relative error 1e-5, float64 within 1e-12); a block's
result must not depend on the rest of the batch (bit-identical rows when
the plan holds that block alone); triangular solves with IC(0) factors
per block match the oracle in both directions."""
import numpy as np
import pytest
import torch

import oracle
from paper_2212_05159_amd import batch as bt
from paper_2212_05159_amd import capi
from paper_2212_05159_amd import gen
from paper_2212_05159_amd import sparse as sp

from _util import TOL, assert_close, rel_err, to_dev, upcast

pytestmark = pytest.mark.gpu


def _one_long_row(n, length, seed):
    # row n//2 holds `length` entries, every other row at most 2
    rng = np.random.default_rng(seed)
    r = [np.full(length, n // 2)]
    c = [rng.choice(n, size=length, replace=False)]
    for i in range(n):
        if i != n // 2 and i % 3:
            k = 1 + (i % 2)
            r.append(np.full(k, i))
            c.append(rng.choice(n, size=k, replace=False))
    r, c = np.concatenate(r), np.concatenate(c)
    return gen._from_coo(n, n, r, c, rng.standard_normal(len(r)))


@pytest.fixture(scope="module")
def blocks():
    geo = bt.geometric_batch(8, n_range=(300, 5000), k_range=(6, 14))
    skew = [gen.power_law_rows(n, s, alpha=1.1, max_len=m, empty=e)
            for n, s, m, e in ((6000, 1, 5000, 0.0), (3000, 2, 2900, 0.3), (9000, 3, 8000, 0.1))]
    tiny = [gen.power_law_rows(1, 4), gen._from_coo(2, 2, np.array([0, 1, 1]),
                                                    np.array([1, 0, 1]), np.array([2.0, -1.0, 3.0]))]
    longrow = [_one_long_row(7000, 6500, 5)]
    out = []
    for i in range(8):
        out.append(geo[i])
        if i < 3:
            out.append(skew[i])
    out[2:2] = tiny
    out.append(longrow[0])
    return out


def _variants(name, nb):
    if name == "auto":
        return None
    if name == "mix":
        rng = np.random.default_rng(9)
        return rng.choice([bt.MERGE, bt.STAGED, 1, 2, 3, 4, 5, 6, 7], size=nb).astype(np.int32)
    code = {"merge": bt.MERGE, "staged": bt.STAGED, "rows1": 1, "rows4": 3, "rows16": 5,
            "rows64": 7}[name]
    return np.full(nb, code, np.int32)


VARIANTS = ["auto", "merge", "staged", "rows1", "rows4", "rows16", "rows64", "mix"]


@pytest.mark.parametrize("dtype,k", [(torch.float32, 64), (torch.float64, 40)],
                         ids=["f32k64", "f64k40"])
@pytest.mark.parametrize("vname", VARIANTS)
def test_batched_ops_match_oracle(blocks, dtype, k, vname):
    Bt = bt.Batch(blocks, dtype=dtype)
    for fam in ("spmv", "spmv_t", "spmm", "spmm_t"):
        Bt.set_variants(fam, _variants(vname, Bt.nblocks))
    n = Bt.pattern.nrows
    x = to_dev(gen.normal(n, 1), dtype)
    gy = to_dev(gen.normal(n, 2), dtype)
    X = to_dev(gen.normal((n, k), 3), dtype)
    G = to_dev(gen.normal((n, k), 4), dtype)
    y = Bt.spmv(x)
    gx, gv = Bt.spmv_bwd(x, gy)
    Cm = Bt.spmm(X)
    gX, gvm = Bt.spmm_bwd(X, G)
    torch.cuda.synchronize()
    Ao = upcast(Bt.host, dtype)
    f = lambda t: t.double().cpu().numpy()
    assert_close(y, oracle.spmv(Ao, f(x)), dtype, f"{vname} y")
    gxo, gvo = oracle.spmv_bwd(Ao, f(x), f(gy))
    assert_close(gx, gxo, dtype, f"{vname} gx")
    assert_close(gv, gvo, dtype, f"{vname} gvals")
    assert_close(Cm, oracle.spmm(Ao, f(X)), dtype, f"{vname} C")
    gXo, gvmo = oracle.spmm_bwd(Ao, f(X), f(G))
    assert_close(gX, gXo, dtype, f"{vname} gB")
    assert_close(gvm, gvmo, dtype, f"{vname} gvals(SpMM)")
    # one-output backward forms
    gx1, _ = Bt.spmv_bwd(x, gy, need_vals=False)
    _, gv1 = Bt.spmv_bwd(x, gy, need_x=False)
    gX1, _ = Bt.spmm_bwd(X, G, need_vals=False)
    _, gvm1 = Bt.spmm_bwd(X, G, need_B=False)
    assert torch.equal(gx1, gx) and torch.equal(gv1, gv)
    assert torch.equal(gX1, gX) and torch.equal(gvm1, gvm)
    # the plain whole-batch kernels (the autotuner's other choice per op)
    Bt.impl = {op: "plain" for op in Bt.impl}
    assert_close(Bt.spmv(x), oracle.spmv(Ao, f(x)), dtype, f"{vname} y (plain)")
    gxp, gvp = Bt.spmv_bwd(x, gy)
    assert_close(gxp, gxo, dtype, f"{vname} gx (plain)")
    assert_close(gvp, gvo, dtype, f"{vname} gvals (plain)")
    assert_close(Bt.spmm(X), oracle.spmm(Ao, f(X)), dtype, f"{vname} C (plain)")
    gXp, gvmp = Bt.spmm_bwd(X, G)
    assert_close(gXp, gXo, dtype, f"{vname} gB (plain)")
    assert_close(gvmp, gvmo, dtype, f"{vname} gvals(SpMM) (plain)")
    Bt.impl = {op: "queue" for op in Bt.impl}
    # split backward (A^T products over A^T's plan, value gradients row-wise
    # over A's plan): the same products and sums, so the same bits
    Bt.bwd_split = {"spmv": True, "spmm": True}
    gx2, gv2 = Bt.spmv_bwd(x, gy)
    gX2, gvm2 = Bt.spmm_bwd(X, G)
    _, gv3 = Bt.spmv_bwd(x, gy, need_x=False)
    _, gvm3 = Bt.spmm_bwd(X, G, need_B=False)
    assert torch.equal(gx2, gx) and torch.equal(gv2, gv) and torch.equal(gv3, gv)
    assert torch.equal(gX2, gX) and torch.equal(gvm2, gvm) and torch.equal(gvm3, gvm)


def test_block_result_independent_of_batch(blocks):
    Bt = bt.Batch(blocks, dtype=torch.float32)
    nb = Bt.nblocks
    var = _variants("mix", nb)
    for fam in ("spmv", "spmv_t", "spmm", "spmm_t"):
        Bt.set_variants(fam, var)
    n = Bt.pattern.nrows
    x = to_dev(gen.normal(n, 5), torch.float32)
    gy = to_dev(gen.normal(n, 6), torch.float32)
    X = to_dev(gen.normal((n, 64), 7), torch.float32)
    G = to_dev(gen.normal((n, 64), 8), torch.float32)
    full = (Bt.spmv(x), *Bt.spmv_bwd(x, gy), Bt.spmm(X), *Bt.spmm_bwd(X, G))
    rp = Bt.host.rowptr
    for b in (0, 3, 4, nb - 1):
        alone = np.full(nb, bt.SKIP, np.int32)
        alone[b] = var[b]
        for fam in ("spmv", "spmv_t", "spmm", "spmm_t"):
            Bt.set_variants(fam, alone)
        part = (Bt.spmv(x), *Bt.spmv_bwd(x, gy), Bt.spmm(X), *Bt.spmm_bwd(X, G))
        r0, r1 = int(Bt.block_rowptr[b]), int(Bt.block_rowptr[b + 1])
        e0, e1 = int(rp[r0]), int(rp[r1])
        for i, (a, c) in enumerate(zip(full, part)):
            sl = slice(e0, e1) if i in (2, 5) else slice(r0, r1)
            assert torch.equal(a[sl], c[sl]), (b, i)


def test_single_row_spanning_all_pieces():
    # one row of 40,000 entries in a task: every thread's (and group's)
    # piece ends inside it, so its sum is completed from a 255-long chain
    n = 50_000
    A = _one_long_row(n, 40_000, 11)
    for dtype in (torch.float32, torch.float64):
        Bt = bt.Batch(host=A, block_rowptr=np.array([0, n]), dtype=dtype)
        for fam in ("spmv", "spmv_t", "spmm", "spmm_t"):
            Bt.set_variants(fam, [bt.MERGE])
        x = to_dev(gen.normal(n, 12), dtype)
        X = to_dev(gen.normal((n, 16), 13), dtype)
        Ao = upcast(A, dtype)
        f = lambda t: t.double().cpu().numpy()
        assert_close(Bt.spmv(x), oracle.spmv(Ao, f(x)), dtype, "y")
        assert_close(Bt.spmm(X), oracle.spmm(Ao, f(X)), dtype, "C")
        gx, _ = Bt.spmv_bwd(x, x)
        assert_close(gx, oracle.spmv_bwd(Ao, f(x), f(x))[0], dtype, "gx")
        gX, _ = Bt.spmm_bwd(X, X)
        assert_close(gX, oracle.spmm_bwd(Ao, f(X), f(X))[0], dtype, "gB")


@pytest.fixture(scope="module")
def ic0_blocks():
    # IC(0) factors per block (the oracle's, exactly as the batched tri-solve
    # workload uses them), on uneven geometric-graph Laplacians
    geo = bt.geometric_batch(10, n_range=(200, 6000), k_range=(6, 14), first=20)
    Ls = []
    for blk in geo:
        Lp = gen.tril(blk)
        Ls.append(gen.Csr(Lp.nrows, Lp.ncols, Lp.rowptr, Lp.colind, oracle.ic0(blk, Lp)))
    return Ls


@pytest.mark.parametrize("mode", ["blocks", "levels", "grid"])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_batched_trisolve_ic0_matches_oracle(ic0_blocks, dtype, mode):
    # both batched solve modes: a workgroup per block ("blocks"), and one
    # cooperative launch with grid barriers between the batch's levels
    Bt = bt.Batch(ic0_blocks, dtype=dtype)
    Bt.tri_mode = mode
    n = Bt.pattern.nrows
    T = Bt.A
    b = to_dev(gen.normal(n, 14), dtype)
    g = to_dev(gen.normal(n, 15), dtype)
    x = Bt.trisolve(T, b, True)
    gb, gv = Bt.trisolve_bwd(T, x, g, True)
    To = upcast(Bt.host, dtype)
    xo = oracle.trisolve(To, b.double().cpu().numpy(), True)
    assert_close(x, xo, dtype, "x")
    gbo, gvo = oracle.trisolve_bwd(To, xo, g.double().cpu().numpy(), True)
    assert_close(gb, gbo, dtype, "gb")
    assert_close(gv, gvo, dtype, "gvals")
    # upper-triangular solves (T^T of the factors) through the same launch
    Tu = T.transpose()
    xu = Bt.trisolve(Tu, b, False)
    rpT, ciT, perm = oracle.transpose(Bt.host)
    Tuo = upcast(gen.Csr(n, n, rpT, ciT, Bt.host.vals[perm]), dtype)
    assert_close(xu, oracle.trisolve(Tuo, b.double().cpu().numpy(), False), dtype, "x upper")
    # equal to the library's level-by-level solve of the whole matrix
    x1 = sp.trisolve(T.pattern, T.vals, b, True)
    assert rel_err(x, x1.cpu().numpy()) <= TOL[dtype]
    # the autotuner times the three modes and keeps one; results unchanged
    ms = Bt.autotune_trisolve(T, True, reps=1)
    assert set(ms) == {"blocks", "levels", "grid"} and Bt.tri_mode in ms
    assert_close(Bt.trisolve(T, b, True), xo, dtype, "x (tuned mode)")


def test_batched_autograd_matches_oracle(blocks, ic0_blocks):
    Bt = bt.Batch(blocks, dtype=torch.float64)
    n = Bt.pattern.nrows
    vals = Bt.A.vals.detach().clone().requires_grad_(True)
    x = to_dev(gen.normal(n, 16)).requires_grad_(True)
    X = to_dev(gen.normal((n, 8), 17)).requires_grad_(True)
    t = to_dev(gen.normal(n, 18))
    loss = 0.5 * ((bt.BatchSpMV.apply(Bt, vals, x) - t) ** 2).sum() + \
        (bt.BatchSpMM.apply(Bt, vals, X) ** 2).sum()
    loss.backward()
    A = Bt.host
    xn, Xn, tn = x.detach().cpu().numpy(), X.detach().cpu().numpy(), t.cpu().numpy()
    gy = oracle.spmv(A, xn) - tn
    gx1, gv1 = oracle.spmv_bwd(A, xn, gy)
    gX2, gv2 = oracle.spmm_bwd(A, Xn, 2 * oracle.spmm(A, Xn))
    assert rel_err(vals.grad, gv1 + gv2) < 1e-12
    assert rel_err(x.grad, gx1) < 1e-12
    assert rel_err(X.grad, gX2) < 1e-12
    Lb = bt.Batch(ic0_blocks, dtype=torch.float64)
    lv = Lb.A.vals.detach().clone().requires_grad_(True)
    b = to_dev(gen.normal(Lb.pattern.nrows, 19)).requires_grad_(True)
    xs = bt.BatchTriSolve.apply(Lb, Lb.pattern, lv, b, True)
    (xs ** 2).sum().backward()
    xo = oracle.trisolve(Lb.host, b.detach().cpu().numpy(), True)
    gbo, gvo = oracle.trisolve_bwd(Lb.host, xo, 2 * xo, True)
    assert rel_err(b.grad, gbo) < 1e-12 and rel_err(lv.grad, gvo) < 1e-12


def test_autotuned_variants_match_oracle(blocks):
    Bt = bt.Batch(blocks, dtype=torch.float32)
    res = Bt.autotune(k=64, reps=1)
    assert set(res) == {"spmv", "spmv_t", "spmm", "spmm_t"}
    assert set(Bt.bwd_times) == {"spmv", "spmm"}
    assert set(Bt.impl_times) == {"spmv", "spmv_bwd", "spmm", "spmm_bwd"}
    assert all(Bt.impl[op] == v["impl"] in ("queue", "plain") for op, v in Bt.impl_times.items())
    classes = set(Bt.block_classes())
    for fam, per in res.items():
        assert set(per) == classes
        assert all(v[0] in bt.CANDIDATES[fam] for v in per.values())
    n = Bt.pattern.nrows
    x = to_dev(gen.normal(n, 20), torch.float32)
    X = to_dev(gen.normal((n, 64), 21), torch.float32)
    Ao = upcast(Bt.host, torch.float32)
    assert_close(Bt.spmv(x), oracle.spmv(Ao, x.double().cpu().numpy()), torch.float32, "y")
    assert_close(Bt.spmm(X), oracle.spmm(Ao, X.double().cpu().numpy()), torch.float32, "C")
    gX, gvm = Bt.spmm_bwd(X, X)
    gXo, gvmo = oracle.spmm_bwd(Ao, X.double().cpu().numpy(), X.double().cpu().numpy())
    assert_close(gX, gXo, torch.float32, "gB")
    assert_close(gvm, gvmo, torch.float32, "gvals")


def test_plan_argument_errors(blocks):
    Bt = bt.Batch(blocks[:4], dtype=torch.float32)
    d = Bt.pattern.desc(Bt.A.vals)
    ws = capi._ws(capi.csr_batch_plan_workspace(d, 4, 1024), "cuda")
    bad = Bt.block_rowptr.copy()
    bad[-1] -= 1  # does not end at the matrix's rows
    with pytest.raises(capi.CsradError):
        capi.csr_batch_plan_build(d, bad, None, 1024, ws)
    with pytest.raises(capi.CsradError):
        capi.csr_batch_plan_build(d, Bt.block_rowptr, np.full(4, 11, np.int32), 1024, ws)
    with pytest.raises(capi.CsradError):  # workspace too small
        capi.csr_batch_plan_build(d, Bt.block_rowptr, None, 1024, ws[:64])
    plan = capi.csr_batch_plan_build(d, Bt.block_rowptr, None, 1024, ws)
    assert plan.ntasks >= 4 and plan.nblocks == 4
    y = torch.empty(Bt.pattern.nrows + 5, device="cuda")
    other = bt.Batch(blocks[4:6], dtype=torch.float32)
    with pytest.raises(capi.CsradError):  # a plan of another matrix
        capi.csr_batch_spmv_fwd(other.pattern.desc(other.A.vals), plan, y, y)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_batched_ic0_matches_oracle(dtype):
    geo = bt.geometric_batch(9, n_range=(200, 6000), k_range=(6, 14), first=40)
    lows = [gen.tril(b) for b in geo]
    Bt = bt.Batch(lows, dtype=dtype)
    Lv = Bt.ic0(Bt.A)
    want = np.concatenate([oracle.ic0(upcast(b, dtype), lo) for b, lo in zip(geo, lows)])
    assert_close(Lv, want, dtype, "IC(0)")
    # the 1D Poisson matrix has no fill: IC(0) is its exact Cholesky factor
    # (L_ii = sqrt((i+1)/i), L_{i+1,i} = -sqrt(i/(i+1)), 1-based)
    A1 = gen.poisson1d(300)
    P1 = bt.Batch([gen.tril(A1)], dtype=torch.float64)
    L1 = P1.ic0(P1.A).cpu().numpy()
    i = np.arange(1, 301)
    assert np.allclose(L1[0::2], np.sqrt((i + 1) / i), rtol=1e-13)
    assert np.allclose(L1[1::2], -np.sqrt(i[:-1] / (i[:-1] + 1)), rtol=1e-13)
