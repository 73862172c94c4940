"""Parity at the sizes the benchmark runs.

* The 128^3 benchmark step (3D Poisson, n = 2,097,152, nnz = 14,581,760;
  SpMM with 64 columns; the Galerkin product P^T A P with 8-aggregation;
  solves with tril of the red-black ordered A), run exactly as timed --
  autotuned plans, three concurrent chains -- against the float64 oracle
  on the same float32 inputs: every integer output bit-exact (A's
  transpose, the patterns of A P and P^T A P, the level sets), every
  float32 output within infinity-norm relative error 1e-5.  At this size
  the SpGEMM kernels sweep their capped grids many times over and the SpMM
  kernels run the autotuner's traversal plans.
* Differentiated CG on 2D anisotropic Q1 diffusion 512^2 (eps 1e-3, angle
  pi/4, n = 262,144), K = 100, loss 0.5 ||x_K - t||^2: float64 values
  against the oracle and central differences; float32 values with float64
  dots against the oracle with the normwise bound of the float32 reading.
* Prefix sums over more than 2048 tiles of 2048 items (the unfused scan)
  inside the sparse + sparse and transpose symbolic passes."""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

import bench
import oracle
from paper_2212_05159_amd import autotune
from paper_2212_05159_amd import cg as cgmod
from paper_2212_05159_amd import gen
from paper_2212_05159_amd import sparse as sp

from _util import rel_err, to_dev, upcast

pytestmark = pytest.mark.gpu

F32_TOL = 1e-5


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def step128():
    h = bench.make_inputs(128, 64)
    d = bench.Device(h)
    P0 = sp.Pattern(d.n, d.n, d.A_rp, d.A_ci)
    autotune.tune_spmm(P0, d.A_v, d.B, d.G, reps=2, use_cache=False)
    d.plan_fwd, d.plan_bwd = P0.plan("spmm_fwd"), P0.plan("spmm_bwd")
    d.spmv_bwd_mode = autotune.tune_spmv_bwd(P0, d.A_v, d.x, d.gy, reps=2, use_cache=False)[0]
    d.streams = tuple(torch.cuda.Stream() for _ in range(3))
    d.pool = cf.ThreadPoolExecutor(2)
    outs = {}
    print(f"[fullsize] 128^3 step, plans {d.plan_fwd} / {d.plan_bwd}, spmv bwd {d.spmv_bwd_mode}",
          flush=True)
    bench.run_step_streams(d, [bench.Marks(False) for _ in range(3)], outs)
    torch.cuda.synchronize()
    d.pool.shutdown()
    got = {k: _np(v) for k, v in outs.items()}
    f = lambda a: np.asarray(a, np.float64)
    A, P, L = h["A"], h["P"], h["L"]
    Af = gen.Csr(A.nrows, A.ncols, A.rowptr, A.colind, f(A.vals))
    return h, d, got, Af, P, L, f


def test_step128_spmv_spmm(step128):
    h, d, got, Af, P, L, f = step128
    y = oracle.spmv(Af, f(h["x"]))
    assert rel_err(got["y"], y) <= F32_TOL
    gx, gv = oracle.spmv_bwd(Af, f(h["x"]), f(h["gy"]))
    assert rel_err(got["gx"], gx) <= F32_TOL
    assert rel_err(got["gv"], gv) <= F32_TOL
    B, G = f(h["B"]), f(h["G"])
    C = oracle.spmm(Af, B)
    assert rel_err(got["C"], C) <= F32_TOL
    del C
    gB, gvm = oracle.spmm_bwd(Af, B, G)
    assert rel_err(got["gB"], gB) <= F32_TOL
    assert rel_err(got["gvm"], gvm) <= F32_TOL


def test_step128_galerkin(step128):
    h, d, got, Af, P, L, f = step128
    rpAP, ciAP, vAP = oracle.spgemm(Af, P)
    assert len(ciAP) == 10_911_744
    assert np.array_equal(got["rpAP"], rpAP) and np.array_equal(got["ciAP"], ciAP)
    assert rel_err(got["vAP"], vAP) <= F32_TOL
    rpT, ciT, perm = oracle.transpose(P)
    Pt = gen.Csr(P.ncols, P.nrows, rpT, ciT, P.vals[perm])
    AP = gen.Csr(Af.nrows, P.ncols, rpAP, ciAP, vAP)
    rpC, ciC, vC = oracle.spgemm(Pt, AP)
    assert len(ciC) == 1_794_048
    assert np.array_equal(got["rpC"], rpC) and np.array_equal(got["ciC"], ciC)
    assert rel_err(got["vC"], vC) <= F32_TOL
    # coarse operator of the 128^3 Poisson matrix: 7-point stencil on the
    # 16 x 128 x 128 aggregate grid, 34 on the diagonal, -1 (x), -8 (y, z)
    assert set(np.unique(got["vC"]).tolist()) == {34.0, -1.0, -8.0}
    gPt, gAP = oracle.spgemm_bwd(Pt, AP, rpC, ciC, f(h["V"]))
    assert rel_err(got["gPt"], gPt) <= F32_TOL
    assert rel_err(got["gAP"], gAP) <= F32_TOL
    gA, gP = oracle.spgemm_bwd(Af, P, rpAP, ciAP, gAP)
    assert rel_err(got["gA"], gA) <= F32_TOL
    assert rel_err(got["gP"], gP) <= F32_TOL


def test_step128_transpose_levels_trisolve(step128):
    h, d, got, Af, P, L, f = step128
    PA = sp.Pattern(d.n, d.n, d.A_rp, d.A_ci)
    PAt, permA = PA.transpose()
    rpT, ciT, perm = oracle.transpose(Af)
    assert np.array_equal(_np(PAt.rowptr), rpT)
    assert np.array_equal(_np(PAt.colind), ciT)
    assert np.array_equal(_np(permA), perm)
    PL = sp.Pattern(d.n, d.n, d.L_rp, d.L_ci)
    PLt, permL = PL.transpose()  # the general (column-block) form at 8.4M entries
    rpT, ciT, perm = oracle.transpose(L)
    assert np.array_equal(_np(PLt.rowptr), rpT)
    assert np.array_equal(_np(PLt.colind), ciT)
    assert np.array_equal(_np(permL), perm)
    nl, lph, lptr, lrows, lor = PL.levels(True)
    lor_o, lptr_o, lrows_o = oracle.levels(L, True)
    assert nl == 2
    assert np.array_equal(lph, lptr_o) and np.array_equal(_np(lptr), lptr_o)
    assert np.array_equal(_np(lrows), lrows_o) and np.array_equal(_np(lor), lor_o)
    Lf = gen.Csr(L.nrows, L.ncols, L.rowptr, L.colind, f(L.vals).astype(np.float32).astype(np.float64))
    xL = oracle.trisolve(Lf, f(h["bL"]), True)
    assert rel_err(got["xL"], xL) <= F32_TOL
    gbL, gvL = oracle.trisolve_bwd(Lf, xL, f(h["gL"]), True)
    assert rel_err(got["gbL"], gbL) <= F32_TOL
    assert rel_err(got["gvL"], gvL) <= F32_TOL


# ----------------------------------------------------------------------
# Differentiated CG at 512^2, K = 100
# ----------------------------------------------------------------------
@pytest.fixture(scope="module")
def q1_512():
    A = gen.anisotropic_q1(512, 1e-3, np.pi / 4)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(A.nrows)
    t = rng.standard_normal(A.nrows)
    return A, b, t


def _gpu_cg(A, b, t, dtype, K=100):
    Ad = sp.CsrTensor.from_host(A, dtype=dtype, requires_grad=True)
    bd = to_dev(b, dtype).requires_grad_(True)
    x = cgmod.cg_solve(Ad, bd, K)
    (0.5 * ((x - to_dev(t, dtype)) ** 2).sum()).backward()
    return _np(x), _np(Ad.vals.grad), _np(bd.grad)


def test_cg512_float64_matches_oracle_and_central_differences(q1_512):
    A, b, t = q1_512
    K = 100
    print("[fullsize] CG 512^2 K=100 float64", flush=True)
    x, gv, gb = _gpu_cg(A, b, t, torch.float64, K)
    xo = oracle.cg(A, b, K)
    gvo, gbo = oracle.cg_bwd(A, b, K, gx=xo - t)
    ex, egv, egb = rel_err(x, xo), rel_err(gv, gvo), rel_err(gb, gbo)
    print(f"[fullsize] float64 rel errs x {ex:.2e} gvals {egv:.2e} gb {egb:.2e}", flush=True)
    assert ex < 1e-10 and egv < 1e-9 and egb < 1e-9
    # central differences of the GPU's own float64 forward along random
    # directions on a few values and on b
    rng = np.random.default_rng(11)
    vals = torch.as_tensor(A.vals, dtype=torch.float64, device="cuda")
    bd = to_dev(b)
    td = to_dev(t)
    Pat = sp.Pattern.from_host(A)

    def loss(v, bb):
        x = cgmod.cg_solve(sp.CsrTensor(Pat, v), bb, K)
        return float(0.5 * ((x - td) ** 2).sum())

    for trial in range(3):
        e = rng.choice(A.nnz, 4, replace=False)
        dv = torch.zeros_like(vals)
        dv[torch.as_tensor(e, device="cuda")] = torch.as_tensor(
            rng.standard_normal(4) * np.abs(A.vals[e]), device="cuda")
        # the loss is ~1e9 (x_K of an ill-conditioned system) and carries
        # rounding noise of ~1e-3, so the steps are sized to keep both the
        # noise and the truncation error below the bar (measured on the
        # oracle: 3e-6 for the values with h = 1e-5, 1e-7 for b with 1e-2)
        h = 1e-5
        fd = (loss(vals + h * dv, bd) - loss(vals - h * dv, bd)) / (2 * h)
        an = float((torch.as_tensor(gv, device="cuda") * dv).sum())
        assert abs(fd - an) <= 5e-5 * abs(an), (trial, fd, an)
        j = rng.choice(A.nrows, 4, replace=False)
        db = torch.zeros_like(bd)
        db[torch.as_tensor(j, device="cuda")] = torch.as_tensor(rng.standard_normal(4), device="cuda")
        h = 1e-2
        fd = (loss(vals, bd + h * db) - loss(vals, bd - h * db)) / (2 * h)
        an = float((torch.as_tensor(gb, device="cuda") * db).sum())
        assert abs(fd - an) <= 1e-5 * abs(an), (trial, fd, an)


def test_cg512_float32_within_normwise_bound(q1_512):
    # Float32 values and vectors with float64 dot products, against the
    # oracle on the float32-rounded system: 100 float32 steps lose
    # orthogonality differently from float64 ones, so the bar is the
    # normwise 1e-3 of the float32 reading, not the element bound.
    A, b, t = q1_512
    K = 100
    print("[fullsize] CG 512^2 K=100 float32", flush=True)
    x, gv, gb = _gpu_cg(A, b, t, torch.float32, K)
    Ao = upcast(A, torch.float32)
    bo = b.astype(np.float32).astype(np.float64)
    to = t.astype(np.float32).astype(np.float64)
    xo = oracle.cg(Ao, bo, K)
    gvo, gbo = oracle.cg_bwd(Ao, bo, K, gx=xo - to)
    nrm = lambda a, r: float(np.linalg.norm(np.asarray(a, np.float64) - r) / np.linalg.norm(r))
    ex, egv, egb = nrm(x, xo), nrm(gv, gvo), nrm(gb, gbo)
    print(f"[fullsize] float32 normwise rel errs x {ex:.2e} gvals {egv:.2e} gb {egb:.2e}", flush=True)
    assert ex <= 1e-3 and egv <= 1e-3 and egb <= 1e-3


# ----------------------------------------------------------------------
# Prefix sums beyond the fused path (> 2048 tiles of 2048 items)
# ----------------------------------------------------------------------
def test_unfused_scan_in_symbolic_passes():
    m = 5_000_000  # 2442 tiles of 2048 row counts
    A = gen.random_rows(m, 1 << 20, 2, seed=31)
    B = gen.random_rows(m, 1 << 20, 2, seed=32)
    print(f"[fullsize] sparse + sparse with {m} rows", flush=True)
    Ad = sp.CsrTensor.from_host(A, dtype=torch.float32)
    Bd = sp.CsrTensor.from_host(B, dtype=torch.float32)
    PC, vC = sp.spadd(Ad.pattern, Ad.vals, Bd.pattern, Bd.vals, 1.0, -2.0)
    rpC, ciC, vCo = oracle.spadd(upcast(A, torch.float32), upcast(B, torch.float32), 1.0, -2.0)
    assert np.array_equal(_np(PC.rowptr), rpC) and np.array_equal(_np(PC.colind), ciC)
    assert np.array_equal(_np(vC), vCo.astype(np.float32))
    # transpose of a 65536 x 5M random pattern: 2442 column blocks of 2048
    W = gen.random_rows(1 << 16, m, 40, seed=33)
    Wd = sp.Pattern.from_host(W)
    print(f"[fullsize] transpose with {m} columns", flush=True)
    Wt, perm = Wd.transpose()
    rpT, ciT, permo = oracle.transpose(W)
    assert np.array_equal(_np(Wt.rowptr), rpT)
    assert np.array_equal(_np(Wt.colind), ciT)
    assert np.array_equal(_np(perm), permo)
    # more than 2^25 columns: the per-entry form (device-atomic column
    # counts, whose 33.6M-item scan takes the unfused path)
    n2 = (1 << 25) + 12345
    W2 = gen.random_rows(4096, n2, 8, seed=34)
    print(f"[fullsize] transpose with {n2} columns", flush=True)
    W2t, perm2 = sp.Pattern.from_host(W2).transpose()
    rpT, ciT, permo = oracle.transpose(W2)
    assert np.array_equal(_np(W2t.rowptr), rpT)
    assert np.array_equal(_np(W2t.colind), ciT)
    assert np.array_equal(_np(perm2), permo)


def test_spgemm_bwd_batched_float64():
    # 600,000 rows of 7 entries (lanes_for 8): rows x lanes reach 8 times
    # the chip's resident threads, so both backward kernels take U = 4
    # entries per lane; float64 values against the oracle (the float32 form
    # at this size runs inside the 128^3 step above)
    m, n, p = 600_000, 600_000, 80_000
    A = gen.random_rows(m, n, 7, seed=41)
    B = gen.random_rows(n, p, 2, seed=42)
    print(f"[fullsize] SpGEMM VJP, batched entries, {m} rows, float64", flush=True)
    Ad = sp.CsrTensor.from_host(A, dtype=torch.float64)
    Bd = sp.CsrTensor.from_host(B, dtype=torch.float64)
    PC, vC = sp.spgemm(Ad.pattern, Ad.vals, Bd.pattern, Bd.vals)
    # the product itself: B's rows hold 2 entries, so the row merge keeps 4
    # rows in flight per group with a 2-entry list window
    rpo, cio, vo = oracle.spgemm(A, B)
    assert np.array_equal(_np(PC.rowptr), rpo)
    assert np.array_equal(_np(PC.colind), cio)
    assert rel_err(_np(vC), vo) <= 1e-12
    rng = np.random.default_rng(43)
    gC = rng.standard_normal(PC.nnz)
    gA, gB = sp.spgemm_bwd(Ad.pattern, Ad.vals, Bd.pattern, Bd.vals, PC,
                           torch.as_tensor(gC, device="cuda"))
    gAo, gBo = oracle.spgemm_bwd(A, B, _np(PC.rowptr), _np(PC.colind), gC)
    assert rel_err(_np(gA), gAo) <= 1e-12
    assert rel_err(_np(gB), gBo) <= 1e-12
