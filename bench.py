#!/usr/bin/env python3
"""Benchmark of the differentiable CSR hot path on one MI355X.

Workload (the single large operator): the 3D 7-point Poisson matrix on a
128^3 grid (n = 2,097,152, nnz = 14,581,760) in float32, a dense operand B
of n x 64 N(0,1) values, the aggregation prolongator P[i, i // 8] = 1 and
the Galerkin product P^T A P, plus a red-black ordered lower factor for
the triangular solve.  One step runs every op of the path forward and
backward, computing everything that depends only on a pattern afresh:

  transposes of A, P, P^T and L (pattern + permutation, values of P^T);
  SpMV y = A x and its VJP (A^T gy, gy x^T on pat(A));
  SpMM C = A B and its VJP (A^T G, G B^T on pat(A));
  SpGEMM A P and P^T (A P), symbolic + numeric, and both VJPs;
  level sets of L, x = L^{-1} b and its VJP.

value = algorithmic bytes of the step / step time (GB/s); each kernel's
algorithmic bytes count every array it must touch once.  The dominant
kernel (the fused SpMM backward) is also timed on its own with HIP events
on the launch stream for the roofline entry.

Second part (the "pcg" entry): preconditioned CG to ||r||/||b|| <= 1e-6 on
64 held-out 2D anisotropic Q1 diffusion systems of 1024^2 (2x2
four-coloured order, float32 values, float64 vectors), wall time per
system with HIP events, for the learned preconditioner M = L L^T in the
paper's form (L L^T approximates A^-1; the network trained here on 4096
systems of 256^2), the same network untrained, the factor reading of M
(L L^T approximates A, two triangular solves) trained and untrained,
Jacobi and plain CG.  Each timed solve includes building its
preconditioner (network inference, values of L^T, 1/diag); the level sets
of L's pattern are shared by all systems and analysed once beforehand.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
I4 = 4


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ----------------------------------------------------------------------
# Batched uneven blocks: one launch per op over a block-diagonal CSR
# ----------------------------------------------------------------------
def _geometric_block(b):
    from paper_2212_05159_amd import gen
    return gen.geometric_graph_laplacian(b)


def geometric_blocks(nblocks):
    """The first `nblocks` host blocks of the batched workload, built by a
    pool of threads (the k-NN queries and sorts release the GIL)."""
    import concurrent.futures as cf

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        blocks = list(ex.map(_geometric_block, range(nblocks)))
    return blocks, time.perf_counter() - t0


def batched_section(blocks, gen_s, reps=5, skew=None):
    """Batched uneven blocks: random geometric-graph Laplacians + 1e-2 I
    (n from 1k to 64k, kNN with k from 6 to 14), float32, concatenated
    block-diagonally; IC(0) factors per block computed on the GPU.  SpMV and
    SpMM (64 columns) forward and backward and the IC(0) solve forward and
    adjoint, each ONE persistent launch over the plan's work queue, with
    the variants the autotuner picks per class of blocks.  Beside them: the
    same plans with the automatic variants (untuned), the library's
    per-matrix kernels over the whole concatenation (one launch per op, one
    per level for the solves), and the ops launched block by block.  With
    `skew` (blocks with heavy-tailed row lengths), SpMV and SpMM forward and
    backward there under row-split, merge-path and the tuned choice."""
    import torch
    from paper_2212_05159_amd import batch as bt, gen
    from paper_2212_05159_amd import sparse as sp

    nblocks = len(blocks)
    t0 = time.perf_counter()
    B = bt.Batch(blocks)
    Lh = gen.tril(B.host)
    LB = bt.Batch(host=Lh, block_rowptr=B.block_rowptr)
    Lv = LB.ic0(LB.A)  # IC(0) of each block on the GPU
    L = sp.CsrTensor(LB.pattern, Lv)
    torch.cuda.synchronize()
    if not bool(torch.isfinite(Lv).all()):
        raise RuntimeError("IC(0) broke down on a block")
    n, nnz, nnzL = B.host.nrows, B.host.nnz, Lh.nnz
    k = 64
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    rnd = lambda *shape: torch.randn(*shape, generator=g, device="cuda", dtype=torch.float32)
    x, gy, bL, gL = rnd(n), rnd(n), rnd(n), rnd(n)
    X, G = rnd(n, k), rnd(n, k)
    P, v = B.pattern, B.A.vals
    P.transpose()
    L.pattern.transpose()
    nl = L.pattern.levels(True)[0]
    xL = torch.empty_like(bL)
    setup_s = time.perf_counter() - t0
    log(f"batched: {nblocks} blocks, n={n} nnz={nnz}, IC(0) nnz={nnzL} ({nl} levels), "
        f"setup {setup_s:.1f} s")

    V, I = 4, I4
    pat = lambda rows, z: (rows + 1) * I + z * I
    model = {"spmv fwd": pat(n, nnz) + nnz * V + 2 * n * V,
             "spmv bwd": pat(n, nnz) + nnz * (I + 2 * V) + 3 * n * V,
             "spmm fwd": pat(n, nnz) + nnz * V + 2 * n * k * V,
             "spmm bwd": pat(n, nnz) + nnz * (I + 2 * V) + 3 * n * k * V,
             "trisolve fwd": pat(n, nnzL) + nnzL * V + 2 * n * V + n * I,
             "trisolve bwd": (pat(n, nnzL) + nnzL * (I + V) + 2 * n * V + n * I)
             + (pat(n, nnzL) + nnzL * I + 2 * n * V + nnzL * V)}

    def batched_ops(Bt):
        return {
            "spmv fwd": lambda: Bt.spmv(x),
            "spmv bwd": lambda: Bt.spmv_bwd(x, gy),
            "spmm fwd": lambda: Bt.spmm(X),
            "spmm bwd": lambda: Bt.spmm_bwd(X, G),
            "trisolve fwd": lambda: LB.trisolve(L, bL, True),
            "trisolve bwd": lambda: LB.trisolve_bwd(L, xL, gL, True),
        }

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, r=reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(r):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    def table(ops):
        out = {}
        for name, fn in ops.items():
            ms = timed(fn)
            out[name] = {"ms": round(ms, 4), "GB/s": round(model[name] / (ms * 1e-3) / 1e9, 1)}
        return out

    xL.copy_(LB.trisolve(L, bL, True))
    untuned = table(batched_ops(B))
    t1 = time.perf_counter()
    tune = B.autotune(k=k, reps=3)
    tri_modes = LB.autotune_trisolve(L, True, reps=3)
    tune_s = time.perf_counter() - t1
    tuned = table(batched_ops(B))
    # the library's per-matrix kernels over the whole concatenation
    whole = table({
        "spmv fwd": lambda: sp.spmv(P, v, x),
        "spmv bwd": lambda: sp.spmv_bwd(P, v, x, gy),
        "spmm fwd": lambda: sp.spmm(P, v, X),
        "spmm bwd": lambda: sp.spmm_bwd(P, v, X, G),
        "trisolve fwd": lambda: sp.trisolve(L.pattern, Lv, bL, True),
        "trisolve bwd": lambda: sp.trisolve_bwd(L.pattern, Lv, xL, gL, True),
    })
    # the same six ops launched block by block (per-block patterns, values
    # and transposes made beforehand)
    per = []
    rp, rpL = B.host.rowptr, Lh.rowptr
    for bi in range(nblocks):
        r0, r1 = int(B.block_rowptr[bi]), int(B.block_rowptr[bi + 1])
        e_0, e_1 = int(rp[r0]), int(rp[r1])
        f_0, f_1 = int(rpL[r0]), int(rpL[r1])
        Pb = sp.Pattern(r1 - r0, r1 - r0, (P.rowptr[r0:r1 + 1] - e_0).contiguous(),
                        (P.colind[e_0:e_1] - r0).contiguous())
        PLb = sp.Pattern(r1 - r0, r1 - r0, (L.pattern.rowptr[r0:r1 + 1] - f_0).contiguous(),
                         (L.pattern.colind[f_0:f_1] - r0).contiguous())
        Pb.transpose()
        PLb.transpose()
        PLb.levels(True)
        per.append((Pb, v[e_0:e_1], PLb, Lv[f_0:f_1], slice(r0, r1)))
    xs, gys, Xs, Gs, bLs, xLs, gLs = (t.contiguous() for t in (x, gy, X, G, bL, xL, gL))

    def per_block():
        for Pb, vb, PLb, lvb, sl in per:
            sp.spmv(Pb, vb, xs[sl])
            sp.spmv_bwd(Pb, vb, xs[sl], gys[sl])
            sp.spmm(Pb, vb, Xs[sl])
            sp.spmm_bwd(Pb, vb, Xs[sl], Gs[sl])
            sp.trisolve(PLb, lvb, bLs[sl], True)
            sp.trisolve_bwd(PLb, lvb, xLs[sl], gLs[sl], True)

    per_ms = timed(per_block, r=max(1, reps // 2))
    tot = lambda t: sum(r["ms"] for r in t.values())
    res = {
        "workload": f"{nblocks} random geometric-graph Laplacians + 1e-2 I (n in [1024, 65536], "
                    f"kNN k in [6, 14]), float32, block-diagonal: n={n}, nnz={nnz}; IC(0) factor per "
                    f"block (nnz={nnzL}, {nl} levels at most); SpMM with k={k}",
        "tuned": tuned,
        "untuned": untuned,
        "whole_matrix_kernels": whole,
        "batched_ms": round(tot(tuned), 4),
        "batched_GB/s": round(sum(model.values()) / (tot(tuned) * 1e-3) / 1e9, 1),
        "untuned_ms": round(tot(untuned), 4),
        "whole_matrix_ms": round(tot(whole), 4),
        "per_block_ms": round(per_ms, 4),
        "speedup_vs_per_block": round(per_ms / tot(tuned), 2),
        # launches: one per SpMV/SpMM op (two for a split backward through
        # the queue); the solves 3 (per-block: forward, adjoint, value
        # gradients) or 2 (cooperative), or one per wide level (grid: None)
        "launches_per_step": None if LB.tri_mode == "grid" else (
            4 + sum(int(v["split"]) for op, v in B.bwd_times.items()
                    if B.impl[op + "_bwd"] == "queue") + (3 if LB.tri_mode == "blocks" else 2)),
        "op_impl": {op: {k2: (round(v2, 4) if isinstance(v2, float) else v2)
                         for k2, v2 in v.items()} for op, v in B.impl_times.items()},
        "trisolve_modes_ms": {m: round(v, 4) for m, v in tri_modes.items()},
        "trisolve_mode": LB.tri_mode,
        "backward_split": {op: {k2: (round(v2, 4) if isinstance(v2, float) else v2)
                                for k2, v2 in v.items()} for op, v in B.bwd_times.items()},
        "variants": {fam: {f"{c[0]}/{'uneven' if c[1] else 'even'}": v[0] for c, v in per_cls.items()}
                     for fam, per_cls in tune.items()},
        "tune_s": round(tune_s, 1),
        "generation_s": round(gen_s, 1),
        "setup_s": round(setup_s, 1),
    }
    log(f"batched: tuned {res['batched_ms']} ms ({res['batched_GB/s']} GB/s), untuned "
        f"{res['untuned_ms']} ms, whole-matrix kernels {res['whole_matrix_ms']} ms, "
        f"block by block {res['per_block_ms']} ms")
    del per, B, LB, L, X, G
    torch.cuda.empty_cache()
    if skew:
        res["uneven_rows"] = skew_section(skew, reps)
    return res


def skew_section(blocks, reps):
    """SpMV and SpMM (64 columns) forward and backward over blocks with
    heavy-tailed row lengths, with every block row-split, every block
    merge-path, the plain per-matrix kernels over the concatenation, and the
    autotuner's choice."""
    import torch
    from paper_2212_05159_amd import batch as bt

    B = bt.Batch(blocks)
    n, nnz, k = B.host.nrows, B.host.nnz, 64
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    x = torch.randn(n, generator=g, device="cuda")
    X = torch.randn(n, k, generator=g, device="cuda")
    B.pattern.transpose()
    V, I = 4, I4
    pat = lambda rows, z: (rows + 1) * I + z * I
    model = {"spmv fwd": pat(n, nnz) + nnz * V + 2 * n * V,
             "spmv bwd": pat(n, nnz) + nnz * (I + 2 * V) + 3 * n * V,
             "spmm fwd": pat(n, nnz) + nnz * V + 2 * n * k * V,
             "spmm bwd": pat(n, nnz) + nnz * (I + 2 * V) + 3 * n * k * V}
    ops = {"spmv fwd": lambda: B.spmv(x), "spmv bwd": lambda: B.spmv_bwd(x, x),
           "spmm fwd": lambda: B.spmm(X), "spmm bwd": lambda: B.spmm_bwd(X, X)}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def run(label):
        out = {}
        for name, fn in ops.items():
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            ms = float(np.median(ts))
            out[name] = {"ms": round(ms, 4), "GB/s": round(model[name] / (ms * 1e-3) / 1e9, 1)}
        return out

    res = {"workload": f"{len(blocks)} blocks with heavy-tailed row lengths (len = floor(u^(-1/1.1)), "
                       f"at most n/2), n in [1024, 65536]: n={n}, nnz={nnz}, longest row "
                       f"{int(B.block_maxrow.max())}; float32, k={k}"}
    for label, var in (("row_split", bt.rows_variant(8)), ("merge_path", bt.MERGE)):
        for fam in ("spmv", "spmv_t", "spmm", "spmm_t"):
            v = var if fam.startswith("spmv") else (bt.rows_variant(16) if var != bt.MERGE else var)
            B.set_variants(fam, np.full(B.nblocks, v, np.int32))
        res[label] = run(label)
    # the library's per-matrix kernels over the whole concatenation
    B.impl = {op: "plain" for op in B.impl}
    res["plain"] = run("plain")
    B.autotune(k=k, reps=3)
    res["tuned"] = run("tuned")
    res["op_impl"] = {op: v["impl"] for op, v in B.impl_times.items()}
    log("uneven rows: " + ", ".join(f"{lab} spmm fwd {res[lab]['spmm fwd']['ms']} ms"
                                     for lab in ("row_split", "merge_path", "plain", "tuned"))
        + f"; kept {res['op_impl']}")
    return res


def skew_blocks(nblocks):
    """Blocks with heavy-tailed row lengths: per block b, default_rng([6, b])
    draws n ~ U{1024..65536}; gen.power_law_rows(n, [6, b, 1], alpha 1.1,
    at most n/2 entries per row)."""
    from paper_2212_05159_amd import gen

    out = []
    for b in range(nblocks):
        n = int(np.random.default_rng([6, b]).integers(1024, 65537))
        out.append(gen.power_law_rows(n, [6, b, 1], alpha=1.1, max_len=n // 2))
    return out


# ----------------------------------------------------------------------
# Differentiated CG: K steps forward, hand-written reverse, sqrt(K) checkpoints
# ----------------------------------------------------------------------
def cg_section(N=512, K=100, reps=5, graph=False):
    """x_K of K CG steps on 2D anisotropic Q1 diffusion (eps 1e-3, angle
    pi/4, N^2 unknowns, float32 values, float64 dots), loss 0.5 ||x_K - t||^2
    backpropagated to the matrix values and b with checkpoints every
    ceil(sqrt(K)) steps.  Steps are launched eagerly (one library call per
    step launches its three kernels, faster than the GPU runs them); a
    captured graph would add its capture to every solve."""
    import torch
    from paper_2212_05159_amd import cg as cgmod, gen
    from paper_2212_05159_amd import sparse as sp

    A = gen.anisotropic_q1(N, 1e-3, np.pi / 4)
    rng = np.random.default_rng(4)
    Ad = sp.CsrTensor.from_host(A, dtype=torch.float32)
    b = torch.as_tensor(rng.standard_normal(A.nrows), dtype=torch.float32, device="cuda")
    t = torch.as_tensor(rng.standard_normal(A.nrows), dtype=torch.float32, device="cuda")
    vals = Ad.vals.detach().clone().requires_grad_(True)
    bb = b.clone().requires_grad_(True)
    Av = sp.CsrTensor(Ad.pattern, vals)
    Ad.pattern.transpose()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))

    def run():
        vals.grad = None
        bb.grad = None
        x = cgmod.cg_solve(Av, bb, K, graph=graph)
        e1.record()
        (0.5 * (x - t).pow(2).sum()).backward()
        return x

    run()
    torch.cuda.synchronize()
    fwd, tot = [], []
    for _ in range(reps):
        e0.record()
        run()
        e2.record()
        torch.cuda.synchronize()
        fwd.append(e0.elapsed_time(e1))
        tot.append(e0.elapsed_time(e2))
    n, nnz = A.nrows, A.nnz
    V, I = 4, I4
    # per step: product with p.q (pattern, values, p gathered, q), update of
    # x and r, r.r, p = r + beta p (vectors read or written once each)
    fwd_step = (n + 1) * I + nnz * (I + V) + 2 * n * V + 6 * n * V + n * V + 3 * n * V
    f_ms, t_ms = float(np.median(fwd)), float(np.median(tot))
    return {
        "workload": f"2D anisotropic Q1 diffusion {N}^2 (n={n}, nnz={nnz}), eps 1e-3, angle pi/4, "
                    f"float32 values, float64 dots; {K} CG steps, loss 0.5||x_K - t||^2, gradients "
                    f"to the values and b, checkpoints every {int(np.ceil(np.sqrt(K)))} steps",
        "K": K,
        "forward_ms": round(f_ms, 4),
        "forward_backward_ms": round(t_ms, 4),
        "forward_us_per_step": round(1e3 * f_ms / K, 2),
        "backward_us_per_step": round(1e3 * (t_ms - f_ms) / K, 2),
        "forward_GB/s": round(fwd_step * K / (f_ms * 1e-3) / 1e9, 1),
    }


def spadd_section(A, reps=10):
    """Sparse + sparse on the Poisson operator: C = A - 0.5 B with B a
    uniform random pattern of 7 draws per row (N(0,1) values), float32.
    Times the union pattern (symbolic, which ends in a host sync), the
    numeric pass with and without writing C's columns, and the VJP to
    both value arrays, each with HIP events on the stream."""
    import torch
    from paper_2212_05159_amd import capi, gen
    from paper_2212_05159_amd import sparse as sp

    B = gen.random_rows(A.nrows, A.ncols, 7, seed=2)
    Ad = sp.CsrTensor.from_host(A, dtype=torch.float32)
    Bd = sp.CsrTensor.from_host(B, dtype=torch.float32)
    dA, dB = Ad.pattern.desc(Ad.vals), Bd.pattern.desc(Bd.vals)
    m, na, nb = A.nrows, A.nnz, B.nnz
    ws = capi._ws(capi.csr_spadd_workspace(dA, dB), Ad.vals.device)
    rpC = torch.empty(m + 1, dtype=torch.int32, device="cuda")
    nc = capi.csr_spadd_symbolic(dA, dB, rpC, ws)
    ciC = torch.empty(nc, dtype=torch.int32, device="cuda")
    vC = torch.empty(nc, dtype=torch.float32, device="cuda")
    Cp = sp.Pattern(m, A.ncols, rpC, ciC)
    dC = Cp.desc()
    gC = torch.randn(nc, dtype=torch.float32, device="cuda")
    gA = torch.empty(na, dtype=torch.float32, device="cuda")
    gB = torch.empty(nb, dtype=torch.float32, device="cuda")
    ops = {
        "symbolic": lambda: capi.csr_spadd_symbolic(dA, dB, rpC, ws),
        "fwd": lambda: capi.csr_spadd_fwd(dA, dB, 1.0, -0.5, rpC, ciC, vC),
        "fwd_values_only": lambda: capi.csr_spadd_fwd(dA, dB, 1.0, -0.5, rpC, None, vC),
        "bwd": lambda: capi.csr_spadd_bwd(dA, dB, dC, 1.0, -0.5, gC, gA, gB),
    }
    rp3 = 3 * 4 * (m + 1)
    algo = {  # bytes each pass must move at least once
        "symbolic": rp3 + 4 * (na + nb),
        "fwd": rp3 + 8 * (na + nb) + 8 * nc,
        "fwd_values_only": rp3 + 8 * (na + nb) + 4 * nc,
        "bwd": rp3 + 8 * (na + nb) + 4 * nc,  # A's and B's columns, V, gA and gB
    }
    res = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for name, fn in ops.items():
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        gbs = algo[name] / (ms * 1e-3) / 1e9
        res[name] = {"ms": round(ms, 4), "GB": round(algo[name] / 1e9, 4), "GB/s": round(gbs, 1),
                     "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
    res["workload"] = (f"C = A - 0.5 B, A the 3D 7-point Poisson operator (n={m}, nnz={na}), B a "
                       f"uniform random pattern of 7 draws per row (nnz={nb}), float32; "
                       f"nnz(C)={nc}")
    return res


def spai_section(grids=(256, 1024)):
    """Sparse approximate inverse by direct minimisation on the 2D 5-point
    Poisson matrix (float32): from M = mask(A), steepest descent with exact
    steps until ||grad|| < 0.01, timed whole (HIP events around the solve,
    one host read of the gradient norm per iteration) after one untimed
    solve; 256^2 is the largest size of the paper's timing study."""
    import torch
    from paper_2212_05159_amd import gen
    from paper_2212_05159_amd import sparse as sp
    from paper_2212_05159_amd.spai import Spai

    out = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for N in grids:
        A = gen.poisson2d(N, N)
        prob = Spai(sp.CsrTensor.from_host(A, dtype=torch.float32))
        prob.solve(tol=0.01, max_iter=200)
        torch.cuda.synchronize()
        e0.record()
        _, info = prob.solve(tol=0.01, max_iter=200)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out[f"{N}^2"] = {"n": A.nrows, "nnz": A.nnz, "iterations": info["iters"],
                         "converged": info["converged"], "loss_start": info["history"][0],
                         "loss": round(info["loss"], 4), "solve_ms": round(ms, 3),
                         "ms_per_iteration": round(ms / max(info["iters"], 1), 4)}
    out["workload"] = ("||I - M A||_F^2 over mask(M) = mask(A), 2D 5-point Poisson, float32, "
                       "from M = mask(A) to ||grad|| < 0.01")
    return out


def gcn_section(sizes=(2708, 19717, 89250, 343565, 914231), C=128, epochs=20):
    """Training epochs of the two-layer GCN (hidden 16, 6 classes, dropout
    0.5, Adam with L2 5e-4) on synthetic random geometric graphs (k = 4
    nearest neighbours, union-symmetrised: about 5 incident edges per node)
    with the node counts of the paper's GCN timings; C input features
    (noisy one-hot of a spatial class), 20 labelled nodes per class.  One
    epoch is the forward pass, the backward pass and the optimiser step;
    HIP events around `epochs` epochs after 3 untimed ones."""
    import torch
    from paper_2212_05159_amd import gcn, gen
    from paper_2212_05159_amd import sparse as sp

    out = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for n in sizes:
        A = gen.geometric_graph(n, 4, seed=[11, n])
        y = gen.node_classes(A.points, 6, seed=[12, n])
        rng = np.random.default_rng([13, n])
        X = torch.as_tensor(0.6 * np.eye(C, dtype=np.float32)[y] +
                            rng.standard_normal((n, C), dtype=np.float32), device="cuda")
        mask = np.zeros(n, bool)
        for c in range(6):
            idx = np.flatnonzero(y == c)
            mask[rng.choice(idx, min(20, len(idx)), replace=False)] = True
        G = sp.CsrTensor.from_host(A)
        G.pattern.transpose()  # the SpMM backward's transpose, built once per graph
        labels = torch.as_tensor(y, device="cuda")
        tm = torch.as_tensor(mask, device="cuda")
        model = gcn.GCN(C, 16, 6, seed=0)
        gcn.train(model, G, X, labels, tm, epochs=3)
        torch.cuda.synchronize()
        e0.record()
        hist = gcn.train(model, G, X, labels, tm, epochs=epochs)
        e1.record()
        torch.cuda.synchronize()
        out[str(n)] = {"nnz": A.nnz, "edges_per_node": round(A.nnz / n, 2),
                       "ms_per_epoch": round(e0.elapsed_time(e1) / epochs, 4),
                       "loss": round(hist[-1], 4)}
    out["workload"] = (f"two-layer GCN (C={C} -> 16 -> 6), random geometric graphs (kNN k=4, "
                       f"union-symmetrised), float32; ms per training epoch (forward, backward, "
                       f"Adam step) over {epochs} epochs")
    return out


# ----------------------------------------------------------------------
# Measured HBM traffic of the dominant kernel (committed counter summary)
# ----------------------------------------------------------------------
COUNTERS = os.path.join(ROOT, "profiles", "spmm_poisson128_counters.md")
SPMM_SRC = os.path.join(ROOT, "paper_2212_05159_amd", "csrc", "spmm.hip")


def measured_traffic(kernel, plan):
    """Bytes per launch of `kernel` under traversal `plan` from the counter
    summary, or None when the summary is missing, lists no such plan, or
    was taken on a different version of the kernel source."""
    import hashlib

    try:
        text = open(COUNTERS).read().splitlines()
        src = hashlib.sha256(open(SPMM_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    if f"spmm_source_sha256: {src}" not in text:
        return None
    key = f"traffic {kernel} {'natural' if plan is None else '(%d, %d)' % tuple(plan)}:"
    for line in text:
        if line.startswith(key):
            return int(float(line.split(":")[1]))
    return None


# ----------------------------------------------------------------------
# PCG time to 1e-6: learned preconditioner vs Jacobi
# ----------------------------------------------------------------------
def pcg_section(n_eval, n_train, train_steps, systems):
    import torch
    from paper_2212_05159_amd import learned
    from paper_2212_05159_amd import pcg as pcgmod
    from paper_2212_05159_amd import sparse as sp

    t0 = time.perf_counter()
    model = learned.MPNN(seed=1)
    untrained = learned.MPNN(seed=1)
    val = learned.held_out(learned.Q1Family(n_train), 4, 52)
    every = max(50, train_steps // 16)
    hist = learned.train(model, N=n_train, steps=train_steps, lr=3e-3, nit=16, seed=5,
                         val_systems=val, eval_every=every)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log(f"trained the network: {train_steps} systems of {n_train}^2 in {train_s:.1f} s "
        f"(loss {np.mean(hist[:20]):.4f} -> {np.mean(hist[-20:]):.4f}; selected parameters: "
        f"{model.selected_score:.1f} mean validation iterations)")
    # the approximate-inverse form of the same network (M = L L^T ~ A^{-1})
    t0 = time.perf_counter()
    model_inv = learned.MPNN(seed=1, form="fsai")
    hist_inv = learned.train(model_inv, N=n_train, steps=train_steps, lr=3e-3, nit=16, seed=5,
                             val_systems=val, eval_every=every)
    torch.cuda.synchronize()
    train_inv_s = time.perf_counter() - t0
    log(f"trained the inverse-form network in {train_inv_s:.1f} s (loss "
        f"{np.mean(hist_inv[:20]):.4f} -> {np.mean(hist_inv[-20:]):.4f}; selected parameters: "
        f"{model_inv.selected_score:.1f} mean validation iterations)")
    fam = learned.Q1Family(n_eval)
    t0 = time.perf_counter()
    nl = fam.Lpat.levels(True)[0]
    fam.Lpat.transpose()
    torch.cuda.synchronize()
    analysis_ms = (time.perf_counter() - t0) * 1e3
    untrained_inv = learned.MPNN(seed=1, form="fsai")
    # "learned": the paper's form (Section 4.3: M = L L^T approximates A^-1,
    # applied by two sparse products); "factor_*": the factor reading (M
    # approximates A, two level-scheduled triangular solves)
    methods = ("learned", "untrained", "factor_learned", "factor_untrained", "jacobi", "cg")
    maxit = 40000

    def solve(key, A, b, cap=maxit):
        if key in ("factor_learned", "factor_untrained"):
            net = model if key == "factor_learned" else untrained
            with torch.no_grad():
                L = sp.CsrTensor(fam.Lpat, net(A, fam.Lpat))
            # the factor step (a dozen launches) runs faster from the stream
            # than replayed from a captured graph; the short Jacobi and plain
            # steps run faster from the graph: each method runs its faster way
            return pcgmod.pcg(A, b, "factor", L=L, tol=1e-6, maxit=cap, chunk=50, graph=False)
        if key in ("learned", "untrained"):
            net = model_inv if key == "learned" else untrained_inv
            with torch.no_grad():
                L = sp.CsrTensor(fam.Lpat, net(A, fam.Lpat))
            return pcgmod.pcg(A, b, "fsai", L=L, tol=1e-6, maxit=cap, chunk=50, graph=False)
        return pcgmod.pcg(A, b, "jacobi" if key == "jacobi" else "none", tol=1e-6, maxit=cap,
                          chunk=50, graph=True)

    times = {k: [] for k in methods}
    iters = {k: [] for k in methods}
    fallbacks = 0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for j in range(systems):
        rng = np.random.default_rng([5, 1, j])
        eps, theta = learned.Q1Family.sample(rng)
        A, _ = fam.system(eps, theta)
        b = torch.as_tensor(rng.standard_normal(fam.P.nrows), device="cuda")
        if j == 0:
            for key in methods:  # warm-up: allocator, graph capture paths
                solve(key, A, b, cap=100)
        for key in methods:
            torch.cuda.synchronize()
            e0.record()
            x, info = solve(key, A, b)
            e1.record()
            torch.cuda.synchronize()
            if not info["converged"]:
                raise RuntimeError(f"{key} PCG did not reach 1e-6 on system {j}: {info}")
            fallbacks += int(info.get("fallback", False))
            times[key].append(e0.elapsed_time(e1))
            iters[key].append(info["iters"])
        if j < 4 or j + 1 == systems or (j + 1) % 16 == 0:
            log(f"pcg system {j}: eps {eps:.2e} theta {theta:.2f} " +
                " ".join(f"{k} {times[k][-1]:.1f} ms/{iters[k][-1]} it" for k in methods))
    med = {k: round(float(np.median(v)), 3) for k, v in times.items()}
    return {
        "workload": f"2D anisotropic Q1 diffusion {n_eval}^2 (n={fam.P.nrows}, nnz={fam.P.nnz}), "
                    f"2x2 four-coloured order, float32 values, float64 vectors; L on tril(A) "
                    f"(nnz={fam.Lpat.nnz}, {nl} levels)",
        "systems": systems, "tol": 1e-6,
        "median_ms": med,
        "median_iterations": {k: float(np.median(v)) for k, v in iters.items()},
        "methods": {"factor_learned": "trained network, factor form (M = L L^T ~ A, two level-scheduled "
                               "triangular solves)",
                    "factor_untrained": "the same network untrained: symmetric Gauss-Seidel factor",
                    "learned": "trained network, the inverse form of Section 4.3 (M = L L^T ~ A^-1, "
                            "two sparse products)",
                    "untrained": "the inverse-form network untrained: first-order inverse "
                                      "factor D^-1 (D - A_L) D^-1/2",
                    "jacobi": "Jacobi-PCG", "cg": "plain CG"},
        "learned_speedup_vs_jacobi": round(med["jacobi"] / med["learned"], 3),
        "learned_speedup_vs_untrained": round(med["untrained"] / med["learned"], 3),
        "training_gain_iterations": round(float(np.median(iters["untrained"])) /
                                          float(np.median(iters["learned"])), 3),
        "factor_learned_speedup_vs_jacobi": round(med["jacobi"] / med["factor_learned"], 3),
        "factor_training_gain_iterations": round(float(np.median(iters["factor_untrained"])) /
                                                 float(np.median(iters["factor_learned"])), 3),
        "fallbacks": fallbacks,
        "level_analysis_ms": round(analysis_ms, 3),
        "train": {"systems": train_steps, "grid": n_train, "lr": 3e-3, "pcg_steps_in_loss": 16,
                  "selection": "best mean PCG iterations on 4 held-out systems of the training grid",
                  "seconds": round(train_inv_s, 2),
                  "validation_iterations": model_inv.selected_score,
                  "factor_seconds": round(train_s, 2),
                  "factor_validation_iterations": model.selected_score},
    }


# ----------------------------------------------------------------------
# Inputs
# ----------------------------------------------------------------------
def make_inputs(N: int, k: int):
    from paper_2212_05159_amd import gen

    t0 = time.time()
    A = gen.poisson3d(N)
    n = A.nrows
    P = gen.aggregation(n, 8)
    L = gen.tril(gen.permute_sym(A, gen.red_black_3d(N)))
    rng = np.random.default_rng(2)
    B = rng.standard_normal((n, k), dtype=np.float32)
    G = rng.standard_normal((n, k), dtype=np.float32)
    x = rng.standard_normal(n, dtype=np.float32)
    gy = rng.standard_normal(n, dtype=np.float32)
    bL = rng.standard_normal(n, dtype=np.float32)
    gL = rng.standard_normal(n, dtype=np.float32)
    nc = P.ncols
    nnz_c = nc + 2 * (N // 8 - 1) * N * N + 4 * (N // 8) * (N - 1) * N  # nnz(P^T A P)
    V = rng.standard_normal(nnz_c, dtype=np.float32)
    log(f"inputs: n={n} nnz(A)={A.nnz} nnz(L)={L.nnz} k={k} ({time.time() - t0:.1f}s)")
    return dict(A=A, P=P, L=L, B=B, G=G, x=x, gy=gy, bL=bL, gL=gL, V=V, N=N, k=k, n=n, nc=nc)


class Device:
    """The inputs resident in HBM."""

    def __init__(self, h):
        import torch

        def t(a, dt=None):
            return torch.as_tensor(np.ascontiguousarray(a)).cuda() if dt is None else \
                torch.as_tensor(np.ascontiguousarray(a)).to(dt).cuda()

        f32 = torch.float32
        self.n, self.nc, self.k = h["n"], h["nc"], h["k"]
        self.A_rp, self.A_ci, self.A_v = t(h["A"].rowptr), t(h["A"].colind), t(h["A"].vals, f32)
        self.P_rp, self.P_ci, self.P_v = t(h["P"].rowptr), t(h["P"].colind), t(h["P"].vals, f32)
        self.L_rp, self.L_ci, self.L_v = t(h["L"].rowptr), t(h["L"].colind), t(h["L"].vals, f32)
        for name in ("B", "G", "x", "gy", "bL", "gL", "V"):
            setattr(self, name, t(h[name]))
        self.nnzA, self.nnzL, self.nnzP = h["A"].nnz, h["L"].nnz, h["P"].nnz


# ----------------------------------------------------------------------
# Algorithmic bytes per op (each array the op must touch, once; I = 4 B
# index, V = 4 B value).
# ----------------------------------------------------------------------
def byte_model(d, nnz_ap, nnz_c, nlev):
    V = 4
    n, nc, k = d.n, d.nc, d.k
    nA, nP, nL = d.nnzA, d.nnzP, d.nnzL

    def pat(rows, nnz):
        return (rows + 1) * I4 + nnz * I4

    def transpose(rows, cols, nnz):
        return pat(rows, nnz) + pat(cols, nnz) + nnz * I4

    def spgemm_sym(m, A_nnz, Bm, B_nnz):
        return pat(m, A_nnz) + pat(Bm, B_nnz) + (m + 1) * I4

    def spgemm_num(m, A_nnz, Bm, B_nnz, C_nnz):
        return pat(m, A_nnz) + A_nnz * V + pat(Bm, B_nnz) + B_nnz * V + (m + 1) * I4 + C_nnz * (I4 + V)

    def spgemm_bwd(m, acols, A_nnz, Bm, B_nnz, C_nnz):
        ka = pat(m, A_nnz) + pat(Bm, B_nnz) + B_nnz * V + pat(m, C_nnz) + C_nnz * V + A_nnz * V
        kb = pat(Bm, B_nnz) + pat(acols, A_nnz) + A_nnz * (I4 + V) + pat(m, C_nnz) + C_nnz * V + B_nnz * V
        return ka + kb

    b = {}
    b["transpose A"] = transpose(n, n, nA)
    b["transpose P"] = transpose(n, nc, nP)
    b["transpose vals P"] = nP * (I4 + 2 * V)
    b["spmv fwd"] = pat(n, nA) + nA * V + 2 * n * V
    b["spmv bwd"] = pat(n, nA) + nA * 2 * V + 3 * n * V
    b["spmm fwd"] = pat(n, nA) + nA * V + 2 * n * k * V
    b["spmm bwd"] = pat(n, nA) + nA * 2 * V + 3 * n * k * V
    b["spgemm A.P"] = spgemm_sym(n, nA, n, nP) + spgemm_num(n, nA, n, nP, nnz_ap)
    b["spgemm Pt.AP"] = spgemm_sym(nc, nP, n, nnz_ap) + spgemm_num(nc, nP, n, nnz_ap, nnz_c)
    b["transpose Pt"] = transpose(nc, n, nP)
    b["spgemm bwd Pt.AP"] = spgemm_bwd(nc, n, nP, n, nnz_ap, nnz_c)
    b["spgemm bwd A.P"] = spgemm_bwd(n, n, nA, n, nP, nnz_ap)
    b["transpose L"] = transpose(n, n, nL)
    b["levels L"] = 2 * pat(n, nL) + 2 * n * I4 + (nlev + 1) * I4
    b["trisolve fwd"] = pat(n, nL) + nL * V + 2 * n * V + n * I4
    b["trisolve bwd"] = (pat(n, nL) + nL * (I4 + V) + 2 * n * V + n * I4) + \
        (pat(n, nL) + nL * I4 + 2 * n * V + nL * V)
    return b


# ----------------------------------------------------------------------
# One step
# ----------------------------------------------------------------------
class Marks:
    """HIP events recorded on the current stream between ops."""

    def __init__(self, enabled):
        import torch
        self.torch = torch
        self.enabled = enabled
        self.ev = []

    def mark(self, name):
        if self.enabled:
            e = self.torch.cuda.Event(enable_timing=True)
            e.record()
            self.ev.append((name, e))

    def durations(self):
        out = {}
        for (_, a), (name, b) in zip(self.ev[:-1], self.ev[1:]):
            out[name] = out.get(name, 0.0) + a.elapsed_time(b)
        return out


def _keep(outs, **kw):
    if outs is not None:
        outs.update(kw)


def run_step(d, marks, outs=None):
    """One step, every op in sequence on the current stream (per-op event
    marks give an exact attribution of the step time).  With outs (a dict),
    the step's outputs are stored in it."""
    from paper_2212_05159_amd import sparse as sp

    marks.mark("start")
    PA = sp.Pattern(d.n, d.n, d.A_rp, d.A_ci)
    PP = sp.Pattern(d.n, d.nc, d.P_rp, d.P_ci)
    PL = sp.Pattern(d.n, d.n, d.L_rp, d.L_ci)
    PA.transpose()
    marks.mark("transpose A")
    PPt, _ = PP.transpose()
    marks.mark("transpose P")
    vPt = sp.transpose_vals(PP, d.P_v)
    marks.mark("transpose vals P")
    y = sp.spmv(PA, d.A_v, d.x)
    marks.mark("spmv fwd")
    gx, gv = sp.spmv_bwd(PA, d.A_v, d.x, d.gy, mode=d.spmv_bwd_mode)
    marks.mark("spmv bwd")
    C = sp.spmm(PA, d.A_v, d.B, plan=d.plan_fwd)
    marks.mark("spmm fwd")
    gB, gvm = sp.spmm_bwd(PA, d.A_v, d.B, d.G, plan=d.plan_bwd)
    marks.mark("spmm bwd")
    PAP, vAP = sp.spgemm(PA, d.A_v, PP, d.P_v)
    marks.mark("spgemm A.P")
    PC, vC = sp.spgemm(PPt, vPt, PAP, vAP)
    marks.mark("spgemm Pt.AP")
    PPt.transpose()
    marks.mark("transpose Pt")
    gPt, gAP = sp.spgemm_bwd(PPt, vPt, PAP, vAP, PC, d.V)
    marks.mark("spgemm bwd Pt.AP")
    gA, gP = sp.spgemm_bwd(PA, d.A_v, PP, d.P_v, PAP, gAP)
    marks.mark("spgemm bwd A.P")
    PL.transpose()
    marks.mark("transpose L")
    nl = PL.levels(True)[0]
    marks.mark("levels L")
    xL = sp.trisolve(PL, d.L_v, d.bL, True)
    marks.mark("trisolve fwd")
    gbL, gvL = sp.trisolve_bwd(PL, d.L_v, xL, d.gL, True)
    marks.mark("trisolve bwd")
    _keep(outs, y=y, gx=gx, gv=gv, C=C, gB=gB, gvm=gvm, rpAP=PAP.rowptr, ciAP=PAP.colind, vAP=vAP,
          rpC=PC.rowptr, ciC=PC.colind, vC=vC, gPt=gPt, gAP=gAP, gA=gA, gP=gP, xL=xL, gbL=gbL, gvL=gvL)
    return PAP.nnz, PC.nnz, nl


def run_step_streams(d, chain_marks, outs=None):
    """The same step as three independent chains on their own HIP streams
    (default priority), joined at the end on the current stream:
      1. A's transpose, SpMV and SpMM forward and backward (HBM-bound);
      2. the Galerkin product P^T A P forward and backward (its symbolic
         passes synchronise their own stream);
      3. L's transpose, level sets and the triangular solves (the level
         analysis synchronises its own stream).
    Chains 2 and 3 are driven by two host threads (d.pool), so their
    synchronisations hold up neither each other nor chain 1; library calls
    release the interpreter lock while they wait.  The one cross-chain
    input, A's cached transpose (the SpGEMM VJP of A P needs it), is made
    before the threads start and handed over with an event.  chain_marks:
    three Marks, each recording on its chain's stream."""
    import torch
    from paper_2212_05159_amd import sparse as sp

    main = torch.cuda.current_stream()
    s1, s2, s3 = d.streams
    start = torch.cuda.Event()
    start.record(main)
    for st in d.streams:
        st.wait_event(start)
    m1, m2, m3 = chain_marks
    PA = sp.Pattern(d.n, d.n, d.A_rp, d.A_ci)
    PP = sp.Pattern(d.n, d.nc, d.P_rp, d.P_ci)
    PL = sp.Pattern(d.n, d.n, d.L_rp, d.L_ci)
    with torch.cuda.stream(s1):
        m1.mark("start")
        PA.transpose()
        m1.mark("transpose A")
        tA = torch.cuda.Event()
        tA.record(s1)

    def chain2():
        with torch.cuda.stream(s2):
            m2.mark("start")
            PPt, _ = PP.transpose()
            m2.mark("transpose P")
            vPt = sp.transpose_vals(PP, d.P_v)
            m2.mark("transpose vals P")
            PAP, vAP = sp.spgemm(PA, d.A_v, PP, d.P_v)
            m2.mark("spgemm A.P")
            PC, vC = sp.spgemm(PPt, vPt, PAP, vAP)
            m2.mark("spgemm Pt.AP")
            PPt.transpose()
            m2.mark("transpose Pt")
            gPt, gAP = sp.spgemm_bwd(PPt, vPt, PAP, vAP, PC, d.V)
            m2.mark("spgemm bwd Pt.AP")
            s2.wait_event(tA)
            gA, gP = sp.spgemm_bwd(PA, d.A_v, PP, d.P_v, PAP, gAP)
            m2.mark("spgemm bwd A.P")
            _keep(outs, rpAP=PAP.rowptr, ciAP=PAP.colind, vAP=vAP, rpC=PC.rowptr, ciC=PC.colind,
                  vC=vC,
                  gPt=gPt, gAP=gAP, gA=gA, gP=gP)
            return PAP.nnz, PC.nnz

    def chain3():
        with torch.cuda.stream(s3):
            m3.mark("start")
            PL.transpose()
            m3.mark("transpose L")
            nl = PL.levels(True)[0]
            m3.mark("levels L")
            xL = sp.trisolve(PL, d.L_v, d.bL, True)
            m3.mark("trisolve fwd")
            gbL, gvL = sp.trisolve_bwd(PL, d.L_v, xL, d.gL, True)
            m3.mark("trisolve bwd")
            _keep(outs, xL=xL, gbL=gbL, gvL=gvL)
            return nl

    f2 = d.pool.submit(chain2)
    f3 = d.pool.submit(chain3)
    with torch.cuda.stream(s1):
        y = sp.spmv(PA, d.A_v, d.x)
        m1.mark("spmv fwd")
        gx, gv = sp.spmv_bwd(PA, d.A_v, d.x, d.gy, mode=d.spmv_bwd_mode)
        m1.mark("spmv bwd")
        C = sp.spmm(PA, d.A_v, d.B, plan=d.plan_fwd)
        m1.mark("spmm fwd")
        gB, gvm = sp.spmm_bwd(PA, d.A_v, d.B, d.G, plan=d.plan_bwd)
        m1.mark("spmm bwd")
        _keep(outs, y=y, gx=gx, gv=gv, C=C, gB=gB, gvm=gvm)
    nnz_ap, nnz_c = f2.result()
    nl = f3.result()
    for st in d.streams:
        done = torch.cuda.Event()
        done.record(st)
        main.wait_event(done)
    return nnz_ap, nnz_c, nl


# ----------------------------------------------------------------------
# Oracle on the host (CPU baseline)
# ----------------------------------------------------------------------
def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(h, bytes_total, seconds=10.0):
    """The float64 oracle timed on the host over whole steps of the same
    workload: its OpenMP build on all host cores (the reported value; row-
    parallel loops only, the A^T products and SpGEMM stay serial) and its
    single-threaded build (the paper's CPU setting), about `seconds` of work
    each, at least one step; median step time of each leg."""
    import oracle
    from paper_2212_05159_amd import gen

    oracle.build()
    A, P, L = h["A"], h["P"], h["L"]
    f = lambda a: np.asarray(a, np.float64)
    Af = gen.Csr(A.nrows, A.ncols, A.rowptr, A.colind, f(A.vals))
    B, G = f(h["B"]), f(h["G"])

    def one_step():
        oracle.transpose(Af)
        rpT, ciT, perm = oracle.transpose(P)
        Pt = gen.Csr(P.ncols, P.nrows, rpT, ciT, P.vals[perm])
        oracle.spmv(Af, f(h["x"]))
        oracle.spmv_bwd(Af, f(h["x"]), f(h["gy"]))
        oracle.spmm(Af, B)
        oracle.spmm_bwd(Af, B, G)
        rpAP, ciAP, vAP = oracle.spgemm(Af, P)
        AP = gen.Csr(A.nrows, P.ncols, rpAP, ciAP, vAP)
        rpC, ciC, _ = oracle.spgemm(Pt, AP)
        oracle.transpose(Pt)
        _, gAP = oracle.spgemm_bwd(Pt, AP, rpC, ciC, f(h["V"]))
        oracle.spgemm_bwd(Af, P, rpAP, ciAP, gAP)
        oracle.transpose(L)
        oracle.levels(L, True)
        xL = oracle.trisolve(L, f(h["bL"]), True)
        oracle.trisolve_bwd(L, xL, f(h["gL"]), True)

    def leg(threads):
        oracle.use_threads(threads)
        try:
            nth = oracle.threads()
            ts = []
            t0 = time.perf_counter()
            while not ts or time.perf_counter() - t0 < seconds:
                t1 = time.perf_counter()
                one_step()
                ts.append(time.perf_counter() - t1)
        finally:
            oracle.use_threads(False)
        dt = float(np.median(ts))
        return {"value": round(bytes_total / dt / 1e9, 3), "unit": "GB/s", "cores": nth,
                "seconds": round(dt, 3), "steps": len(ts)}

    allc = leg(True)
    one = leg(False)
    return {**allc, "kind": "oracle", "cpu": _cpu_model(), "host_cpus": os.cpu_count(),
            "single_thread": one,
            "sample": f"whole steps of the same workload (every op of the step), median step time; "
                      f"{allc['steps']} steps on {allc['cores']} threads (OpenMP build: loops over "
                      f"independent rows split among threads, A^T products, transposes, SpGEMM and "
                      f"solves serial) and {one['steps']} on one thread (the paper's CPU setting), "
                      f"float64"}


def calibrate(millions):
    """valsT[t] = vals[perm[t]] with perm = identity: reads 8 bytes and
    writes 4 bytes per value, once each."""
    import torch
    from paper_2212_05159_amd import capi

    n = millions * 1000 * 1000
    perm = torch.arange(n, dtype=torch.int32, device="cuda")
    vals = torch.ones(n, dtype=torch.float32, device="cuda")
    out = torch.empty_like(vals)
    rp = torch.zeros(2, dtype=torch.int32, device="cuda")
    d = capi.csrad_csr(1, n, n, capi.F32, rp.data_ptr(), perm.data_ptr(), vals.data_ptr())
    for _ in range(3):
        capi.csr_transpose_vals(d, perm, out)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "k_gather_vals", "values": n, "read_bytes": 8 * n,
                      "write_bytes": 4 * n}), flush=True)


# ----------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--k", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pcg", action="store_true", help="skip the PCG time-to-1e-6 part")
    ap.add_argument("--pcg-grid", type=int, default=1024)
    ap.add_argument("--pcg-systems", type=int, default=64)
    ap.add_argument("--train-grid", type=int, default=256)
    ap.add_argument("--train-steps", type=int, default=4096,
                    help="training systems (one Adam step each) per network")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-blocks part")
    ap.add_argument("--no-cg", action="store_true", help="skip the differentiated-CG part")
    ap.add_argument("--no-spadd", action="store_true", help="skip the sparse + sparse part")
    ap.add_argument("--no-spai", action="store_true", help="skip the sparse-approximate-inverse part")
    ap.add_argument("--no-gcn", action="store_true", help="skip the graph-convolution part")
    ap.add_argument("--serial", action="store_true",
                    help="run the step's ops in sequence on one stream (exact per-op attribution) "
                         "instead of three concurrent chains")
    ap.add_argument("--batched-blocks", type=int, default=512,
                    help="number of the 512 geometric-graph blocks in the batched part")
    ap.add_argument("--skew-blocks", type=int, default=64,
                    help="blocks with heavy-tailed row lengths in the batched part (0: none)")
    ap.add_argument("--calibrate", type=int, default=0, metavar="M",
                    help="only run a copy-like kernel over M million float32 values "
                         "(identity-permutation gather: 12 bytes per value) to calibrate "
                         "hardware byte counters, then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    host_blocks = None
    if not args.no_batched and not args.calibrate:
        # host inputs of the batched part first (a thread pool; the host
        # work overlaps nothing on the GPU)
        host_blocks = geometric_blocks(args.batched_blocks)
        log(f"built {args.batched_blocks} geometric-graph blocks in {host_blocks[1]:.1f} s")
        skew = skew_blocks(args.skew_blocks) if args.skew_blocks else None

    import torch
    from paper_2212_05159_amd import capi

    capi.load()
    if args.calibrate:
        calibrate(args.calibrate)
        return
    h = make_inputs(args.grid, args.k)
    d = Device(h)
    torch.cuda.synchronize()

    # Setup (outside the timed region): the autotuner picks traversal plans
    # for the SpMM kernels on this pattern.
    from paper_2212_05159_amd import autotune
    from paper_2212_05159_amd import sparse as sp
    P0 = sp.Pattern(d.n, d.n, d.A_rp, d.A_ci)
    tuned = autotune.tune_spmm(P0, d.A_v, d.B, d.G, reps=3, use_cache=False)
    d.plan_fwd, d.plan_bwd = P0.plan("spmm_fwd"), P0.plan("spmm_bwd")
    d.spmv_bwd_mode = autotune.tune_spmv_bwd(P0, d.A_v, d.x, d.gy, reps=3, use_cache=False)[0]
    log(f"autotuned plans: {tuned}, SpMV backward: {d.spmv_bwd_mode}")

    d.streams = tuple(torch.cuda.Stream() for _ in range(3))
    d.pool = cf.ThreadPoolExecutor(2)  # host threads of the step's chains 2 and 3

    def step(enabled):
        if args.serial:
            mk = [Marks(enabled)]
            return run_step(d, mk[0]), mk
        mk = [Marks(enabled) for _ in range(3)]
        return run_step_streams(d, mk), mk

    for i in range(args.warmup):
        step(False)
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    # Timed region: exactly `steps` steps (three concurrent chains unless
    # --serial), bracketed by synchronisations.  Python's cyclic garbage
    # collector is paused over the timed and attribution passes (collected
    # just before), as timeit does: a collection pass is host-side noise of
    # tens of milliseconds that would otherwise land inside one step.
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    t_start.record()
    w0 = time.perf_counter()
    for i in range(args.steps):
        (nnz_ap, nnz_c, nlev), _ = step(False)
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    log(f"{args.steps} steps: {ms_step:.3f} ms/step (wall {wall / args.steps * 1e3:.3f} ms/step)")

    # Attribution pass: the same number of steps with every op in sequence
    # on one stream and HIP events between ops (events on overlapping
    # streams would time the interleaving, not the kernels).  The per-op
    # breakdown and the dominant kernel's roofline come from this pass.
    marks_all = []
    a_start = torch.cuda.Event(enable_timing=True)
    a_end = torch.cuda.Event(enable_timing=True)
    # one untimed step first: the pass runs on another stream than the timed
    # chains, and its first step grows the allocator's pool for that stream
    run_step(d, Marks(False))
    torch.cuda.synchronize()
    a_start.record()
    last_outs = {}
    for i in range(args.steps):
        mk = Marks(True)
        run_step(d, mk, last_outs if i + 1 == args.steps else None)
        marks_all.append(mk)
    a_end.record()
    torch.cuda.synchronize()
    serial_ms = a_start.elapsed_time(a_end) / args.steps
    gc.enable()
    log(f"attribution pass (one stream): {serial_ms:.3f} ms/step")

    # intermediate products of the two SpGEMMs, from the last attribution
    # step's A P: sum over A's entries of the length of the P row each
    # selects, and sum over k of len(P row k) * len(AP row k) for P^T (A P)
    with torch.no_grad():
        lenP = (d.P_rp[1:] - d.P_rp[:-1]).long()
        lenAP = (last_outs["rpAP"][1:] - last_outs["rpAP"][:-1]).long()
        products = {"A.P": int(lenP[d.A_ci.long()].sum()), "Pt.AP": int((lenP * lenAP).sum())}
    bm = byte_model(d, nnz_ap, nnz_c, nlev)
    total_bytes = sum(bm.values())
    # per op the median over the attribution steps (a one-off host stall in
    # one step, e.g. an allocation, would otherwise spread over the mean)
    per_op = {}
    for mk in marks_all:
        for kname, v in mk.durations().items():
            per_op.setdefault(kname, []).append(v)
    op_ms = {kname: float(np.median(v)) for kname, v in per_op.items()}
    breakdown = {kname: {"ms": round(op_ms[kname], 4), "GB": round(bm[kname] / 1e9, 4),
                         "GB/s": round(bm[kname] / (op_ms[kname] * 1e-3) / 1e9, 1)}
                 for kname in bm}
    value = total_bytes / (ms_step * 1e-3) / 1e9

    # Roofline of the dominant kernel: k_spmm_bwd_coop alone, 20 warm-up
    # launches, then the median of 60 launches timed with HIP events on the
    # stream it runs on, against its
    # minimum algorithmic bytes ((m+1)I + nnz(I+2V) + 3nkV: pattern, values
    # read and value gradients written once, G read, B read, gB written).
    from paper_2212_05159_amd import sparse as sp
    dom = "spmm bwd"
    PA = sp.Pattern(d.n, d.n, d.A_rp, d.A_ci)
    gB_buf, gv_buf = torch.empty_like(d.G), torch.empty_like(d.A_v)
    PAt, permA = PA.transpose()
    from paper_2212_05159_amd import capi as _capi
    dA, dAt = PA.desc(d.A_v), PAt.desc(dtype=d.A_v.dtype)

    def dom_launch():
        _capi.csr_spmm_bwd(dA, dAt, permA, d.k, d.B, d.k, d.G, d.k, gB_buf, d.k, gv_buf,
                           d.plan_bwd)

    stream = torch.cuda.current_stream()
    for _ in range(20):  # warm-up launches
        dom_launch()
    torch.cuda.synchronize()
    reps_dom = []
    for _ in range(60):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        dom_launch()
        e1.record(stream)
        e1.synchronize()
        reps_dom.append(e0.elapsed_time(e1))
    dom_ms = float(np.median(reps_dom))
    achieved = bm[dom] / (dom_ms * 1e-3) / 1e9
    bwd_plan = tuned["spmm_bwd"][0]
    roofline = {"bound": "hbm", "kernel": "k_spmm_bwd_coop (fused A^T G and G B^T on pat(A))",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic("k_spmm_bwd_coop", bwd_plan),
                "bytes_per_launch": bm[dom], "median_ms": round(dom_ms, 4), "launches": 60,
                "plan": "natural" if bwd_plan is None else list(bwd_plan)}
    for kname in breakdown:
        breakdown[kname]["frac"] = round(breakdown[kname]["GB/s"] / HBM_PEAK_GBS, 4)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host (one step) ...")
        cpu = cpu_baseline(h, total_bytes)
        log(f"oracle: {cpu['seconds']} s per step on {cpu['cores']} threads, "
            f"{cpu['single_thread']['seconds']} s on one ({cpu['cpu']})")

    pcg = None
    if not args.no_pcg:
        log("PCG time-to-1e-6 part ...")
        pcg = pcg_section(args.pcg_grid, args.train_grid, args.train_steps, args.pcg_systems)

    batched = None
    if not args.no_batched:
        log(f"batched part ({args.batched_blocks} blocks) ...")
        batched = batched_section(*host_blocks, skew=skew)
        host_blocks = skew = None

    cgres = None
    if not args.no_cg:
        log("differentiated-CG part ...")
        cgres = cg_section()
        log(f"CG: {cgres['forward_ms']} ms forward, {cgres['forward_backward_ms']} ms forward+backward")

    spadd = None
    if not args.no_spadd:
        log("sparse + sparse part ...")
        spadd = spadd_section(h["A"])
        log("spadd: " + ", ".join(f"{k} {v['ms']} ms ({v['GB/s']} GB/s)"
                                  for k, v in spadd.items() if isinstance(v, dict)))

    spai = None
    if not args.no_spai:
        log("sparse approximate inverse part ...")
        spai = spai_section()
        log("spai: " + ", ".join(f"{k} {v['iterations']} it {v['solve_ms']} ms"
                                 for k, v in spai.items() if isinstance(v, dict)))

    gcnres = None
    if not args.no_gcn:
        log("graph-convolution part ...")
        gcnres = gcn_section()
        log("gcn: " + ", ".join(f"N={k} {v['ms_per_epoch']} ms/epoch"
                                for k, v in gcnres.items() if isinstance(v, dict)))

    out = {
        "metric": "fwd+bwd sparse-op GB/s (% HBM peak); PCG time-to-1e-6: learned vs Jacobi",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"3D 7-point Poisson {args.grid}^3 (n={d.n}, nnz={d.nnzA}) float32: "
                               f"SpMV and SpMM (k={args.k}) fwd+bwd, Galerkin P^T A P with 8-aggregation "
                               f"(SpGEMM symbolic+numeric+bwd), transposes, red-black L level sets + "
                               f"tri-solve fwd+bwd",
                   "grid": args.grid, "k": args.k, "nnz_A": d.nnzA, "nnz_AP": nnz_ap,
                   "nnz_PtAP": nnz_c, "spgemm_products": products, "nnz_L": d.nnzL,
                   "levels_L": nlev,
                   "spmm_plans": {op: (list(c) if c else "natural") for op, (c, _) in tuned.items()},
                   "spmv_bwd_mode": d.spmv_bwd_mode,
                   "streams": 1 if args.serial else 3,
                   "serial_ms_per_step": round(serial_ms, 4)},
        "frac_hbm_peak": round(value / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "pcg": pcg,
        "batched": batched,
        "cg": cgres,
        "spadd": spadd,
        "spai": spai,
        "gcn": gcnres,
        "breakdown": breakdown,
        "step_bytes": total_bytes,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
