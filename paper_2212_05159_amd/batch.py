"""Batches of independent CSR matrices of uneven sizes as one block-diagonal
matrix, with every op (SpMV and SpMM forward and backward, the triangular
solve and its adjoint) run as ONE persistent launch over a work queue
(``csr_batch_*`` in the library), or, where the autotuner measures it
faster, as the library's per-matrix kernel over the whole concatenation
(one launch as well, one traversal for every block; for the solve, one
grid launch per wide level of the batch).

A plan cuts the blocks into row-aligned tasks of about equal cost (rows +
stored entries), ordered by block cost, largest first; each task carries
its block's traversal variant (row-split with G lanes per row, rows staged
in LDS, or merge-path).  ``Batch.autotune`` picks the variant per class of
blocks (blocks grouped by mean row length and by how uneven their rows
are) by timing each candidate on a plan that holds only that class's
blocks.

Rows of different blocks never interact, so a block's result does not
depend on the rest of the batch; the row-split and staged variants give
the same bits as the library's per-matrix kernels with the same
traversal, and the merge-path variant a deterministic result of its own.
"""
from __future__ import annotations

import numpy as np
import torch

from . import capi
from . import gen
from . import sparse as sp

# variant codes of the plan (see csr_batch_plan_build)
SKIP, AUTO, MERGE, STAGED = -1, 0, 8, 9


def rows_variant(G):
    """Row-split variant with G lanes per row (G a power of two <= 64)."""
    return int(np.log2(G)) + 1


# path items (rows + entries) per task of each op family
BUDGET = {"spmv": 16384, "spmv_t": 16384, "spmm": 2048, "spmm_t": 2048, "tri": 0}

# candidates the autotuner times per class
CANDIDATES = {
    "spmv": (STAGED, rows_variant(4), rows_variant(8), rows_variant(16), MERGE),
    "spmv_t": (rows_variant(4), rows_variant(8), rows_variant(16), MERGE),
    "spmm": (rows_variant(16), MERGE),
    "spmm_t": (rows_variant(16), MERGE),
}


class _Plan:
    def __init__(self, P, brp, variants, budget, dtype):
        d = P.desc(dtype=dtype)
        self.ws = capi._ws(capi.csr_batch_plan_workspace(d, len(brp) - 1, budget), P.device)
        self.plan = capi.csr_batch_plan_build(d, brp, variants, budget, self.ws)


class Batch:
    def __init__(self, blocks=None, dtype=torch.float32, device="cuda", host=None,
                 block_rowptr=None):
        """blocks: list of square host Csr matrices (or host= the block-
        diagonal Csr with block_rowptr=)."""
        if blocks is not None:
            host, block_rowptr = gen.block_diag(blocks)
        self.host = host
        self.block_rowptr = np.asarray(block_rowptr, dtype=np.int32)
        self.nblocks = len(self.block_rowptr) - 1
        self.A = sp.CsrTensor.from_host(host, dtype=dtype, device=device)
        self.dtype = dtype
        self.variants = {}
        # backward of SpMV / SpMM split into the A^T product over A^T's plan
        # and a row-wise value-gradient pass over A's plan (else one fused
        # pass over A^T); set by autotune
        self.bwd_split = {"spmv": False, "spmm": False}
        # triangular solves: "blocks" (a workgroup per block, levels in
        # order inside it), "levels" (one cooperative launch, all
        # workgroups on each level of the batch, grid barriers between) or
        # "grid" (the library's level-scheduled solve of the whole
        # block-diagonal matrix: one grid launch per wide level of the
        # batch); set by autotune_trisolve
        self.tri_mode = "blocks"
        # per op: "queue" (the persistent launch over the plan's work queue,
        # per-block variants) or "plain" (the library's per-matrix kernel
        # over the whole concatenation: also one launch, one traversal for
        # every block); set by autotune, which keeps the faster
        self.impl = {"spmv": "queue", "spmv_bwd": "queue", "spmm": "queue", "spmm_bwd": "queue"}
        self._plans = {}
        self._tri = {}
        rows = np.diff(self.block_rowptr).astype(np.int64)
        rp = np.asarray(host.rowptr, np.int64)
        lens = np.diff(rp)
        self.block_nnz = rp[self.block_rowptr[1:]] - rp[self.block_rowptr[:-1]]
        self.block_rows = rows
        self.block_maxrow = np.array([lens[a:b].max() if b > a else 0
                                      for a, b in zip(self.block_rowptr[:-1],
                                                      self.block_rowptr[1:])], np.int64)

    @property
    def pattern(self):
        return self.A.pattern

    def split(self, v):
        """Per-block views of a vector (or rows of a matrix) over the batch."""
        return [v[int(a):int(b)] for a, b in zip(self.block_rowptr[:-1], self.block_rowptr[1:])]

    def concat(self, parts):
        return torch.cat(list(parts), dim=0)

    # ------------------------------------------------------------------
    def block_classes(self):
        """Class of each block: (floor(log2(mean row length)), uneven),
        uneven meaning the longest row exceeds 8x the mean."""
        mean = self.block_nnz / np.maximum(self.block_rows, 1)
        lg = np.floor(np.log2(np.maximum(mean, 1.0))).astype(int)
        uneven = self.block_maxrow > 8 * np.maximum(mean, 1.0)
        return [(int(a), bool(b)) for a, b in zip(lg, uneven)]

    def _pattern_for(self, family):
        return self.pattern.transpose()[0] if family.endswith("_t") else self.pattern

    def plan(self, family, variants=None):
        """The plan of an op family ("spmv", "spmm" over A; "spmv_t",
        "spmm_t" over A^T) with the chosen (or given) per-block variants."""
        if variants is not None:
            return _Plan(self._pattern_for(family), self.block_rowptr, variants, BUDGET[family],
                         self.dtype)
        if family not in self._plans:
            self._plans[family] = _Plan(self._pattern_for(family), self.block_rowptr,
                                        self.variants.get(family), BUDGET[family], self.dtype)
        return self._plans[family]

    def set_variants(self, family, variants):
        self.variants[family] = None if variants is None else np.asarray(variants, np.int32)
        self._plans.pop(family, None)

    # ------------------------------------------------------------------
    # Ops (functional forms; one launch each)
    # ------------------------------------------------------------------
    def spmv(self, x, vals=None):
        vals = self.A.vals if vals is None else vals
        sp._check_vals(self.pattern, vals)
        sp._check_dense(x, vals, (self.pattern.ncols,), "x")
        if self.impl["spmv"] == "plain":
            return sp.spmv(self.pattern, vals, x)
        y = torch.empty(self.pattern.nrows, dtype=vals.dtype, device=vals.device)
        capi.csr_batch_spmv_fwd(self.pattern.desc(vals), self.plan("spmv").plan, x, y)
        return y

    def spmv_bwd(self, x, gy, vals=None, need_x=True, need_vals=True):
        vals = self.A.vals if vals is None else vals
        P = self.pattern
        sp._check_vals(P, vals)
        sp._check_dense(gy, vals, (P.nrows,), "gy")
        if need_vals:
            sp._check_dense(x, vals, (P.ncols,), "x")
        if self.impl["spmv_bwd"] == "plain":
            return sp.spmv_bwd(P, vals, x, gy, need_x=need_x, need_vals=need_vals)
        Pt, perm = P.transpose()
        gx = torch.empty(P.ncols, dtype=vals.dtype, device=vals.device) if need_x else None
        gv = torch.empty(P.nnz, dtype=vals.dtype, device=vals.device) if need_vals else None
        split = self.bwd_split["spmv"] and need_vals
        if need_x or not split:
            capi.csr_batch_spmv_bwd(P.desc(vals), Pt.desc(dtype=vals.dtype), perm,
                                    self.plan("spmv_t").plan, x, gy, gx, None if split else gv)
        if split:
            capi.csr_batch_sddmv(P.desc(vals), self.plan("spmv").plan, x, gy, gv)
        return gx, gv

    def spmm(self, B, vals=None):
        vals = self.A.vals if vals is None else vals
        sp._check_vals(self.pattern, vals)
        k = sp._cols(B, "B")
        sp._check_dense(B, vals, (self.pattern.ncols, k), "B")
        if self.impl["spmm"] == "plain":
            return sp.spmm(self.pattern, vals, B)
        out = torch.empty(self.pattern.nrows, k, dtype=vals.dtype, device=vals.device)
        capi.csr_batch_spmm_fwd(self.pattern.desc(vals), self.plan("spmm").plan, k, B,
                                B.stride(0), out, out.stride(0))
        return out

    def spmm_bwd(self, B, gC, vals=None, need_B=True, need_vals=True):
        vals = self.A.vals if vals is None else vals
        P = self.pattern
        sp._check_vals(P, vals)
        k = sp._cols(gC, "gC")
        sp._check_dense(gC, vals, (P.nrows, k), "gC")
        if need_vals:
            sp._check_dense(B, vals, (P.ncols, k), "B")
        if self.impl["spmm_bwd"] == "plain":
            return sp.spmm_bwd(P, vals, B, gC, need_B=need_B, need_vals=need_vals)
        Pt, perm = P.transpose()
        gB = torch.empty(P.ncols, k, dtype=vals.dtype, device=vals.device) if need_B else None
        gv = torch.empty(P.nnz, dtype=vals.dtype, device=vals.device) if need_vals else None
        split = self.bwd_split["spmm"] and need_vals
        if need_B or not split:
            capi.csr_batch_spmm_bwd(P.desc(vals), Pt.desc(dtype=vals.dtype), perm,
                                    self.plan("spmm_t").plan, k, B,
                                    B.stride(0) if B is not None else k, gC, gC.stride(0), gB,
                                    gB.stride(0) if gB is not None else k, None if split else gv)
        if split:
            capi.csr_batch_sddmm(P.desc(vals), self.plan("spmm").plan, k, B, B.stride(0), gC,
                                 gC.stride(0), gv)
        return gB, gv

    # ------------------------------------------------------------------
    # Triangular solves with a block-diagonal factor T on the same blocks
    # ------------------------------------------------------------------
    def _tri_setup(self, PT, lower):
        key = (id(PT), bool(lower))
        hit = self._tri.get(key)
        if hit is not None and hit[0] is PT:
            return hit[1:]
        nl, lph, lp, lr, _ = PT.levels(lower)
        plan = _Plan(PT, self.block_rowptr, None, 0, self.dtype)
        lv = capi._ws(capi.csr_batch_levels_workspace(self.nblocks, nl), PT.device)
        capi.csr_batch_levels(plan.plan, nl, lp, lr, lv)
        self._tri[key] = (PT, plan, nl, lr, lv)
        return plan, nl, lr, lv

    def trisolve(self, T, b, lower=True):
        """x = T^{-1} b for a block-diagonal triangular CsrTensor T on this
        batch's blocks."""
        PT = T.pattern
        sp._check_square(PT, "batch trisolve")
        sp._check_vals(PT, T.vals)
        sp._check_dense(b, T.vals, (PT.nrows,), "b")
        if self.tri_mode == "grid":
            return sp.trisolve(PT, T.vals, b, lower)
        x = torch.empty_like(b)
        if self.tri_mode == "levels":
            nl, _, lp, lr, _ = PT.levels(lower)
            capi.csr_batch_trisolve_levels_fwd(PT.desc(T.vals), nl, lp, lr, b, x)
            return x
        plan, nl, lr, lv = self._tri_setup(PT, lower)
        capi.csr_batch_trisolve_fwd(PT.desc(T.vals), plan.plan, nl, lr, lv, b, x)
        return x

    def trisolve_bwd(self, T, x, gx, lower=True, need_vals=True):
        PT = T.pattern
        sp._check_square(PT, "batch trisolve_bwd")
        sp._check_vals(PT, T.vals)
        sp._check_dense(x, T.vals, (PT.nrows,), "x")
        sp._check_dense(gx, T.vals, (PT.nrows,), "gx")
        if self.tri_mode == "grid":
            return sp.trisolve_bwd(PT, T.vals, x, gx, lower, need_vals)
        Pt, perm = PT.transpose()
        gb = torch.empty_like(gx)
        gv = torch.empty(PT.nnz, dtype=T.vals.dtype, device=T.vals.device) if need_vals else None
        if self.tri_mode == "levels":
            nl, _, lp, lr, _ = PT.levels(lower)
            capi.csr_batch_trisolve_levels_bwd(PT.desc(T.vals), Pt.desc(dtype=T.vals.dtype), perm,
                                               nl, lp, lr, x, gx, gb, gv)
            return gb, gv
        plan, nl, lr, lv = self._tri_setup(PT, lower)
        capi.csr_batch_trisolve_bwd(PT.desc(T.vals), Pt.desc(dtype=T.vals.dtype), perm, plan.plan,
                                    nl, lr, lv, x, gx, gb, gv)
        return gb, gv

    def ic0(self, Alow):
        """IC(0) factor values on the pattern of Alow = tril(A) (a
        CsrTensor on this batch's blocks, diagonal last in every row), one
        workgroup per block over the levels of the lower solve."""
        P = Alow.pattern
        sp._check_square(P, "batch ic0")
        sp._check_vals(P, Alow.vals)
        plan, nl, lr, lv = self._tri_setup(P, True)
        out = torch.empty_like(Alow.vals)
        capi.csr_batch_ic0(P.desc(Alow.vals), plan.plan, nl, lr, lv, out)
        return out

    # ------------------------------------------------------------------
    # Autotuner
    # ------------------------------------------------------------------
    def autotune(self, families=("spmv", "spmv_t", "spmm", "spmm_t"), k=64, reps=3, seed=0):
        """Per class of blocks (block_classes), times every candidate
        variant of each op family on a plan holding only that class's
        blocks and keeps the fastest; then the fused or split backward, and
        per op the persistent launch or the plain whole-batch kernel
        (impl_times).  Returns {family: {class: (variant, ms)}}."""
        for op in self.impl:  # the queue's own timings below run through the queue
            self.impl[op] = "queue"
        classes = self.block_classes()
        keys = sorted(set(classes))
        dev = self.A.vals.device
        g = torch.Generator(device=dev)
        g.manual_seed(seed)
        n = self.pattern.nrows
        x = torch.randn(n, generator=g, device=dev, dtype=self.dtype)
        gy = torch.randn(n, generator=g, device=dev, dtype=self.dtype)
        B = G = None
        if any(f.startswith("spmm") for f in families):
            B = torch.randn(n, k, generator=g, device=dev, dtype=self.dtype)
            G = torch.randn(n, k, generator=g, device=dev, dtype=self.dtype)
        P = self.pattern
        vals = self.A.vals
        Pt, perm = P.transpose()
        out = {}
        for fam in families:
            chosen = np.zeros(self.nblocks, np.int32)
            out[fam] = {}
            for key in keys:
                member = np.array([c == key for c in classes])
                timed = []
                for cand in CANDIDATES[fam]:
                    var = np.where(member, cand, SKIP).astype(np.int32)
                    plan_obj = self.plan(fam, var)  # owns the plan's device memory
                    pl = plan_obj.plan
                    if fam == "spmv":
                        y = torch.empty(n, dtype=self.dtype, device=dev)
                        run = lambda: capi.csr_batch_spmv_fwd(P.desc(vals), pl, x, y)
                    elif fam == "spmv_t":
                        gx = torch.empty(n, dtype=self.dtype, device=dev)
                        gv = torch.empty(P.nnz, dtype=self.dtype, device=dev)
                        run = lambda: capi.csr_batch_spmv_bwd(P.desc(vals), Pt.desc(dtype=self.dtype),
                                                              perm, pl, x, gy, gx, gv)
                    elif fam == "spmm":
                        Cm = torch.empty(n, k, dtype=self.dtype, device=dev)
                        run = lambda: capi.csr_batch_spmm_fwd(P.desc(vals), pl, k, B, k, Cm, k)
                    else:
                        gB = torch.empty(n, k, dtype=self.dtype, device=dev)
                        gv = torch.empty(P.nnz, dtype=self.dtype, device=dev)
                        run = lambda: capi.csr_batch_spmm_bwd(P.desc(vals), Pt.desc(dtype=self.dtype),
                                                              perm, pl, k, B, k, G, k, gB, k, gv)
                    timed.append((cand, _time(run, reps)))
                    torch.cuda.current_stream().synchronize()
                    del plan_obj
                cand, ms = min(timed, key=lambda t: t[1])
                chosen[member] = cand
                out[fam][key] = (int(cand), ms, [(int(c), round(t, 4)) for c, t in timed])
            self.set_variants(fam, chosen)
        # fused vs split backward, on the tuned plans
        self.bwd_times = {}
        for op in ("spmv", "spmm"):
            if op not in families or op + "_t" not in families:
                continue
            ms = {}
            for split in (False, True):
                self.bwd_split[op] = split
                if op == "spmv":
                    ms[split] = _time(lambda: self.spmv_bwd(x, gy), reps)
                else:
                    ms[split] = _time(lambda: self.spmm_bwd(B, G), reps)
            self.bwd_split[op] = ms[True] < ms[False]
            self.bwd_times[op] = {"fused_ms": ms[False], "split_ms": ms[True],
                                  "split": self.bwd_split[op]}
        # per op, the tuned persistent launch against the plain kernel over
        # the whole concatenation: keep the faster
        self.impl_times = {}
        runs = {"spmv": ("spmv", lambda: self.spmv(x)),
                "spmv_bwd": ("spmv_t", lambda: self.spmv_bwd(x, gy)),
                "spmm": ("spmm", lambda: self.spmm(B)),
                "spmm_bwd": ("spmm_t", lambda: self.spmm_bwd(B, G))}
        for op, (fam, fn) in runs.items():
            if fam not in families:
                continue
            ms = {}
            for impl in ("queue", "plain"):
                self.impl[op] = impl
                ms[impl] = _time(fn, reps)
            self.impl[op] = min(ms, key=ms.get)
            self.impl_times[op] = {"queue_ms": ms["queue"], "plain_ms": ms["plain"],
                                   "impl": self.impl[op]}
        return out


    def autotune_trisolve(self, T, lower=True, reps=3, seed=0):
        """Times the batched solve modes (forward + adjoint) with the factor
        T on this batch's blocks and keeps the fastest; returns {mode:
        ms}."""
        dev = T.vals.device
        g = torch.Generator(device=dev)
        g.manual_seed(seed)
        n = T.pattern.nrows
        b = torch.randn(n, generator=g, device=dev, dtype=T.vals.dtype)
        gx = torch.randn(n, generator=g, device=dev, dtype=T.vals.dtype)
        ms = {}
        for mode in ("blocks", "levels", "grid"):
            self.tri_mode = mode
            try:
                x = self.trisolve(T, b, lower)
                ms[mode] = _time(lambda: (self.trisolve(T, b, lower),
                                          self.trisolve_bwd(T, x, gx, lower)), reps)
            except capi.CsradError:
                # the runtime may refuse a cooperative launch (a grid the
                # chip cannot hold at once): that mode is then unavailable
                if mode == "blocks":
                    raise
                ms[mode] = float("inf")
        self.tri_mode = min(ms, key=ms.get)
        return ms


def _time(fn, reps):
    fn()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        s.record()
        fn()
        e.record()
        e.synchronize()
        best = min(best, s.elapsed_time(e))
    return best


# ----------------------------------------------------------------------
# Autograd over the batched ops (values and dense operands differentiable)
# ----------------------------------------------------------------------
class BatchSpMV(torch.autograd.Function):
    @staticmethod
    def forward(ctx, batch, vals, x):
        ctx.batch = batch
        ctx.save_for_backward(vals, x)
        return batch.spmv(x.contiguous(), vals)

    @staticmethod
    def backward(ctx, gy):
        vals, x = ctx.saved_tensors
        gx, gv = ctx.batch.spmv_bwd(x.contiguous(), gy.contiguous(), vals,
                                    need_x=ctx.needs_input_grad[2],
                                    need_vals=ctx.needs_input_grad[1])
        return None, gv, gx


class BatchSpMM(torch.autograd.Function):
    @staticmethod
    def forward(ctx, batch, vals, B):
        ctx.batch = batch
        ctx.save_for_backward(vals, B)
        return batch.spmm(B.contiguous(), vals)

    @staticmethod
    def backward(ctx, gC):
        vals, B = ctx.saved_tensors
        gB, gv = ctx.batch.spmm_bwd(B.contiguous(), gC.contiguous(), vals,
                                    need_B=ctx.needs_input_grad[2],
                                    need_vals=ctx.needs_input_grad[1])
        return None, gv, gB


class BatchTriSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, batch, PT, vals, b, lower):
        T = sp.CsrTensor(PT, vals)
        x = batch.trisolve(T, b.contiguous(), lower)
        ctx.batch, ctx.PT, ctx.lower = batch, PT, lower
        ctx.save_for_backward(vals, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        vals, x = ctx.saved_tensors
        gb, gv = ctx.batch.trisolve_bwd(sp.CsrTensor(ctx.PT, vals), x, gx.contiguous(), ctx.lower,
                                        need_vals=ctx.needs_input_grad[2])
        return None, None, gv, gb, None


def geometric_batch(nblocks, n_range=(1024, 65536), k_range=(6, 14), first=0):
    """Host blocks of the batched workload: random geometric-graph
    Laplacians + 1e-2 I (gen.geometric_graph_laplacian), blocks first ..
    first + nblocks - 1."""
    return [gen.geometric_graph_laplacian(b, n_range=n_range, k_range=k_range)
            for b in range(first, first + nblocks)]
