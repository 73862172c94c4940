"""CSR tensors on the GPU and their differentiable operations.

``Pattern`` is an immutable device CSR pattern (rowptr, colind) that caches
what only depends on the pattern: its transpose (pattern + permutation)
and triangular level sets.  ``CsrTensor`` pairs a pattern with a value
array that may require grad; ``@`` dispatches to SpMV (vector), SpDMM
(matrix) or SpSpMM (CsrTensor), and ``solve_triangular`` to the level-
scheduled solve.  Each op is a ``torch.autograd.Function`` whose forward and
backward call the HIP library through ``capi``; gradients of sparse inputs
are value arrays on the input's own pattern (Section 3.1, Table 1).
"""
from __future__ import annotations

import numpy as np
import torch

from . import capi


class Pattern:
    def __init__(self, nrows, ncols, rowptr, colind):
        assert rowptr.dtype == torch.int32 and colind.dtype == torch.int32
        self.nrows, self.ncols = int(nrows), int(ncols)
        self.rowptr, self.colind = rowptr, colind
        self._t = None
        self._levels = {}
        self._plans = {}
        self._stats = None

    @property
    def nnz(self):
        return int(self.colind.numel())

    @property
    def device(self):
        return self.rowptr.device

    def desc(self, vals=None, dtype=torch.float32):
        return capi.desc(self.nrows, self.ncols, self.rowptr, self.colind, vals,
                         dtype=vals.dtype if vals is not None else dtype)

    def transpose(self):
        """(Pattern of A^T, perm) with valsT = vals[perm]; cached."""
        if self._t is None:
            d = self.desc()
            rpT = torch.empty(self.ncols + 1, dtype=torch.int32, device=self.device)
            ciT = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
            perm = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
            ws = capi._ws(capi.csr_transpose_workspace(d), self.device)
            capi.csr_transpose(d, rpT, ciT, perm, ws)
            self._t = (Pattern(self.ncols, self.nrows, rpT, ciT), perm)
        return self._t

    def stats(self):
        """(longest row, bandwidth, non-empty rows, nnz); cached."""
        if self._stats is None:
            ws = torch.empty(64, dtype=torch.uint8, device=self.device)
            self._stats = capi.csr_pattern_stats(self.desc(), ws)
        return self._stats

    def plan(self, op):
        """Traversal plan chosen for ``op`` (set by the autotuner), or None."""
        return self._plans.get(op)

    def set_plan(self, op, plan):
        self._plans[op] = plan

    def levels(self, lower=True):
        """Level sets of the triangular solve; cached per orientation.
        Returns (nlevels, level_ptr_host ndarray, level_ptr, level_rows,
        level_of_row)."""
        key = bool(lower)
        if key not in self._levels:
            Tt, _ = self.transpose()
            n = self.nrows
            lor = torch.empty(n, dtype=torch.int32, device=self.device)
            lptr = torch.empty(n + 1, dtype=torch.int32, device=self.device)
            lrows = torch.empty(n, dtype=torch.int32, device=self.device)
            d = self.desc()
            ws = capi._ws(capi.csr_trisolve_workspace(d), self.device)
            lph = np.empty(n + 1, dtype=np.int32)
            nl = capi.csr_trisolve_analyze(d, int(key), Tt.desc(), lor, lptr, lrows, ws, lph)
            self._levels[key] = (nl, lph[: nl + 1].copy(), lptr[: nl + 1], lrows, lor)
        return self._levels[key]

    @classmethod
    def from_host(cls, m, device="cuda"):
        return cls(m.nrows, m.ncols, torch.as_tensor(np.asarray(m.rowptr, np.int32), device=device),
                   torch.as_tensor(np.asarray(m.colind, np.int32), device=device))


# ----------------------------------------------------------------------
# Argument checks.  The C ABI receives bare pointers and cannot tell a
# host pointer, a short buffer or another value type from a valid operand,
# so every functional form checks its tensors here and raises before any
# launch.
# ----------------------------------------------------------------------

def _check_vals(P, vals, what="vals"):
    if not torch.is_tensor(vals):
        raise TypeError(f"{what}: expected a tensor, got {type(vals).__name__}")
    if vals.dtype not in (torch.float32, torch.float64):
        raise TypeError(f"{what}: value type must be float32 or float64, got {vals.dtype}")
    if vals.device.type != "cuda":
        raise TypeError(f"{what}: must be on a CUDA device, got {vals.device}")
    if P.rowptr.device != vals.device or P.colind.device != vals.device:
        raise TypeError(f"{what}: on {vals.device}, pattern on {P.rowptr.device}")
    if vals.dim() != 1 or vals.numel() != P.nnz or not vals.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous vector of nnz = {P.nnz} values, "
                         f"got shape {tuple(vals.shape)}")


def _check_dense(t, ref, shape, what):
    """t must be a tensor on ref's device with ref's dtype and the given
    shape (rows may carry a leading dimension >= the column count, but the
    columns must be unit-stride)."""
    if not torch.is_tensor(t):
        raise TypeError(f"{what}: expected a tensor, got {type(t).__name__}")
    if t.device != ref.device:
        raise TypeError(f"{what}: on {t.device}, expected {ref.device}")
    if t.dtype != ref.dtype:
        raise TypeError(f"{what}: dtype {t.dtype}, expected {ref.dtype} (the values' type)")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.dim() == 1 and t.numel() > 0 and t.stride(0) != 1:
        raise ValueError(f"{what}: must be contiguous")
    if t.dim() == 2 and t.numel() > 0 and (t.stride(1) != 1 or t.stride(0) < t.shape[1]):
        raise ValueError(f"{what}: rows must be unit-stride with a leading dimension >= "
                         f"{t.shape[1]}")


def _cols(t, what):
    if not torch.is_tensor(t) or t.dim() != 2:
        raise ValueError(f"{what}: expected a 2-D tensor")
    if t.shape[1] <= 0:
        raise ValueError(f"{what}: needs at least one column")
    return int(t.shape[1])


# ----------------------------------------------------------------------
# Functional forms (allocate outputs, call the library).
# ----------------------------------------------------------------------

def spmv(P, vals, x):
    _check_vals(P, vals)
    _check_dense(x, vals, (P.ncols,), "x")
    y = torch.empty(P.nrows, dtype=vals.dtype, device=vals.device)
    capi.csr_spmv_fwd(P.desc(vals), x, y)
    return y


def spmv_bwd(P, vals, x, gy, need_x=True, need_vals=True, use_transpose=True, mode=None):
    """(gx, gvals).  mode "fused" or "split" (see autotune.tune_spmv_bwd)
    overrides the pattern's tuned choice; both give the same bits."""
    _check_vals(P, vals)
    _check_dense(gy, vals, (P.nrows,), "gy")
    if need_vals:
        _check_dense(x, vals, (P.ncols,), "x")
    mode = mode if mode is not None else P.plan("spmv_bwd")
    gx = torch.empty(P.ncols, dtype=vals.dtype, device=vals.device) if need_x else None
    gv = torch.empty(P.nnz, dtype=vals.dtype, device=vals.device) if need_vals else None
    if use_transpose:
        Pt, perm = P.transpose()
        if need_x and need_vals and mode == "split":
            # A^T gy over A^T and the value gradient row-wise over A, the two
            # passes in one launch (the autotuner's choice for patterns with
            # a scattered transpose)
            capi.csr_spmv_bwd_split(P.desc(vals), Pt.desc(dtype=vals.dtype), perm, x, gy, gx, gv)
        else:
            capi.csr_spmv_bwd(P.desc(vals), Pt.desc(dtype=vals.dtype), perm, x, gy, gx, gv)
    else:
        capi.csr_spmv_bwd(P.desc(vals), None, None, x, gy, gx, gv)
    return gx, gv


def spmm(P, vals, B, plan=None):
    _check_vals(P, vals)
    k = _cols(B, "B")
    _check_dense(B, vals, (P.ncols, k), "B")
    out = torch.empty(P.nrows, k, dtype=vals.dtype, device=vals.device)
    capi.csr_spmm_fwd(P.desc(vals), k, B, B.stride(0), out, out.stride(0),
                      plan if plan is not None else P.plan("spmm_fwd"))
    return out


def spmm_bwd(P, vals, B, gC, need_B=True, need_vals=True, plan=None):
    _check_vals(P, vals)
    k = _cols(gC, "gC")
    _check_dense(gC, vals, (P.nrows, k), "gC")
    if need_vals:
        _check_dense(B, vals, (P.ncols, k), "B")
    gB = torch.empty(P.ncols, k, dtype=vals.dtype, device=vals.device) if need_B else None
    gv = torch.empty(P.nnz, dtype=vals.dtype, device=vals.device) if need_vals else None
    Pt, perm = P.transpose() if need_B else (None, None)
    capi.csr_spmm_bwd(P.desc(vals), Pt.desc(dtype=vals.dtype) if Pt is not None else None, perm, k,
                      B, B.stride(0) if B is not None else k, gC, gC.stride(0), gB,
                      gB.stride(0) if gB is not None else k, gv,
                      plan if plan is not None else P.plan("spmm_bwd" if need_B else "sddmm"))
    return gB, gv


def transpose_vals(P, vals):
    """Values of A^T in the order of P.transpose()'s pattern."""
    _check_vals(P, vals)
    _, perm = P.transpose()
    out = torch.empty_like(vals)
    capi.csr_transpose_vals(P.desc(vals), perm, out)
    return out


def spgemm(PA, valsA, PB, valsB):
    """C = A B.  Returns (Pattern of C, valsC)."""
    _check_vals(PA, valsA, "valsA")
    _check_vals(PB, valsB, "valsB")
    if PA.ncols != PB.nrows:
        raise ValueError(f"spgemm: inner dimensions differ ({PA.ncols} vs {PB.nrows})")
    if valsA.dtype != valsB.dtype:
        raise TypeError("spgemm: operands differ in value type")
    dA, dB = PA.desc(valsA), PB.desc(valsB)
    ws = capi._ws(capi.csr_spgemm_workspace(dA, dB), valsA.device)
    rpC = torch.empty(PA.nrows + 1, dtype=torch.int32, device=valsA.device)
    bins = np.empty(capi.SPGEMM_BINS, dtype=np.int32)  # row classes, reused by the numeric call
    nnz = capi.csr_spgemm_symbolic(dA, dB, rpC, ws, bins)
    ciC = torch.empty(nnz, dtype=torch.int32, device=valsA.device)
    vC = torch.empty(nnz, dtype=valsA.dtype, device=valsA.device)
    capi.csr_spgemm_fwd(dA, dB, rpC, ciC, vC, ws, bins)
    return Pattern(PA.nrows, PB.ncols, rpC, ciC), vC


def spgemm_bwd(PA, valsA, PB, valsB, PC, gC, need_A=True, need_B=True):
    _check_vals(PA, valsA, "valsA")
    _check_vals(PB, valsB, "valsB")
    _check_dense(gC, valsA, (PC.nnz,), "gC")
    gA = torch.empty(PA.nnz, dtype=valsA.dtype, device=valsA.device) if need_A else None
    gB = torch.empty(PB.nnz, dtype=valsB.dtype, device=valsB.device) if need_B else None
    At, permA = PA.transpose() if need_B else (None, None)
    capi.csr_spgemm_bwd(PA.desc(valsA), PB.desc(valsB),
                        At.desc(dtype=valsA.dtype) if At is not None else None, permA,
                        PC.desc(dtype=valsA.dtype), gC, gA, gB)
    return gA, gB


def spadd(PA, valsA, PB, valsB, alpha=1.0, beta=1.0):
    """C = alpha A + beta B on the union pattern.  Returns (Pattern of C, valsC).

    The union pattern is cached on PA for PB (patterns are immutable), so a
    repeated sum recomputes values only."""
    if PA.nrows != PB.nrows or PA.ncols != PB.ncols:
        raise ValueError("spadd: operands differ in shape")
    _check_vals(PA, valsA, "valsA")
    _check_vals(PB, valsB, "valsB")
    if valsA.dtype != valsB.dtype:
        raise TypeError("spadd: operands differ in value type")
    dA, dB = PA.desc(valsA), PB.desc(valsB)
    key = ("spadd", id(PB))
    hit = PA.plan(key)
    if hit is not None and hit[0] is PB:
        PC, cols = hit[1], None
    else:
        dev = valsA.device
        ws = capi._ws(capi.csr_spadd_workspace(dA, dB), dev)
        rpC = torch.empty(PA.nrows + 1, dtype=torch.int32, device=dev)
        nnz = capi.csr_spadd_symbolic(dA, dB, rpC, ws)
        PC = Pattern(PA.nrows, PA.ncols, rpC,
                     torch.empty(nnz, dtype=torch.int32, device=dev))
        cols = PC.colind
    vC = torch.empty(PC.nnz, dtype=valsA.dtype, device=valsA.device)
    capi.csr_spadd_fwd(dA, dB, alpha, beta, PC.rowptr, cols, vC)
    if cols is not None:
        PA.set_plan(key, (PB, PC))
    return PC, vC


def spadd_bwd(PA, PB, PC, gC, alpha=1.0, beta=1.0, need_A=True, need_B=True, dtype=None):
    dtype = dtype or gC.dtype
    if not torch.is_tensor(gC) or gC.device.type != "cuda":
        raise TypeError("spadd_bwd: gC must be a CUDA tensor")
    _check_dense(gC, torch.empty(0, dtype=dtype, device=gC.device), (PC.nnz,), "gC")
    gA = torch.empty(PA.nnz, dtype=dtype, device=gC.device) if need_A else None
    gB = torch.empty(PB.nnz, dtype=dtype, device=gC.device) if need_B else None
    capi.csr_spadd_bwd(PA.desc(dtype=dtype), PB.desc(dtype=dtype), PC.desc(dtype=dtype), alpha,
                       beta, gC, gA, gB)
    return gA, gB


def _check_square(P, what):
    if P.nrows != P.ncols:
        raise ValueError(f"{what}: the triangular matrix must be square, got {P.nrows}x{P.ncols}")


def trisolve(P, vals, b, lower=True):
    _check_square(P, "trisolve")
    _check_vals(P, vals)
    _check_dense(b, vals, (P.nrows,), "b")
    nl, lph, lp, lr, _ = P.levels(lower)
    x = torch.empty_like(b)
    capi.csr_trisolve_fwd(P.desc(vals), int(lower), nl, lph, lp, lr, b, x)
    return x


def trisolve_bwd(P, vals, x, gx, lower=True, need_vals=True):
    _check_square(P, "trisolve_bwd")
    _check_vals(P, vals)
    _check_dense(x, vals, (P.nrows,), "x")
    _check_dense(gx, vals, (P.nrows,), "gx")
    nl, lph, lp, lr, _ = P.levels(lower)
    Pt, perm = P.transpose()
    gb = torch.empty_like(gx)
    gv = torch.empty(P.nnz, dtype=vals.dtype, device=vals.device) if need_vals else None
    capi.csr_trisolve_bwd(P.desc(vals), int(lower), Pt.desc(dtype=vals.dtype), perm, nl, lph, lp,
                          lr, x, gx, gb, gv)
    return gb, gv


# ----------------------------------------------------------------------
# Autograd functions: differentiable inputs are value arrays and dense
# operands; patterns are constants.
# ----------------------------------------------------------------------

class SpMV(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, vals, x):
        ctx.P = P
        ctx.save_for_backward(vals, x)
        return spmv(P, vals, x.contiguous())

    @staticmethod
    def backward(ctx, gy):
        vals, x = ctx.saved_tensors
        gx, gv = spmv_bwd(ctx.P, vals, x.contiguous(), gy.contiguous(),
                          need_x=ctx.needs_input_grad[2], need_vals=ctx.needs_input_grad[1])
        return None, gv, gx


class SpMVT(torch.autograd.Function):
    """y = A^T x through the library's transpose product (the input-gradient
    kernel of SpMV).  VJP: g_x = A g, g_vals[(i,j)] = x_i g_j on pat(A)."""

    @staticmethod
    def forward(ctx, P, vals, x):
        ctx.P = P
        x = x.contiguous()
        ctx.save_for_backward(vals, x)
        y, _ = spmv_bwd(P, vals, x, x, need_x=True, need_vals=False)
        return y

    @staticmethod
    def backward(ctx, g):
        vals, x = ctx.saved_tensors
        g = g.contiguous()
        gx = spmv(ctx.P, vals, g) if ctx.needs_input_grad[2] else None
        gv = None
        if ctx.needs_input_grad[1]:
            # the value gradient of SpMV with its roles swapped: g_y -> x, x -> g
            _, gv = spmv_bwd(ctx.P, vals, g, x, need_x=False, need_vals=True)
        return None, gv, gx


class SpMM(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, vals, B):
        ctx.P = P
        ctx.save_for_backward(vals, B)
        return spmm(P, vals, B.contiguous())

    @staticmethod
    def backward(ctx, gC):
        vals, B = ctx.saved_tensors
        gB, gv = spmm_bwd(ctx.P, vals, B.contiguous(), gC.contiguous(),
                          need_B=ctx.needs_input_grad[2], need_vals=ctx.needs_input_grad[1])
        return None, gv, gB


class SpGEMM(torch.autograd.Function):
    """Returns the value array of C; its pattern is stored on ``out_pattern``."""

    @staticmethod
    def forward(ctx, PA, valsA, PB, valsB, out_pattern):
        PC, vC = spgemm(PA, valsA, PB, valsB)
        out_pattern.append(PC)
        ctx.PA, ctx.PB, ctx.PC = PA, PB, PC
        ctx.save_for_backward(valsA, valsB)
        return vC

    @staticmethod
    def backward(ctx, gC):
        valsA, valsB = ctx.saved_tensors
        gA, gB = spgemm_bwd(ctx.PA, valsA, ctx.PB, valsB, ctx.PC, gC.contiguous(),
                            need_A=ctx.needs_input_grad[1], need_B=ctx.needs_input_grad[3])
        return None, gA, None, gB, None


class SpAdd(torch.autograd.Function):
    """alpha A + beta B; returns the value array of C, whose pattern is
    stored on ``out_pattern``."""

    @staticmethod
    def forward(ctx, PA, valsA, PB, valsB, alpha, beta, out_pattern):
        PC, vC = spadd(PA, valsA, PB, valsB, alpha, beta)
        out_pattern.append(PC)
        ctx.PA, ctx.PB, ctx.PC, ctx.alpha, ctx.beta = PA, PB, PC, alpha, beta
        return vC

    @staticmethod
    def backward(ctx, gC):
        gA, gB = spadd_bwd(ctx.PA, ctx.PB, ctx.PC, gC.contiguous(), ctx.alpha, ctx.beta,
                           need_A=ctx.needs_input_grad[1], need_B=ctx.needs_input_grad[3])
        return None, gA, None, gB, None, None, None


class TriSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, vals, b, lower):
        x = trisolve(P, vals, b.contiguous(), lower)
        ctx.P, ctx.lower = P, lower
        ctx.save_for_backward(vals, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        vals, x = ctx.saved_tensors
        gb, gv = trisolve_bwd(ctx.P, vals, x, gx.contiguous(), ctx.lower,
                              need_vals=ctx.needs_input_grad[1])
        return None, gv, gb, None


class CsrTensor:
    """A CSR matrix on the GPU: constant pattern, (possibly trainable) values."""

    def __init__(self, pattern: Pattern, vals: torch.Tensor):
        assert vals.numel() == pattern.nnz
        self.pattern, self.vals = pattern, vals

    @property
    def shape(self):
        return (self.pattern.nrows, self.pattern.ncols)

    @classmethod
    def from_host(cls, m, dtype=torch.float32, device="cuda", requires_grad=False):
        P = Pattern.from_host(m, device)
        v = torch.as_tensor(np.asarray(m.vals), device=device).to(dtype)
        return cls(P, v.requires_grad_(requires_grad))

    def __matmul__(self, other):
        if isinstance(other, CsrTensor):
            box = []
            vC = SpGEMM.apply(self.pattern, self.vals, other.pattern, other.vals, box)
            return CsrTensor(box[0], vC)
        if other.dim() == 1:
            return SpMV.apply(self.pattern, self.vals, other)
        return SpMM.apply(self.pattern, self.vals, other)

    def add(self, other, alpha=1.0, beta=1.0):
        """alpha self + beta other on the union of the two patterns."""
        box = []
        vC = SpAdd.apply(self.pattern, self.vals, other.pattern, other.vals, float(alpha),
                         float(beta), box)
        return CsrTensor(box[0], vC)

    def __add__(self, other):
        return self.add(other, 1.0, 1.0)

    def __sub__(self, other):
        return self.add(other, 1.0, -1.0)

    def __mul__(self, scalar):
        return CsrTensor(self.pattern, self.vals * scalar)

    __rmul__ = __mul__

    def __neg__(self):
        return CsrTensor(self.pattern, -self.vals)

    def row_sum(self):
        """Row sums (the SpMV A 1; differentiable in the values)."""
        ones = torch.ones(self.pattern.ncols, dtype=self.vals.dtype, device=self.vals.device)
        return SpMV.apply(self.pattern, self.vals, ones)

    def diagonal(self):
        """The stored diagonal as a dense vector (zero where not stored;
        differentiable in the values)."""
        P = self.pattern
        n = min(P.nrows, P.ncols)
        rows = torch.repeat_interleave(torch.arange(P.nrows, device=self.vals.device),
                                       (P.rowptr[1:] - P.rowptr[:-1]).long())
        on = rows == P.colind.long()
        out = torch.zeros(n, dtype=self.vals.dtype, device=self.vals.device)
        return out.index_put((rows[on],), self.vals[on])

    def tmatvec(self, x):
        """A^T x (differentiable in the values and x)."""
        return SpMVT.apply(self.pattern, self.vals, x)

    def solve_triangular(self, b, lower=True):
        return TriSolve.apply(self.pattern, self.vals, b, lower)

    def transpose(self):
        """A^T with its values gathered by the library (not differentiable)."""
        Pt, _ = self.pattern.transpose()
        return CsrTensor(Pt, transpose_vals(self.pattern, self.vals.detach()))


def eye(n, k=0, dtype=torch.float32, device="cuda"):
    """n x n matrix with ones on diagonal k (k > 0 above the main diagonal)."""
    i = torch.arange(max(0, -k), min(n, n - k), device=device, dtype=torch.int32)
    counts = torch.zeros(n, dtype=torch.int32, device=device)
    counts[i.long()] = 1
    rowptr = torch.zeros(n + 1, dtype=torch.int32, device=device)
    rowptr[1:] = torch.cumsum(counts, 0, dtype=torch.int32)
    P = Pattern(n, n, rowptr, (i + k).to(torch.int32))
    return CsrTensor(P, torch.ones(P.nnz, dtype=dtype, device=device))


def diag(v):
    """Diagonal matrix with the entries of v as its values (differentiable:
    the values are v itself)."""
    n = v.numel()
    ar = torch.arange(n + 1, dtype=torch.int32, device=v.device)
    return CsrTensor(Pattern(n, n, ar, ar[:n].clone()), v)

