"""Sparse approximate inverse by direct minimisation (Section 4.6).

Minimises l(M) = ||I - M A||_F^2 over the stored values of M with
mask(M) = mask(A), starting from M = mask(A) (every stored value 1), by
steepest descent until the gradient norm falls below a tolerance (0.01 in
the paper).  Every product runs in the library's kernels:

  C = M A            SpSpMM numeric (the pattern of C and the row classes
                     are computed once: M's pattern never changes)
  R = I - C          Sp + Sp (union pattern cached after the first call)
  l = sum R_ij^2
  g_C = -2 R on pat(C)            Sp + Sp VJP
  g_M = (g_C A^T) masked to pat(M)  SpSpMM VJP

The loss is quadratic in M, so the step along -g has a closed form: with
G the gradient, l(M - tG) = ||R + t G A||^2 is least at
t = ||G||^2 / (2 ||G A||^2), one more SpSpMM numeric pass (G A has the
pattern of M A).
"""
from __future__ import annotations

import numpy as np
import torch

from . import capi
from . import sparse as sp


class Spai:
    """The SPAI problem for one matrix A (CsrTensor, square)."""

    def __init__(self, A):
        if A.pattern.nrows != A.pattern.ncols:
            raise ValueError("SPAI needs a square matrix")
        self.A = A
        self.P = A.pattern  # mask(M) = mask(A)
        n = self.P.nrows
        dev = A.vals.device
        self.n = n
        self.dA = self.P.desc(A.vals)
        dM = self.P.desc(dtype=A.vals.dtype)
        self.ws = capi._ws(capi.csr_spgemm_workspace(dM, self.dA), dev)
        self.bins = np.empty(capi.SPGEMM_BINS, dtype=np.int32)
        rpC = torch.empty(n + 1, dtype=torch.int32, device=dev)
        nnz = capi.csr_spgemm_symbolic(dM, self.dA, rpC, self.ws, self.bins)
        self.PC = sp.Pattern(n, n, rpC, torch.empty(nnz, dtype=torch.int32, device=dev))
        self.vC = torch.empty(nnz, dtype=A.vals.dtype, device=dev)
        ar = torch.arange(n + 1, dtype=torch.int32, device=dev)
        self.PI = sp.Pattern(n, n, ar, ar[:n].clone())
        self.ones = torch.ones(n, dtype=A.vals.dtype, device=dev)

    def product(self, Mv, out):
        """out = values of M A on self.PC for M on mask(A) with values Mv."""
        capi.csr_spgemm_fwd(self.P.desc(Mv), self.dA, self.PC.rowptr, self.PC.colind, out,
                            self.ws, self.bins)
        return out

    def loss_grad(self, Mv):
        """(loss, gradient on mask(A)); the loss is a 0-d device tensor."""
        self.product(Mv, self.vC)
        PR, vR = sp.spadd(self.PI, self.ones, self.PC, self.vC, 1.0, -1.0)
        loss = (vR * vR).sum()
        _, gC = sp.spadd_bwd(self.PI, self.PC, PR, 2.0 * vR, 1.0, -1.0, need_A=False)
        gM, _ = sp.spgemm_bwd(self.P, Mv, self.P, self.A.vals, self.PC, gC, need_B=False)
        return loss, gM

    def step_length(self, G):
        """Exact minimiser t of l(M - t G) for the gradient G."""
        GA = self.product(G, torch.empty_like(self.vC))
        return (G * G).sum() / (2.0 * (GA * GA).sum())

    def solve(self, M0=None, tol=0.01, max_iter=1000):
        """Steepest descent with exact steps from M0 (default mask(A)) until
        ||grad|| < tol.  Returns (values of M, info with the loss history)."""
        Mv = (torch.ones_like(self.A.vals) if M0 is None else M0.clone()).contiguous()
        losses, gnorm = [], None
        for it in range(max_iter + 1):
            loss, g = self.loss_grad(Mv)
            gn = torch.linalg.norm(g)
            losses.append(loss)
            gnorm = float(gn)  # one host read per iteration: the stopping test
            if gnorm < tol or it == max_iter:
                break
            Mv = Mv - self.step_length(g) * g
        hist = [float(v) for v in torch.stack(losses).cpu()]
        return Mv, {"iters": len(hist) - 1, "loss": hist[-1], "grad_norm": gnorm,
                    "history": hist, "converged": gnorm < tol}
