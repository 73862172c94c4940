"""Preconditioned CG to a relative-residual tolerance (Section 4.3).

``pcg(A, b, precond=...)`` runs the library's device-resident PCG steps in
chunks, reading the device state once per chunk (the steps after
convergence are no-ops).  Preconditioners: ``"jacobi"`` (1/diag(A)),
``"factor"`` with a lower-triangular ``L`` (M = L L^T approximating A,
z = L^{-T} L^{-1} r by two level-scheduled solves per step), ``"fsai"``
with a lower-triangular ``L`` (the form Section 4.3 learns: M = L L^T
approximating A^{-1}, z = L (L^T r) by two sparse products) and
``"none"``.  A breakdown (non-positive curvature or a
non-finite value, e.g. from an indefinite learned M) falls back to
Jacobi-PCG when ``fallback`` is set.  Vectors and dots are float64; the
matrix values may be float32.
"""
from __future__ import annotations

import numpy as np
import torch

from . import capi
from . import sparse as sp

_KIND = {"jacobi": 0, "factor": 1, "none": 2, "fsai": 3}


class PCG:
    """A reusable PCG context for one matrix and preconditioner."""

    def __init__(self, A, precond="jacobi", L=None, graph=False):
        self.A = A
        self.P = A.pattern
        self.Ad = A.pattern.desc(A.vals)
        self.n = A.pattern.nrows
        dev = A.vals.device
        self.kind = _KIND[precond]
        self.dinv = None
        self.Lkeep = None
        if self.kind == 0:
            self.dinv = torch.empty(self.n, dtype=torch.float64, device=dev)
            capi.csr_diag_inv(self.Ad, self.dinv)
            self.pc = (0, self.dinv, None, None, None, 0, None, None, None)
        elif self.kind == 1:
            if L is None:
                raise ValueError("factor preconditioner needs L")
            nl, lph, lp, lr, _ = L.pattern.levels(True)
            Lt, perm = L.pattern.transpose()
            # L^T's values once, so the adjoint solve reads them directly
            Ltv = sp.transpose_vals(L.pattern, L.vals)
            Ld, Ltd = L.pattern.desc(L.vals), Lt.desc(Ltv)
            self.Lkeep = (L, Lt, Ltv, Ld, Ltd, lph, lp, lr, perm)
            self.pc = (1, None, Ld, Ltd, perm, nl, lph, lp, lr)
        elif self.kind == 3:
            if L is None:
                raise ValueError("fsai preconditioner needs L")
            Lt, perm = L.pattern.transpose()
            Ltv = sp.transpose_vals(L.pattern, L.vals)
            Ld, Ltd = L.pattern.desc(L.vals), Lt.desc(Ltv)
            self.Lkeep = (L, Lt, Ltv, Ld, Ltd, perm)
            self.pc = (3, None, Ld, Ltd, perm, 0, None, None, None)
        else:
            self.pc = (2, None, None, None, None, 0, None, None, None)
        if self.kind in (1, 3):
            bytes_ = capi.csr_pcg_workspace(self.Ad, self.pc[2], self.pc[5], self.pc[6])
        else:
            bytes_ = capi.csr_pcg_workspace(self.Ad)
        self.ws = capi._ws(bytes_, dev)
        f = lambda: torch.empty(self.n, dtype=torch.float64, device=dev)
        self.x, self.r, self.z, self.p, self.q = f(), f(), f(), f(), f()
        self.scal = torch.zeros(16, dtype=torch.float64, device=dev)
        self.graph = graph
        self._g = None

    def _step(self, hist):
        capi.csr_pcg_step(self.Ad, self.pc, self.x, self.r, self.z, self.p, self.q, self.scal,
                          hist, self.ws)

    def solve(self, b, tol=1e-6, maxit=10000, chunk=25, record=False):
        b = b.to(torch.float64).contiguous()
        self.b = b
        hist = torch.zeros(maxit, dtype=torch.float64, device=b.device) if record else None
        capi.csr_pcg_init(self.Ad, self.pc, b, self.x, self.r, self.z, self.p, tol, self.scal,
                          self.ws)
        g = None
        if self.graph and not record:
            if self._g is None or self._g[0] != chunk:
                # capture `chunk` steps as one graph (recorded, not
                # executed); every replay reads the same state buffers
                cg = torch.cuda.CUDAGraph()
                with torch.cuda.graph(cg):
                    for _ in range(chunk):
                        self._step(None)
                self._g = (chunk, cg)
            g = self._g[1]
        it = 0
        while it < maxit:
            n = min(chunk, maxit - it)
            if g is not None and n == chunk:
                g.replay()
            else:
                for _ in range(n):
                    self._step(hist)
            it += n
            st = self.scal.cpu().numpy()
            if st[6] != 0.0:
                break
        st = self.scal.cpu().numpy()
        info = dict(iters=int(st[8]), res=float(st[5]), converged=bool(st[6] and not st[7]),
                    breakdown=bool(st[7]))
        if record:
            info["hist"] = hist[: info["iters"]].cpu().numpy()
        return self.x, info


def pcg(A, b, precond="jacobi", L=None, tol=1e-6, maxit=10000, chunk=25, fallback=True,
        record=False, graph=False):
    """Solves A x = b by PCG.  Returns (x, info)."""
    solver = PCG(A, precond, L, graph=graph)
    x, info = solver.solve(b, tol, maxit, chunk, record)
    info["fallback"] = False
    if info["breakdown"] and fallback and precond != "jacobi":
        x, info2 = PCG(A, "jacobi").solve(b, tol, maxit, chunk, record)
        info2["fallback"] = True
        info2["first_try"] = info
        return x, info2
    return x, info
