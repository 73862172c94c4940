"""Differentiable conjugate gradients on the GPU (Section 4.3's solver).

``cg_solve(A, b, K)`` runs K CG steps from x0 = 0 and returns x_K; its
backward applies the hand-written reverse of every step (the library's
``csr_cg_step_bwd``), so gradients reach the matrix values (per stored
entry) and b.  Memory: the forward keeps (r, p, rho) every c = ceil(sqrt(K))
steps; the backward recomputes one segment at a time from its checkpoint,
storing that segment's (p_t, q_t, r_{t+1}) through the step kernels' save
outputs, then undoes its steps in reverse.  Forward steps are
bit-reproducible, so the checkpointed gradient equals the fully stored one
exactly.  With ``graph=True`` one checkpoint segment (c forward steps) is
captured in a HIP graph and replayed per segment (scalars stay on the
device; no host synchronisation); a shorter last segment runs eagerly.
"""
from __future__ import annotations

import math

import torch

from . import capi


class _Solver:
    def __init__(self, P, vals, b):
        self.P, self.vals, self.b = P, vals, b
        self.A = P.desc(vals)
        self.n = P.nrows
        self.ws = capi._ws(capi.csr_cg_workspace(self.A), vals.device)

    def _new_state(self):
        e = lambda: torch.empty_like(self.b)
        st = dict(x=e(), r=e(), p=e(), q=e(),
                  scal=torch.zeros(8, dtype=torch.float64, device=self.b.device),
                  step=torch.zeros(1, dtype=torch.int32, device=self.b.device))
        capi.csr_cg_init(self.A, self.b, st["x"], st["r"], st["p"], st["scal"], st["step"], self.ws)
        return st

    def _step(self, st, hist, p_save=None, r_save=None, q=None):
        capi.csr_cg_step(self.A, st["x"], st["r"], st["p"], st["q"] if q is None else q, p_save,
                         r_save, st["scal"], st["step"], hist, self.ws)

    def forward(self, K, ckpt_every=None, store_all=False, keep_residuals=False, graph=False):
        """Returns (x_K, saved) where saved holds what the backward needs."""
        c = ckpt_every or max(1, math.ceil(math.sqrt(K)))
        hist = torch.zeros(max(K, 1), 5, dtype=torch.float64, device=self.b.device)
        st = self._new_state()
        R = torch.empty(K, self.n, dtype=self.b.dtype, device=self.b.device) if keep_residuals else None
        full = None
        if store_all:
            full = [torch.empty(K, self.n, dtype=self.b.dtype, device=self.b.device) for _ in range(3)]
        ckpts = []
        g = None
        if graph and not store_all and not keep_residuals and K >= c:
            # capture one checkpoint segment (c steps); each replay advances
            # the device step counter c times
            g = torch.cuda.CUDAGraph()
            probe = {k: v.clone() for k, v in st.items()}
            hist_probe = torch.zeros_like(hist)
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                self._step(probe, hist_probe)  # warm-up outside the capture
            torch.cuda.current_stream().wait_stream(s)
            with torch.cuda.graph(g):
                for _ in range(c):
                    self._step(st, hist)
        t = 0
        while t < K:
            if t % c == 0 and not store_all:
                ckpts.append((st["r"].clone(), st["p"].clone(), st["scal"].clone()))
            if g is not None and t + c <= K:
                g.replay()
                t += c
                continue
            if store_all:
                self._step(st, hist, p_save=full[0][t], r_save=full[2][t], q=full[1][t])
            else:
                self._step(st, hist, r_save=None if R is None else R[t])
            t += 1
        return st["x"], dict(c=c, hist=hist, ckpts=ckpts, full=full, R=R, K=K)

    def backward(self, saved, gx=None, gR=None):
        """Reverse sweep; returns (gvals, gb)."""
        K, c, hist = saved["K"], saved["c"], saved["hist"]
        dev, dt = self.b.device, self.b.dtype
        Pt, perm = self.P.transpose()
        vT = torch.empty_like(self.vals)  # A^T's values, gathered once per sweep
        capi.csr_transpose_vals(self.A, perm, vT)
        At = Pt.desc(vT)
        z = lambda: torch.zeros(self.n, dtype=dt, device=dev)
        xb = gx.clone().to(dt) if gx is not None else z()
        rb, pb, qb = z(), z(), z()
        scal_b = torch.zeros(8, dtype=torch.float64, device=dev)
        gv = torch.zeros(self.P.nnz, dtype=dt, device=dev)

        def undo(t, p_t, q_t, r_t1):
            capi.csr_cg_step_bwd(self.A, At, p_t, q_t, r_t1, hist[t],
                                 None if gR is None else gR[t], xb, rb, pb, qb, scal_b, gv, self.ws)

        if saved["full"] is not None:
            Pf, Qf, Rf = saved["full"]
            for t in reversed(range(K)):
                undo(t, Pf[t], Qf[t], Rf[t])
        else:
            segP = torch.empty(c, self.n, dtype=dt, device=dev)
            segQ = torch.empty_like(segP)
            segR = torch.empty_like(segP)
            xd = z()
            stepd = torch.zeros(1, dtype=torch.int32, device=dev)
            for s in reversed(range(len(saved["ckpts"]))):
                t0, t1 = s * c, min(K, (s + 1) * c)
                r_w, p_w, sc_w = saved["ckpts"][s]  # consumed in place
                st = dict(x=xd, r=r_w, p=p_w, q=None, scal=sc_w, step=stepd)
                for i in range(t1 - t0):
                    self._step(st, None, p_save=segP[i], r_save=segR[i], q=segQ[i])
                for i in reversed(range(t1 - t0)):
                    undo(t0 + i, segP[i], segQ[i], segR[i])
        gb = torch.empty_like(self.b)
        capi.csr_cg_finish_bwd(self.A, self.b, rb, pb, scal_b, gb)
        return gv, gb


class CGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, P, vals, b, K, ckpt_every, store_all, graph):
        sol = _Solver(P, vals.detach(), b.detach().contiguous())
        x, saved = sol.forward(K, ckpt_every, store_all, graph=graph)
        ctx.sol, ctx.saved = sol, saved
        return x

    @staticmethod
    def backward(ctx, gx):
        gv, gb = ctx.sol.backward(ctx.saved, gx=gx.contiguous())
        ctx.sol = ctx.saved = None
        return None, gv, gb, None, None, None, None


def cg_solve(A, b, K, ckpt_every=None, store_all=False, graph=False):
    """x_K of K CG steps on the CsrTensor A (differentiable in A.vals and b)."""
    return CGSolve.apply(A.pattern, A.vals, b, int(K), ckpt_every, bool(store_all), bool(graph))


def cg_with_residuals(A, b, K):
    """(x_K, R) with R[t] = r_{t+1}; not an autograd op: use ``residual_grads``
    for the reverse sweep with upstream gradients on x_K and R."""
    sol = _Solver(A.pattern, A.vals.detach(), b.detach().contiguous())
    x, saved = sol.forward(K, store_all=False, keep_residuals=True)
    return x, saved["R"], (sol, saved)


def residual_grads(handle, gx=None, gR=None):
    sol, saved = handle
    return sol.backward(saved, gx=gx, gR=gR)
