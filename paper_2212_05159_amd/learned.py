"""Learned IC(0)-shaped preconditioner: a message-passing network on A's
graph emits the values of a lower-triangular factor L on tril(A)'s pattern
(M = L L^T, applied by two triangular solves), trained by backpropagation
through a few PCG iterations with the residual-history loss of Section 4.3.

Network (hidden width 32, bf16 matrix-core dense layers, float32 elsewhere):
  Ahat = D^{-1/2} A D^{-1/2};  X0 = node inputs (csr_mpnn_prep)
  H0 = relu(X0 W0 + b0)
  H_l = relu([H_{l-1}, Ahat H_{l-1}] W_l + b_l),  l = 1..3   (SpMM aggregation)
  P = H3 Wp;  t_ij = <P_i, H3_j> on tril(A)                    (SDDMM readout)
  L_ij = sqrt(A_ii) Ahat_ij (1 + t_ij) (j < i),  L_ii = sqrt(A_ii)(softplus(t_ii + c) + delta)
With Wp = 0 the factor is the symmetric Gauss-Seidel one, L = (D + tril_strict A) D^{-1/2}.
Every sparse product and dense layer runs in the library's kernels (SpMM,
its backward, SDDMM, tri-solves, MFMA layers); PyTorch holds the tensors,
the scalar/vector glue of the loss, and Adam.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import capi
from . import gen
from . import sparse as sp

HIDDEN = 32
LAYERS = 3
C0 = math.log(math.e - 1.0)  # softplus(C0) = 1
DELTA = 1e-3


# ----------------------------------------------------------------------
# Autograd wrappers over the library
# ----------------------------------------------------------------------
class Dense(torch.autograd.Function):
    @staticmethod
    def forward(ctx, X1, X2, W, b, relu):
        n, K1 = X1.shape
        K2 = 0 if X2 is None else X2.shape[1]
        Y = torch.empty(n, HIDDEN, dtype=torch.float32, device=X1.device)
        capi.csr_dense_fwd(n, K1, X1, X1.stride(0), K2, X2, K2 if X2 is None else X2.stride(0),
                           W, b, int(relu), Y)
        ctx.save_for_backward(X1, X2 if X2 is not None else torch.empty(0), W, Y)
        ctx.has2, ctx.hasb, ctx.relu = X2 is not None, b is not None, relu
        return Y

    @staticmethod
    def backward(ctx, dY):
        X1, X2, W, Y = ctx.saved_tensors
        X2 = X2 if ctx.has2 else None
        n, K1 = X1.shape
        K2 = 0 if X2 is None else X2.shape[1]
        dY = dY.contiguous()
        dX1 = torch.empty_like(X1) if ctx.needs_input_grad[0] else None
        dX2 = torch.empty_like(X2) if (X2 is not None and ctx.needs_input_grad[1]) else None
        dW = torch.empty_like(W)
        db = torch.empty(HIDDEN, dtype=torch.float32, device=W.device) if ctx.hasb else None
        ws = capi._ws(capi.csr_dense_workspace(n), W.device)
        capi.csr_dense_bwd(n, K1, X1, X1.stride(0), K2, X2, K2 if X2 is None else X2.stride(0),
                           W, Y, dY, int(ctx.relu), dX1, dX2, dW, db, ws)
        return dX1, dX2, dW, db, None


class SDDMM(torch.autograd.Function):
    """t[e] = <P[i,:], H[j,:]> for the entries e = (i, j) of pattern S."""

    @staticmethod
    def forward(ctx, S, P, H):
        k = P.shape[1]
        t = torch.empty(S.nnz, dtype=P.dtype, device=P.device)
        capi.csr_spmm_bwd(S.desc(dtype=P.dtype), None, None, k, H, H.stride(0), P, P.stride(0),
                          None, k, t)
        ctx.S = S
        ctx.save_for_backward(P, H)
        return t

    @staticmethod
    def backward(ctx, gt):
        P, H = ctx.saved_tensors
        S = ctx.S
        gt = gt.contiguous()
        # dP = G H and dH = G^T P with G the sparse matrix of gt on S
        dP = sp.spmm(S, gt, H)
        dH, _ = sp.spmm_bwd(S, gt, None, P, need_B=True, need_vals=False)
        return None, dP, dH


class Readout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, t, Lpat, ahatL, dsqrt):
        Lv = torch.empty_like(t)
        capi.csr_mpnn_readout(Lpat.desc(dtype=torch.float32), ahatL, dsqrt, t, C0, DELTA, Lv)
        ctx.Lpat = Lpat
        ctx.save_for_backward(t, ahatL, dsqrt)
        return Lv

    @staticmethod
    def backward(ctx, gL):
        t, ahatL, dsqrt = ctx.saved_tensors
        gt = torch.empty_like(t)
        capi.csr_mpnn_readout_bwd(ctx.Lpat.desc(dtype=torch.float32), ahatL, dsqrt, t, C0,
                                  gL.contiguous(), gt)
        return gt, None, None, None


class TriSolveT(torch.autograd.Function):
    """y = T^{-T} b for lower-triangular T (the second solve of M^{-1})."""

    @staticmethod
    def forward(ctx, P, vals, b):
        nl, lph, lp, lr, _ = P.levels(True)
        Pt, perm = P.transpose()
        y = torch.empty_like(b)
        capi.csr_trisolve_bwd(P.desc(vals), 1, Pt.desc(dtype=vals.dtype), perm, nl, lph, lp, lr,
                              None, b.contiguous(), y, None)
        ctx.P = P
        ctx.save_for_backward(vals, y)
        return y

    @staticmethod
    def backward(ctx, g):
        vals, y = ctx.saved_tensors
        w = sp.trisolve(ctx.P, vals, g.contiguous(), True)       # T^{-1} g
        gv = None
        if ctx.needs_input_grad[1]:
            # d/dT_ij of <g, T^{-T} b> = -y_i w_j on T's pattern
            _, gv = sp.spmv_bwd(ctx.P, vals, w, -y, need_x=False, need_vals=True,
                                use_transpose=False)
        return None, gv, w


# ----------------------------------------------------------------------
# The network
# ----------------------------------------------------------------------
class MPNN(torch.nn.Module):
    """form "factor": L approximates A's Cholesky factor (M^{-1} = L^{-T} L^{-1}).
    form "fsai": the approximate-inverse form of Section 4.3 (M = L L^T
    approximates A^{-1}); the readout's factor F is mapped entrywise to
    L_ii = F_ii / d_i and L_ij = -F_ij / d_i, so the untrained network gives
    the first-order inverse factor L = D^{-1} (D - A_L) D^{-1/2} (A_L the
    strictly lower part of A, up to the 1e-3 on the diagonal)."""

    def __init__(self, seed=0, device="cuda", form="factor"):
        super().__init__()
        self.form = form
        g = torch.Generator().manual_seed(seed)

        def init(k, scale=1.0):
            return torch.nn.Parameter((torch.randn(k, HIDDEN, generator=g) * scale / math.sqrt(k))
                                      .to(device))

        self.W0 = init(16)
        self.b0 = torch.nn.Parameter(torch.zeros(HIDDEN, device=device))
        self.Ws = torch.nn.ParameterList([init(2 * HIDDEN) for _ in range(LAYERS)])
        self.bs = torch.nn.ParameterList([torch.nn.Parameter(torch.zeros(HIDDEN, device=device))
                                          for _ in range(LAYERS)])
        self.Wp = torch.nn.Parameter(torch.zeros(HIDDEN, HIDDEN, device=device))

    def prepare(self, A, Lpat):
        """Scaled matrix and inputs for A (CsrTensor, float32)."""
        n = A.pattern.nrows
        dev = A.vals.device
        ahat = torch.empty_like(A.vals)
        ahatL = torch.empty(Lpat.nnz, dtype=torch.float32, device=dev)
        dsqrt = torch.empty(n, dtype=torch.float32, device=dev)
        X0 = torch.empty(n, 16, dtype=torch.float32, device=dev)
        capi.csr_mpnn_prep(A.pattern.desc(A.vals), Lpat.desc(dtype=torch.float32), ahat, ahatL,
                           dsqrt, X0)
        return ahat, ahatL, dsqrt, X0

    def forward(self, A, Lpat, prep=None):
        """Values of L on Lpat (differentiable in the parameters)."""
        ahat, ahatL, dsqrt, X0 = prep if prep is not None else self.prepare(A, Lpat)
        H = Dense.apply(X0, None, self.W0, self.b0, True)
        for W, b in zip(self.Ws, self.bs):
            AH = sp.SpMM.apply(A.pattern, ahat, H)
            H = Dense.apply(H, AH, W, b, True)
        P = Dense.apply(H, None, self.Wp, None, False)
        t = SDDMM.apply(Lpat, P, H)
        F = Readout.apply(t, Lpat, ahatL, dsqrt)
        if self.form == "fsai":
            F = F * inverse_factor_scale(Lpat, dsqrt)
        return F


def inverse_factor_scale(Lpat, dsqrt):
    """Per-entry scale of the approximate-inverse mapping: 1/d_i on the
    diagonal, -1/d_i below it (d_i = dsqrt_i^2)."""
    n = Lpat.nrows
    rows = torch.repeat_interleave(torch.arange(n, device=dsqrt.device),
                                   (Lpat.rowptr[1:] - Lpat.rowptr[:-1]).long())
    sign = torch.where(rows == Lpat.colind.long(), 1.0, -1.0).to(dsqrt.dtype)
    return sign / (dsqrt * dsqrt)[rows]


# ----------------------------------------------------------------------
# Loss: residual history of a few PCG iterations (Section 4.3)
# ----------------------------------------------------------------------
def loss_weights(nit, gamma):
    w = np.array([gamma ** (nit - i) for i in range(1, nit + 1)])
    return w / w.sum()


class _PcgStart(torch.autograd.Function):
    """(rho_0, ||b||) with rho_0 = b.z_0 (b is data)."""

    @staticmethod
    def forward(ctx, b, z, ws):
        scal = torch.empty(2, dtype=torch.float64, device=b.device)
        capi.csr_pcgl_start(b, z.contiguous(), scal, ws)
        ctx.save_for_backward(b)
        return scal[0:1], scal[1:2]

    @staticmethod
    def backward(ctx, grho, gbn):
        (b,) = ctx.saved_tensors
        gz = torch.empty_like(b)
        capi.csr_pcgl_start_bwd(b, None, None if grho is None else grho.contiguous(), gz)
        return None, gz, None


class _PcgRes(torch.autograd.Function):
    """One iteration's update of r and of the loss accumulator (see
    csr_pcgl_res_fwd)."""

    @staticmethod
    def forward(ctx, p, q, r, rho, acc, w, bnorm, ws):
        r1 = torch.empty_like(r)
        scal = torch.empty(3, dtype=torch.float64, device=r.device)
        acc1 = torch.empty(1, dtype=torch.float64, device=r.device)
        capi.csr_pcgl_res_fwd(p, q, r, rho, w, bnorm, acc, r1, scal, acc1, ws)
        ctx.w, ctx.ws = w, ws
        ctx.save_for_backward(p, q, r1, rho, scal, bnorm)
        return r1, acc1

    @staticmethod
    def backward(ctx, gr1, gacc1):
        p, q, r1, rho, scal, bnorm = ctx.saved_tensors
        if gacc1 is None:
            gacc1 = torch.zeros(1, dtype=torch.float64, device=p.device)
        gr, gq, gp = torch.empty_like(r1), torch.empty_like(q), torch.empty_like(p)
        grho = torch.empty(1, dtype=torch.float64, device=p.device)
        capi.csr_pcgl_res_bwd(p, q, r1, rho, scal, ctx.w, bnorm,
                              None if gr1 is None else gr1.contiguous(), gacc1.contiguous(), gr,
                              gq, gp, grho, ctx.ws)
        return gp, gq, gr, grho, gacc1, None, None, None


class _PcgDir(torch.autograd.Function):
    """rho' = r'.z', p' = z' + (rho'/rho) p (see csr_pcgl_dir_fwd)."""

    @staticmethod
    def forward(ctx, r1, z1, rho, p, ws):
        z1 = z1.contiguous()
        rho1 = torch.empty(1, dtype=torch.float64, device=r1.device)
        p1 = torch.empty_like(p)
        capi.csr_pcgl_dir_fwd(r1, z1, rho, p, rho1, p1, ws)
        ctx.ws = ws
        ctx.save_for_backward(r1, z1, rho, p, rho1)
        return rho1, p1

    @staticmethod
    def backward(ctx, grho1, gp1):
        r1, z1, rho, p, rho1 = ctx.saved_tensors
        gr1, gz1, gp = torch.empty_like(r1), torch.empty_like(z1), torch.empty_like(p)
        grho = torch.empty(1, dtype=torch.float64, device=p.device)
        capi.csr_pcgl_dir_bwd(r1, z1, rho, p, rho1, None if gp1 is None else gp1.contiguous(),
                              None if grho1 is None else grho1.contiguous(), gr1, gz1, gp, grho,
                              ctx.ws)
        return gr1, gz1, grho, gp, None


def pcg_residual_loss(A, Lpat, Lv, b, nit=4, gamma=0.6, form="factor"):
    """sum_i w_i ||r_i|| / ||b|| over nit PCG iterations with M = L L^T.

    form "factor": M approximates A and z = L^{-T} L^{-1} r (two triangular
    solves); form "fsai": M approximates A^{-1}, the form Section 4.3
    learns, and z = L (L^T r) (two sparse products).  Every step runs in
    the library: the products and solves, and the iteration's dot
    products, updates and norms (csr_pcgl_*), each with its hand-written
    reverse; the result is a one-element float64 tensor."""
    def minv(r):
        if form == "fsai":
            return sp.SpMV.apply(Lpat, Lv, sp.SpMVT.apply(Lpat, Lv, r))
        return TriSolveT.apply(Lpat, Lv, sp.TriSolve.apply(Lpat, Lv, r, True))

    w = loss_weights(nit, gamma)
    b = b.contiguous()
    ws = capi._ws(capi.csr_pcgl_workspace(b.numel()), b.device)
    z = minv(b)
    rho, bnorm = _PcgStart.apply(b, z, ws)
    bnorm = bnorm.detach()
    acc = torch.zeros(1, dtype=torch.float64, device=b.device)
    r, p = b, z
    for i in range(nit):
        q = sp.SpMV.apply(A.pattern, A.vals, p)
        r, acc = _PcgRes.apply(p, q, r, rho, acc, float(w[i]), bnorm, ws)
        if i + 1 < nit:
            z = minv(r)
            rho, p = _PcgDir.apply(r, z, rho, p, ws)
    return acc[0]


# ----------------------------------------------------------------------
# Systems: anisotropic Q1 diffusion in 2x2 four-coloured order
# ----------------------------------------------------------------------
class Q1Family:
    """All systems of one grid size share the pattern; values depend on
    (eps, theta) through the nine stencil weights."""

    def __init__(self, N, device="cuda"):
        self.N = N
        base = gen.anisotropic_q1(N, 0.5, 0.3)  # any generic coefficients: pattern + types
        # stencil type of each entry: neighbour offset (dy, dx) -> 0..8
        rows = base.row_of_entry()
        iy, ix = np.divmod(rows, N)
        jy, jx = np.divmod(base.colind, N)
        dy, dx = jy - iy, jx - ix
        types = (dy + 1) * 3 + (dx + 1)
        perm = gen.four_color_2d(N)
        A4 = gen.permute_sym(gen.Csr(base.nrows, base.ncols, base.rowptr, base.colind,
                                     types.astype(np.float64)), perm)
        self.types = A4.vals.astype(np.int64)
        self.pattern_host = gen.Csr(A4.nrows, A4.ncols, A4.rowptr, A4.colind,
                                    np.zeros(A4.nnz))
        self.P = sp.Pattern.from_host(self.pattern_host, device)
        self.Lpat = sp.Pattern.from_host(gen.tril(self.pattern_host), device)
        self.device = device

    @staticmethod
    def weights(eps, theta):
        cs, sn = np.cos(theta), np.sin(theta)
        a = cs * cs + eps * sn * sn
        c = sn * sn + eps * cs * cs
        b = (1.0 - eps) * cs * sn
        w = np.zeros(9)
        # index (dy+1)*3 + (dx+1)
        w[4] = 4 * (a + c) / 3
        w[3] = w[5] = -2 * a / 3 + c / 3
        w[1] = w[7] = a / 3 - 2 * c / 3
        w[8] = w[0] = -(a + c) / 6 - b / 2
        w[6] = w[2] = -(a + c) / 6 + b / 2
        return w

    def system(self, eps, theta, dtype=torch.float32):
        v = self.weights(eps, theta)[self.types]
        return sp.CsrTensor(self.P, torch.as_tensor(v, device=self.device).to(dtype)), v

    @staticmethod
    def sample(rng):
        return 10.0 ** rng.uniform(-4.0, 0.0), rng.uniform(0.0, np.pi)


def held_out(fam, count, seed):
    """`count` systems of the family with their right-hand sides, drawn from
    default_rng([seed, j]) (float32 values, float64 b)."""
    out = []
    for j in range(count):
        rng = np.random.default_rng([seed, j])
        eps, theta = Q1Family.sample(rng)
        A, _ = fam.system(eps, theta)
        out.append((A, torch.as_tensor(rng.standard_normal(fam.P.nrows), device=fam.device)))
    return out


def mean_iterations(model, fam, systems, tol=1e-6):
    """Mean PCG iterations to tol with the network's factor."""
    from . import pcg as pcgmod

    its = []
    with torch.no_grad():
        for A, b in systems:
            L = sp.CsrTensor(fam.Lpat, model(A, fam.Lpat))
            _, info = pcgmod.pcg(A, b, getattr(model, "form", "factor"), L=L, tol=tol,
                                 fallback=False)
            its.append(info["iters"] if info["converged"] else float("inf"))
    return float(np.mean(its))


def train(model, N=256, steps=200, lr=1e-3, nit=4, gamma=0.6, seed=5, log_every=0, t_budget=None,
          val_systems=None, eval_every=50):
    """Adam on the residual-history loss over freshly drawn systems
    (eps log-uniform in [1e-4, 1], theta uniform in [0, pi], b ~ N(0,1)).

    With val_systems (a list of (A, b) of the same grid), the parameters
    are scored every eval_every steps (and before the first) by the mean
    PCG iterations to 1e-6 on those systems, and the best-scoring ones are
    kept (model selection on held-out systems; the untrained network is a
    candidate).  Returns the loss history."""
    import time

    fam = Q1Family(N, model.W0.device)
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    history = []
    best = None
    if val_systems is not None:
        best = (mean_iterations(model, fam, val_systems),
                {k: v.detach().clone() for k, v in model.state_dict().items()})
    t0 = time.time()
    for step in range(steps):
        rng = np.random.default_rng([seed, 0, step])
        eps, theta = Q1Family.sample(rng)
        A, _ = fam.system(eps, theta)
        b = torch.as_tensor(rng.standard_normal(fam.P.nrows), device=A.vals.device).float()
        opt.zero_grad()
        Lv = model(A, fam.Lpat)
        loss = pcg_residual_loss(A, fam.Lpat, Lv, b, nit, gamma,
                                 form=getattr(model, "form", "factor"))
        loss.backward()
        opt.step()
        history.append(float(loss.detach()))
        if log_every and step % log_every == 0:
            print(f"[train] step {step} loss {history[-1]:.4f}", flush=True)
        last = step + 1 == steps or (t_budget is not None and time.time() - t0 > t_budget)
        if val_systems is not None and ((step + 1) % eval_every == 0 or last):
            score = mean_iterations(model, fam, val_systems)
            if score < best[0]:
                best = (score, {k: v.detach().clone() for k, v in model.state_dict().items()})
        if last:
            break
    if best is not None:
        model.load_state_dict(best[1])
        model.selected_score = best[0]
    return history
