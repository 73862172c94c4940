"""Float64 CPU reference of the learned-preconditioner network and its
PCG residual-history loss (Section 4.3 loss).  TEST INFRASTRUCTURE ONLY.

Plain PyTorch CPU ops in float64, written from the equations, with
autograd providing reference gradients; no code is shared with the HIP
path.  The network's stated precision is bf16 operands with wide
accumulation, so with rounding=True every dense product X W rounds both
operands to bfloat16 and accumulates in float64, and its backward rounds
the incoming gradient G the same way (dX = r(G) r(W)^T, dW = r(X)^T r(G));
bias gradients, the message sums, the readout and the loss stay float64.
rounding=False gives the plain float64 network (finite-difference pins).

Equations (hidden width 32, three message-passing layers):
  d_i = A_ii, Ahat_ij = A_ij / sqrt(d_i d_j)
  X0_i = [1, sum_{j!=i} |Ahat_ij|, sum_{j!=i} Ahat_ij, (deg_i - 1)/8,
          sum_{j<i} Ahat_ij, sum_{j<i} |Ahat_ij|, #{j<i}/8,
          sum_{j>i} Ahat_ij, sum_{j>i} |Ahat_ij|, #{j>i}/8, 0 x 6]
  H0 = relu(X0 W0 + b0);  H_l = relu([H, Ahat H] W_l + b_l)
  P = H Wp;  t_ij = P_i . H_j on tril(A)
  L_ij = sqrt(d_i) Ahat_ij (1 + t_ij) (j < i),  L_ii = sqrt(d_i)(softplus(t_ii + c) + delta)
"""
from __future__ import annotations

import math

import numpy as np
import torch

C0 = math.log(math.e - 1.0)
DELTA = 1e-3


def bf16(w):
    return torch.as_tensor(np.asarray(w, np.float32)).to(torch.bfloat16).to(torch.float64)


def _r(t):
    """Round a float64 tensor to bfloat16 (through float32) and back."""
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


class _Bf16Product(torch.autograd.Function):
    """X @ W on bf16-rounded operands, float64 accumulation, both ways."""

    @staticmethod
    def forward(ctx, X, W):
        Xr, Wr = _r(X), _r(W)
        ctx.save_for_backward(Xr, Wr)
        return Xr @ Wr

    @staticmethod
    def backward(ctx, G):
        Xr, Wr = ctx.saved_tensors
        Gr = _r(G)
        return Gr @ Wr.T, Xr.T @ Gr


def _rows(rowptr):
    return torch.as_tensor(np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr)))


def prep(A, Lpat):
    """(ahat, ahatL, dsqrt, X0) as float64 tensors."""
    rows = _rows(A.rowptr)
    cols = torch.as_tensor(np.asarray(A.colind, np.int64))
    v = torch.as_tensor(np.asarray(A.vals, np.float64))
    n = A.nrows
    d = torch.zeros(n, dtype=torch.float64)
    diag = rows == cols
    d[rows[diag]] = v[diag]
    ahat = v / torch.sqrt(d[rows] * d[cols])
    off = ~diag
    s1 = torch.zeros(n, dtype=torch.float64).index_add_(0, rows[off], ahat[off].abs())
    s2 = torch.zeros(n, dtype=torch.float64).index_add_(0, rows[off], ahat[off])
    deg = torch.as_tensor(np.diff(A.rowptr), dtype=torch.float64)
    X0 = torch.zeros(n, 16, dtype=torch.float64)
    X0[:, 0] = 1.0
    X0[:, 1] = s1
    X0[:, 2] = s2
    X0[:, 3] = (deg - 1) / 8.0
    # where the node sits in the solve order: neighbours before / after it
    for k, m in ((4, cols < rows), (7, cols > rows)):
        X0[:, k] = torch.zeros(n, dtype=torch.float64).index_add_(0, rows[m], ahat[m])
        X0[:, k + 1] = torch.zeros(n, dtype=torch.float64).index_add_(0, rows[m], ahat[m].abs())
        X0[:, k + 2] = torch.zeros(n, dtype=torch.float64).index_add_(
            0, rows[m], torch.ones(int(m.sum()), dtype=torch.float64)) / 8.0
    # tril entries are the leading entries of each row
    key = {(int(r), int(c)): e for e, (r, c) in enumerate(zip(rows.tolist(), cols.tolist()))}
    Lrows = _rows(Lpat.rowptr)
    idx = torch.as_tensor([key[(int(r), int(c))] for r, c in zip(Lrows.tolist(), Lpat.colind)],
                          dtype=torch.int64)
    return ahat, ahat[idx], torch.sqrt(d), X0


def factor(A, Lpat, params, rounding=True):
    """L values on Lpat (float64, differentiable in the float64 copies of
    the parameters returned alongside; dense products on bf16-rounded
    operands unless rounding is False)."""
    cast = lambda w: torch.as_tensor(np.asarray(w, np.float64))
    mm = _Bf16Product.apply if rounding else torch.matmul
    p = {k: ([cast(w).clone().requires_grad_(True) for w in v] if isinstance(v, list)
             else cast(v).clone().requires_grad_(True)) for k, v in params.items()
         if k in ("W0", "Ws", "Wp")}
    b0 = torch.as_tensor(np.asarray(params["b0"], np.float64)).requires_grad_(True)
    bs = [torch.as_tensor(np.asarray(b, np.float64)).requires_grad_(True) for b in params["bs"]]
    ahat, ahatL, dsqrt, X0 = prep(A, Lpat)
    rows = _rows(A.rowptr)
    cols = torch.as_tensor(np.asarray(A.colind, np.int64))
    n = A.nrows

    def agg(H):
        return torch.zeros_like(H).index_add_(0, rows, ahat[:, None] * H[cols])

    H = torch.relu(mm(X0, p["W0"]) + b0)
    for W, b in zip(p["Ws"], bs):
        H = torch.relu(mm(torch.cat([H, agg(H)], dim=1), W) + b)
    P = mm(H, p["Wp"])
    Lr = _rows(Lpat.rowptr)
    Lc = torch.as_tensor(np.asarray(Lpat.colind, np.int64))
    t = (P[Lr] * H[Lc]).sum(1)
    off = Lc < Lr
    L = torch.where(off, dsqrt[Lr] * ahatL * (1 + t),
                    dsqrt[Lr] * (torch.nn.functional.softplus(t + C0) + DELTA))
    leaves = dict(W0=p["W0"], b0=b0, Ws=p["Ws"], bs=bs, Wp=p["Wp"])
    return L, leaves


def _dense_lower(Lpat, Lv, n):
    M = torch.zeros(n, n, dtype=torch.float64)
    M = M.index_put((_rows(Lpat.rowptr), torch.as_tensor(np.asarray(Lpat.colind, np.int64))), Lv)
    return M


def pcg_loss(A, Lpat, Lv, b, nit=4, gamma=0.6, form="factor"):
    """Residual-history loss of nit PCG iterations (dense float64; small
    systems only).  form "factor": M = L L^T approximates A, so the
    preconditioned residual is z = L^{-T} L^{-1} r (two triangular solves);
    form "fsai": M = L L^T approximates A^{-1} (Section 4.3), z = L L^T r."""
    n = A.nrows
    Ad = torch.as_tensor(A.todense())
    Ld = _dense_lower(Lpat, Lv, n)
    b = torch.as_tensor(np.asarray(b, np.float64))

    def minv(r):
        if form == "fsai":
            return Ld @ (Ld.T @ r)
        y = torch.linalg.solve_triangular(Ld, r[:, None], upper=False)
        return torch.linalg.solve_triangular(Ld.T, y, upper=True)[:, 0]

    w = np.array([gamma ** (nit - i) for i in range(1, nit + 1)])
    w = w / w.sum()
    x = torch.zeros(n, dtype=torch.float64)
    r = b.clone()
    z = minv(r)
    p = z
    rho = r @ z
    loss = 0.0
    bn = torch.linalg.norm(b)
    for i in range(nit):
        q = Ad @ p
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        loss = loss + float(w[i]) * torch.linalg.norm(r) / bn
        if i + 1 < nit:
            z = minv(r)
            rn = r @ z
            p = z + (rn / rho) * p
            rho = rn
    return loss
