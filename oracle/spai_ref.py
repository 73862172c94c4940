"""Float64 CPU reference of the sparse approximate inverse by direct
minimisation (Section 4.6).  TEST INFRASTRUCTURE ONLY.

The loss l(M) = ||I - M A||_F^2 over the stored values of M, with
mask(M) = mask(A), and its gradient are composed from the oracle's pinned
sparse routines in the order the definition reads: C = M A (SpSpMM),
R = I - C (Sp + Sp), l = sum of R's squared values; the VJP runs back
through Sp + Sp and SpSpMM.  The optimum comes from the row-wise split of
the loss that the section states: row i of I - M A is e_i^T - m_i^T A, so
each row of M solves its own dense least-squares problem over the columns
that mask(A) allows in that row."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2212_05159_amd import gen


def _identity(n):
    return gen.Csr(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                   np.ones(n))


def loss_and_grad(A, Mv):
    """(loss, gradient on mask(A)) for M with A's pattern and values Mv."""
    n = A.nrows
    M = gen.Csr(n, n, A.rowptr, A.colind, np.asarray(Mv, np.float64))
    rpC, ciC, vC = oracle.spgemm(M, A)
    C = gen.Csr(n, n, rpC, ciC, vC)
    rpR, ciR, vR = oracle.spadd(_identity(n), C, 1.0, -1.0)
    loss = float(np.sum(vR * vR))
    _, gC = oracle.spadd_bwd(_identity(n), C, rpR, ciR, 2.0 * vR, 1.0, -1.0, want_A=False)
    gM, _ = oracle.spgemm_bwd(M, A, rpC, ciC, gC, want_B=False)
    return loss, gM


def optimum(A):
    """Values of the minimiser on mask(A), row by row by dense least squares."""
    n = A.nrows
    Ad = A.todense()
    out = np.empty(A.nnz)
    for i in range(n):
        S = A.colind[A.rowptr[i]:A.rowptr[i + 1]]
        e = np.zeros(n)
        e[i] = 1.0
        x, *_ = np.linalg.lstsq(Ad[S, :].T, e, rcond=None)
        out[A.rowptr[i]:A.rowptr[i + 1]] = x
    return out
