"""Pins of the oracle's preconditioned CG beyond its first step, with
preconditioners that are not a multiple of the identity.

Reference: the preconditioned conjugate-gradient iteration of Section 4.3
(Saad, Iterative Methods for Sparse Linear Systems, Algorithm 9.1), written
out densely with NumPy: M^{-1} is applied as an explicit dense operator
(Jacobi: D^{-1}; factor form: (L L^T)^{-1} through two dense triangular
solves; inverse form: L L^T as two dense products).  With a non-constant
diagonal or a general L, r.z is not proportional to r.r, so these runs
separate the step length beta = (r'.z')/(r.z) from any variant that takes
it from r.r -- a test below shows such a variant leaves the 1e-12 band at
once.

Tolerance: both sides run the same iteration in float64 on preconditioned
systems with kappa(M^{-1} A) below 100; they differ only in the summation
order of the products, so the residual histories (normalised to
||r_0|| = ||b||) agree to well under 1e-12 absolute over every step taken.
(Plain CG is left to the other CG pins: there r.z = r.r, and on the
variable-coefficient system its 80-odd steps come close to n, where the
loss of orthogonality makes the history itself rounding-sensitive.)
"""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_2212_05159_amd import gen


def _variable_diffusion(nx, ny, seed):
    """Five-point finite-volume diffusion -div(k grad u) with a random
    coefficient field k in [0.1, 10] on the cell faces (log-uniform) and a
    small shift; SPD with a strongly varying diagonal."""
    rng = np.random.default_rng(seed)
    kx = 10.0 ** rng.uniform(-1, 1, size=(ny, nx + 1))
    ky = 10.0 ** rng.uniform(-1, 1, size=(ny + 1, nx))
    n = nx * ny
    D = np.zeros((n, n))
    for iy in range(ny):
        for ix in range(nx):
            i = iy * nx + ix
            D[i, i] += kx[iy, ix] + kx[iy, ix + 1] + ky[iy, ix] + ky[iy + 1, ix] + 0.05
            if ix > 0:
                D[i, i - 1] = -kx[iy, ix]
            if ix < nx - 1:
                D[i, i + 1] = -kx[iy, ix + 1]
            if iy > 0:
                D[i, i - nx] = -ky[iy, ix]
            if iy < ny - 1:
                D[i, i + nx] = -ky[iy + 1, ix]
    r, c = np.nonzero(D)
    return gen._from_coo(n, n, r, c, D[r, c])


def _random_spd(n, seed):
    rng = np.random.default_rng(seed)
    M = (rng.random((n, n)) < 0.15) * rng.standard_normal((n, n))
    S = np.triu(M, 1)
    S = S + S.T
    S += np.diag(np.abs(S).sum(1) * rng.uniform(1.05, 4.0, n) + 0.1)
    r, c = np.nonzero(S)
    return gen._from_coo(n, n, r, c, S[r, c])


def _factor(A, orc, seed, pert=0.1):
    """A general lower factor for M = L L^T ~ A: IC(0) on tril(A) with each
    diagonal entry scaled by U(1 - pert, 1 + pert) and each off-diagonal one
    by 1 + pert N(0,1) (neither a Cholesky factor nor a scaled identity)."""
    rng = np.random.default_rng(seed)
    Lp = gen.tril(A)
    diag = Lp.colind == Lp.row_of_entry()
    lv = orc.ic0(A, Lp) * np.where(diag, rng.uniform(1 - pert, 1 + pert, Lp.nnz),
                                   1 + pert * rng.standard_normal(Lp.nnz))
    return gen.Csr(Lp.nrows, Lp.ncols, Lp.rowptr, Lp.colind, lv)


def _inverse_factor(A, seed, pert=0.3):
    """A general lower L for the inverse form M = L L^T ~ A^{-1}: the
    first-order inverse factor D^{-1}(D - A_L)D^{-1/2} on tril(A), i.e.
    L_ii = d_i^{-1/2}, L_ij = -A_ij / (d_i d_j^{1/2}), each entry perturbed
    as in _factor."""
    rng = np.random.default_rng(seed)
    Lp = gen.tril(A)
    rows = Lp.row_of_entry()
    diag = Lp.colind == rows
    d = A.todense().diagonal()
    lv = np.where(diag, 1.0 / np.sqrt(d[rows]), -Lp.vals / (d[rows] * np.sqrt(d[Lp.colind])))
    lv = lv * np.where(diag, rng.uniform(1 - pert, 1 + pert, Lp.nnz),
                       1 + pert * rng.standard_normal(Lp.nnz))
    return gen.Csr(Lp.nrows, Lp.ncols, Lp.rowptr, Lp.colind, lv)


def _prec(A, orc, mode):
    if mode == "factor":
        L = _factor(A, orc, 74)
    elif mode == "fsai":
        L = _inverse_factor(A, 75)
    else:
        return None, None
    return L, L.todense()


def _dense_pcg(Ad, b, apply_minv, tol, maxit, beta_from_rr=False):
    """Saad's Algorithm 9.1 with x_0 = 0 on dense arrays.  Returns the
    iterate and the history of ||r_t|| / ||b||."""
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_minv(r)
    p = z.copy()
    rz = r @ z
    bn = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bn]
    while hist[-1] > tol and len(hist) <= maxit:
        q = Ad @ p
        alpha = rz / (p @ q)
        x = x + alpha * p
        r_new = r - alpha * q
        z = apply_minv(r_new)
        rz_new = r_new @ z
        beta = (r_new @ r_new) / (r @ r) if beta_from_rr else rz_new / rz
        p = z + beta * p
        r, rz = r_new, rz_new
        hist.append(np.linalg.norm(r) / bn)
    return x, np.array(hist)


def _minv(mode, Ad, Ld):
    if mode == "jacobi":
        d = np.diag(Ad).copy()
        return lambda r: r / d
    if mode == "factor":
        return lambda r: sla.solve_triangular(Ld.T, sla.solve_triangular(Ld, r, lower=True),
                                              lower=False)
    if mode == "fsai":
        return lambda r: Ld @ (Ld.T @ r)
    return lambda r: r.copy()


def _systems():
    A1 = _variable_diffusion(10, 9, 71)
    A2 = _random_spd(70, 72)
    return [("variable-diffusion", A1), ("random-spd", A2)]


@pytest.mark.parametrize("name,A", _systems())
@pytest.mark.parametrize("mode", ["jacobi", "factor", "fsai"])
def test_pcg_histories_match_dense_algorithm(orc, name, A, mode):
    Ad = A.todense()
    d = np.diag(Ad)
    assert d.max() / d.min() > 3.0  # the diagonal is far from constant
    b = gen.normal(A.nrows, 73)
    L, Ld = _prec(A, orc, mode)
    tol = 1e-10
    x_or, it_or, h_or = orc.pcg(A, b, mode, L=L, tol=tol, maxit=500)
    x_ref, h_ref = _dense_pcg(Ad, b, _minv(mode, Ad, Ld), tol, 500)
    assert it_or == len(h_ref) - 1 and it_or > 10
    assert np.abs(h_or - h_ref).max() <= 1e-12
    assert np.linalg.norm(x_or - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
    assert np.linalg.norm(Ad @ x_or - b) <= 2 * tol * np.linalg.norm(b)


@pytest.mark.parametrize("mode", ["jacobi", "factor", "fsai"])
def test_dense_pin_separates_beta_from_rr(orc, mode):
    """The pin is sharp: a PCG that took beta from r.r (a plausible slip)
    differs from the oracle by far more than the 1e-12 band within a few
    steps, for each preconditioner with a non-scalar M."""
    A = _variable_diffusion(10, 9, 71)
    Ad = A.todense()
    b = gen.normal(A.nrows, 73)
    L, Ld = _prec(A, orc, mode)
    _, _, h_or = orc.pcg(A, b, mode, L=L, tol=1e-10, maxit=500)
    _, h_bad = _dense_pcg(Ad, b, _minv(mode, Ad, Ld), 1e-10, 500, beta_from_rr=True)
    k = min(len(h_or), len(h_bad), 6)
    assert np.abs(h_or[:k] - h_bad[:k]).max() > 1e-6
