"""GPU parity for sparse + sparse (Section 3.1.4; Table 1, Sp + Sp rows).

Both sides evaluate alpha A_ij + beta B_ij (and alpha V_ij, beta V_ij) in
float64 with each product and the sum rounded separately; the GPU rounds
that once more to the value type.  So the union pattern must match the
oracle bit for bit, float64 values and gradients too, and float32 values
must equal the oracle's float64 results rounded to float32."""
import numpy as np
import pytest
import torch

import oracle
from paper_2212_05159_amd import capi, gen
from paper_2212_05159_amd import sparse as sp

from _util import rounded, to_dev, upcast

pytestmark = pytest.mark.gpu
DTYPES = [torch.float32, torch.float64]


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build()


def _pairs():
    # (name, A, B): row lengths chosen to hit every lane count (4..64),
    # rows longer than one chunk, empty rows and ragged grid tails.
    yield "rand_ragged", gen.random_csr(777, 523, 0.01, seed=1, empty_rows=0.2), \
        gen.random_csr(777, 523, 0.012, seed=2, empty_rows=0.3)
    yield "lanes16", gen.random_csr(1000, 900, 0.012, seed=3), gen.random_csr(1000, 900, 0.01, seed=4)
    yield "lanes32", gen.random_csr(333, 700, 0.04, seed=5), gen.random_csr(333, 700, 0.03, seed=6)
    yield "lanes64_long", gen.random_csr(70, 600, 0.4, seed=7, empty_rows=0.1), \
        gen.random_csr(70, 600, 0.3, seed=8)
    yield "long_rows", gen.random_csr(300, 4000, 0.001, seed=9, long_rows=3, long_len=3000), \
        gen.random_csr(300, 4000, 0.002, seed=10, long_rows=2, long_len=2500)
    P = gen.poisson3d(12)
    yield "poisson_plus_random", P, gen.random_rows(P.nrows, P.ncols, 7, seed=11)
    yield "poisson_minus_identity", P, gen._from_coo(P.nrows, P.ncols, np.arange(P.nrows),
                                                     np.arange(P.nrows), np.ones(P.nrows))
    yield "same_pattern", P, gen.Csr(P.nrows, P.ncols, P.rowptr, P.colind,
                                     gen.normal(P.nnz, seed=12))
    yield "one", gen.random_csr(1, 1, 1.0, seed=13), gen.random_csr(1, 1, 0.0, seed=14)
    yield "A_empty", gen.random_csr(50, 40, 0.0, seed=15), gen.random_csr(50, 40, 0.1, seed=16)
    yield "both_empty", gen.random_csr(9, 7, 0.0, seed=17), gen.random_csr(9, 7, 0.0, seed=18)


PAIRS = list(_pairs())
COEFS = [(1.0, 1.0), (0.75, -1.3), (2.0, 0.0)]


def _exact(gpu, ref, dtype, what):
    g = gpu.detach().cpu().numpy()
    r = np.asarray(ref)
    if dtype == torch.float32:
        r = r.astype(np.float32)
    assert g.shape == r.shape, what
    bad = np.flatnonzero(g != r)
    assert bad.size == 0, f"{what}: {bad.size} mismatches, first at {bad[:5]}"


def _run(A, B, alpha, beta, dtype, seed=0):
    Ad = sp.CsrTensor.from_host(A, dtype=dtype)
    Bd = sp.CsrTensor.from_host(B, dtype=dtype)
    Cp, vC = sp.spadd(Ad.pattern, Ad.vals, Bd.pattern, Bd.vals, alpha, beta)
    Ao, Bo = upcast(A, dtype), upcast(B, dtype)
    rp, ci, vo = oracle.spadd(Ao, Bo, alpha, beta)
    np.testing.assert_array_equal(Cp.rowptr.cpu().numpy(), rp)
    np.testing.assert_array_equal(Cp.colind.cpu().numpy(), ci)
    _exact(vC, vo, dtype, "vals")
    gC = rounded(gen.normal(len(ci), seed=seed + 99), dtype)
    gA, gB = sp.spadd_bwd(Ad.pattern, Bd.pattern, Cp, to_dev(gC, dtype), alpha, beta)
    gAo, gBo = oracle.spadd_bwd(Ao, Bo, rp, ci, gC, alpha, beta)
    _exact(gA, gAo, dtype, "gA")
    _exact(gB, gBo, dtype, "gB")
    return Ad, Bd, Cp


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("alpha,beta", COEFS)
@pytest.mark.parametrize("name,A,B", PAIRS, ids=[p[0] for p in PAIRS])
def test_spadd_fwd_bwd(name, A, B, alpha, beta, dtype):
    _run(A, B, alpha, beta, dtype)


def test_spadd_values_only_second_call():
    """A repeated sum reuses the cached union pattern (no column write)."""
    A = gen.random_csr(500, 400, 0.02, seed=20)
    B = gen.random_csr(500, 400, 0.02, seed=21)
    Ad, Bd, Cp = _run(A, B, 1.0, -0.5, torch.float32)
    v3 = A.vals.astype(np.float32) * np.float32(3.0)
    Cp2, v2 = sp.spadd(Ad.pattern, to_dev(v3), Bd.pattern, Bd.vals, 1.0, -0.5)
    assert Cp2 is Cp
    A3 = gen.Csr(A.nrows, A.ncols, A.rowptr, A.colind, v3.astype(np.float64))
    _, _, vo = oracle.spadd(A3, upcast(B, torch.float32), 1.0, -0.5)
    _exact(v2, vo, torch.float32, "vals")


def test_spadd_gradients_through_autograd():
    """The Jacobi example's tridiagonal, assembled from shifted identities
    with operators: 2 I - I_{+1} - I_{-1}, then a loss on its values."""
    N = 300

    def eye(k):
        i = np.arange(max(0, -k), min(N, N - k))
        return gen._from_coo(N, N, i, i + k, np.ones(len(i)))

    I0, Ip, Im = (sp.CsrTensor.from_host(eye(k), requires_grad=True) for k in (0, 1, -1))
    T = I0 * 2.0 - Ip - Im
    ref = gen.poisson1d(N)
    np.testing.assert_array_equal(T.pattern.colind.cpu().numpy(), ref.colind)
    np.testing.assert_array_equal(T.vals.detach().cpu().numpy(), ref.vals.astype(np.float32))
    w = to_dev(gen.normal(T.pattern.nnz, seed=5), torch.float32)
    (T.vals * w).sum().backward()
    wn = w.cpu().numpy().astype(np.float64)
    rp, ci = ref.rowptr, ref.colind
    # d loss / d I_k values: the coefficient of I_k (2, -1, -1) times w at (i, i+k)
    for Ik, k, coef in ((I0, 0, 2.0), (Ip, 1, -1.0), (Im, -1, -1.0)):
        rows = np.arange(max(0, -k), min(N, N - k))
        pos = np.array([rp[i] + np.searchsorted(ci[rp[i]:rp[i + 1]], i + k) for i in rows])
        np.testing.assert_array_equal(Ik.vals.grad.cpu().numpy(), (coef * wn[pos]).astype(np.float32))


def test_spadd_full_size_poisson128_plus_random7():
    """The measured workload at full size: 3D 7-point Poisson 128^3 plus a
    random pattern with 7 draws per row, C = A - 0.5 B in float32."""
    A = gen.poisson3d(128)
    B = gen.random_rows(A.nrows, A.ncols, 7, seed=2)
    _run(A, B, 1.0, -0.5, torch.float32, seed=3)


def test_spadd_argument_errors():
    A = sp.CsrTensor.from_host(gen.random_csr(10, 12, 0.2, seed=1))
    B = sp.CsrTensor.from_host(gen.random_csr(10, 13, 0.2, seed=2))
    with pytest.raises(ValueError):
        sp.spadd(A.pattern, A.vals, B.pattern, B.vals)
    dA, dB = A.pattern.desc(A.vals), B.pattern.desc(B.vals)
    with pytest.raises(capi.CsradError):
        capi.csr_spadd_workspace(dA, dB)
