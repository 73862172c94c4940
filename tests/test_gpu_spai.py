"""GPU parity of the sparse approximate inverse by direct minimisation
(Section 4.6): loss and gradient against the float64 reference composed
from the oracle, the explicit gradient against autograd through the
CsrTensor operators (I - M @ A), and the paper's 8x8 experiment: from
M = mask(A), steepest descent reaches ||grad|| < 0.01 in about 20
iterations at the row-wise least-squares optimum."""
import numpy as np
import pytest
import torch

import oracle
from oracle import spai_ref
from paper_2212_05159_amd import gen
from paper_2212_05159_amd import sparse as sp
from paper_2212_05159_amd.spai import Spai

from _util import rel_err, to_dev, upcast

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build()


MATS = [("poisson12x10", lambda: gen.poisson2d(12, 10)),
        ("rand_ragged", lambda: gen.random_csr(300, 300, 0.02, seed=3, empty_rows=0.1)),
        ("q1_aniso", lambda: gen.anisotropic_q1(20, 1e-2, 0.5))]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("name,mk", MATS, ids=[m[0] for m in MATS])
def test_spai_loss_and_gradient_match_reference(name, mk, dtype):
    A = mk()
    Ao = upcast(A, dtype)
    Mv = np.asarray(gen.normal(A.nnz, seed=5), np.float64)
    if dtype == torch.float32:
        Mv = Mv.astype(np.float32).astype(np.float64)
    prob = Spai(sp.CsrTensor.from_host(A, dtype=dtype))
    loss, g = prob.loss_grad(to_dev(Mv, dtype))
    lo, go = spai_ref.loss_and_grad(Ao, Mv)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert abs(float(loss) - lo) <= tol * lo
    assert rel_err(g, go) <= tol


def test_spai_gradient_equals_autograd_through_operators():
    A = gen.poisson2d(10, 9)
    Ad = sp.CsrTensor.from_host(A, dtype=torch.float64)
    Mv = to_dev(0.2 * gen.normal(A.nnz, seed=6), torch.float64)
    _, g = Spai(Ad).loss_grad(Mv)
    n = A.nrows
    I = sp.CsrTensor.from_host(gen.Csr(n, n, np.arange(n + 1, dtype=np.int32),
                                       np.arange(n, dtype=np.int32), np.ones(n)),
                               dtype=torch.float64)
    M = sp.CsrTensor(Ad.pattern, Mv.clone().requires_grad_(True))
    R = I - M @ Ad
    (R.vals * R.vals).sum().backward()
    np.testing.assert_allclose(M.vals.grad.cpu().numpy(), g.cpu().numpy(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_paper_8x8_spai(dtype):
    A = gen.poisson2d(8, 8)
    prob = Spai(sp.CsrTensor.from_host(A, dtype=dtype))
    Mv, info = prob.solve(tol=0.01)
    lopt, _ = spai_ref.loss_and_grad(A, spai_ref.optimum(A))
    print(f"{info['iters']} iterations, loss {info['history'][0]:.1f} -> {info['loss']:.6f} "
          f"(least-squares optimum {lopt:.6f})")
    assert info["converged"] and info["history"][0] == 3032.0
    assert info["iters"] <= 30
    assert abs(info["loss"] - lopt) <= 1e-5 * lopt
    assert rel_err(Mv, spai_ref.optimum(A)) < 1e-3


def test_spai_64x64_float32_reaches_optimum():
    A = gen.poisson2d(64, 64)
    prob = Spai(sp.CsrTensor.from_host(A, dtype=torch.float32))
    _, info = prob.solve(tol=0.01, max_iter=200)
    lopt, _ = spai_ref.loss_and_grad(A, spai_ref.optimum(A))
    assert info["converged"]
    assert abs(info["loss"] - lopt) <= 1e-4 * lopt
