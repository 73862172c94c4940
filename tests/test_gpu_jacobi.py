"""The entry-wise weighted Jacobi example (Section 4.1) written with the
library's operator forms, as in the paper's listing: A = 2 I - I_{+1} -
I_{-1}, D^{-1} = diag(1 / diagonal(A)), Omega = diag(omega), one relaxation
step g = (I - Omega D^{-1} A) x (the section's equation; SpSpMM, Sp + Sp and
SpMV with their VJPs), loss g^T A g.  Checked against the dense float64
reference: the loss and its gradient in omega, and 300 Adam steps (lr
1e-2, one seeded unit test vector per step), whose weights must agree and
show the section's pattern (end nodes weighted highest, interior near
2/3)."""
import numpy as np
import pytest
import torch

from oracle import jacobi_ref
from paper_2212_05159_amd import gen
from paper_2212_05159_amd import sparse as sp

pytestmark = pytest.mark.gpu
N = 16


def _setup():
    dt = torch.float64
    A = sp.eye(N, dtype=dt) * 2.0 - sp.eye(N, k=1, dtype=dt) - sp.eye(N, k=-1, dtype=dt)
    I = sp.eye(N, dtype=dt)
    Dinv = sp.diag(1.0 / A.diagonal())
    return A, I, Dinv


def _loss(A, I, Dinv, omega, x):
    Omega = sp.diag(omega)
    g = (I - Omega @ Dinv @ A) @ x
    return g @ (A @ g)


def test_operator_forms_build_the_1d_matrix():
    A, I, Dinv = _setup()
    ref = gen.poisson1d(N)
    np.testing.assert_array_equal(A.pattern.rowptr.cpu().numpy(), ref.rowptr)
    np.testing.assert_array_equal(A.pattern.colind.cpu().numpy(), ref.colind)
    np.testing.assert_array_equal(A.vals.cpu().numpy(), ref.vals)
    np.testing.assert_array_equal(Dinv.vals.cpu().numpy(), np.full(N, 0.5))
    np.testing.assert_array_equal(A.row_sum().cpu().numpy(), ref.todense().sum(1))


def test_jacobi_loss_and_gradient_match_reference():
    A, I, Dinv = _setup()
    rng = np.random.default_rng(3)
    om = 0.5 + 0.4 * rng.random(N)
    x = rng.standard_normal(N)
    omega = torch.as_tensor(om, device="cuda").requires_grad_(True)
    loss = _loss(A, I, Dinv, omega, torch.as_tensor(x, device="cuda"))
    loss.backward()
    omr = torch.as_tensor(om).requires_grad_(True)
    lr_ = jacobi_ref.step_loss(torch.as_tensor(gen.poisson1d(N).todense()), omr, torch.as_tensor(x))
    lr_.backward()
    assert abs(float(loss) - float(lr_)) <= 1e-13 * abs(float(lr_))
    np.testing.assert_allclose(omega.grad.cpu().numpy(), omr.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_jacobi_training_matches_reference():
    A, I, Dinv = _setup()
    Ad = torch.as_tensor(gen.poisson1d(N).todense())
    omega = torch.ones(N, dtype=torch.float64, device="cuda", requires_grad=True)
    omr = torch.ones(N, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([omega], lr=1e-2)
    optr = torch.optim.Adam([omr], lr=1e-2)
    rng = np.random.default_rng(0)
    for _ in range(300):
        x = rng.standard_normal(N)
        x /= np.linalg.norm(x)
        opt.zero_grad()
        _loss(A, I, Dinv, omega, torch.as_tensor(x, device="cuda")).backward()
        opt.step()
        optr.zero_grad()
        jacobi_ref.step_loss(Ad, omr, torch.as_tensor(x)).backward()
        optr.step()
    w = omega.detach().cpu().numpy()
    np.testing.assert_allclose(w, omr.detach().numpy(), atol=1e-8)
    print("weights", np.round(w, 3))
    interior = w[1:-1]
    assert min(w[0], w[-1]) > interior.max()
    assert 0.5 < interior.mean() < 0.75
