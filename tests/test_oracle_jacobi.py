"""Pins for the dense reference of the entry-wise Jacobi example (Section
4.1): zero weights leave x unchanged (loss x^T A x); for a scalar weight
and an eigenvector v of A_N (D = 2I) the step scales v by 1 - omega
lambda / 2, so the loss is (1 - omega lambda / 2)^2 lambda ||v||^2; the
gradient matches central differences."""
import numpy as np
import torch

from oracle import jacobi_ref
from paper_2212_05159_amd import gen

N = 16


def _A():
    return torch.as_tensor(gen.poisson1d(N).todense())


def test_zero_weights_leave_x():
    A = _A()
    x = torch.as_tensor(gen.normal(N, seed=1))
    assert abs(float(jacobi_ref.step_loss(A, torch.zeros(N, dtype=torch.float64), x))
               - float(x @ (A @ x))) < 1e-13


def test_eigenvector_closed_form():
    A = _A()
    k = 3
    lam = 2.0 - 2.0 * np.cos(k * np.pi / (N + 1))
    v = torch.as_tensor(np.sin(k * np.pi * np.arange(1, N + 1) / (N + 1)))
    for omega in (0.5, 2.0 / 3.0, 1.0):
        got = float(jacobi_ref.step_loss(A, torch.full((N,), omega, dtype=torch.float64), v))
        want = (1.0 - omega * lam / 2.0) ** 2 * lam * float(v @ v)
        assert abs(got - want) < 1e-12 * max(1.0, want)


def test_gradient_matches_central_differences():
    A = _A()
    rng = np.random.default_rng(2)
    om = torch.as_tensor(0.5 + 0.3 * rng.random(N)).requires_grad_(True)
    x = torch.as_tensor(rng.standard_normal(N))
    jacobi_ref.step_loss(A, om, x).backward()
    h = 1e-6
    for i in (0, 7, 15):
        p, m = om.detach().clone(), om.detach().clone()
        p[i] += h
        m[i] -= h
        fd = (float(jacobi_ref.step_loss(A, p, x)) - float(jacobi_ref.step_loss(A, m, x))) / (2 * h)
        assert abs(fd - float(om.grad[i])) < 1e-8
