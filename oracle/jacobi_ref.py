"""Float64 CPU reference of the entry-wise weighted Jacobi example
(Section 4.1).  TEST INFRASTRUCTURE ONLY.

Dense PyTorch CPU ops written from the equations: one relaxation step with
a zero right-hand side, g(x; Omega) = (I - Omega D^{-1} A) x, and the loss
g^T A g for a test vector x; autograd gives the gradient in the weights."""
from __future__ import annotations

import torch


def step_loss(Ad, omega, x):
    """Ad: dense float64 A; omega: weights (n); x: test vector (n)."""
    n = Ad.shape[0]
    Dinv = torch.diag(1.0 / torch.diagonal(Ad))
    g = (torch.eye(n, dtype=torch.float64) - torch.diag(omega) @ Dinv @ Ad) @ x
    return g @ (Ad @ g)
