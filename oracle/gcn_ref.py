"""Float64 CPU reference of the graph-convolution layer (Section 4.4).
TEST INFRASTRUCTURE ONLY.

The layer's equation written out densely with plain PyTorch CPU ops:
  X' = Dt^{-1/2} At Dt^{-1/2} X Theta + bias,  At = A + I,
  Dt = the diagonal of At's row sums (the degree matrix of At),
with autograd giving the reference gradients."""
from __future__ import annotations

import numpy as np
import torch


def dense(A):
    return torch.as_tensor(A.todense(), dtype=torch.float64)


def layer(Ad, X, Theta, bias):
    """Ad: dense float64 adjacency (n x n); X (n x C), Theta (C x F), bias (F)."""
    n = Ad.shape[0]
    At = Ad + torch.eye(n, dtype=torch.float64)
    d = At.sum(dim=1)
    Dm = torch.diag(d ** -0.5)
    return Dm @ At @ Dm @ X @ Theta + bias
