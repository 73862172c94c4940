"""Graph convolution (Section 4.4) on the library's sparse kernels.

One layer computes X' = Dt^{-1/2} (A + I) Dt^{-1/2} X Theta + bias with
Dt the degree matrix of A + I, in the order of the paper's listing:
  d   = (row_sum(A) + 1)^{-1/2}     row_sum is the SpMV A 1
  Y   = d * (X Theta)                a dense GEMM, then a row scaling
  X'  = d * (A Y + Y) + bias         the SpMM A Y (its backward is A^T G
                                     over A's cached transpose)
A's values may be trainable (row_sum and the SpMM differentiate in them).

``GCN`` is the two-layer network of the section's experiment: ReLU after
the first layer, dropout between the layers, a sigmoid after the second,
cross-entropy over the labelled nodes, Adam with L2 regularisation.
"""
from __future__ import annotations

import numpy as np
import torch

from . import sparse as sp


def row_sum(A):
    """Row sums of a CsrTensor (the SpMV A 1)."""
    return A.row_sum()


class GCNConv(torch.nn.Module):
    def __init__(self, in_channels, out_channels, generator=None, device="cuda"):
        super().__init__()
        self.weights = torch.nn.Parameter(
            torch.randn(in_channels, out_channels, generator=generator).to(device)
            / np.sqrt(in_channels))
        self.bias = torch.nn.Parameter(torch.zeros(out_channels, device=device))

    def forward(self, graph, X, d=None):
        """graph: CsrTensor adjacency; d: precomputed (row_sum + 1)^{-1/2}."""
        if d is None:
            d = (row_sum(graph) + 1.0) ** -0.5
        Y = d[:, None] * (X @ self.weights)
        AY = sp.SpMM.apply(graph.pattern, graph.vals, Y.contiguous())
        return d[:, None] * (AY + Y) + self.bias


class GCN(torch.nn.Module):
    """Two GCN layers (hidden width 16 in the paper's experiment)."""

    def __init__(self, in_channels, hidden, classes, seed=0, dropout=0.5, device="cuda"):
        super().__init__()
        g = torch.Generator().manual_seed(seed)
        self.conv1 = GCNConv(in_channels, hidden, g, device)
        self.conv2 = GCNConv(hidden, classes, g, device)
        self.dropout = dropout

    def forward(self, graph, X, d=None):
        if d is None:
            d = (row_sum(graph) + 1.0) ** -0.5
        H = torch.relu(self.conv1(graph, X, d))
        H = torch.nn.functional.dropout(H, self.dropout, self.training)
        return torch.sigmoid(self.conv2(graph, H, d))


def train(model, graph, X, labels, train_mask, epochs=200, lr=0.01, weight_decay=5e-4):
    """Adam on the cross-entropy of the labelled nodes; the degree scaling
    is computed once (the graph is fixed).  Returns the loss history."""
    opt = torch.optim.Adam(model.parameters(), lr=lr, weight_decay=weight_decay)
    with torch.no_grad():
        d = (row_sum(graph) + 1.0) ** -0.5
    hist = []
    model.train()
    for _ in range(epochs):
        opt.zero_grad()
        out = model(graph, X, d)
        loss = torch.nn.functional.cross_entropy(out[train_mask], labels[train_mask])
        loss.backward()
        opt.step()
        hist.append(loss.detach())
    model.eval()
    return [float(v) for v in torch.stack(hist).cpu()]


def accuracy(model, graph, X, labels, mask):
    with torch.no_grad():
        pred = model(graph, X).argmax(dim=1)
    return float((pred[mask] == labels[mask]).float().mean())
