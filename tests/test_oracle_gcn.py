"""Pins for the dense graph-convolution reference (Section 4.4).

Independent checks: a graph without edges reduces the layer to
X Theta + bias; on a k-regular graph Dt^{-1/2} At Dt^{-1/2} = At/(k+1), so
a constant feature column stays constant and one node's output is the
mean of its closed neighbourhood (written out by hand for a cycle);
the propagation matrix is symmetric with largest eigenvalue 1 (its
eigenvector Dt^{1/2} 1); gradients match central differences."""
import numpy as np
import torch

from oracle import gcn_ref
from paper_2212_05159_amd import gen


def _cycle(n):
    i = np.arange(n)
    return gen._from_coo(n, n, np.concatenate([i, i]), np.concatenate([(i + 1) % n, (i - 1) % n]),
                         np.ones(2 * n))


def test_empty_graph_is_dense_layer():
    n, C, F = 7, 5, 3
    A = gen.Csr(n, n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    rng = np.random.default_rng(0)
    X, W, b = (torch.as_tensor(rng.standard_normal(s)) for s in ((n, C), (C, F), (F,)))
    np.testing.assert_allclose(gcn_ref.layer(gcn_ref.dense(A), X, W, b).numpy(),
                               (X @ W + b).numpy(), rtol=1e-14, atol=1e-14)


def test_cycle_is_closed_neighbourhood_mean():
    n = 9
    A = _cycle(n)
    rng = np.random.default_rng(1)
    X = torch.as_tensor(rng.standard_normal((n, 4)))
    I = torch.eye(4, dtype=torch.float64)
    Y = gcn_ref.layer(gcn_ref.dense(A), X, I, torch.zeros(4, dtype=torch.float64)).numpy()
    x = X.numpy()
    for i in range(n):
        want = (x[(i - 1) % n] + x[i] + x[(i + 1) % n]) / 3.0
        np.testing.assert_allclose(Y[i], want, rtol=1e-13, atol=1e-13)


def test_propagation_spectrum():
    A = gen.geometric_graph(60, 4, seed=2)
    n = A.nrows
    I = torch.eye(n, dtype=torch.float64)
    P = gcn_ref.layer(gcn_ref.dense(A), I, I, torch.zeros(n, dtype=torch.float64)).numpy()
    np.testing.assert_allclose(P, P.T, atol=1e-14)
    ev = np.linalg.eigvalsh(P)
    assert abs(ev[-1] - 1.0) < 1e-12 and ev[0] > -1.0
    v = np.sqrt(A.todense().sum(1) + 1.0)
    np.testing.assert_allclose(P @ v, v, rtol=1e-12)


def test_gradients_match_central_differences():
    A = gen.geometric_graph(25, 3, seed=3)
    rng = np.random.default_rng(4)
    Ad = gcn_ref.dense(A)
    X = torch.as_tensor(rng.standard_normal((25, 6))).requires_grad_(True)
    W = torch.as_tensor(rng.standard_normal((6, 4))).requires_grad_(True)
    b = torch.as_tensor(rng.standard_normal(4)).requires_grad_(True)
    T = torch.as_tensor(rng.standard_normal((25, 4)))
    (gcn_ref.layer(Ad, X, W, b) * T).sum().backward()
    h = 1e-6
    for t, idx in ((X, (3, 2)), (W, (5, 1)), (b, (2,))):
        with torch.no_grad():
            t[idx] += h
            fp = float((gcn_ref.layer(Ad, X, W, b) * T).sum())
            t[idx] -= 2 * h
            fm = float((gcn_ref.layer(Ad, X, W, b) * T).sum())
            t[idx] += h
        assert abs((fp - fm) / (2 * h) - float(t.grad[idx])) < 1e-7
