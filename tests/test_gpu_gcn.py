"""GPU parity of the graph-convolution layer (Section 4.4) against the
dense float64 reference (forward, and gradients to X, Theta, bias and the
adjacency values through autograd), and a semi-supervised training run of
the section's two-layer network on a synthetic graph: a random geometric
graph (about 5 incident edges per node) whose classes are spatial regions
and whose features are a noisy one-hot of the class; 20 labelled nodes per
class, as in the section's experiment."""
import numpy as np
import pytest
import torch

from oracle import gcn_ref
from paper_2212_05159_amd import gcn, gen
from paper_2212_05159_amd import sparse as sp

from _util import rel_err, to_dev

pytestmark = pytest.mark.gpu

def _weighted_symmetric(n, density, seed):
    """Symmetric random graph with positive weights and some isolated nodes."""
    R = gen.random_csr(n, n, density, seed=seed, empty_rows=0.1).todense()
    S = np.abs(R + R.T)
    np.fill_diagonal(S, 0.0)
    r, c = np.nonzero(S)
    return gen._from_coo(n, n, r, c, S[r, c])


GRAPHS = [("geo500", lambda: gen.geometric_graph(500, 4, seed=1)),
          ("rand_weighted", lambda: _weighted_symmetric(300, 0.02, 2))]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("name,mk", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_gcn_layer_matches_reference(name, mk, dtype):
    A = mk()
    n, C, F = A.nrows, 24, 7
    rng = np.random.default_rng(3)
    Xh, Wh, bh, Th = (rng.standard_normal(s) for s in ((n, C), (C, F), (F,), (n, F)))
    if dtype == torch.float32:
        Xh, Wh, bh, Th, vh = (a.astype(np.float32).astype(np.float64)
                              for a in (Xh, Wh, bh, Th, A.vals))
    else:
        vh = A.vals
    G = sp.CsrTensor(sp.Pattern.from_host(A), to_dev(vh, dtype).requires_grad_(True))
    layer = gcn.GCNConv(C, F, device="cuda").to(dtype)
    with torch.no_grad():
        layer.weights.copy_(to_dev(Wh, dtype))
        layer.bias.copy_(to_dev(bh, dtype))
    X = to_dev(Xh, dtype).requires_grad_(True)
    Y = layer(G, X)
    (Y * to_dev(Th, dtype)).sum().backward()

    Ah = gen.Csr(n, n, A.rowptr, A.colind, vh)
    Ad = gcn_ref.dense(Ah).requires_grad_(True)
    Xr, Wr, br = (torch.as_tensor(a).requires_grad_(True) for a in (Xh, Wh, bh))
    Yr = gcn_ref.layer(Ad, Xr, Wr, br)
    (Yr * torch.as_tensor(Th)).sum().backward()
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert rel_err(Y, Yr.detach().numpy()) < tol
    assert rel_err(X.grad, Xr.grad.numpy()) < tol
    assert rel_err(layer.weights.grad, Wr.grad.numpy()) < tol
    assert rel_err(layer.bias.grad, br.grad.numpy()) < tol
    rows = np.repeat(np.arange(n), np.diff(A.rowptr))
    assert rel_err(G.vals.grad, Ad.grad.numpy()[rows, A.colind]) < tol


def test_gcn_semi_supervised_training():
    n, classes, C = 3000, 6, 32
    A = gen.geometric_graph(n, 4, seed=5)
    y = gen.node_classes(A.points, classes, seed=6)
    rng = np.random.default_rng(7)
    Xh = 0.6 * np.eye(C)[y] + rng.standard_normal((n, C))
    train_idx = np.concatenate([rng.choice(np.flatnonzero(y == c), 20, replace=False)
                                for c in range(classes)])
    mask = np.zeros(n, bool)
    mask[train_idx] = True
    G = sp.CsrTensor.from_host(A)
    X = to_dev(Xh, torch.float32)
    labels = torch.as_tensor(y, device="cuda")
    tm = torch.as_tensor(mask, device="cuda")
    model = gcn.GCN(C, 16, classes, seed=0)
    hist = gcn.train(model, G, X, labels, tm, epochs=200)
    acc = gcn.accuracy(model, G, X, labels, ~tm)
    # the features alone: a linear read of the noisy one-hot
    feat_acc = float(np.mean(Xh[:, :classes].argmax(1)[~mask] == y[~mask]))
    print(f"loss {hist[0]:.3f} -> {hist[-1]:.3f}; test accuracy {acc:.3f} "
          f"(features alone {feat_acc:.3f}, chance {1 / classes:.3f})")
    assert hist[-1] < hist[0]
    assert acc > feat_acc + 0.2
