"""Pins for the float64 reference of the learned-preconditioner network and
its PCG loss (CPU): the zero-readout network is the closed-form symmetric
Gauss-Seidel factor, an exact factor drives the loss to zero, the loss
weights follow gamma^(Nit-i), and autograd gradients agree with central
differences."""
import numpy as np
import torch

from oracle import mpnn_ref
from paper_2212_05159_amd import gen


def _params(seed, wp_scale=0.0):
    rng = np.random.default_rng(seed)
    return dict(W0=rng.standard_normal((16, 32)) / 4, b0=rng.standard_normal(32) * 0.1,
                Ws=[rng.standard_normal((64, 32)) / 8 for _ in range(3)],
                bs=[rng.standard_normal(32) * 0.1 for _ in range(3)],
                Wp=rng.standard_normal((32, 32)) * wp_scale)


def _system(N=8, eps=1e-2, theta=0.4):
    A = gen.permute_sym(gen.anisotropic_q1(N, eps, theta), gen.four_color_2d(N))
    return A, gen.tril(A)


def test_zero_readout_is_symmetric_gauss_seidel():
    A, Lp = _system()
    L, _ = mpnn_ref.factor(A, Lp, _params(0, 0.0))
    rows = Lp.row_of_entry()
    d = np.zeros(A.nrows)
    d[rows[Lp.colind == rows]] = Lp.vals[Lp.colind == rows]
    # (D + strict lower) D^{-1/2}: entry (i,j) -> A_ij / sqrt(d_j), diagonal sqrt(d_i)(1 + delta)
    want = np.where(Lp.colind < rows, Lp.vals / np.sqrt(d[Lp.colind]),
                    np.sqrt(d[rows]) * (1.0 + mpnn_ref.DELTA))
    np.testing.assert_allclose(L.detach().numpy(), want, rtol=1e-12)


def test_exact_factor_gives_zero_loss():
    A, _ = _system(6)
    r, c = np.nonzero(np.ones((A.nrows, A.nrows)))
    Ad = A.todense()
    Lfull = np.linalg.cholesky(Ad)
    Lp = gen.tril(gen._from_coo(A.nrows, A.nrows, r, c, Ad[r, c]))
    Lv = torch.as_tensor(Lfull[Lp.row_of_entry(), Lp.colind])
    loss = mpnn_ref.pcg_loss(A, Lp, Lv, np.random.default_rng(1).standard_normal(A.nrows))
    assert float(loss) < 1e-12


def test_loss_gradients_match_central_differences():
    A, Lp = _system(6)
    prm = _params(2, 0.05)
    b = np.random.default_rng(3).standard_normal(A.nrows)
    L, leaves = mpnn_ref.factor(A, Lp, prm, rounding=False)
    loss = mpnn_ref.pcg_loss(A, Lp, L, b)
    loss.backward()
    h = 1e-6
    for name, idx in [("Wp", (0, 0)), ("Wp", (3, 7)), ("W0", (1, 5)), ("b0", (4,))]:
        g = leaves[name].grad.numpy()[idx]
        vals = []
        for s in (+1, -1):
            q = {k: ([w.copy() for w in v] if isinstance(v, list) else np.array(v, copy=True))
                 for k, v in prm.items()}
            q[name][idx] += s * h
            Lq, _ = mpnn_ref.factor(A, Lp, q, rounding=False)
            vals.append(float(mpnn_ref.pcg_loss(A, Lp, Lq.detach(), b)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g) < 1e-6 * max(1.0, abs(fd)), (name, idx, fd, g)


def test_bf16_product_is_plain_product_on_bf16_exact_inputs():
    # Operands and gradient exact in bf16 (small integers over powers of
    # two): rounding is the identity, so the rounded product and its
    # gradients must equal the plain float64 product's (pins the operand
    # order and transposes of the backward).
    rng = np.random.default_rng(0)
    X = torch.tensor(rng.integers(-8, 9, (7, 5)) / 4.0, requires_grad=True)
    W = torch.tensor(rng.integers(-8, 9, (5, 3)) / 8.0, requires_grad=True)
    G = torch.tensor(rng.integers(-4, 5, (7, 3)) / 2.0)
    Y = mpnn_ref._Bf16Product.apply(X, W)
    Y.backward(G)
    assert torch.equal(Y, X.detach() @ W.detach())
    assert torch.equal(X.grad, G @ W.detach().T)
    assert torch.equal(W.grad, X.detach().T @ G)
    # and a value off the bf16 grid is rounded (8 significant bits)
    x = torch.tensor([[1.0 + 2.0 ** -10]], requires_grad=True)
    assert float(mpnn_ref._Bf16Product.apply(x, torch.ones(1, 1)).detach()) == 1.0


def test_node_inputs_by_hand():
    # tridiag(-1, 2, -1) on 3 nodes: every off-diagonal scaled entry is
    # -1/sqrt(2*2) = -1/2; the lower/upper split follows the row order.
    A = gen._from_coo(3, 3, [0, 0, 1, 1, 1, 2, 2], [0, 1, 0, 1, 2, 1, 2],
                      [2.0, -1.0, -1.0, 2.0, -1.0, -1.0, 2.0])
    _, _, dsqrt, X0 = mpnn_ref.prep(A, gen.tril(A))
    h = -0.5
    want = np.array([
        [1, 0.5, h, 1 / 8, 0, 0, 0, h, 0.5, 1 / 8],
        [1, 1.0, 2 * h, 2 / 8, h, 0.5, 1 / 8, h, 0.5, 1 / 8],
        [1, 0.5, h, 1 / 8, h, 0.5, 1 / 8, 0, 0, 0],
    ])
    assert np.allclose(X0[:, :10].numpy(), want, rtol=0, atol=1e-15)
    assert np.all(X0[:, 10:].numpy() == 0)
    assert np.allclose(dsqrt.numpy(), np.sqrt(2.0))
