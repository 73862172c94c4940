"""GPU parity of the learned-preconditioner network against its float64
reference (oracle/mpnn_ref.py), and the gain it brings once trained.

The bf16 dense layers are held to 1e-2 (infinity-norm relative); with
inputs that are exact in bf16 (small integers, eighths) the matrix-core
products are exact, which pins the lane layout of the MFMA operands."""
import numpy as np
import pytest
import torch

from oracle import mpnn_ref
from paper_2212_05159_amd import gen
from paper_2212_05159_amd import learned
from paper_2212_05159_amd import pcg as pcgmod
from paper_2212_05159_amd import sparse as sp

from _util import rel_err, to_dev

pytestmark = pytest.mark.gpu


def _dense_ref(X, W, b, relu):
    Y = X @ W + (0 if b is None else b)
    return np.maximum(Y, 0) if relu else Y


@pytest.mark.parametrize("n,K1,K2", [(32, 16, 0), (1000, 32, 32), (77, 16, 0), (4099, 32, 32)])
def test_dense_layer_exact_lane_layout(n, K1, K2):
    rng = np.random.default_rng(n)
    X1 = rng.integers(-3, 4, (n, K1)).astype(np.float32)
    X2 = rng.integers(-3, 4, (n, K2)).astype(np.float32) if K2 else None
    W = (rng.integers(-8, 9, (K1 + K2, 32)) / 8).astype(np.float32)
    b = (rng.integers(-4, 5, 32) / 4).astype(np.float32)
    X = X1 if X2 is None else np.concatenate([X1, X2], 1)
    X1d = to_dev(X1).requires_grad_(True)
    X2d = to_dev(X2).requires_grad_(True) if X2 is not None else None
    Wd, bd = to_dev(W).requires_grad_(True), to_dev(b).requires_grad_(True)
    Y = learned.Dense.apply(X1d, X2d, Wd, bd, True)
    assert np.array_equal(Y.detach().cpu().numpy(), _dense_ref(X, W, b, True))
    G = (rng.integers(-2, 3, (n, 32)) / 2).astype(np.float32)
    Y.backward(to_dev(G))
    Gm = G * (_dense_ref(X, W, b, True) > 0)
    assert np.array_equal(Wd.grad.cpu().numpy(), X.T @ Gm)
    assert np.array_equal(bd.grad.cpu().numpy(), Gm.sum(0))
    dX = Gm @ W.T
    assert np.array_equal(X1d.grad.cpu().numpy(), dX[:, :K1])
    if X2 is not None:
        assert np.array_equal(X2d.grad.cpu().numpy(), dX[:, K1:])


def test_dense_layer_random_within_bf16_tolerance():
    rng = np.random.default_rng(1)
    n = 5000
    X1, X2 = rng.standard_normal((n, 32)), rng.standard_normal((n, 32))
    W, b = rng.standard_normal((64, 32)) / 8, rng.standard_normal(32) * 0.1
    Y = learned.Dense.apply(to_dev(X1, torch.float32), to_dev(X2, torch.float32),
                            to_dev(W, torch.float32), to_dev(b, torch.float32), False)
    assert rel_err(Y, _dense_ref(np.concatenate([X1, X2], 1), W, b, False)) < 1e-2


def test_sddmm_autograd():
    A = gen.random_csr(300, 300, 0.02, seed=2)
    S = sp.Pattern.from_host(A)
    rng = np.random.default_rng(3)
    P, H = rng.standard_normal((300, 32)), rng.standard_normal((300, 32))
    Pd = to_dev(P, torch.float64).requires_grad_(True)
    Hd = to_dev(H, torch.float64).requires_grad_(True)
    t = learned.SDDMM.apply(S, Pd, Hd)
    rows = A.row_of_entry()
    assert rel_err(t, (P[rows] * H[A.colind]).sum(1)) < 1e-12
    g = rng.standard_normal(A.nnz)
    t.backward(to_dev(g))
    Gd = np.zeros((300, 300))
    Gd[rows, A.colind] = g
    assert rel_err(Pd.grad, Gd @ H) < 1e-12
    assert rel_err(Hd.grad, Gd.T @ P) < 1e-12


def _params(seed, wp_scale):
    rng = np.random.default_rng(seed)
    return dict(W0=rng.standard_normal((16, 32)) / 4, b0=rng.standard_normal(32) * 0.1,
                Ws=[rng.standard_normal((64, 32)) / 8 for _ in range(3)],
                bs=[rng.standard_normal(32) * 0.1 for _ in range(3)],
                Wp=rng.standard_normal((32, 32)) * wp_scale)


def _load(model, prm):
    with torch.no_grad():
        model.W0.copy_(torch.as_tensor(prm["W0"]))
        model.b0.copy_(torch.as_tensor(prm["b0"]))
        for w, v in zip(model.Ws, prm["Ws"]):
            w.copy_(torch.as_tensor(v))
        for w, v in zip(model.bs, prm["bs"]):
            w.copy_(torch.as_tensor(v))
        model.Wp.copy_(torch.as_tensor(prm["Wp"]))


@pytest.mark.parametrize("N", [16, 40])
def test_network_and_loss_gradients_match_reference(N):
    fam = learned.Q1Family(N)
    A, vals = fam.system(3e-3, 0.9)
    Ah = gen.Csr(fam.pattern_host.nrows, fam.pattern_host.ncols, fam.pattern_host.rowptr,
                 fam.pattern_host.colind, vals.astype(np.float32).astype(np.float64))
    Lph = gen.tril(Ah)
    prm = _params(4, 0.05)
    model = learned.MPNN()
    _load(model, prm)
    b = np.random.default_rng(5).standard_normal(Ah.nrows)
    Lv = model(A, fam.Lpat)
    loss = learned.pcg_residual_loss(A, fam.Lpat, Lv, to_dev(b, torch.float32))
    loss.backward()
    # the reference rounds the operands of every dense product to bf16 as
    # the matrix cores do; the rest differs by float32 vs float64 arithmetic
    Lo, leaves = mpnn_ref.factor(Ah, Lph, prm)
    errs = {"L": rel_err(Lv, Lo.detach().numpy())}
    lo = mpnn_ref.pcg_loss(Ah, Lph, Lo, b)
    lo.backward()
    errs["loss"] = abs(float(loss.detach()) - float(lo.detach())) / abs(float(lo.detach()))
    for name in ("Wp", "W0", "b0"):
        errs[name] = rel_err(getattr(model, name).grad, leaves[name].grad.numpy())
    for l in range(3):
        errs[f"Ws{l}"] = rel_err(model.Ws[l].grad, leaves["Ws"][l].grad.numpy())
        errs[f"bs{l}"] = rel_err(model.bs[l].grad, leaves["bs"][l].grad.numpy())
    print("relative errors", {k: f"{v:.2e}" for k, v in errs.items()})
    assert all(v < 1e-2 for v in errs.values()), errs


def test_untrained_network_is_gauss_seidel_factor():
    fam = learned.Q1Family(24)
    A, vals = fam.system(1e-2, 0.3)
    model = learned.MPNN()
    with torch.no_grad():
        Lv = model(A, fam.Lpat)
    Ah = gen.Csr(fam.pattern_host.nrows, fam.pattern_host.ncols, fam.pattern_host.rowptr,
                 fam.pattern_host.colind, vals.astype(np.float32).astype(np.float64))
    T = gen.tril(Ah)
    rows = T.row_of_entry()
    d = np.zeros(T.nrows)
    d[rows[T.colind == rows]] = T.vals[T.colind == rows]
    want = np.where(T.colind < rows, T.vals / np.sqrt(d[T.colind]),
                    np.sqrt(d[rows]) * (1 + learned.DELTA))
    assert rel_err(Lv, want) < 1e-6


def test_prep_matches_reference():
    fam = learned.Q1Family(20)
    A, vals = fam.system(2e-2, 1.1)
    Ah = gen.Csr(fam.pattern_host.nrows, fam.pattern_host.ncols, fam.pattern_host.rowptr,
                 fam.pattern_host.colind, vals.astype(np.float32).astype(np.float64))
    ahat, ahatL, dsqrt, X0 = learned.MPNN().prepare(A, fam.Lpat)
    ro = mpnn_ref.prep(Ah, gen.tril(Ah))
    for got, want in zip((ahat, ahatL, dsqrt, X0), ro):
        assert rel_err(got, want.numpy()) < 1e-6


def _validation(fam, model, systems, nit):
    with torch.no_grad():
        return float(np.mean([float(learned.pcg_residual_loss(A, fam.Lpat, model(A, fam.Lpat),
                                                              b, nit)) for A, b in systems]))


@pytest.fixture(scope="module")
def trained_48():
    """Short training on 48x48 systems of the family and PCG iteration
    counts to 1e-6 on six held-out systems for the trained factor, the
    untrained (symmetric Gauss-Seidel) factor and Jacobi."""
    N, nit = 48, 6
    fam = learned.Q1Family(N)
    held = []
    for j in range(6):
        rng = np.random.default_rng([5, 1, j])
        eps, theta = learned.Q1Family.sample(rng)
        A, _ = fam.system(eps, theta)
        held.append((A, to_dev(rng.standard_normal(fam.P.nrows), torch.float32)))
    model, untrained = learned.MPNN(seed=1), learned.MPNN(seed=1)
    before = _validation(fam, model, held, nit)
    learned.train(model, N=N, steps=300, lr=3e-3, nit=nit, seed=7)
    after = _validation(fam, model, held, nit)
    its = {"trained": [], "untrained": [], "jacobi": []}
    for A, b in held:
        with torch.no_grad():
            for key, net in (("trained", model), ("untrained", untrained)):
                L = sp.CsrTensor(fam.Lpat, net(A, fam.Lpat).detach())
                _, info = pcgmod.pcg(A, b, "factor", L=L, tol=1e-6, fallback=False)
                assert info["converged"]
                its[key].append(info["iters"])
        _, info = pcgmod.pcg(A, b, "jacobi", tol=1e-6)
        its["jacobi"].append(info["iters"])
    print("held-out loss", before, "->", after, "iterations", its)
    return before, after, its


def test_training_lowers_held_out_loss_and_beats_jacobi(trained_48):
    # The residual-history loss the training minimises drops on held-out
    # systems of the family, and the trained factor needs fewer PCG
    # iterations to 1e-6 than Jacobi.
    before, after, its = trained_48
    assert after < 0.98 * before
    assert np.mean(its["trained"]) < np.mean(its["jacobi"])


@pytest.mark.xfail(strict=True, reason=(
    "training does not yet beat its own starting point in PCG iterations: in 2x2 four-coloured "
    "order the tril(A) factor family is at its ceiling at the symmetric Gauss-Seidel factor "
    "(exact IC(0) is only ~6% better), and at 1024^2 the trained factor took 1403 median "
    "iterations against 1387.5 untrained"))
def test_trained_factor_beats_untrained_factor(trained_48):
    # What training gains over the method without it: fewer PCG iterations
    # to 1e-6 on held-out systems than the untrained network's factor.
    _, _, its = trained_48
    assert np.mean(its["trained"]) < np.mean(its["untrained"])


@pytest.fixture(scope="module")
def trained_inverse_48():
    """The inverse form of Section 4.3 (M = L L^T ~ A^{-1}): short training
    on 48x48 systems with model selection on four validation systems, then
    PCG iteration counts on six other held-out systems for the trained
    network, the untrained one (the first-order inverse factor) and Jacobi."""
    N, nit = 48, 6
    fam = learned.Q1Family(N)
    held = learned.held_out(fam, 6, 61)
    val = learned.held_out(fam, 4, 62)
    model = learned.MPNN(seed=1, form="fsai")
    untrained = learned.MPNN(seed=1, form="fsai")
    learned.train(model, N=N, steps=400, lr=3e-3, nit=nit, seed=7, val_systems=val,
                  eval_every=50)
    its = {"trained": [], "untrained": [], "jacobi": []}
    for A, b in held:
        with torch.no_grad():
            for key, net in (("trained", model), ("untrained", untrained)):
                L = sp.CsrTensor(fam.Lpat, net(A, fam.Lpat).detach())
                _, info = pcgmod.pcg(A, b, "fsai", L=L, tol=1e-6, fallback=False)
                assert info["converged"]
                its[key].append(info["iters"])
        _, info = pcgmod.pcg(A, b, "jacobi", tol=1e-6)
        its["jacobi"].append(info["iters"])
    print("inverse form: validation", model.selected_score, "held-out iterations", its)
    return its


def test_training_gains_over_untrained_inverse_form(trained_inverse_48):
    # What training gains over the method without it, in the inverse form:
    # fewer PCG iterations to 1e-6 on held-out systems than the untrained
    # network's first-order inverse factor, and fewer than Jacobi.
    its = trained_inverse_48
    assert np.mean(its["trained"]) < np.mean(its["untrained"])
    assert np.mean(its["trained"]) < np.mean(its["jacobi"])
