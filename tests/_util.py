"""Shared helpers for the GPU parity tests (no method arithmetic of their
own: residual checks and rounding bands call the oracle)."""
import numpy as np
import torch

from paper_2212_05159_amd import gen

# Float32 bar: infinity-norm relative error max|gpu - ref| / max|ref| per
# output array against the float64 oracle on the same (exactly upcast)
# inputs.  Float64 runs are held to 1e-12.
TOL = {torch.float32: 1e-5, torch.float64: 1e-12}


def rel_err(gpu, ref):
    g = np.asarray(gpu.detach().double().cpu().numpy() if torch.is_tensor(gpu) else gpu, np.float64)
    r = np.asarray(ref, np.float64)
    if r.size == 0:
        assert g.size == 0
        return 0.0
    scale = np.abs(r).max()
    diff = np.abs(g - r).max()
    return float(diff / scale) if scale > 0 else float(diff)


def assert_close(gpu, ref, dtype, what=""):
    e = rel_err(gpu, ref)
    assert e <= TOL[dtype], f"{what}: rel err {e:.3e} > {TOL[dtype]:.0e}"


def to_dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def upcast(m, dtype):
    """The matrix as the GPU sees it (values rounded to dtype), in float64."""
    return gen.Csr(m.nrows, m.ncols, m.rowptr, m.colind,
                   m.vals.astype(np.float32).astype(np.float64) if dtype == torch.float32 else m.vals)


def rounded(a, dtype):
    a = np.asarray(a)
    return a.astype(np.float32).astype(np.float64) if dtype == torch.float32 else a.astype(np.float64)


def true_residual(A_host, x, b):
    """||b - A x|| / ||b|| on the host, A x by the float64 oracle."""
    import oracle

    xs = np.asarray(x.detach().cpu().numpy() if torch.is_tensor(x) else x, np.float64)
    bs = np.asarray(b.detach().cpu().numpy() if torch.is_tensor(b) else b, np.float64)
    return float(np.linalg.norm(bs - oracle.spmv(A_host, xs)) / np.linalg.norm(bs))


def pcg_rounding_band(A_host, b, mode, L=None, tol=1e-8, trials=3, seed=0, maxit=10000):
    """How far the oracle's own PCG moves when its right-hand side is
    perturbed at the level of float64 rounding (each entry times
    1 + 2^-52 xi, xi ~ N(0,1)): per history entry and for x, the largest
    deviation over a few perturbations, plus the spread of the iteration
    counts.  A GPU run takes every sum in another order, which perturbs the
    iteration by the same order of magnitude at every step; this band is the
    problem's own sensitivity to such perturbations."""
    import oracle

    b = np.asarray(b, np.float64)
    x0, it0, h0 = oracle.pcg(A_host, b, mode, L=L, tol=tol, maxit=maxit)
    rng = np.random.default_rng(seed)
    hb = np.zeros(len(h0))
    xb = 0.0
    its = [it0]
    for _ in range(trials):
        bp = b * (1.0 + 2.0 ** -52 * rng.standard_normal(b.shape))
        x1, it1, h1 = oracle.pcg(A_host, bp, mode, L=L, tol=tol, maxit=maxit)
        m = min(len(h0), len(h1))
        hb[:m] = np.maximum(hb[:m], np.abs(h1[:m] - h0[:m]))
        xb = max(xb, float(np.abs(x1 - x0).max() / np.abs(x0).max()))
        its.append(it1)
    return {"x": x0, "iters": it0, "hist": h0, "hist_band": hb, "x_band": xb,
            "iter_spread": max(its) - min(its)}


def assert_pcg_f64_parity(info, x, ref, what=""):
    """The float64 PCG bar: every history entry within 10x the oracle's own
    rounding band plus 1e-12 (the history is normalised so that entry 0 is
    1), x within 10x its band plus 1e-12 relative, and the step count
    within one step plus the band's spread."""
    assert abs(info["iters"] - ref["iters"]) <= 1 + ref["iter_spread"], (what, info["iters"],
                                                                       ref["iters"])
    m = min(info["iters"], ref["iters"])
    got = np.asarray(info["hist"][:m])
    want = ref["hist"][1:m + 1]
    band = 10.0 * ref["hist_band"][1:m + 1] + 1e-12
    bad = np.nonzero(np.abs(got - want) > band)[0]
    assert bad.size == 0, (f"{what}: history differs beyond the rounding band at steps "
                           f"{bad[:5] + 1}: {np.abs(got - want)[bad[:5]]} > {band[bad[:5]]}")
    e = rel_err(x, ref["x"])
    assert e <= 10.0 * ref["x_band"] + 1e-12, (what, e, ref["x_band"])
