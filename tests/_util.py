"""Shared helpers for the GPU parity tests (no method arithmetic here)."""
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
