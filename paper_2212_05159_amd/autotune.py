"""Autotuner for the dense-operand kernels' traversal plans.

Candidates come from the pattern's statistics (csr_pattern_stats): natural
row order always, and when the bandwidth is large (long-range couplings at
a fixed row offset, as in structured-grid operators) tiled orders with
row_stride = bandwidth and several tile heights.  Each candidate is timed
with HIP events on the current stream (the kernels' own launches, after one
warm-up call), the fastest is stored on the Pattern and in a JSON cache
keyed by GPU architecture and pattern/operand signature.  A plan changes
only the order in which rows are visited, never a result.
"""
from __future__ import annotations

import json
import os

import torch

from . import capi

_CACHE_PATH = os.environ.get("CSRAD_TUNE_CACHE",
                             os.path.join(os.path.expanduser("~"), ".cache", "csrad", "tune.json"))
_TILES = (1024, 2048, 4096, 8192)
_FAR = 4096  # bandwidth above which tiled orders are worth trying


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName
    except Exception:  # pragma: no cover
        return "unknown"


def _load_cache():
    try:
        with open(_CACHE_PATH) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c):
    try:
        os.makedirs(os.path.dirname(_CACHE_PATH), exist_ok=True)
        tmp = _CACHE_PATH + ".tmp"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, _CACHE_PATH)
    except OSError:
        pass


def candidates(P):
    """Plans worth timing for the rows of pattern P."""
    maxrow, bw, _, _ = P.stats()
    out = [None]
    if bw >= _FAR:
        for t in _TILES:
            if t < bw:
                out.append((int(bw), t))
    return out


def _plan_obj(c):
    return None if c is None else capi.csrad_plan(c[0], c[1])


def _time(fn, reps):
    fn()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        s.record()
        fn()
        e.record()
        e.synchronize()
        best = min(best, s.elapsed_time(e))
    return best


def tune_spmm(P, vals, B, G, reps=3, use_cache=True):
    """Chooses plans for SpMM forward (rows of A) and the fused backward
    (rows of A^T) with operands like B (n x k) and G (m x k); stores them on
    P and returns {op: (candidate, ms)}."""
    from . import sparse as sp

    k = B.shape[1]
    Pt, _ = P.transpose()
    key_base = f"{_arch()}|{P.nrows}x{P.ncols}|nnz{P.nnz}|{tuple(P.stats())}|k{k}|{vals.dtype}"
    cache = _load_cache() if use_cache else {}
    result = {}
    jobs = {
        "spmm_fwd": (candidates(P), lambda pl: sp.spmm(P, vals, B, plan=_plan_obj(pl) or capi.csrad_plan(0, 0))),
        "spmm_bwd": (candidates(Pt), lambda pl: sp.spmm_bwd(P, vals, B, G, plan=_plan_obj(pl) or capi.csrad_plan(0, 0))),
    }
    for op, (cands, run) in jobs.items():
        key = f"{key_base}|{op}"
        if key in cache:
            c = cache[key]["plan"]
            c = None if c is None else tuple(c)
            result[op] = (c, cache[key]["ms"])
        else:
            timed = [(c, _time(lambda c=c: run(c), reps)) for c in cands]
            c, ms = min(timed, key=lambda t: t[1])
            result[op] = (c, ms)
            cache[key] = {"plan": c, "ms": ms, "all": [[list(t[0]) if t[0] else None, t[1]] for t in timed]}
        P.set_plan(op, _plan_obj(result[op][0]))
    if use_cache:
        _save_cache(cache)
    return result


def tune_spmv_bwd(P, vals, x, gy, reps=3, use_cache=True):
    """Chooses how the SpMV backward forms its two gradients when both are
    wanted: "fused" (one pass over A^T writes the value gradient through
    the permutation) or "split" (A^T gy over A^T, the value gradient in a
    second, row-wise pass over A with coalesced writes).  Patterns whose
    transpose permutation is local (structured grids) favour the fused
    pass; scattered ones (random graphs) the split.  Results are the same
    bit for bit either way.  Stores the choice on P; returns (choice, ms)."""
    from . import sparse as sp

    key = f"{_arch()}|{P.nrows}x{P.ncols}|nnz{P.nnz}|{tuple(P.stats())}|{vals.dtype}|spmv_bwd"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        choice, ms = cache[key]["mode"], cache[key]["ms"]
    else:
        timed = []
        for mode in ("fused", "split"):
            P.set_plan("spmv_bwd", mode)
            timed.append((mode, _time(lambda: sp.spmv_bwd(P, vals, x, gy), reps)))
        choice, ms = min(timed, key=lambda t: t[1])
        cache[key] = {"mode": choice, "ms": ms, "all": [list(t) for t in timed]}
        if use_cache:
            _save_cache(cache)
    P.set_plan("spmv_bwd", choice)
    return choice, ms
