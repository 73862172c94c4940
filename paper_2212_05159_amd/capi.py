"""Thin ctypes binding over libcsrad.so.

The functions here carry the C names of the ABI declared in
``include/csrad.h`` and only marshal arguments: device tensors become raw
pointers, PyTorch allocates outputs and workspaces, and the current torch
stream is passed through.  Every arithmetic step runs in the library's HIP
kernels.  The library must be built (``paper_2212_05159_amd.build``); a
missing library is an error, never a fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcsrad.so")

F32, F64 = 0, 1
_DT = {torch.float32: F32, torch.float64: F64}


class csrad_csr(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("ncols", C.c_int32), ("nnz", C.c_int32),
                ("dtype", C.c_int32), ("rowptr", C.c_void_p), ("colind", C.c_void_p),
                ("vals", C.c_void_p)]


class csrad_plan(C.Structure):
    _fields_ = [("row_stride", C.c_int32), ("row_tile", C.c_int32)]


class csrad_batch_plan(C.Structure):
    _fields_ = [("nrows", C.c_int32), ("nblocks", C.c_int32), ("ntasks", C.c_int32),
                ("cus", C.c_int32), ("tasks", C.c_void_p), ("counters", C.c_void_p),
                ("block_rowptr", C.c_void_p)]


_lib = None

_SIGS = {
    "csr_status_string": (C.c_char_p, [C.c_int]),
    "csr_spmv_fwd": (C.c_int, [C.c_void_p] * 4),
    "csr_spmv_bwd": (C.c_int, [C.c_void_p] * 8),
    "csr_spmv_bwd_split": (C.c_int, [C.c_void_p] * 8),
    "csr_spmm_fwd": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                               C.c_int64, C.c_void_p, C.c_void_p]),
    "csr_spmm_bwd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                               C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                               C.c_void_p, C.c_void_p, C.c_void_p]),
    "csr_pattern_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_void_p, C.c_size_t,
                                    C.c_void_p]),
    "csr_transpose_workspace": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "csr_transpose": (C.c_int, [C.c_void_p] * 5 + [C.c_size_t, C.c_void_p]),
    "csr_transpose_vals": (C.c_int, [C.c_void_p] * 4),
    "csr_transpose_noalloc": (C.c_int, [C.c_void_p] * 5),
    "csr_noalloc_scratch_bytes": (C.c_size_t, []),
    "csr_spgemm_workspace": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]),
    "csr_spgemm_symbolic": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(C.c_int64), C.c_void_p, C.c_void_p, C.c_size_t,
                                      C.c_void_p]),
    "csr_spgemm_fwd": (C.c_int, [C.c_void_p] * 7 + [C.c_size_t, C.c_void_p]),
    "csr_spgemm_bwd": (C.c_int, [C.c_void_p] * 9),
    "csr_spadd_workspace": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]),
    "csr_spadd_symbolic": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64),
                                     C.c_void_p, C.c_size_t, C.c_void_p]),
    "csr_spadd_fwd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_void_p]),
    "csr_spadd_bwd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "csr_trisolve_workspace": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "csr_trisolve_analyze": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.POINTER(C.c_int32),
                                       C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "csr_trisolve_fwd": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "csr_trisolve_bwd": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p]),
    "csr_cg_workspace": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "csr_cg_init": (C.c_int, [C.c_void_p] * 8 + [C.c_size_t, C.c_void_p]),
    "csr_cg_step": (C.c_int, [C.c_void_p] * 10 + [C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]),
    "csr_cg_step_bwd": (C.c_int, [C.c_void_p] * 14 + [C.c_size_t, C.c_void_p]),
    "csr_cg_finish_bwd": (C.c_int, [C.c_void_p] * 7),
    "csr_pcg_workspace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                    C.POINTER(C.c_size_t)]),
    "csr_diag_inv": (C.c_int, [C.c_void_p] * 3),
    "csr_pcg_init": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_int32] + [C.c_void_p] * 8
                     + [C.c_double, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "csr_pcg_step": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.c_int32] + [C.c_void_p] * 10
                     + [C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]),
    "csr_dense_workspace": (C.c_int, [C.c_int32, C.POINTER(C.c_size_t)]),
    "csr_dense_fwd": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                C.c_int64, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                C.c_void_p]),
    "csr_dense_bwd": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                C.c_int64] + [C.c_void_p] * 3 + [C.c_int32] + [C.c_void_p] * 5
                      + [C.c_size_t, C.c_void_p]),
    "csr_mpnn_prep": (C.c_int, [C.c_void_p] * 7),
    "csr_mpnn_readout": (C.c_int, [C.c_void_p] * 4 + [C.c_float, C.c_float, C.c_void_p,
                                                      C.c_void_p]),
    "csr_mpnn_readout_bwd": (C.c_int, [C.c_void_p] * 4 + [C.c_float] + [C.c_void_p] * 3),
    "csr_validate": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_void_p, C.c_size_t,
                               C.c_void_p]),
    "csr_batch_plan_workspace": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32,
                                           C.POINTER(C.c_size_t)]),
    "csr_batch_plan_build": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                       C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "csr_batch_spmv_fwd": (C.c_int, [C.c_void_p] * 5),
    "csr_batch_spmv_bwd": (C.c_int, [C.c_void_p] * 9),
    "csr_batch_spmm_fwd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64,
                                     C.c_void_p, C.c_int64, C.c_void_p]),
    "csr_batch_spmm_bwd": (C.c_int, [C.c_void_p] * 4 + [C.c_int32, C.c_void_p, C.c_int64,
                                                         C.c_void_p, C.c_int64, C.c_void_p,
                                                         C.c_int64, C.c_void_p, C.c_void_p]),
    "csr_batch_sddmv": (C.c_int, [C.c_void_p] * 6),
    "csr_batch_sddmm": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64,
                                  C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "csr_batch_trisolve_levels_fwd": (C.c_int, [C.c_void_p, C.c_int32] + [C.c_void_p] * 5),
    "csr_batch_trisolve_levels_bwd": (C.c_int, [C.c_void_p] * 3 + [C.c_int32] + [C.c_void_p] * 7),
    "csr_batch_levels_workspace": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "csr_batch_levels": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_size_t, C.c_void_p]),
    "csr_batch_trisolve_fwd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                         C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                         C.c_void_p]),
    "csr_batch_trisolve_bwd": (C.c_int, [C.c_void_p] * 4 + [C.c_int32, C.c_void_p, C.c_void_p,
                                                             C.c_size_t] + [C.c_void_p] * 5),
    "csr_batch_ic0": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                C.c_size_t, C.c_void_p, C.c_void_p]),
    "csr_pcgl_workspace": (C.c_int, [C.c_int32, C.POINTER(C.c_size_t)]),
    "csr_pcgl_start": (C.c_int, [C.c_int32, C.c_int32] + [C.c_void_p] * 4
                       + [C.c_size_t, C.c_void_p]),
    "csr_pcgl_res_fwd": (C.c_int, [C.c_int32, C.c_int32] + [C.c_void_p] * 4
                         + [C.c_double] + [C.c_void_p] * 6 + [C.c_size_t, C.c_void_p]),
    "csr_pcgl_res_bwd": (C.c_int, [C.c_int32, C.c_int32] + [C.c_void_p] * 5
                         + [C.c_double] + [C.c_void_p] * 8 + [C.c_size_t, C.c_void_p]),
    "csr_pcgl_dir_fwd": (C.c_int, [C.c_int32, C.c_int32] + [C.c_void_p] * 7
                         + [C.c_size_t, C.c_void_p]),
    "csr_pcgl_dir_bwd": (C.c_int, [C.c_int32, C.c_int32] + [C.c_void_p] * 12
                         + [C.c_size_t, C.c_void_p]),
    "csr_pcgl_start_bwd": (C.c_int, [C.c_int32, C.c_int32] + [C.c_void_p] * 5),
}


def exported_symbols():
    return list(_SIGS)


def load():
    """Loads libcsrad.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2212_05159_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class CsradError(RuntimeError):
    def __init__(self, fn, status):
        self.status = status
        super().__init__(f"{fn}: {load().csr_status_string(status).decode()} (status {status})")


def _check(fn, status):
    if status != 0:
        raise CsradError(fn, status)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def desc(nrows, ncols, rowptr, colind, vals=None, dtype=None):
    """Host descriptor of a device CSR matrix (tensors must stay alive)."""
    dt = dtype if dtype is not None else vals.dtype
    if dt not in _DT:
        raise TypeError(f"unsupported value type {dt}")
    d = csrad_csr(int(nrows), int(ncols), int(colind.numel()), _DT[dt], rowptr.data_ptr(),
                  colind.data_ptr() if colind.numel() else None,
                  _ptr(vals) if vals is not None and vals.numel() else None)
    return d


def _ws(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# ----------------------------------------------------------------------
# C-named entry points (tensor marshalling only).
# ----------------------------------------------------------------------

def csr_spmv_fwd(A, x, y):
    _check("csr_spmv_fwd", load().csr_spmv_fwd(C.byref(A), _ptr(x), _ptr(y), _stream()))


def csr_spmv_bwd(A, At, perm, x, gy, gx, gvals):
    _check("csr_spmv_bwd", load().csr_spmv_bwd(C.byref(A), C.byref(At) if At is not None else None,
                                               _ptr(perm), _ptr(x), _ptr(gy), _ptr(gx),
                                               _ptr(gvals), _stream()))


def csr_spmv_bwd_split(A, At, perm, x, gy, gx, gvals):
    _check("csr_spmv_bwd_split", load().csr_spmv_bwd_split(C.byref(A), C.byref(At), _ptr(perm),
                                                           _ptr(x), _ptr(gy), _ptr(gx),
                                                           _ptr(gvals), _stream()))


def _plan(plan):
    return None if plan is None else C.byref(plan)


def csr_spmm_fwd(A, k, B, ldb, Cout, ldc, plan=None):
    _check("csr_spmm_fwd", load().csr_spmm_fwd(C.byref(A), int(k), _ptr(B), int(ldb), _ptr(Cout),
                                               int(ldc), _plan(plan), _stream()))


def csr_spmm_bwd(A, At, perm, k, B, ldb, gC, ldgc, gB, ldgb, gvals, plan=None):
    _check("csr_spmm_bwd", load().csr_spmm_bwd(C.byref(A), C.byref(At) if At is not None else None,
                                               _ptr(perm), int(k), _ptr(B), int(ldb), _ptr(gC),
                                               int(ldgc), _ptr(gB), int(ldgb), _ptr(gvals),
                                               _plan(plan), _stream()))


def csr_pattern_stats(A, work):
    st = (C.c_int64 * 4)()
    _check("csr_pattern_stats", load().csr_pattern_stats(C.byref(A), st, _ptr(work), work.numel(),
                                                         _stream()))
    return list(st)


def csr_transpose_workspace(A):
    n = C.c_size_t(0)
    _check("csr_transpose_workspace", load().csr_transpose_workspace(C.byref(A), C.byref(n)))
    return n.value


def csr_transpose(A, rowptrT, colindT, perm, work):
    _check("csr_transpose", load().csr_transpose(C.byref(A), _ptr(rowptrT), _ptr(colindT),
                                                 _ptr(perm), _ptr(work), work.numel(), _stream()))


def csr_transpose_noalloc(A, rowptrT, colindT, perm):
    _check("csr_transpose_noalloc", load().csr_transpose_noalloc(
        C.byref(A), _ptr(rowptrT), _ptr(colindT), _ptr(perm), _stream()))


def csr_noalloc_scratch_bytes():
    return int(load().csr_noalloc_scratch_bytes())


def csr_transpose_vals(A, perm, valsT):
    _check("csr_transpose_vals", load().csr_transpose_vals(C.byref(A), _ptr(perm), _ptr(valsT),
                                                           _stream()))


def csr_spgemm_workspace(A, B):
    n = C.c_size_t(0)
    _check("csr_spgemm_workspace", load().csr_spgemm_workspace(C.byref(A), C.byref(B), C.byref(n)))
    return n.value


SPGEMM_BINS = 9


def _host_i32(a, size):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous and a.size >= size
    return a.ctypes.data_as(C.c_void_p)


def csr_spgemm_symbolic(A, B, C_rowptr, work, bins_host=None):
    """Returns nnz(C); bins_host (int32 ndarray of SPGEMM_BINS, or None)
    receives the row classes for csr_spgemm_fwd."""
    nnz = C.c_int64(0)
    _check("csr_spgemm_symbolic", load().csr_spgemm_symbolic(
        C.byref(A), C.byref(B), _ptr(C_rowptr), C.byref(nnz), _host_i32(bins_host, SPGEMM_BINS),
        _ptr(work), work.numel(), _stream()))
    return nnz.value


def csr_spgemm_fwd(A, B, C_rowptr, C_colind, C_vals, work, bins_host=None):
    _check("csr_spgemm_fwd", load().csr_spgemm_fwd(
        C.byref(A), C.byref(B), _ptr(C_rowptr), _ptr(C_colind), _ptr(C_vals),
        _host_i32(bins_host, SPGEMM_BINS), _ptr(work), work.numel(), _stream()))


def csr_spgemm_bwd(A, B, At, permA, Cpat, gC, gA, gB):
    _check("csr_spgemm_bwd", load().csr_spgemm_bwd(C.byref(A), C.byref(B),
                                                   C.byref(At) if At is not None else None,
                                                   _ptr(permA), C.byref(Cpat), _ptr(gC), _ptr(gA),
                                                   _ptr(gB), _stream()))


def csr_spadd_workspace(A, B):
    n = C.c_size_t(0)
    _check("csr_spadd_workspace", load().csr_spadd_workspace(C.byref(A), C.byref(B), C.byref(n)))
    return n.value


def csr_spadd_symbolic(A, B, C_rowptr, work):
    """Returns nnz(C) of the union pattern (synchronises the stream)."""
    nnz = C.c_int64(0)
    _check("csr_spadd_symbolic", load().csr_spadd_symbolic(
        C.byref(A), C.byref(B), _ptr(C_rowptr), C.byref(nnz), _ptr(work), work.numel(),
        _stream()))
    return nnz.value


def csr_spadd_fwd(A, B, alpha, beta, C_rowptr, C_colind, C_vals):
    _check("csr_spadd_fwd", load().csr_spadd_fwd(
        C.byref(A), C.byref(B), float(alpha), float(beta), _ptr(C_rowptr), _ptr(C_colind),
        _ptr(C_vals), _stream()))


def csr_spadd_bwd(A, B, Cpat, alpha, beta, gC, gA, gB):
    _check("csr_spadd_bwd", load().csr_spadd_bwd(
        C.byref(A), C.byref(B), C.byref(Cpat), float(alpha), float(beta), _ptr(gC), _ptr(gA),
        _ptr(gB), _stream()))


def csr_trisolve_workspace(T):
    n = C.c_size_t(0)
    _check("csr_trisolve_workspace", load().csr_trisolve_workspace(C.byref(T), C.byref(n)))
    return n.value


def csr_trisolve_analyze(T, lower, Tt, level_of_row, level_ptr, level_rows, work,
                         level_ptr_host=None):
    """Returns nlevels; level_ptr_host (int32 ndarray of n+1 entries, or
    None) receives the level pointers on the host."""
    nl = C.c_int32(0)
    lph = None
    if level_ptr_host is not None:
        assert level_ptr_host.dtype == np.int32 and level_ptr_host.flags.c_contiguous
        assert level_ptr_host.size >= T.nrows + 1
        lph = level_ptr_host.ctypes.data_as(C.c_void_p)
    _check("csr_trisolve_analyze", load().csr_trisolve_analyze(
        C.byref(T), int(lower), C.byref(Tt), _ptr(level_of_row), _ptr(level_ptr),
        _ptr(level_rows), C.byref(nl), lph, _ptr(work), work.numel(), _stream()))
    return nl.value


def csr_trisolve_fwd(T, lower, nlevels, level_ptr_host, level_ptr, level_rows, b, x):
    _check("csr_trisolve_fwd", load().csr_trisolve_fwd(
        C.byref(T), int(lower), int(nlevels), level_ptr_host.ctypes.data, _ptr(level_ptr),
        _ptr(level_rows), _ptr(b), _ptr(x), _stream()))


def csr_trisolve_bwd(T, lower, Tt, perm, nlevels, level_ptr_host, level_ptr, level_rows, x, gx,
                     gb, gvals):
    _check("csr_trisolve_bwd", load().csr_trisolve_bwd(
        C.byref(T), int(lower), C.byref(Tt), _ptr(perm), int(nlevels),
        level_ptr_host.ctypes.data, _ptr(level_ptr), _ptr(level_rows), _ptr(x), _ptr(gx),
        _ptr(gb), _ptr(gvals), _stream()))


def csr_cg_workspace(A):
    n = C.c_size_t(0)
    _check("csr_cg_workspace", load().csr_cg_workspace(C.byref(A), C.byref(n)))
    return n.value


def csr_cg_init(A, b, x, r, p, scal, step, work):
    _check("csr_cg_init", load().csr_cg_init(C.byref(A), _ptr(b), _ptr(x), _ptr(r), _ptr(p),
                                             _ptr(scal), _ptr(step), _ptr(work), work.numel(),
                                             _stream()))


def csr_cg_step(A, x, r, p, q, p_save, r_save, scal, step, hist, work):
    _check("csr_cg_step", load().csr_cg_step(
        C.byref(A), _ptr(x), _ptr(r), _ptr(p), _ptr(q), _ptr(p_save), _ptr(r_save), _ptr(scal),
        _ptr(step), _ptr(hist), 0 if hist is None else hist.shape[0], _ptr(work), work.numel(),
        _stream()))


def csr_cg_step_bwd(A, At, p, q, r1, step_hist, gR, xb, rb, pb, qb, scal, gvals, work):
    _check("csr_cg_step_bwd", load().csr_cg_step_bwd(
        C.byref(A), C.byref(At), _ptr(p), _ptr(q), _ptr(r1), _ptr(step_hist),
        _ptr(gR), _ptr(xb), _ptr(rb), _ptr(pb), _ptr(qb), _ptr(scal), _ptr(gvals), _ptr(work),
        work.numel(), _stream()))


def csr_cg_finish_bwd(A, b, rb, pb, scal, gb):
    _check("csr_cg_finish_bwd", load().csr_cg_finish_bwd(C.byref(A), _ptr(b), _ptr(rb), _ptr(pb),
                                                         _ptr(scal), _ptr(gb), _stream()))


def csr_pcg_workspace(A, L=None, nlevels=0, level_ptr_host=None):
    n = C.c_size_t(0)
    _check("csr_pcg_workspace", load().csr_pcg_workspace(
        C.byref(A), C.byref(L) if L is not None else None, int(nlevels),
        level_ptr_host.ctypes.data if level_ptr_host is not None else None, C.byref(n)))
    return n.value


def csr_diag_inv(A, dinv):
    _check("csr_diag_inv", load().csr_diag_inv(C.byref(A), _ptr(dinv), _stream()))


def _pc_args(pc):
    """(kind, dinv, L, Lt, perm, nlevels, lp_host, lp, rows) -> ctypes values."""
    kind, dinv, L, Lt, perm, nl, lph, lp, rows = pc
    return (int(kind), _ptr(dinv), None if L is None else C.byref(L),
            None if Lt is None else C.byref(Lt), _ptr(perm), int(nl),
            None if lph is None else lph.ctypes.data, _ptr(lp), _ptr(rows))


def csr_pcg_init(A, pc, b, x, r, z, p, tol, scal, work):
    _check("csr_pcg_init", load().csr_pcg_init(C.byref(A), *_pc_args(pc), _ptr(b), _ptr(x),
                                               _ptr(r), _ptr(z), _ptr(p), float(tol), _ptr(scal),
                                               _ptr(work), work.numel(), _stream()))


def csr_pcg_step(A, pc, x, r, z, p, q, scal, hist, work):
    _check("csr_pcg_step", load().csr_pcg_step(
        C.byref(A), *_pc_args(pc), _ptr(x), _ptr(r), _ptr(z), _ptr(p), _ptr(q), _ptr(scal),
        _ptr(hist), 0 if hist is None else hist.numel(), _ptr(work), work.numel(), _stream()))


def csr_dense_workspace(n):
    nb = C.c_size_t(0)
    _check("csr_dense_workspace", load().csr_dense_workspace(int(n), C.byref(nb)))
    return nb.value


def csr_dense_fwd(n, K1, X1, ld1, K2, X2, ld2, W, b, relu, Y):
    _check("csr_dense_fwd", load().csr_dense_fwd(int(n), int(K1), _ptr(X1), int(ld1), int(K2),
                                                 _ptr(X2), int(ld2), _ptr(W), _ptr(b), int(relu),
                                                 _ptr(Y), _stream()))


def csr_dense_bwd(n, K1, X1, ld1, K2, X2, ld2, W, Y, dY, relu, dX1, dX2, dW, db, work):
    _check("csr_dense_bwd", load().csr_dense_bwd(
        int(n), int(K1), _ptr(X1), int(ld1), int(K2), _ptr(X2), int(ld2), _ptr(W), _ptr(Y),
        _ptr(dY), int(relu), _ptr(dX1), _ptr(dX2), _ptr(dW), _ptr(db), _ptr(work),
        0 if work is None else work.numel(), _stream()))


def csr_mpnn_prep(A, Lpat, ahat, ahatL, dsqrt, X0):
    _check("csr_mpnn_prep", load().csr_mpnn_prep(C.byref(A), C.byref(Lpat), _ptr(ahat),
                                                 _ptr(ahatL), _ptr(dsqrt), _ptr(X0), _stream()))


def csr_mpnn_readout(Lpat, ahatL, dsqrt, t, c, delta, Lv):
    _check("csr_mpnn_readout", load().csr_mpnn_readout(C.byref(Lpat), _ptr(ahatL), _ptr(dsqrt),
                                                       _ptr(t), float(c), float(delta), _ptr(Lv),
                                                       _stream()))


def csr_mpnn_readout_bwd(Lpat, ahatL, dsqrt, t, c, gL, gt):
    _check("csr_mpnn_readout_bwd", load().csr_mpnn_readout_bwd(
        C.byref(Lpat), _ptr(ahatL), _ptr(dsqrt), _ptr(t), float(c), _ptr(gL), _ptr(gt),
        _stream()))


def csr_validate(A, work):
    bad = C.c_int32(0)
    st = load().csr_validate(C.byref(A), C.byref(bad), _ptr(work), work.numel(), _stream())
    if st not in (0, -3):
        _check("csr_validate", st)
    return st, bad.value


# ----------------------------------------------------------------------
# Batched (block-diagonal) operators.
# ----------------------------------------------------------------------

def csr_batch_plan_workspace(A, nblocks, budget):
    n = C.c_size_t(0)
    _check("csr_batch_plan_workspace",
           load().csr_batch_plan_workspace(C.byref(A), int(nblocks), int(budget), C.byref(n)))
    return n.value


def csr_batch_plan_build(A, block_rowptr_host, variants_host, budget, work):
    """Returns a csrad_batch_plan pointing into `work` (the struct keeps a
    reference to `work`)."""
    brp = np.ascontiguousarray(block_rowptr_host, dtype=np.int32)
    var = None if variants_host is None else np.ascontiguousarray(variants_host, dtype=np.int32)
    plan = csrad_batch_plan()
    _check("csr_batch_plan_build",
           load().csr_batch_plan_build(C.byref(A), int(len(brp) - 1), brp.ctypes.data,
                                       None if var is None else var.ctypes.data, int(budget),
                                       _ptr(work), work.numel(), C.byref(plan), _stream()))
    # the plan's task array and queue counters live in `work`: the struct
    # holds the tensor so that the memory cannot be reused while any holder
    # of the plan may still launch with it
    plan._work = work
    return plan


def csr_batch_spmv_fwd(A, plan, x, y):
    _check("csr_batch_spmv_fwd",
           load().csr_batch_spmv_fwd(C.byref(A), C.byref(plan), _ptr(x), _ptr(y), _stream()))


def csr_batch_spmv_bwd(A, At, perm, planT, x, gy, gx, gvals):
    _check("csr_batch_spmv_bwd",
           load().csr_batch_spmv_bwd(C.byref(A), C.byref(At), _ptr(perm), C.byref(planT), _ptr(x),
                                     _ptr(gy), _ptr(gx), _ptr(gvals), _stream()))


def csr_batch_sddmv(A, plan, x, gy, gvals):
    _check("csr_batch_sddmv",
           load().csr_batch_sddmv(C.byref(A), C.byref(plan), _ptr(x), _ptr(gy), _ptr(gvals),
                                  _stream()))


def csr_batch_sddmm(A, plan, k, B, ldb, gC, ldgc, gvals):
    _check("csr_batch_sddmm",
           load().csr_batch_sddmm(C.byref(A), C.byref(plan), int(k), _ptr(B), int(ldb), _ptr(gC),
                                  int(ldgc), _ptr(gvals), _stream()))


def csr_batch_trisolve_levels_fwd(T, nlevels, level_ptr, level_rows, b, x):
    _check("csr_batch_trisolve_levels_fwd",
           load().csr_batch_trisolve_levels_fwd(C.byref(T), int(nlevels), _ptr(level_ptr),
                                                _ptr(level_rows), _ptr(b), _ptr(x), _stream()))


def csr_batch_trisolve_levels_bwd(T, Tt, perm, nlevels, level_ptr, level_rows, x, gx, gb, gvals):
    _check("csr_batch_trisolve_levels_bwd",
           load().csr_batch_trisolve_levels_bwd(C.byref(T), C.byref(Tt), _ptr(perm), int(nlevels),
                                                _ptr(level_ptr), _ptr(level_rows), _ptr(x),
                                                _ptr(gx), _ptr(gb), _ptr(gvals), _stream()))


def csr_batch_spmm_fwd(A, plan, k, B, ldb, Cout, ldc):
    _check("csr_batch_spmm_fwd",
           load().csr_batch_spmm_fwd(C.byref(A), C.byref(plan), int(k), _ptr(B), int(ldb),
                                     _ptr(Cout), int(ldc), _stream()))


def csr_batch_spmm_bwd(A, At, perm, planT, k, B, ldb, gC, ldgc, gB, ldgb, gvals):
    _check("csr_batch_spmm_bwd",
           load().csr_batch_spmm_bwd(C.byref(A), C.byref(At), _ptr(perm), C.byref(planT), int(k),
                                     _ptr(B), int(ldb), _ptr(gC), int(ldgc), _ptr(gB), int(ldgb),
                                     _ptr(gvals), _stream()))


def csr_batch_levels_workspace(nblocks, nlevels):
    n = C.c_size_t(0)
    _check("csr_batch_levels_workspace",
           load().csr_batch_levels_workspace(int(nblocks), int(nlevels), C.byref(n)))
    return n.value


def csr_batch_levels(plan, nlevels, level_ptr, level_rows, work):
    _check("csr_batch_levels",
           load().csr_batch_levels(C.byref(plan), int(nlevels), _ptr(level_ptr), _ptr(level_rows),
                                   _ptr(work), work.numel(), _stream()))


def csr_batch_trisolve_fwd(T, plan, nlevels, level_rows, lv_work, b, x):
    _check("csr_batch_trisolve_fwd",
           load().csr_batch_trisolve_fwd(C.byref(T), C.byref(plan), int(nlevels), _ptr(level_rows),
                                         _ptr(lv_work), lv_work.numel(), _ptr(b), _ptr(x),
                                         _stream()))


def csr_batch_trisolve_bwd(T, Tt, perm, plan, nlevels, level_rows, lv_work, x, gx, gb, gvals):
    _check("csr_batch_trisolve_bwd",
           load().csr_batch_trisolve_bwd(C.byref(T), C.byref(Tt), _ptr(perm), C.byref(plan),
                                         int(nlevels), _ptr(level_rows), _ptr(lv_work),
                                         lv_work.numel(), _ptr(x), _ptr(gx), _ptr(gb),
                                         _ptr(gvals), _stream()))


def csr_batch_ic0(Alow, plan, nlevels, level_rows, lv_work, Lvals):
    _check("csr_batch_ic0",
           load().csr_batch_ic0(C.byref(Alow), C.byref(plan), int(nlevels), _ptr(level_rows),
                                _ptr(lv_work), lv_work.numel(), _ptr(Lvals), _stream()))


# ----------------------------------------------------------------------
# PCG unroll steps of the residual-history loss (vectors of one dtype,
# float64 device scalars).
# ----------------------------------------------------------------------

def csr_pcgl_workspace(n):
    nb = C.c_size_t(0)
    _check("csr_pcgl_workspace", load().csr_pcgl_workspace(int(n), C.byref(nb)))
    return nb.value


def _dt(t):
    return _DT[t.dtype]


def csr_pcgl_start(b, z, scal, work):
    _check("csr_pcgl_start", load().csr_pcgl_start(b.numel(), _dt(b), _ptr(b), _ptr(z), _ptr(scal),
                                                   _ptr(work), work.numel(), _stream()))


def csr_pcgl_res_fwd(p, q, r, rho, w, bnorm, acc, r1, scal, acc1, work):
    _check("csr_pcgl_res_fwd", load().csr_pcgl_res_fwd(
        p.numel(), _dt(p), _ptr(p), _ptr(q), _ptr(r), _ptr(rho), float(w), _ptr(bnorm), _ptr(acc),
        _ptr(r1), _ptr(scal), _ptr(acc1), _ptr(work), work.numel(), _stream()))


def csr_pcgl_res_bwd(p, q, r1, rho, scal, w, bnorm, gr1, gacc1, gr, gq, gp, grho, work):
    _check("csr_pcgl_res_bwd", load().csr_pcgl_res_bwd(
        p.numel(), _dt(p), _ptr(p), _ptr(q), _ptr(r1), _ptr(rho), _ptr(scal), float(w),
        _ptr(bnorm), _ptr(gr1), _ptr(gacc1), _ptr(gr), _ptr(gq), _ptr(gp), _ptr(grho), _ptr(work),
        work.numel(), _stream()))


def csr_pcgl_dir_fwd(r1, z1, rho, p, rho1, p1, work):
    _check("csr_pcgl_dir_fwd", load().csr_pcgl_dir_fwd(
        r1.numel(), _dt(r1), _ptr(r1), _ptr(z1), _ptr(rho), _ptr(p), _ptr(rho1), _ptr(p1),
        _ptr(work), work.numel(), _stream()))


def csr_pcgl_dir_bwd(r1, z1, rho, p, rho1, gp1, grho1, gr1, gz1, gp, grho, work):
    _check("csr_pcgl_dir_bwd", load().csr_pcgl_dir_bwd(
        r1.numel(), _dt(r1), _ptr(r1), _ptr(z1), _ptr(rho), _ptr(p), _ptr(rho1), _ptr(gp1),
        _ptr(grho1), _ptr(gr1), _ptr(gz1), _ptr(gp), _ptr(grho), _ptr(work), work.numel(),
        _stream()))


def csr_pcgl_start_bwd(b, gp0, grho0, gz0):
    _check("csr_pcgl_start_bwd", load().csr_pcgl_start_bwd(
        b.numel(), _dt(b), _ptr(b), _ptr(gp0), _ptr(grho0), _ptr(gz0), _stream()))
