"""FP64 CPU oracle (test infrastructure only).

Thin ctypes wrappers over ``liboracle.so`` (built from ``oracle.c`` with gcc).
Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the HIP product path never does.

All wrappers take and return NumPy arrays; matrices are
``paper_2212_05159_amd.gen.Csr``-like objects (nrows, ncols, rowptr,
colind, vals).  Values are upcast to float64 (exact for float32 inputs).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SO_OMP = os.path.join(_HERE, "liboracle_omp.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lib = None
_libs = {}
_threads = False

_I32P = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_F64P = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


class _Nullable:
    """ndpointer that also accepts None (passed as NULL)."""

    def __init__(self, base):
        self.base = base

    def from_param(self, obj):
        if obj is None:
            return None
        return self.base.from_param(obj)


_F64N = _Nullable(_F64P)
_I32N = _Nullable(_I32P)


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (single-threaded, -O2) and, from the
    same source, liboracle_omp.so with OpenMP (row-parallel loops; used
    only to time the oracle on all host cores)."""
    for so, extra in ((_SO, []), (_SO_OMP, ["-fopenmp"])):
        if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(_SRC):
            tmp = so + ".tmp"
            subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", *extra,
                                   "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, so)
    return _SO


def threads() -> int:
    """Threads the current build's row-parallel loops use."""
    return int(_load().or_threads())


def use_threads(on: bool) -> None:
    """Route later calls to the OpenMP build (on) or the single-threaded
    one (off, the default).  Both return the same bits."""
    global _threads, _lib
    _threads = bool(on)
    _lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    so = _SO_OMP if _threads else _SO
    if so in _libs:
        _lib = _libs[so]
        return _lib
    if not os.path.exists(so):
        build()
    lib = C.CDLL(so)
    i32, i64, dbl, cint = C.c_int32, C.c_int64, C.c_double, C.c_int
    sig = {
        "or_spmv": (None, [i32, _I32P, _I32P, _F64P, _F64P, _F64P]),
        "or_spmv_bwd": (None, [i32, i32, _I32P, _I32P, _F64P, _F64P, _F64P, _F64N, _F64N]),
        "or_spmm": (None, [i32, i32, _I32P, _I32P, _F64P, _F64P, _F64P]),
        "or_spmm_bwd": (None, [i32, i32, i32, _I32P, _I32P, _F64P, _F64P, _F64P, _F64N, _F64N]),
        "or_transpose": (None, [i32, i32, _I32P, _I32P, _I32P, _I32P, _I32P]),
        "or_spgemm_rowptr": (i64, [i32, i32, _I32P, _I32P, _I32P, _I32P, _I32P]),
        "or_spgemm_fill": (cint, [i32, i32, _I32P, _I32P, _F64P, _I32P, _I32P, _F64P,
                                  _I32P, _I32P, _F64P]),
        "or_spgemm_bwd": (cint, [i32, i32, i32, _I32P, _I32P, _F64P, _I32P, _I32P, _F64P,
                                 _I32P, _I32P, _F64P, _F64N, _F64N]),
        "or_spadd_rowptr": (i64, [i32, i32, _I32P, _I32P, _I32P, _I32P, _I32P]),
        "or_spadd_fill": (cint, [i32, i32, _I32P, _I32P, _F64P, _I32P, _I32P, _F64P, dbl, dbl,
                                 _I32P, _I32P, _F64P]),
        "or_spadd_bwd": (cint, [i32, i32, _I32P, _I32P, _I32P, _I32P, _I32P, _I32P, _F64P, dbl,
                                dbl, _F64N, _F64N]),
        "or_levels": (i32, [i32, _I32P, _I32P, cint, _I32P, _I32P, _I32P]),
        "or_trisolve": (i32, [i32, _I32P, _I32P, _F64P, cint, _F64P, _F64P]),
        "or_trisolve_bwd": (i32, [i32, _I32P, _I32P, _F64P, cint, _F64P, _F64P, _F64P, _F64N]),
        "or_cg": (cint, [i32, _I32P, _I32P, _F64P, _F64P, i32, _F64P, _F64N, _F64N, _F64N, _F64N]),
        "or_cg_bwd": (cint, [i32, _I32P, _I32P, _F64P, _F64P, i32, _F64N, _F64N, _F64P, _F64P]),
        "or_pcg": (i32, [i32, _I32P, _I32P, _F64P, _F64P, cint, _I32N, _I32N, _F64N, dbl, i32,
                         _F64P, _F64N]),
        "or_ic0": (i32, [i32, _I32P, _I32P, _F64P, _I32P, _I32P, _F64P]),
        "or_paper_loss": (dbl, [i32, dbl, _F64P, dbl, _F64P]),
        "or_threads": (cint, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _libs[so] = lib
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _csr(A):
    return A.nrows, A.ncols, _i32(A.rowptr), _i32(A.colind), _f64(A.vals)


def spmv(A, x):
    m, n, rp, ci, v = _csr(A)
    y = np.empty(m)
    _load().or_spmv(m, rp, ci, v, _f64(x), y)
    return y


def spmv_bwd(A, x, gy, want_x=True, want_vals=True):
    m, n, rp, ci, v = _csr(A)
    gx = np.empty(n) if want_x else None
    gv = np.empty(len(ci)) if want_vals else None
    _load().or_spmv_bwd(m, n, rp, ci, v, _f64(x), _f64(gy), gx, gv)
    return gx, gv


def spmm(A, B):
    m, n, rp, ci, v = _csr(A)
    B = _f64(B)
    k = B.shape[1]
    Cm = np.empty((m, k))
    _load().or_spmm(m, k, rp, ci, v, B, Cm)
    return Cm


def spmm_bwd(A, B, G, want_B=True, want_vals=True):
    m, n, rp, ci, v = _csr(A)
    B, G = _f64(B), _f64(G)
    k = B.shape[1]
    gB = np.empty((n, k)) if want_B else None
    gv = np.empty(len(ci)) if want_vals else None
    _load().or_spmm_bwd(m, n, k, rp, ci, v, B, G, gB, gv)
    return gB, gv


def transpose(A):
    """Returns (rowptrT, colindT, perm)."""
    m, n, rp, ci, _ = _csr(A)
    rpT = np.empty(n + 1, np.int32)
    ciT = np.empty(len(ci), np.int32)
    perm = np.empty(len(ci), np.int32)
    _load().or_transpose(m, n, rp, ci, rpT, ciT, perm)
    return rpT, ciT, perm


def spgemm(A, B):
    """Returns (rowptrC, colindC, valsC) of C = A B."""
    m, n, rpA, ciA, vA = _csr(A)
    _, p, rpB, ciB, vB = _csr(B)
    lib = _load()
    rpC = np.empty(m + 1, np.int32)
    nnz = lib.or_spgemm_rowptr(m, p, rpA, ciA, rpB, ciB, rpC)
    if nnz < 0:
        raise MemoryError("oracle spgemm")
    ciC = np.empty(nnz, np.int32)
    vC = np.empty(nnz)
    if lib.or_spgemm_fill(m, p, rpA, ciA, vA, rpB, ciB, vB, rpC, ciC, vC) != 0:
        raise MemoryError("oracle spgemm")
    return rpC, ciC, vC


def spgemm_bwd(A, B, rpC, ciC, gC, want_A=True, want_B=True):
    m, n, rpA, ciA, vA = _csr(A)
    _, p, rpB, ciB, vB = _csr(B)
    gA = np.empty(len(ciA)) if want_A else None
    gB = np.empty(len(ciB)) if want_B else None
    rc = _load().or_spgemm_bwd(m, n, p, rpA, ciA, vA, rpB, ciB, vB, _i32(rpC), _i32(ciC),
                               _f64(gC), gA, gB)
    if rc != 0:
        raise MemoryError("oracle spgemm_bwd")
    return gA, gB


def spadd(A, B, alpha=1.0, beta=1.0):
    """Returns (rowptrC, colindC, valsC) of C = alpha A + beta B on the
    union of the two patterns."""
    m, n, rpA, ciA, vA = _csr(A)
    _, _, rpB, ciB, vB = _csr(B)
    lib = _load()
    rpC = np.empty(m + 1, np.int32)
    nnz = lib.or_spadd_rowptr(m, n, rpA, ciA, rpB, ciB, rpC)
    if nnz < 0:
        raise MemoryError("oracle spadd")
    ciC = np.empty(nnz, np.int32)
    vC = np.empty(nnz)
    if lib.or_spadd_fill(m, n, rpA, ciA, vA, rpB, ciB, vB, float(alpha), float(beta),
                         rpC, ciC, vC) != 0:
        raise MemoryError("oracle spadd")
    return rpC, ciC, vC


def spadd_bwd(A, B, rpC, ciC, gC, alpha=1.0, beta=1.0, want_A=True, want_B=True):
    m, n, rpA, ciA, _ = _csr(A)
    _, _, rpB, ciB, _ = _csr(B)
    gA = np.empty(len(ciA)) if want_A else None
    gB = np.empty(len(ciB)) if want_B else None
    if _load().or_spadd_bwd(m, n, rpA, ciA, rpB, ciB, _i32(rpC), _i32(ciC), _f64(gC),
                            float(alpha), float(beta), gA, gB) != 0:
        raise MemoryError("oracle spadd_bwd")
    return gA, gB


def levels(T, lower=True):
    """Returns (level_of_row, level_ptr, level_rows)."""
    n, _, rp, ci, _ = _csr(T)
    lor = np.empty(n, np.int32)
    lptr = np.empty(n + 1, np.int32)
    lrows = np.empty(n, np.int32)
    nl = _load().or_levels(n, rp, ci, int(bool(lower)), lor, lptr, lrows)
    return lor, lptr[: nl + 1].copy(), lrows


def trisolve(T, b, lower=True):
    n, _, rp, ci, v = _csr(T)
    x = np.empty(n)
    rc = _load().or_trisolve(n, rp, ci, v, int(bool(lower)), _f64(b), x)
    if rc != 0:
        raise ZeroDivisionError(f"diagonal of row {rc - 1} not stored")
    return x


def trisolve_bwd(T, x, gx, lower=True, want_vals=True):
    n, _, rp, ci, v = _csr(T)
    gb = np.empty(n)
    gv = np.empty(len(ci)) if want_vals else None
    rc = _load().or_trisolve_bwd(n, rp, ci, v, int(bool(lower)), _f64(x), _f64(gx), gb, gv)
    if rc != 0:
        raise ZeroDivisionError(f"diagonal of row {rc - 1} not stored")
    return gb, gv


def cg(A, b, K, want_history=False):
    """K steps of CG from x0 = 0.  Returns x_K (and r_1..r_K if asked)."""
    n, _, rp, ci, v = _csr(A)
    x = np.empty(n)
    R = np.empty((K, n)) if want_history else None
    _load().or_cg(n, rp, ci, v, _f64(b), K, x, R, None, None, None)
    return (x, R) if want_history else x


def cg_bwd(A, b, K, gx=None, gR=None):
    """Reverse mode of ``cg``: returns (gvals, gb)."""
    n, _, rp, ci, v = _csr(A)
    gv = np.empty(len(ci))
    gb = np.empty(n)
    _load().or_cg_bwd(n, rp, ci, v, _f64(b), K, None if gx is None else _f64(gx),
                      None if gR is None else _f64(gR), gv, gb)
    return gv, gb


def pcg(A, b, mode="jacobi", L=None, tol=1e-6, maxit=10000):
    """Returns (x, iterations, history) ; iterations = -1 on breakdown."""
    n, _, rp, ci, v = _csr(A)
    m = {"jacobi": 0, "factor": 1, "none": 2, "fsai": 3}[mode]
    x = np.empty(n)
    hist = np.full(maxit + 1, np.nan)
    if m in (1, 3):
        _, _, lrp, lci, lv = _csr(L)
    else:
        lrp = lci = lv = None
    it = _load().or_pcg(n, rp, ci, v, _f64(b), m, lrp, lci, lv, float(tol), int(maxit), x, hist)
    return x, int(it), hist[: (it + 1 if it >= 0 else maxit + 1)]


def ic0(A, Lpat):
    """IC(0) values on the lower pattern Lpat (diagonal last per row)."""
    n, _, rp, ci, v = _csr(A)
    lrp, lci = _i32(Lpat.rowptr), _i32(Lpat.colind)
    lv = np.empty(len(lci))
    rc = _load().or_ic0(n, rp, ci, v, lrp, lci, lv)
    if rc != 0:
        raise ArithmeticError(f"IC(0) breakdown at row {rc - 1}")
    return lv


def paper_loss(rnorms, bnorm, gamma=0.6):
    r = _f64(rnorms)
    w = np.empty(len(r))
    val = _load().or_paper_loss(len(r), float(gamma), r, float(bnorm), w)
    return val, w
