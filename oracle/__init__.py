"""Reference Posit(N,2) arithmetic and reference BLAS/LAPACK routines.

TEST INFRASTRUCTURE ONLY.  This package wraps the C oracle in
``posit_oracle.c``: a plain, slow, obviously correct CPU implementation written
from the definition of the posit format (paper, Section 2, Eq. (1)) and of
GEMM (Section 3, Eq. (2)).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  The GPU library neither imports
nor links it, and it imports nothing from the GPU library.

All posit values are numpy ``uint32`` arrays holding raw bit patterns (the
N-bit pattern in the low N bits).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["posit_oracle.c", "ref_lapack.c"]

NAR32 = 0x80000000
ONE32 = 0x40000000


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with gcc + OpenMP."""
    if force or not os.path.exists(_LIB_PATH):
        srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall",
             "-o", tmp] + srcs + ["-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        u32, i32, i64, dbl = ctypes.c_uint32, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        vp = ctypes.c_void_p
        for name in ("oracle_posit_add", "oracle_posit_sub", "oracle_posit_mul",
                     "oracle_posit_div"):
            f = getattr(L, name)
            f.argtypes, f.restype = [i32, u32, u32], u32
        for name in ("oracle_posit_sqrt", "oracle_posit_neg"):
            f = getattr(L, name)
            f.argtypes, f.restype = [i32, u32], u32
        L.oracle_posit_from_double.argtypes, L.oracle_posit_from_double.restype = [i32, dbl], u32
        L.oracle_posit_to_double.argtypes, L.oracle_posit_to_double.restype = [i32, u32], dbl
        L.oracle_posit_fields.argtypes = [i32, u32] + [ctypes.POINTER(i32)] * 4 + [ctypes.POINTER(u32)]
        L.oracle_posit_fields.restype = i32
        L.oracle_vec_from_double.argtypes = [i32, i64, vp, vp]
        L.oracle_vec_to_double.argtypes = [i32, i64, vp, vp]
        L.oracle_vec_binop.argtypes = [i32, i32, i64, vp, vp, vp]
        L.oracle_gemm.argtypes = [i32, i32, i64, i64, i64, u32, vp, i64, vp, i64, u32, vp, i64]
        L.oracle_gemm_entries.argtypes = [i32, i32, i64, u32, vp, i64, vp, i64, u32, i64,
                                          vp, vp, vp, vp]
        L.oracle_num_threads.restype = i32
        if hasattr(L, "oracle_getrf"):
            L.oracle_getrf.argtypes = [i64, i64, vp, i64, vp, vp]
            L.oracle_getrs.argtypes = [i64, i64, vp, i64, vp, vp, i64]
            L.oracle_potrf.argtypes = [i64, i64, vp, i64, vp]
            L.oracle_potrs.argtypes = [i64, i64, vp, i64, vp, i64]
            L.oracle_getrs_trans.argtypes = [i64, i64, vp, i64, vp, vp, i64]
            L.oracle_potrf_upper.argtypes = [i64, i64, vp, i64, vp]
            L.oracle_potrf_upper.restype = i32
            L.oracle_potrs_upper.argtypes = [i64, i64, vp, i64, vp, i64]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _ld(a: np.ndarray) -> int:
    """Row stride in elements of a row-major 2-D array (unit column stride)."""
    if a.size == 0:
        return max(1, a.shape[1])
    assert a.strides[1] == 4, "matrices must have unit column stride"
    return a.strides[0] // 4


# ---- scalar operations -------------------------------------------------------

def add(a: int, b: int, N: int = 32) -> int:
    return lib().oracle_posit_add(N, a, b)


def sub(a: int, b: int, N: int = 32) -> int:
    return lib().oracle_posit_sub(N, a, b)


def mul(a: int, b: int, N: int = 32) -> int:
    return lib().oracle_posit_mul(N, a, b)


def div(a: int, b: int, N: int = 32) -> int:
    return lib().oracle_posit_div(N, a, b)


def sqrt(a: int, N: int = 32) -> int:
    return lib().oracle_posit_sqrt(N, a)


def neg(a: int, N: int = 32) -> int:
    return lib().oracle_posit_neg(N, a)


def from_double(x: float, N: int = 32) -> int:
    return lib().oracle_posit_from_double(N, float(x))


def to_double(p: int, N: int = 32) -> float:
    return lib().oracle_posit_to_double(N, p)


def fields(p: int, N: int = 32):
    """(kind, sign, k, e, fs, f) with kind 0 normal, 1 zero, 2 NaR."""
    s, k, e, fs = (ctypes.c_int() for _ in range(4))
    f = ctypes.c_uint32()
    kind = lib().oracle_posit_fields(N, p, ctypes.byref(s), ctypes.byref(k),
                                     ctypes.byref(e), ctypes.byref(fs), ctypes.byref(f))
    return kind, s.value, k.value, e.value, fs.value, f.value


# ---- array operations ----------------------------------------------------------

def vec_from_double(x, N: int = 32) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(x.shape, dtype=np.uint32)
    lib().oracle_vec_from_double(N, x.size, _ptr(x), _ptr(out))
    return out


def vec_to_double(p, N: int = 32) -> np.ndarray:
    p = np.ascontiguousarray(p, dtype=np.uint32)
    out = np.empty(p.shape, dtype=np.float64)
    lib().oracle_vec_to_double(N, p.size, _ptr(p), _ptr(out))
    return out


_OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "sqrt": 4}


def vec_op(op: str, a, b=None, N: int = 32) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = a if b is None else np.ascontiguousarray(b, dtype=np.uint32)
    assert a.shape == b.shape
    out = np.empty(a.shape, dtype=np.uint32)
    lib().oracle_vec_binop(N, _OPS[op], a.size, _ptr(a), _ptr(b), _ptr(out))
    return out


# ---- Rgemm ---------------------------------------------------------------------

def gemm(A, B, C, alpha: int = ONE32, beta: int = ONE32, transa: bool = False,
         transb: bool = False, m=None, n=None, k=None) -> np.ndarray:
    """Return a new array: alpha*op(A)*op(B) + beta*C in Posit(32,2).

    A, B, C are 2-D uint32 arrays in row-major order; their row strides are
    the leading dimensions.  m, n, k default to the shapes implied by op()."""
    A = np.asarray(A, dtype=np.uint32)
    B = np.asarray(B, dtype=np.uint32)
    Cout = np.array(C, dtype=np.uint32, copy=True, order="C")
    if m is None:
        m = A.shape[1] if transa else A.shape[0]
    if k is None:
        k = A.shape[0] if transa else A.shape[1]
    if n is None:
        n = B.shape[0] if transb else B.shape[1]
    lda, ldb = _ld(A), _ld(B)
    lib().oracle_gemm(int(transa), int(transb), m, n, k, alpha, A.ctypes.data, lda,
                      B.ctypes.data, ldb, beta, Cout.ctypes.data, Cout.shape[1])
    return Cout


def gemm_entries(A, B, rows, cols, Cin, alpha: int = ONE32, beta: int = ONE32,
                 transa: bool = False, transb: bool = False, k=None) -> np.ndarray:
    """Oracle Rgemm results for the listed (row, col) entries only."""
    A = np.asarray(A, dtype=np.uint32)
    B = np.asarray(B, dtype=np.uint32)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    Cin = np.ascontiguousarray(Cin, dtype=np.uint32)
    if k is None:
        k = A.shape[0] if transa else A.shape[1]
    out = np.empty(rows.shape, dtype=np.uint32)
    lib().oracle_gemm_entries(int(transa), int(transb), k, alpha, A.ctypes.data,
                              _ld(A), B.ctypes.data, _ld(B), beta,
                              rows.size, _ptr(rows), _ptr(cols), _ptr(Cin), _ptr(out))
    return out


def num_threads() -> int:
    return lib().oracle_num_threads()


# ---- factorisations and solves --------------------------------------------------

def getrf(A, nb: int = 256):
    """Blocked LU with partial pivoting (order in ref_lapack.c).
    Returns (LU, ipiv (0-based int32), info)."""
    A = np.array(A, dtype=np.uint32, copy=True, order="C")
    n = A.shape[0]
    assert A.shape == (n, n)
    ipiv = np.zeros(n, dtype=np.int32)
    info = np.zeros(1, dtype=np.int32)
    lib().oracle_getrf(n, nb, _ptr(A), n, _ptr(ipiv), _ptr(info))
    return A, ipiv, int(info[0])


def getrs(LU, ipiv, B, trans: bool = False):
    """Solve A X = B (trans: A^T X = B) with the factors of getrf."""
    LU = np.ascontiguousarray(LU, dtype=np.uint32)
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    X = np.array(B, dtype=np.uint32, copy=True, order="C")
    if X.ndim == 1:
        X = X.reshape(-1, 1)
    n = LU.shape[0]
    f = lib().oracle_getrs_trans if trans else lib().oracle_getrs
    f(n, X.shape[1], _ptr(LU), n, _ptr(ipiv), _ptr(X), X.shape[1])
    return X


def potrf(A, nb: int = 256, upper: bool = False):
    """Blocked Cholesky (order in ref_lapack.c).  Returns (L, info) (upper:
    (U, info) with A = U^T U); only the factor's triangle is meaningful, the
    rest is A's."""
    A = np.array(A, dtype=np.uint32, copy=True, order="C")
    n = A.shape[0]
    info = np.zeros(1, dtype=np.int32)
    if upper:
        if lib().oracle_potrf_upper(n, nb, _ptr(A), n, _ptr(info)) != 0:
            raise MemoryError("oracle_potrf_upper: no memory for the transposed copy")
    else:
        lib().oracle_potrf(n, nb, _ptr(A), n, _ptr(info))
    return A, int(info[0])


def potrs(L, B, upper: bool = False):
    """Solve A X = B with the factor of potrf (upper: U with A = U^T U)."""
    L = np.ascontiguousarray(L, dtype=np.uint32)
    X = np.array(B, dtype=np.uint32, copy=True, order="C")
    if X.ndim == 1:
        X = X.reshape(-1, 1)
    n = L.shape[0]
    f = lib().oracle_potrs_upper if upper else lib().oracle_potrs
    f(n, X.shape[1], _ptr(L), n, _ptr(X), X.shape[1])
    return X
