"""ctypes binding of libposit32.so (C ABI in include/posit32.h).

Argument marshalling only: every operation runs in the HIP library on the
caller's current torch stream.  Posit(32,2) values are carried in
``torch.int32`` device tensors holding the raw bit patterns (a signed view of
the uint32 pattern).  Scalars (alpha, beta) are Python ints holding patterns.
If the library has not been built, or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# POSIT32_LIB may name another build of the same library (same C ABI)
LIB_PATH = os.environ.get("POSIT32_LIB") or os.path.join(HERE, "libposit32.so")

NAR = 0x80000000
ONE = 0x40000000
ZERO = 0
MINUS_ONE = 0xC0000000

OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_SQRT = range(5)

_lib = None

REQ_LU, REQ_CHOL = 0, 1
E_NOMEM = -4000
E_BUSY = -5000


class Posit32Error(RuntimeError):
    """A library call returned a nonzero status; ``code`` holds it (None when
    the library itself could not be loaded)."""

    def __init__(self, msg: str, code: int | None = None):
        super().__init__(msg)
        self.code = code


TUNE_BUCKETS = 8


class Tuning(ctypes.Structure):
    """posit32_vbatch_tuning: the sub-panel width of the batched kernels per
    size bucket (a system of order n takes sub[b] of the first bucket with
    n <= max_n[b]).  Any table gives the same result bits."""
    _fields_ = [("buckets", ctypes.c_int32), ("max_n", ctypes.c_int32 * TUNE_BUCKETS),
                ("sub", ctypes.c_int32 * TUNE_BUCKETS)]

    @classmethod
    def make(cls, max_n, sub) -> "Tuning":
        if len(max_n) != len(sub) or not 1 <= len(sub) <= TUNE_BUCKETS:
            raise ValueError("max_n and sub need the same length, 1..8")
        t = cls()
        t.buckets = len(sub)
        for b, (m, w) in enumerate(zip(max_n, sub)):
            t.max_n[b] = int(m)
            t.sub[b] = int(w)
        return t

    def to_dict(self) -> dict:
        return {"max_n": list(self.max_n)[:self.buckets], "sub": list(self.sub)[:self.buckets]}


class VBatchDesc(ctypes.Structure):
    """posit32_vbatch: descriptor of one call of posit32_vbatched."""
    _fields_ = [("kind", ctypes.c_int32), ("factor", ctypes.c_int32), ("solve", ctypes.c_int32),
                ("count", ctypes.c_int32), ("max_n", ctypes.c_int32), ("nb", ctypes.c_int64),
                ("n", ctypes.c_void_p), ("nrhs", ctypes.c_void_p), ("A", ctypes.c_void_p),
                ("lda", ctypes.c_void_p), ("ipiv", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("ldb", ctypes.c_void_p), ("info", ctypes.c_void_p)]


class QueueCfg(ctypes.Structure):
    _fields_ = [("device_bytes", ctypes.c_int64), ("max_batch", ctypes.c_int32),
                ("nb", ctypes.c_int32), ("batch_max_n", ctypes.c_int32),
                ("tuning", ctypes.c_void_p), ("max_pending", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("keep", ctypes.c_int32), ("n", ctypes.c_int64),
                ("nrhs", ctypes.c_int64), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("factor", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("info", ctypes.c_int32), ("factor", ctypes.c_uint64),
                ("submit_s", ctypes.c_double), ("start_s", ctypes.c_double),
                ("done_s", ctypes.c_double)]


class QueueStats(ctypes.Structure):
    _fields_ = [("pending", ctypes.c_int64), ("inflight_batches", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("systems_done", ctypes.c_int64),
                ("pool_bytes", ctypes.c_int64), ("pool_used", ctypes.c_int64),
                ("resident_factors", ctypes.c_int64), ("error", ctypes.c_int32)]


def lib() -> ctypes.CDLL:
    """Load libposit32.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise Posit32Error(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32
    L.posit32_version.restype = i32
    L.posit32_strerror.argtypes = [i32]
    L.posit32_strerror.restype = ctypes.c_char_p
    L.posit32_gemm.argtypes = [vp, i32, i32, i64, i64, i64, u32, vp, i64, vp, i64, u32, vp, i64]
    L.posit32_gemm.restype = i32
    L.posit32_from_f64.argtypes = [vp, i64, vp, vp]
    L.posit32_to_f64.argtypes = [vp, i64, vp, vp]
    L.posit32_elementwise.argtypes = [vp, i32, i64, vp, vp, vp]
    L.posit32_getrf.argtypes = [vp, i64, i64, vp, i64, vp, vp]
    L.posit32_getrf_noalloc.argtypes = [vp, i64, i64, vp, i64, vp, vp]
    L.posit32_getrf_phases.argtypes = [vp, i64, i64, vp, i64, vp, vp, vp]
    L.posit32_getrf_phases.restype = i32
    L.posit32_getrs_group.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.posit32_getrs_group.restype = i32
    L.posit32_getrf_group.argtypes = [vp, i32, vp, i64, vp, vp, vp, vp]
    L.posit32_getrf_group.restype = i32
    L.posit32_getrf_noalloc.restype = i32
    L.posit32_getrs.argtypes = [vp, i32, i64, i64, vp, i64, vp, vp, i64]
    L.posit32_potrf.argtypes = [vp, i32, i64, i64, vp, i64, vp]
    L.posit32_potrs.argtypes = [vp, i32, i64, i64, vp, i64, vp, i64]
    L.posit32_getrf_vbatched.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp, vp]
    L.posit32_getrs_vbatched.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.posit32_gesv_vbatched.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    L.posit32_potrf_vbatched.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp]
    L.posit32_potrs_vbatched.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp, vp]
    L.posit32_posv_vbatched.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp, vp, vp, vp]
    L.posit32_vbatched.argtypes = [vp, ctypes.POINTER(VBatchDesc), ctypes.POINTER(Tuning)]
    L.posit32_vbatched.restype = i32
    L.posit32_vbatched_default_tuning.argtypes = [i32, ctypes.POINTER(Tuning)]
    L.posit32_vbatched_default_tuning.restype = i32
    L.posit32_queue_create.argtypes = [ctypes.POINTER(QueueCfg), ctypes.POINTER(ctypes.c_void_p)]
    L.posit32_queue_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.posit32_queue_poll.argtypes = [vp, ctypes.c_uint64, vp, ctypes.POINTER(Result)]
    L.posit32_queue_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, vp, ctypes.POINTER(Result)]
    L.posit32_factor_release.argtypes = [vp, ctypes.c_uint64]
    L.posit32_queue_stats.argtypes = [vp, ctypes.POINTER(QueueStats)]
    L.posit32_queue_destroy.argtypes = [vp]
    for f in (L.posit32_queue_create, L.posit32_queue_submit, L.posit32_queue_poll,
              L.posit32_queue_wait, L.posit32_factor_release, L.posit32_queue_stats,
              L.posit32_queue_destroy):
        f.restype = i32
    for f in (L.posit32_from_f64, L.posit32_to_f64, L.posit32_elementwise, L.posit32_getrf,
              L.posit32_getrs, L.posit32_potrf, L.posit32_potrs, L.posit32_getrf_vbatched,
              L.posit32_getrs_vbatched, L.posit32_gesv_vbatched, L.posit32_potrf_vbatched,
              L.posit32_potrs_vbatched, L.posit32_posv_vbatched):
        f.restype = i32
    _lib = L
    return L


def _check(rc: int, what: str) -> None:
    if rc != 0:
        msg = lib().posit32_strerror(rc).decode()
        raise Posit32Error(f"{what} failed with code {rc}: {msg}", rc)


KIND_CODES = {"lu": 0, "chol": 1}
_tunings: dict | None = None
TUNING_DIR = os.path.join(HERE, "tuning")


def default_tuning(kind: str) -> Tuning:
    """The library's built-in sub-panel table for kind "lu" or "chol"."""
    t = Tuning()
    _check(lib().posit32_vbatched_default_tuning(KIND_CODES[kind], ctypes.byref(t)),
           "posit32_vbatched_default_tuning")
    return t


def tuning_file() -> str | None:
    """The tuning file in use: $POSIT32_TUNING (a path, or "builtin" for
    none), else tuning/<arch>.json beside this module if it exists (written by
    paper_2401_14117_amd.autotune for the current GPU)."""
    env = os.environ.get("POSIT32_TUNING")
    if env:
        return None if env == "builtin" else env
    if not torch.cuda.is_available():
        return None
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = os.path.join(TUNING_DIR, f"{arch}.json")
    return path if os.path.exists(path) else None


def active_tuning(kind: str) -> Tuning | None:
    """The measured table for kind from tuning_file(), or None (the library's
    built-in table)."""
    global _tunings
    if _tunings is None:
        _tunings = {}
        path = tuning_file()
        if path is not None:
            import json
            with open(path) as f:
                data = json.load(f)
            for k in KIND_CODES:
                if k in data:
                    _tunings[k] = Tuning.make(data[k]["max_n"], data[k]["sub"])
    return _tunings.get(kind)


def set_active_tuning(kind: str, tuning: Tuning | None) -> None:
    """Replace the table used by VBatch and Queue for kind (None: built-in)."""
    active_tuning(kind)
    if tuning is None:
        _tunings.pop(kind, None)
    else:
        _tunings[kind] = tuning


def _stream(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _ld(t: torch.Tensor) -> int:
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if t.numel() and t.stride(1) != 1:
        raise ValueError("matrices must have unit column stride (row-major)")
    return max(t.stride(0), 1) if t.shape[0] > 1 else max(t.shape[1], 1)


def _is_i32_cuda(t: torch.Tensor) -> None:
    if t.dtype != torch.int32 or not t.is_cuda:
        raise TypeError("posit tensors must be torch.int32 on a CUDA (HIP) device")


def gemm(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor, alpha: int = ONE, beta: int = ONE,
         transa: bool = False, transb: bool = False, stream=None) -> torch.Tensor:
    """In place: C = alpha*op(A)*op(B) + beta*C (Posit(32,2)); returns C."""
    for t in (A, B, C):
        _is_i32_cuda(t)
    m, n = C.shape
    k = A.shape[0] if transa else A.shape[1]
    if (A.shape[1] if transa else A.shape[0]) != m:
        raise ValueError("op(A) rows must equal C rows")
    if (B.shape[1] if transb else B.shape[0]) != k or (B.shape[0] if transb else B.shape[1]) != n:
        raise ValueError("op(B) must be k x n")
    rc = lib().posit32_gemm(_stream(stream), int(transa), int(transb), m, n, k,
                            alpha & 0xFFFFFFFF, _ptr(A), _ld(A), _ptr(B), _ld(B),
                            beta & 0xFFFFFFFF, _ptr(C), _ld(C))
    _check(rc, "posit32_gemm")
    return C


def gemm_raw(transa: int, transb: int, m: int, n: int, k: int, alpha: int, A_ptr, lda: int,
             B_ptr, ldb: int, beta: int, C_ptr, ldc: int, stream=None) -> int:
    """Direct call of the C entry point with raw pointers; returns its code."""
    return lib().posit32_gemm(_stream(stream) if torch.cuda.is_available() else None,
                              transa, transb, m, n, k, alpha & 0xFFFFFFFF, A_ptr, lda,
                              B_ptr, ldb, beta & 0xFFFFFFFF, C_ptr, ldc)


def from_f64(x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if x.dtype != torch.float64 or not x.is_cuda:
        raise TypeError("from_f64 expects a float64 CUDA tensor")
    x = x.contiguous()
    if out is None:
        out = torch.empty(x.shape, dtype=torch.int32, device=x.device)
    else:
        _is_i32_cuda(out)
        if out.numel() != x.numel() or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor with x's number of elements")
    _check(lib().posit32_from_f64(_stream(stream), x.numel(), _ptr(x), _ptr(out)), "posit32_from_f64")
    return out


def to_f64(p: torch.Tensor, stream=None) -> torch.Tensor:
    _is_i32_cuda(p)
    p = p.contiguous()
    out = torch.empty(p.shape, dtype=torch.float64, device=p.device)
    _check(lib().posit32_to_f64(_stream(stream), p.numel(), _ptr(p), _ptr(out)), "posit32_to_f64")
    return out


def elementwise(op: int, a: torch.Tensor, b: torch.Tensor | None = None, stream=None,
                out: torch.Tensor | None = None) -> torch.Tensor:
    _is_i32_cuda(a)
    a = a.contiguous()
    if b is not None:
        _is_i32_cuda(b)
        b = b.contiguous()
        if b.shape != a.shape:
            raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty_like(a)
    else:
        _is_i32_cuda(out)
        if out.shape != a.shape or not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor of a's shape")
    _check(lib().posit32_elementwise(_stream(stream), op, a.numel(), _ptr(a), _ptr(b), _ptr(out)),
           "posit32_elementwise")
    return out


def version() -> int:
    return lib().posit32_version()


def _square(A: torch.Tensor) -> int:
    _is_i32_cuda(A)
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("expected a square matrix")
    return A.shape[0]


def _rhs(B: torch.Tensor, n: int) -> torch.Tensor:
    _is_i32_cuda(B)
    if B.dim() == 1:
        B = B.view(-1, 1)
    if B.shape[0] != n:
        raise ValueError("right-hand side has the wrong number of rows")
    return B


def getrf(A: torch.Tensor, nb: int = 256, stream=None):
    """In place LU with partial pivoting; returns (A, ipiv, info) with ipiv an
    int32 device tensor (0-based) and info a 1-element int32 device tensor."""
    n = _square(A)
    ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    info = torch.empty(1, dtype=torch.int32, device=A.device)
    _check(lib().posit32_getrf(_stream(stream), n, nb, _ptr(A), _ld(A), _ptr(ipiv), _ptr(info)),
           "posit32_getrf")
    return A, ipiv[:n], info


def getrf_phases(A: torch.Tensor, nb: int = 256, stream=None):
    """getrf with its phases timed by HIP events (synchronises the stream);
    returns (A, ipiv, info, {panel, interchanges, u12_solve, trailing_update} in ms)."""
    n = _square(A)
    ipiv = torch.empty(max(n, 1), dtype=torch.int32, device=A.device)
    info = torch.empty(1, dtype=torch.int32, device=A.device)
    ms = (ctypes.c_double * 4)()
    _check(lib().posit32_getrf_phases(_stream(stream), n, nb, _ptr(A), _ld(A), _ptr(ipiv), _ptr(info), ms),
           "posit32_getrf_phases")
    names = ("panel", "interchanges", "u12_solve", "trailing_update")
    return A, ipiv[:n], info, {k: round(v, 3) for k, v in zip(names, ms)}


GROUP_MAX = 16


def getrf_group(As, nb: int = 256, stream=None):
    """In place LU of up to GROUP_MAX independent square matrices advanced
    together (posit32_getrf_group); returns [(A, ipiv, info)] as getrf."""
    if len(As) > GROUP_MAX:
        raise ValueError(f"at most {GROUP_MAX} systems per group")
    count = len(As)
    ns = (ctypes.c_int64 * max(count, 1))(*[_square(A) for A in As])
    ldas = (ctypes.c_int64 * max(count, 1))(*[_ld(A) for A in As])
    ipivs = [torch.empty(max(A.shape[0], 1), dtype=torch.int32, device=A.device) for A in As]
    infos = [torch.empty(1, dtype=torch.int32, device=A.device) for A in As]
    Ap = (ctypes.c_void_p * max(count, 1))(*[A.data_ptr() for A in As])
    Pp = (ctypes.c_void_p * max(count, 1))(*[p.data_ptr() for p in ipivs])
    Ip = (ctypes.c_void_p * max(count, 1))(*[i.data_ptr() for i in infos])
    _check(lib().posit32_getrf_group(_stream(stream), count, ns, nb, Ap, ldas, Pp, Ip), "posit32_getrf_group")
    return [(A, p[:A.shape[0]], i) for A, p, i in zip(As, ipivs, infos)]


def getrs_group(LUs, ipivs, Bs, stream=None):
    """In place A_i X_i = B_i for up to GROUP_MAX systems at once
    (posit32_getrs_group) with the factors of getrf; returns Bs."""
    count = len(LUs)
    if count > GROUP_MAX or len(ipivs) != count or len(Bs) != count:
        raise ValueError(f"at most {GROUP_MAX} systems, one pivot vector and right-hand side each")
    B2 = [_rhs(B, _square(LU)) for LU, B in zip(LUs, Bs)]
    c = max(count, 1)
    ns = (ctypes.c_int64 * c)(*[LU.shape[0] for LU in LUs])
    rs = (ctypes.c_int64 * c)(*[B.shape[1] for B in B2])
    ldas = (ctypes.c_int64 * c)(*[_ld(LU) for LU in LUs])
    ldbs = (ctypes.c_int64 * c)(*[_ld(B) for B in B2])
    P = lambda ts: (ctypes.c_void_p * c)(*[t.data_ptr() for t in ts])
    _check(lib().posit32_getrs_group(_stream(stream), count, ns, rs, P(LUs), ldas, P(ipivs), P(B2), ldbs),
           "posit32_getrs_group")
    return Bs


def getrs(LU: torch.Tensor, ipiv: torch.Tensor, B: torch.Tensor, stream=None,
          trans: bool = False) -> torch.Tensor:
    """In place solve of A X = B (trans: A^T X = B) with the output of getrf;
    B is n x nrhs (or length n)."""
    n = _square(LU)
    B2 = _rhs(B, n)
    _check(lib().posit32_getrs(_stream(stream), int(bool(trans)), n, B2.shape[1], _ptr(LU), _ld(LU),
                               _ptr(ipiv), _ptr(B2), _ld(B2)), "posit32_getrs")
    return B


def potrf(A: torch.Tensor, nb: int = 256, stream=None, upper: bool = False):
    """In place Cholesky, lower (A = L L^T) or upper (A = U^T U); returns
    (A, info)."""
    n = _square(A)
    info = torch.empty(1, dtype=torch.int32, device=A.device)
    _check(lib().posit32_potrf(_stream(stream), int(bool(upper)), n, nb, _ptr(A), _ld(A), _ptr(info)),
           "posit32_potrf")
    return A, info


def potrs(L: torch.Tensor, B: torch.Tensor, stream=None, upper: bool = False) -> torch.Tensor:
    """In place solve with the output of potrf (the same upper flag)."""
    n = _square(L)
    B2 = _rhs(B, n)
    _check(lib().posit32_potrs(_stream(stream), int(bool(upper)), n, B2.shape[1], _ptr(L), _ld(L),
                               _ptr(B2), _ld(B2)), "posit32_potrs")
    return B


class VBatch:
    """Device-side description of a variable-size batch (the pointer, size and
    leading-dimension arrays of the *_vbatched entry points), built once from
    lists of tensors so that repeated calls only launch.

    As: n_i x n_i int32 device matrices (row-major); Bs: optional n_i x nrhs_i
    right-hand sides; lu: allocate pivot vectors for the LU calls.  The
    tensors stay owned by the caller and must outlive the batch."""

    def __init__(self, As, Bs=None, lu: bool = True, device=None):
        dev = device if device is not None else (As[0].device if As else torch.device("cuda"))
        self.count = len(As)
        ns = []
        for A in As:
            ns.append(_square(A))
        self.max_n = max(ns) if ns else 0
        self.n = torch.tensor(ns, dtype=torch.int32, device=dev)
        self.A = torch.tensor([A.data_ptr() for A in As], dtype=torch.int64, device=dev)
        self.lda = torch.tensor([_ld(A) for A in As], dtype=torch.int64, device=dev)
        self.info = torch.zeros(self.count, dtype=torch.int32, device=dev)
        self.ipivs = None
        self.ipiv = None
        if lu:
            self.ipivs = [torch.empty(max(k, 1), dtype=torch.int32, device=dev) for k in ns]
            self.ipiv = torch.tensor([p.data_ptr() for p in self.ipivs], dtype=torch.int64, device=dev)
        self.nrhs = self.B = self.ldb = None
        if Bs is not None:
            if len(Bs) != self.count:
                raise ValueError("one right-hand side per matrix")
            B2 = [_rhs(B, k) for B, k in zip(Bs, ns)]
            self.nrhs = torch.tensor([b.shape[1] for b in B2], dtype=torch.int32, device=dev)
            self.B = torch.tensor([b.data_ptr() for b in B2], dtype=torch.int64, device=dev)
            self.ldb = torch.tensor([_ld(b) for b in B2], dtype=torch.int64, device=dev)
        self._keep = (As, Bs)

    def _need_b(self):
        if self.B is None:
            raise ValueError("this batch has no right-hand sides")

    def _need_piv(self):
        if self.ipiv is None:
            raise ValueError("this batch was built without pivot vectors (lu=False)")

    def run(self, factor: bool, solve: bool, nb: int = 256, tuning=None, stream=None) -> torch.Tensor:
        """One posit32_vbatched call: factor and/or solve every system with the
        sub-panel table `tuning` (a Tuning; None: active_tuning() of this
        batch's kind, else the library's built-in table)."""
        kind = "lu" if self.ipiv is not None else "chol"
        if solve:
            self._need_b()
        if tuning is None:
            tuning = active_tuning(kind)
        d = VBatchDesc(KIND_CODES[kind], int(factor), int(solve), self.count, self.max_n, nb,
                       _ptr(self.n), _ptr(self.nrhs) if solve else None, _ptr(self.A), _ptr(self.lda),
                       _ptr(self.ipiv), _ptr(self.B) if solve else None, _ptr(self.ldb) if solve else None,
                       _ptr(self.info))
        _check(lib().posit32_vbatched(_stream(stream), ctypes.byref(d),
                                      None if tuning is None else ctypes.byref(tuning)),
               "posit32_vbatched")
        return self.info

    # The six calls below go through posit32_vbatched with the active tuning
    # table unless tuned=False, which calls the dedicated entry points (the
    # library's built-in table).  The results are the same bits either way.
    def getrf(self, nb: int = 256, stream=None, tuned: bool = True) -> torch.Tensor:
        self._need_piv()
        if tuned:
            return self.run(True, False, nb, stream=stream)
        _check(lib().posit32_getrf_vbatched(_stream(stream), self.count, self.max_n, nb, _ptr(self.n),
                                            _ptr(self.A), _ptr(self.lda), _ptr(self.ipiv),
                                            _ptr(self.info)), "posit32_getrf_vbatched")
        return self.info

    def getrs(self, stream=None, tuned: bool = True) -> torch.Tensor:
        self._need_piv()
        self._need_b()
        if tuned:
            return self.run(False, True, stream=stream)
        _check(lib().posit32_getrs_vbatched(_stream(stream), self.count, self.max_n, _ptr(self.n),
                                            _ptr(self.nrhs), _ptr(self.A), _ptr(self.lda),
                                            _ptr(self.ipiv), _ptr(self.B), _ptr(self.ldb),
                                            _ptr(self.info)), "posit32_getrs_vbatched")
        return self.info

    def gesv(self, nb: int = 256, stream=None, tuned: bool = True) -> torch.Tensor:
        self._need_piv()
        self._need_b()
        if tuned:
            return self.run(True, True, nb, stream=stream)
        _check(lib().posit32_gesv_vbatched(_stream(stream), self.count, self.max_n, nb, _ptr(self.n),
                                           _ptr(self.nrhs), _ptr(self.A), _ptr(self.lda),
                                           _ptr(self.ipiv), _ptr(self.B), _ptr(self.ldb),
                                           _ptr(self.info)), "posit32_gesv_vbatched")
        return self.info

    def potrf(self, nb: int = 256, stream=None, tuned: bool = True) -> torch.Tensor:
        if tuned:
            return self.run(True, False, nb, stream=stream)
        _check(lib().posit32_potrf_vbatched(_stream(stream), self.count, self.max_n, nb, _ptr(self.n),
                                            _ptr(self.A), _ptr(self.lda), _ptr(self.info)),
               "posit32_potrf_vbatched")
        return self.info

    def potrs(self, stream=None, tuned: bool = True) -> torch.Tensor:
        self._need_b()
        if tuned:
            return self.run(False, True, stream=stream)
        _check(lib().posit32_potrs_vbatched(_stream(stream), self.count, self.max_n, _ptr(self.n),
                                            _ptr(self.nrhs), _ptr(self.A), _ptr(self.lda),
                                            _ptr(self.B), _ptr(self.ldb), _ptr(self.info)),
               "posit32_potrs_vbatched")
        return self.info

    def posv(self, nb: int = 256, stream=None, tuned: bool = True) -> torch.Tensor:
        self._need_b()
        if tuned:
            return self.run(True, True, nb, stream=stream)
        _check(lib().posit32_posv_vbatched(_stream(stream), self.count, self.max_n, nb, _ptr(self.n),
                                           _ptr(self.nrhs), _ptr(self.A), _ptr(self.lda),
                                           _ptr(self.B), _ptr(self.ldb), _ptr(self.info)),
               "posit32_posv_vbatched")
        return self.info


class Queue:
    """Request queue of the library (posit32_queue_*): submit systems from host
    memory (numpy uint32 patterns), collect their solutions later.  Solutions
    are bit-identical to the batched and single-matrix calls."""

    def __init__(self, device_bytes: int = 2 << 30, max_batch: int = 1024, nb: int = 256,
                 batch_max_n: int = 512, max_pending: int = 0):
        import numpy as np  # noqa: F401
        tl, tc = active_tuning("lu"), active_tuning("chol")
        self._tunings = None
        if tl is not None or tc is not None:
            self._tunings = (Tuning * 2)(tl or default_tuning("lu"), tc or default_tuning("chol"))
        cfg = QueueCfg(device_bytes, max_batch, nb, batch_max_n,
                       ctypes.addressof(self._tunings) if self._tunings is not None else None, max_pending)
        h = ctypes.c_void_p()
        _check(lib().posit32_queue_create(ctypes.byref(cfg), ctypes.byref(h)), "posit32_queue_create")
        self._h = h
        self._shapes = {}

    def submit(self, kind: int, B, A=None, keep: bool = False, factor: int = 0) -> int:
        """Queue one system; A (n x n) and B (n x nrhs or n) are numpy arrays of
        posit patterns (copied at once).  Returns the ticket."""
        import numpy as np
        B2 = np.ascontiguousarray(B, dtype=np.uint32)
        if B2.ndim == 1:
            B2 = B2.reshape(-1, 1)
        n, nrhs = B2.shape
        A2 = None if A is None else np.ascontiguousarray(A, dtype=np.uint32)
        if A2 is not None and A2.shape != (n, n):
            raise ValueError("A must be n x n")
        req = Request(kind, int(keep), n, nrhs,
                      None if A2 is None else A2.ctypes.data, B2.ctypes.data, factor)
        t = ctypes.c_uint64()
        _check(lib().posit32_queue_submit(self._h, ctypes.byref(req), ctypes.byref(t)),
               "posit32_queue_submit")
        self._shapes[t.value] = (n, nrhs)
        return t.value

    def _collect(self, ticket: int, call):
        import numpy as np
        n, nrhs = self._shapes[ticket]
        X = np.empty((n, nrhs), dtype=np.uint32)
        res = Result()
        rc = call(X.ctypes.data, ctypes.byref(res))
        if rc == 1:
            return None
        if -1000 < rc < 0:                        # bad ticket or argument
            _check(rc, "posit32_queue_poll/wait")
        del self._shapes[ticket]
        # a request that failed (status != 0) has no solution: X is None
        return {"X": X if res.status == 0 else None, "status": res.status, "info": res.info,
                "factor": res.factor,
                "submit_s": res.submit_s, "start_s": res.start_s, "done_s": res.done_s}

    def poll(self, ticket: int):
        """The result dict once the request is done, else None: X (the n x nrhs
        solution; the unsolved B when info > 0; None when status != 0), status
        (0 or a library error code), info, factor (a resident factor's handle
        or 0) and the submit / start / done times."""
        return self._collect(ticket, lambda x, r: lib().posit32_queue_poll(self._h, ticket, x, r))

    def wait(self, ticket: int, timeout_s: float = -1.0):
        return self._collect(ticket, lambda x, r: lib().posit32_queue_wait(self._h, ticket,
                                                                              timeout_s, x, r))

    def release(self, factor: int) -> None:
        _check(lib().posit32_factor_release(self._h, factor), "posit32_factor_release")

    def stats(self) -> dict:
        st = QueueStats()
        _check(lib().posit32_queue_stats(self._h, ctypes.byref(st)), "posit32_queue_stats")
        return {f: getattr(st, f) for f, _ in QueueStats._fields_}

    def close(self) -> None:
        if self._h:
            _check(lib().posit32_queue_destroy(self._h), "posit32_queue_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
