"""The C-ABI library loads, exports every symbol its header declares, and
rejects invalid arguments before launching anything (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "posit32.h")).read()
    return sorted(set(re.findall(r"\b(posit32_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2401_14117_amd import posit32
    return posit32.lib()


def test_header_symbols_exported(L):
    syms = _declared_symbols()
    assert "posit32_gemm" in syms and len(syms) >= 5
    for s in syms:
        assert hasattr(L, s), s


def test_version_and_strerror(L):
    assert L.posit32_version() >= 100
    assert L.posit32_strerror(0) == b"ok"
    assert b"argument" in L.posit32_strerror(-3)


@pytest.mark.parametrize("args,code", [
    ((2, 0, 4, 4, 4, 8, 4, 8, 4, 8, 4), -2),      # bad transa
    ((0, 7, 4, 4, 4, 8, 4, 8, 4, 8, 4), -3),      # bad transb
    ((0, 0, -1, 4, 4, 8, 4, 8, 4, 8, 4), -4),     # m < 0
    ((0, 0, 4, -1, 4, 8, 4, 8, 4, 8, 4), -5),     # n < 0
    ((0, 0, 4, 4, -1, 8, 4, 8, 4, 8, 4), -6),     # k < 0
    ((0, 0, 4, 4, 4, 8, 3, 8, 4, 8, 4), -9),      # lda < k
    ((1, 0, 5, 4, 4, 8, 4, 8, 4, 8, 5), -9),      # lda < m for A^T
    ((0, 0, 4, 4, 4, 8, 4, 8, 3, 8, 4), -11),     # ldb < n
    ((0, 1, 4, 4, 5, 8, 5, 8, 4, 8, 4), -11),     # ldb < k for B^T
    ((0, 0, 4, 4, 4, 8, 4, 8, 4, 8, 3), -14),     # ldc < n
    ((0, 0, 4, 4, 4, 0, 4, 8, 4, 8, 4), -8),      # A null
    ((0, 0, 4, 4, 4, 8, 4, 0, 4, 8, 4), -10),     # B null
    ((0, 0, 4, 4, 4, 8, 4, 8, 4, 0, 4), -13),     # C null
    ((0, 0, 4, 4, 4, 8, 4, 16, 4, 8, 4), -13),    # C aliases A (A = C = 8)
])
def test_gemm_argument_errors(L, args, code):
    ta, tb, m, n, k, A, lda, B, ldb, C, ldc = args
    # pointers are never dereferenced: validation fails before any launch
    rc = L.posit32_gemm(None, ta, tb, m, n, k, 0x40000000, A or None, lda, B or None, ldb,
                        0x40000000, C or None, ldc)
    assert rc == code


def test_gemm_noop_shapes_return_ok(L):
    # m == 0 or n == 0: nothing to do, null pointers allowed
    assert L.posit32_gemm(None, 0, 0, 0, 5, 5, 0x40000000, None, 5, None, 5, 0, None, 5) == 0
    assert L.posit32_gemm(None, 0, 0, 5, 0, 5, 0x40000000, None, 5, None, 1, 0, None, 1) == 0


def test_other_argument_errors(L):
    assert L.posit32_from_f64(None, -1, None, None) == -2
    assert L.posit32_from_f64(None, 4, None, 8) == -3
    assert L.posit32_to_f64(None, 4, 8, None) == -4
    assert L.posit32_elementwise(None, 9, 4, 8, 8, 8) == -2
    assert L.posit32_elementwise(None, 0, -4, 8, 8, 8) == -3
    assert L.posit32_elementwise(None, 0, 4, 8, None, 8) == -5
    assert L.posit32_from_f64(None, 0, None, None) == 0


def test_factorisation_argument_errors(L):
    # validated on the host before anything is launched (no GPU needed)
    assert L.posit32_getrf(None, -1, 256, 8, 1, 8, 8) == -2
    assert L.posit32_getrf(None, 4, 0, 8, 4, 8, 8) == -3
    assert L.posit32_getrf(None, 4, 257, 8, 4, 8, 8) == -3
    assert L.posit32_getrf(None, 4, 64, None, 4, 8, 8) == -4
    assert L.posit32_getrf(None, 4, 64, 8, 3, 8, 8) == -5
    assert L.posit32_getrf(None, 4, 64, 8, 4, None, 8) == -6
    assert L.posit32_getrf(None, 4, 64, 8, 4, 8, None) == -7
    # the phase-timed getrf validates like getrf, plus its host array
    assert L.posit32_getrf_phases(None, -1, 256, 8, 1, 8, 8, 8) == -2
    assert L.posit32_getrf_phases(None, 4, 64, 8, 4, 8, 8, None) == -8
    # the allocation-free getrf validates exactly like getrf
    assert L.posit32_getrf_noalloc(None, -1, 256, 8, 1, 8, 8) == -2
    assert L.posit32_getrf_noalloc(None, 4, 257, 8, 4, 8, 8) == -3
    assert L.posit32_getrf_noalloc(None, 4, 64, None, 4, 8, 8) == -4
    assert L.posit32_getrf_noalloc(None, 4, 64, 8, 3, 8, 8) == -5
    assert L.posit32_getrf_noalloc(None, 4, 64, 8, 4, None, 8) == -6
    assert L.posit32_getrf_noalloc(None, 4, 64, 8, 4, 8, None) == -7
    assert L.posit32_getrf_noalloc(None, 1 << 24, 64, 8, 1 << 24, 8, 8) == -2
    # getrf_group(stream, count, n[], nb, A[], lda[], ipiv[], info[]) with host arrays
    I64x2, Px2 = ctypes.c_int64 * 2, ctypes.c_void_p * 2
    n2, ld2, p2 = I64x2(4, 3), I64x2(4, 3), Px2(8, 16)
    assert L.posit32_getrf_group(None, 17, n2, 64, p2, ld2, p2, p2) == -2
    assert L.posit32_getrf_group(None, -1, n2, 64, p2, ld2, p2, p2) == -2
    assert L.posit32_getrf_group(None, 0, None, 64, None, None, None, None) == 0
    assert L.posit32_getrf_group(None, 2, None, 64, p2, ld2, p2, p2) == -3
    assert L.posit32_getrf_group(None, 2, I64x2(4, -1), 64, p2, ld2, p2, p2) == -3
    assert L.posit32_getrf_group(None, 2, n2, 0, p2, ld2, p2, p2) == -4
    assert L.posit32_getrf_group(None, 2, n2, 64, Px2(8, None), ld2, p2, p2) == -5
    assert L.posit32_getrf_group(None, 2, n2, 64, Px2(8, 8), ld2, p2, p2) == -5     # shared matrix
    assert L.posit32_getrf_group(None, 2, n2, 64, p2, I64x2(4, 2), p2, p2) == -6
    assert L.posit32_getrf_group(None, 2, n2, 64, p2, ld2, None, p2) == -7
    assert L.posit32_getrf_group(None, 2, n2, 64, p2, ld2, p2, Px2(8, None)) == -8
    # getrs_group(stream, count, n[], nrhs[], LU[], lda[], ipiv[], B[], ldb[])
    r2 = I64x2(1, 2)
    assert L.posit32_getrs_group(None, 17, n2, r2, p2, ld2, p2, p2, r2) == -2
    assert L.posit32_getrs_group(None, 0, None, None, None, None, None, None, None) == 0
    assert L.posit32_getrs_group(None, 2, I64x2(-1, 3), r2, p2, ld2, p2, p2, r2) == -3
    assert L.posit32_getrs_group(None, 2, n2, I64x2(1, 70000), p2, ld2, p2, p2, r2) == -4
    assert L.posit32_getrs_group(None, 2, n2, r2, Px2(None, 8), ld2, p2, p2, r2) == -5
    assert L.posit32_getrs_group(None, 2, n2, r2, p2, I64x2(3, 3), p2, p2, r2) == -6
    assert L.posit32_getrs_group(None, 2, n2, r2, p2, ld2, None, p2, r2) == -7
    assert L.posit32_getrs_group(None, 2, n2, r2, p2, ld2, p2, Px2(8, 8), r2) == -8
    assert L.posit32_getrs_group(None, 2, n2, r2, p2, ld2, p2, p2, I64x2(1, 1)) == -9
    # getrs(stream, op, n, nrhs, LU, lda, ipiv, B, ldb)
    assert L.posit32_getrs(None, 2, 4, 1, 8, 4, 8, 8, 1) == -2
    assert L.posit32_getrs(None, -1, 4, 1, 8, 4, 8, 8, 1) == -2
    assert L.posit32_getrs(None, 1, -1, 1, 8, 4, 8, 8, 1) == -3
    assert L.posit32_getrs(None, 0, 4, -1, 8, 4, 8, 8, 1) == -4
    assert L.posit32_getrs(None, 1, 4, 1, None, 4, 8, 8, 1) == -5
    assert L.posit32_getrs(None, 1, 4, 1, 8, 3, 8, 8, 1) == -6
    assert L.posit32_getrs(None, 1, 4, 1, 8, 4, None, 8, 1) == -7
    assert L.posit32_getrs(None, 1, 4, 1, 8, 4, 8, None, 1) == -8
    assert L.posit32_getrs(None, 0, 4, 2, 8, 4, 8, 8, 1) == -9
    assert L.posit32_getrs(None, 1, 0, 0, None, 1, None, None, 1) == 0
    # potrf(stream, uplo, n, nb, A, lda, info)
    assert L.posit32_potrf(None, 2, 4, 64, 8, 4, 8) == -2
    assert L.posit32_potrf(None, 1, -4, 64, 8, 4, 8) == -3
    assert L.posit32_potrf(None, 1, (1 << 20) + 1, 64, 8, (1 << 20) + 1, 8) == -3
    assert L.posit32_potrf(None, 0, 4, 0, 8, 4, 8) == -4
    assert L.posit32_potrf(None, 1, 4, 64, None, 4, 8) == -5
    assert L.posit32_potrf(None, 1, 4, 64, 8, 2, 8) == -6
    assert L.posit32_potrf(None, 0, 4, 64, 8, 4, None) == -7
    # potrs(stream, uplo, n, nrhs, L, lda, B, ldb)
    assert L.posit32_potrs(None, 3, 4, 2, 8, 4, 8, 2) == -2
    assert L.posit32_potrs(None, 1, -4, 2, 8, 4, 8, 2) == -3
    assert L.posit32_potrs(None, 1, 4, -2, 8, 4, 8, 2) == -4
    assert L.posit32_potrs(None, 1, 4, 2, None, 4, 8, 2) == -5
    assert L.posit32_potrs(None, 1, 4, 2, 8, 1, 8, 2) == -6
    assert L.posit32_potrs(None, 0, 4, 2, 8, 4, None, 2) == -7
    assert L.posit32_potrs(None, 1, 4, 2, 8, 4, 8, 1) == -8
    assert L.posit32_potrs(None, 1, 0, 0, None, 1, None, 1) == 0


def test_vbatched_argument_errors(L):
    # count, max_n, nb and null arrays are checked on the host; count = 0 is a no-op
    assert L.posit32_getrf_vbatched(None, -1, 8, 256, 8, 8, 8, 8, 8) == -2
    assert L.posit32_getrf_vbatched(None, 1 << 24, 8, 256, 8, 8, 8, 8, 8) == -2   # > P32_VBATCH_MAX_COUNT
    assert L.posit32_gesv_vbatched(None, (1 << 24) - 1, 1 << 24, 256, 8, 8, 8, 8, 8, 8, 8, 8) == -3
    assert L.posit32_getrf_vbatched(None, 1, -1, 256, 8, 8, 8, 8, 8) == -3
    assert L.posit32_getrf_vbatched(None, 1, 1 << 24, 256, 8, 8, 8, 8, 8) == -3
    assert L.posit32_getrf_vbatched(None, 1, 8, 0, 8, 8, 8, 8, 8) == -4
    assert L.posit32_getrf_vbatched(None, 1, 8, 256, None, 8, 8, 8, 8) == -5
    assert L.posit32_getrf_vbatched(None, 1, 8, 256, 8, 8, 8, None, 8) == -5
    assert L.posit32_gesv_vbatched(None, 1, 8, 256, 8, None, 8, 8, 8, 8, 8, 8) == -5
    assert L.posit32_posv_vbatched(None, 1, 8, 300, 8, 8, 8, 8, 8, 8, 8) == -4
    assert L.posit32_potrs_vbatched(None, 1, 8, 8, 8, 8, 8, None, 8, 8) == -5
    assert L.posit32_getrs_vbatched(None, 1, 8, 8, 8, 8, 8, 8, 8, 8, None) == -5
    assert L.posit32_potrf_vbatched(None, 0, 0, 256, None, None, None, None) == 0
    assert L.posit32_gesv_vbatched(None, 0, 0, 256, None, None, None, None, None, None, None,
                                   None) == 0


def test_queue_argument_errors(L):
    # configuration and handle checks happen before any device call
    from paper_2401_14117_amd.posit32 import QueueCfg, Request
    import ctypes
    h = ctypes.c_void_p()
    for cfg in (QueueCfg(1 << 10, 16, 256, 512), QueueCfg(1 << 30, 0, 256, 512),
                QueueCfg(1 << 30, 16, 0, 512), QueueCfg(1 << 30, 16, 300, 512),
                QueueCfg(1 << 30, 16, 256, -1), QueueCfg(1 << 30, 16, 256, 512, None, -1)):
        assert L.posit32_queue_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    assert L.posit32_queue_create(None, ctypes.byref(h)) == -1
    t = ctypes.c_uint64()
    assert L.posit32_queue_submit(None, ctypes.byref(Request()), ctypes.byref(t)) == -1
    assert L.posit32_factor_release(None, 1) == -1
    assert L.posit32_queue_destroy(None) == -1
    assert L.posit32_strerror(-4000) == b"the system does not fit the queue's device pool"
    assert L.posit32_strerror(-5000) == b"the queue holds its maximum of unretired requests"


def test_vbatched_descriptor_and_tuning_validation(L):
    """posit32_vbatched checks its descriptor and table on the host (nothing
    is dereferenced or launched when they are invalid)."""
    import ctypes
    from paper_2401_14117_amd import posit32 as P
    ok = dict(kind=0, factor=1, solve=1, count=4, max_n=10, nb=256, n=8, nrhs=8, A=8, lda=8, ipiv=8,
              B=8, ldb=8, info=8)

    def desc(**kw):
        d = dict(ok)
        d.update(kw)
        return P.VBatchDesc(*[d[f] for f, _ in P.VBatchDesc._fields_])

    def call(d, t=None):
        return L.posit32_vbatched(None, None if d is None else ctypes.byref(d),
                                  None if t is None else ctypes.byref(t))

    assert call(None) == -2
    for bad in (dict(kind=2), dict(factor=0, solve=0), dict(factor=2), dict(count=-1), dict(max_n=-1),
                dict(nb=0), dict(nb=257), dict(n=None), dict(ipiv=None), dict(nrhs=None), dict(B=None),
                dict(info=None)):
        assert call(desc(**bad)) == -2, bad
    big = 2**31 - 1
    for t in (P.Tuning.make([big], [0]), P.Tuning.make([big], [65]), P.Tuning.make([50, 50], [8, 8]),
              P.Tuning.make([50, 20], [8, 8])):
        assert call(desc(), t) == -3, t.to_dict()
    t = P.Tuning()
    t.buckets = 9
    assert call(desc(), t) == -3
    t.buckets = 0
    assert call(desc(), t) == -3
    # an empty batch is valid and launches nothing
    assert call(desc(count=0, n=None, A=None, lda=None, ipiv=None, nrhs=None, B=None, ldb=None,
                     info=None), P.Tuning.make([big], [16])) == 0


def test_default_tuning_tables(L):
    from paper_2401_14117_amd import posit32 as P
    for kind in ("lu", "chol"):
        t = P.default_tuning(kind)
        assert 1 <= t.buckets <= P.TUNE_BUCKETS
        mx = list(t.max_n)[:t.buckets]
        assert mx == sorted(mx) and len(set(mx)) == len(mx) and mx[-1] == 2**31 - 1
        assert all(1 <= s <= 64 for s in list(t.sub)[:t.buckets])
    assert L.posit32_vbatched_default_tuning(2, None) == -1
    assert L.posit32_vbatched_default_tuning(0, None) == -2
