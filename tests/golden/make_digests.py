"""Writes tests/golden/digests.json: SHA-256 digests of the oracle's results on
workloads too large to compare inline in a GPU test (the Rgemm sweep's
square cases, the factor + solve cases at n = 1024 and 4096, 10^8 elementwise
pairs per operation, the square root of every non-negative pattern).

Only the oracle (``oracle/``) and the seeded input generators
(``paper_2401_14117_amd/workloads.py``, ``tests/helpers.py``) are called: no
expected value comes from the GPU library.  The GPU tests regenerate the same
inputs, run the library, hash its results the same way and compare.  Each
entry also records the digest of the inputs, so a change of the generators
shows as an input mismatch rather than as a wrong result.

    python tests/golden/make_digests.py [name ...]     (default: every case)

Runs for tens of minutes on a few cores (the n = 4096 factorisations and the
n = 2048 Rgemm dominate); existing entries of other cases are kept.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2401_14117_amd import workloads as W  # noqa: E402
from tests.helpers import stratified_patterns  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "digests.json")

# elementwise: 10 chunks of 10^7 stratified pairs, chunk c from default_rng([9100, c])
EW_CHUNKS, EW_CHUNK = 10, 10_000_000
# square root of every non-negative pattern, 2^27 per chunk
SQRT_CHUNK = 1 << 27


def sha(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).astype(np.asarray(a).dtype.newbyteorder("<")).tobytes())
    return h.hexdigest()


def gemm_inputs(case: W.GemmCase):
    A = W.apply_masks(O.vec_from_double(case.A.values), case.A)
    B = W.apply_masks(O.vec_from_double(case.B.values), case.B)
    C = W.apply_masks(O.vec_from_double(case.C.values), case.C)
    return A, B, C, O.from_double(case.alpha), O.from_double(case.beta)


def case_gemm_square(n: int) -> dict:
    A, B, C, alpha, beta = gemm_inputs(W.gemm_square(n))
    out = O.gemm(A, B, C, alpha, beta)
    return {"inputs": sha(A, B, C), "C": sha(out)}


def lu_inputs(n: int):
    case = W.lu_case(n)
    return O.vec_from_double(case.A), O.vec_from_double(case.b)


def case_lu(n: int) -> dict:
    A, b = lu_inputs(n)
    LU, ipiv, info = O.getrf(A, 256)
    X = O.getrs(LU, ipiv, b)
    XT = O.getrs(LU, ipiv, b, trans=True)
    return {"inputs": sha(A, b), "LU": sha(LU), "ipiv": sha(ipiv.astype(np.int32)), "info": info,
            "X": sha(X), "XT": sha(XT)}


def chol_inputs(n: int):
    case = W.chol_case(n)
    return O.vec_from_double(case.A), O.vec_from_double(case.b)


def case_chol(n: int) -> dict:
    A, b = chol_inputs(n)
    L, info = O.potrf(A, 256)
    X = O.potrs(L, b)
    return {"inputs": sha(A, b), "L": sha(np.tril(L)), "info": info, "X": sha(X)}


def ew_chunk(c: int):
    rng = np.random.default_rng([9100, c])
    a = stratified_patterns(rng, EW_CHUNK)
    b = stratified_patterns(rng, EW_CHUNK)
    return a, b


def case_elementwise() -> dict:
    ops = ("add", "sub", "mul", "div")
    hs = {op: hashlib.sha256() for op in ops}
    hin = hashlib.sha256()
    for c in range(EW_CHUNKS):
        a, b = ew_chunk(c)
        hin.update(a.tobytes())
        hin.update(b.tobytes())
        for op in ops:
            hs[op].update(O.vec_op(op, a, b).tobytes())
    out = {"inputs": hin.hexdigest(), "pairs_per_op": EW_CHUNKS * (EW_CHUNK + 8)}
    out.update({op: h.hexdigest() for op, h in hs.items()})
    return out


def case_sqrt_all() -> dict:
    h = hashlib.sha256()
    for start in range(0, 1 << 31, SQRT_CHUNK):
        a = np.arange(start, start + SQRT_CHUNK, dtype=np.uint32)
        h.update(O.vec_op("sqrt", a).tobytes())
    return {"patterns": "0x00000000 .. 0x7FFFFFFF", "sqrt": h.hexdigest()}


CASES = {
    "gemm_square_n1024": lambda: case_gemm_square(1024),
    "gemm_square_n2048": lambda: case_gemm_square(2048),
    "lu_n1024": lambda: case_lu(1024),
    "chol_n1024": lambda: case_chol(1024),
    "lu_n4096": lambda: case_lu(4096),
    "chol_n4096": lambda: case_chol(4096),
    "elementwise_1e8": case_elementwise,
    "sqrt_all_nonnegative": case_sqrt_all,
}


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names or list(CASES):
        t0 = time.time()
        data[name] = CASES[name]()
        data[name]["oracle_s"] = round(time.time() - t0, 1)
        data[name]["oracle_threads"] = O.num_threads()
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)
        print(f"{name}: {time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
