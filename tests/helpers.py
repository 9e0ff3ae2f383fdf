"""Shared test helpers: moving posit patterns between numpy and the device,
and building seeded inputs through the oracle's own conversion."""
import numpy as np

import oracle as O
from paper_2401_14117_amd import workloads as W


def to_dev(a: np.ndarray):
    import torch
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32).copy()).cuda()


def from_dev(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def oracle_patterns(mat: W.Matrix) -> np.ndarray:
    """Posit(32,2) patterns of a workload matrix, converted by the oracle."""
    p = O.vec_from_double(mat.values)
    return W.apply_masks(p, mat)


def case_patterns(case: W.GemmCase):
    return (oracle_patterns(case.A), oracle_patterns(case.B), oracle_patterns(case.C),
            O.from_double(case.alpha), O.from_double(case.beta))


def stratified_patterns(rng: np.random.Generator, count: int) -> np.ndarray:
    """Random Posit(32,2) patterns with the regime length drawn uniformly
    (every magnitude from minpos to maxpos well represented), plus specials."""
    m = rng.integers(1, 32, count).astype(np.int64)  # regime run length 1..31
    lead = rng.integers(0, 2, count).astype(np.int64)
    tail = rng.integers(0, 1 << 31, count, dtype=np.int64)
    one = np.int64(1)
    run = np.where(lead == 1, ((one << m) - 1) << (31 - m), 0)
    has_term = m < 31
    rest = np.where(has_term, 30 - m, 0)
    term = np.where(has_term & (lead == 0), one << rest, 0)
    body = run | term | np.where(has_term, tail & ((one << rest) - 1), 0)
    neg = rng.integers(0, 2, count).astype(bool)
    pats = np.where(neg, (1 << 32) - body, body) & 0xFFFFFFFF
    specials = np.array([0, 0x80000000, 1, 0x7FFFFFFF, 0xFFFFFFFF, 0x80000001, 0x40000000,
                         0xC0000000], dtype=np.int64)
    return np.concatenate([pats, specials]).astype(np.uint32)
