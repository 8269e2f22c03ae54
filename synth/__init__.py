"""Seeded synthetic GF(2) matrices for tests and benchmarks.

Inputs only: nothing here performs a step of the PLS/RREF method.  Both the CPU
oracle's tests and the GPU path's tests draw their inputs from this module, so
the two sides see identical bits.

Layout: a matrix is a ``numpy.uint64`` array of shape ``(m, stride)``; column
``j`` of row ``i`` is bit ``j % 64`` of word ``A[i, j // 64]`` (LSB first).  Bits
past column ``n`` are zero.

Random numbers: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) used counter-based,
``value(seed, i) = mix64(seed + (i + 1) * 0x9E3779B97F4A7C15)``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gf2synth.c")
_LIB = os.path.join(_HERE, "libgf2synth.so")
_lib = None

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def build(force: bool = False) -> str:
    """Compile the generator with gcc (OpenMP) into ``synth/libgf2synth.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        u64, i64, p = ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p
        lib.synth_splitmix.restype = u64
        lib.synth_splitmix.argtypes = [u64, u64]
        lib.synth_substream.restype = u64
        lib.synth_substream.argtypes = [u64, u64]
        lib.synth_fill_half.restype = None
        lib.synth_fill_half.argtypes = [p, i64, i64, i64, u64]
        lib.synth_fill_bernoulli.restype = None
        lib.synth_fill_bernoulli.argtypes = [p, i64, i64, i64, u64, u64]
        lib.synth_fill_planted.restype = ctypes.c_int
        lib.synth_fill_planted.argtypes = [p, i64, i64, i64, i64, u64, u64, ctypes.c_int]
        _lib = lib
    return _lib


def splitmix(seed: int, i: int) -> int:
    """Pure-Python SplitMix64 value(seed, i); identical to the C generator."""
    z = (seed + (i + 1) * GOLDEN) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def words_per_row(n: int) -> int:
    return (n + 63) // 64


def threshold(p: float) -> int:
    """Integer threshold round(p * 2^32) for Bernoulli(p) bits."""
    return int(round(p * (1 << 32)))


def empty(m: int, n: int, stride: int | None = None) -> np.ndarray:
    stride = words_per_row(n) if stride is None else stride
    if stride < words_per_row(n):
        raise ValueError("stride too small")
    return np.zeros((m, max(stride, 0)), dtype=np.uint64)


def _ptr(a: np.ndarray) -> int:
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def random_half(m: int, n: int, seed: int, stride: int | None = None) -> np.ndarray:
    """iid Bernoulli(1/2) matrix: each word drawn whole from the generator."""
    a = empty(m, n, stride)
    if a.size:
        _load().synth_fill_half(_ptr(a), m, n, a.shape[1], seed & MASK64)
    return a


def random_bernoulli(m: int, n: int, p: float, seed: int, stride: int | None = None) -> np.ndarray:
    """iid Bernoulli(p) matrix, one generator draw per bit.  p = 0.5 uses random_half."""
    if p == 0.5:
        return random_half(m, n, seed, stride)
    a = empty(m, n, stride)
    if a.size:
        _load().synth_fill_bernoulli(_ptr(a), m, n, a.shape[1], seed & MASK64, threshold(p))
    return a


def planted(m: int, n: int, r: int, seed: int, p: float = 0.5, unit: bool = True,
            stride: int | None = None) -> np.ndarray:
    """A = B*C over GF(2), B (m x r), C (r x n) Bernoulli(p).

    With ``unit`` the factors carry r unit rows / columns at seeded positions, so
    rank(A) = r exactly; without it the literal product is returned (rank r with
    overwhelming probability for p = 1/2 and r well below min(m, n))."""
    a = empty(m, n, stride)
    if a.size:
        th = 0 if p == 0.5 else threshold(p)
        rc = _load().synth_fill_planted(_ptr(a), m, n, a.shape[1], r, seed & MASK64, th,
                                        1 if unit else 0)
        if rc != 0:
            raise ValueError("planted: bad arguments")
    return a


def density(a: np.ndarray, n: int) -> float:
    m = a.shape[0]
    if m == 0 or n == 0:
        return 0.0
    w = words_per_row(n)
    bits = np.unpackbits(a[:, :w].view(np.uint8), axis=1).sum()
    return float(bits) / (m * n)


@dataclass
class BatchItem:
    m: int
    n: int
    p: float
    r: int
    seed: int


def batch_shapes(count: int, seed: int, lo: int = 64, hi: int = 2048,
                 densities=(0.5, 0.1, 0.01)) -> list[BatchItem]:
    """Shapes of the batched workload: m, n log-uniform in [lo, hi] (rounded),
    p uniform over ``densities``, planted rank r uniform in [ceil(min/2), min]."""
    out = []
    for t in range(count):
        u = [splitmix(seed, 4 * t + q) for q in range(4)]
        f = [(x >> 11) * (1.0 / (1 << 53)) for x in u]
        m = int(round(math.exp(math.log(lo) + f[0] * (math.log(hi) - math.log(lo)))))
        n = int(round(math.exp(math.log(lo) + f[1] * (math.log(hi) - math.log(lo)))))
        p = densities[u[2] % len(densities)]
        mn = min(m, n)
        rlo = (mn + 1) // 2
        r = rlo + int(u[3] % (mn - rlo + 1))
        out.append(BatchItem(m=m, n=n, p=p, r=r, seed=(seed * 1000003 + t) & MASK64))
    return out


def batch_matrix(item: BatchItem, stride: int | None = None) -> np.ndarray:
    return planted(item.m, item.n, item.r, item.seed, p=item.p, unit=True, stride=stride)


@dataclass(frozen=True)
class PracticeShape:
    name: str
    m: int
    n: int
    p: float
    seed: int


# Shapes and densities of the four "matrices from practice" of Table 2
# (Section 7).  Those matrices are not available; the stand-ins are iid
# Bernoulli(p) matrices of the same size and density, and match them in nothing
# else (the originals come with structure and rank deficiency of their own).
PRACTICE_SHAPES = (
    PracticeShape("table2_row1", 12307, 13508, 0.076, 25),
    PracticeShape("table2_row2", 19907, 29323, 0.067, 30),
    PracticeShape("table2_row3", 29969, 55800, 0.059, 35),
    PracticeShape("table2_row4", 26075, 26407, 0.185, 40),
)


def practice_matrix(shape: PracticeShape, stride: int | None = None) -> np.ndarray:
    return random_bernoulli(shape.m, shape.n, shape.p, shape.seed, stride)

