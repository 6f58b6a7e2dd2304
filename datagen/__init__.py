"""Seeded synthetic inputs: sparse tf-idf document sets and index draws.

This module is the one input source shared by the oracle tests, the GPU tests
and the benchmark.  It holds none of the clustering arithmetic; the generator
itself is plain C (``gen.c``) so that multi-million-document sets are produced
in seconds and identically on every machine.

Workload shapes follow the paper's two document sets (PubMed abstracts:
D = 140,914 terms, 58.95 nonzeros per document; NYT articles: 225.76 nonzeros
per document; Section "Data Sets"), with synthetic Zipf term draws in place of
the real collections, which are not available here.
"""
from __future__ import annotations

import ctypes
import hashlib
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c into libgen.so (plain gcc + OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               os.path.join(_HERE, "gen.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        i64, u64, dbl, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int32
        vp = ctypes.c_void_p
        lib.gen_count.argtypes = [i64, i64, dbl, i64, i64, u64, vp]
        lib.gen_fill.argtypes = [i64, i64, dbl, i64, i64, dbl, u64, vp, vp, vp, vp, vp]
        lib.gen_perm_prefix.argtypes = [i64, i64, u64, u64, vp]
        lib.gen_uniform_labels.argtypes = [i64, i32, u64, u64, vp]
        lib.gen_uniform01.argtypes = [i64, u64, u64, vp]
        for f in (lib.gen_count, lib.gen_fill, lib.gen_perm_prefix, lib.gen_uniform_labels,
                  lib.gen_uniform01):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class CSR:
    """Object set in CSR form: ascending term ids per row, FP32 values."""
    n: int
    d: int
    indptr: np.ndarray   # int64 [n+1]
    indices: np.ndarray  # int32 [nnz]
    values: np.ndarray   # float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def row(self, i: int):
        a, b = int(self.indptr[i]), int(self.indptr[i + 1])
        return self.indices[a:b], self.values[a:b]

    def subset(self, rows) -> "CSR":
        rows = np.asarray(rows, dtype=np.int64)
        lens = self.indptr[rows + 1] - self.indptr[rows]
        ptr = np.zeros(len(rows) + 1, np.int64)
        np.cumsum(lens, out=ptr[1:])
        idx = np.empty(int(ptr[-1]), np.int32)
        val = np.empty(int(ptr[-1]), np.float32)
        for o, i in enumerate(rows):
            a, b = int(self.indptr[i]), int(self.indptr[i + 1])
            idx[ptr[o]:ptr[o + 1]] = self.indices[a:b]
            val[ptr[o]:ptr[o + 1]] = self.values[a:b]
        return CSR(len(rows), self.d, ptr, idx, val)


def generate(n: int, d: int, lam: float, lo: int, hi: int, s: float, seed: int) -> CSR:
    """Synthetic Zipf tf-idf document set (recipe in gen.c's header)."""
    lib = _load()
    length = np.empty(n, np.int64)
    lib.gen_count(n, d, float(lam), lo, hi, seed, _p(length))
    cap = int(length.sum())
    indptr = np.empty(n + 1, np.int64)
    indices = np.empty(max(cap, 1), np.int32)
    values = np.empty(max(cap, 1), np.float32)
    nnz = np.zeros(1, np.int64)
    rc = lib.gen_fill(n, d, float(lam), lo, hi, float(s), seed, _p(length), _p(indptr),
                      _p(indices), _p(values), _p(nnz))
    if rc != 0:
        raise MemoryError("generator allocation failed")
    m = int(nnz[0])
    return CSR(n, d, indptr, indices[:m].copy() if m < cap else indices[:m],
               values[:m].copy() if m < cap else values[:m])


def perm_prefix(n: int, m: int, seed: int, stream: int = 0) -> np.ndarray:
    """First m entries of a seeded uniform permutation of range(n)."""
    out = np.empty(min(m, n), np.int64)
    _load().gen_perm_prefix(n, min(m, n), seed, stream, _p(out))
    return out


def uniform_labels(n: int, k: int, seed: int, stream: int = 1) -> np.ndarray:
    """n seeded labels uniform in [0, k) (a random partition)."""
    out = np.empty(n, np.int32)
    _load().gen_uniform_labels(n, k, seed, stream, _p(out))
    return out


def uniform01(n: int, seed: int, stream: int = 2) -> np.ndarray:
    out = np.empty(n, np.float64)
    _load().gen_uniform01(n, seed, stream, _p(out))
    return out


def seed_objects(x: CSR, k: int, seed: int) -> np.ndarray:
    """k distinct, nonempty, pairwise non-identical object indices.

    Walks a seeded permutation of the objects and skips empty rows and rows
    whose (indices, values) repeat an already chosen one, so the initial means
    hold no exact duplicates.
    """
    out, seen = [], set()
    want = k
    m = min(x.n, 2 * k + 64)
    while True:
        cand = perm_prefix(x.n, m, seed, stream=0)
        out.clear()
        seen.clear()
        for i in cand:
            a, b = int(x.indptr[i]), int(x.indptr[i + 1])
            if a == b:
                continue
            h = hashlib.blake2b(x.indices[a:b].tobytes() + x.values[a:b].tobytes(),
                                digest_size=16).digest()
            if h in seen:
                continue
            seen.add(h)
            out.append(int(i))
            if len(out) == want:
                return np.asarray(out, np.int64)
        if m >= x.n:
            raise ValueError("fewer than k distinct nonempty objects")
        m = min(x.n, 2 * m)


# ---------------------------------------------------------------------------
# Workload presets.  Sizes and distributions are the five benchmark
# configurations of this project; the seed of configuration c is c.
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    d: int
    lam: float
    lo: int
    hi: int
    s: float
    k: int
    iters: int
    seed: int

    def generate(self) -> CSR:
        return generate(self.n, self.d, self.lam, self.lo, self.hi, self.s, self.seed)

    def seeds(self, x: CSR, restart: int = 0) -> np.ndarray:
        return seed_objects(x, self.k, self.seed + 1000 * restart)


WORKLOADS = {
    "small": Workload("small", 20_000, 10_000, 50.0, 5, 200, 1.1, 100, 10, 1),
    "nyt_like": Workload("nyt_like", 300_000, 100_000, 230.0, 10, 2000, 1.05, 10_000, 20, 2),
    "pubmed_8m": Workload("pubmed_8m", 8_000_000, 140_000, 60.0, 3, 1000, 1.1, 10_000, 10, 3),
    "precision": Workload("precision", 2_000_000, 200_000, 120.0, 5, 1500, 1.1, 50_000, 10, 4),
    # the paper's 1M-document PubMed sample shape at k = 10,000: its Lloyd chain
    # still moves hundreds of objects per iteration after 10 iterations
    "pubmed_1m": Workload("pubmed_1m", 1_000_000, 140_000, 60.0, 3, 1000, 1.1, 10_000, 10, 9),
}


def batched_instances(count: int = 96, meta_seed: int = 5, distinct: int = 48,
                      restarted: int = 6, restarts: int = 8):
    """Parameters of the many-instance workload.

    ``distinct`` data sets run once and ``restarted`` data sets run ``restarts``
    times from different initial means (48 + 6 * 8 = 96 instances).  Per data
    set: N ~ U[5e3, 4e5], D ~ U[2e4, 1.5e5], lambda ~ U[30, 250],
    s ~ U[1.0, 1.2], k = round(exp(U[ln 16, ln 8192])), clamped to N // 4;
    nnz clipped to [3, 1000].
    """
    nsets = distinct + restarted
    u = uniform01(5 * nsets, meta_seed, stream=3).reshape(nsets, 5)
    sets = []
    for j in range(nsets):
        n = int(5_000 + u[j, 0] * (400_000 - 5_000))
        d = int(20_000 + u[j, 1] * (150_000 - 20_000))
        lam = 30.0 + u[j, 2] * 220.0
        s = 1.0 + u[j, 3] * 0.2
        k = int(round(math.exp(math.log(16) + u[j, 4] * (math.log(8192) - math.log(16)))))
        k = max(1, min(k, n // 4))
        sets.append(Workload("batch%02d" % j, n, d, lam, 3, 1000, s, k, 15, 100 + j))
    inst = []
    for j, w in enumerate(sets):
        reps = 1 if j < distinct else restarts
        for r in range(reps):
            inst.append((w, r))
    assert len(inst) == count
    return inst
