"""FP64 CPU oracle for inverted-file spherical k-means.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product package.
It shares no code with the GPU library.

* ``ivf_oracle.c`` - the naive sparse IVF (Algorithm 3 of the paper: the
  assignment walk over the means' inverted file and the update step), FP64,
  no FMA contraction, OpenMP over objects / clusters with results independent
  of the thread count; and IVFD's assignment (Algorithm 4: the objects'
  inverted file queried by each mean in turn).
* ``dense.py``     - a dense brute-force cosine Lloyd (Algorithm 2 scored with
  Algorithm 3's tie rule), for tiny inputs; bit-identical to the sparse walk.
* ``exact.py``     - an exact-rational checker (Python ``fractions``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, IEEE FP64 with contraction off)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-ffp-contract=off", "-fno-fast-math",
                               os.path.join(_HERE, "ivf_oracle.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _configure(lib):
    i64, i32, vp, ci = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int
    lib.oracle_assign.argtypes = [i64, i64, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp,
                                  vp, ci]
    lib.oracle_assign.restype = ci
    lib.oracle_scores.argtypes = [i64, vp, vp, i64, vp, vp, vp, i32, vp, vp, vp, vp]
    lib.oracle_scores.restype = ci
    lib.oracle_update.argtypes = [i64, i64, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, i64,
                                  vp, ci]
    lib.oracle_update.restype = i64
    lib.oracle_ivfd_assign.argtypes = [i64, i64, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp,
                                       vp, vp]
    lib.oracle_ivfd_assign.restype = ci
    lib.oracle_term_counts.argtypes = [i64, i64, vp, vp, i32, vp, vp, vp, vp]
    lib.oracle_term_counts.restype = ci
    return lib


def compile_variant(src_text: str, out_path: str) -> str:
    """Compile a (test-planted) variant of the oracle source with the same flags."""
    c_path = out_path + ".c"
    with open(c_path, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-ffp-contract=off", "-fno-fast-math", c_path, "-o", out_path, "-lm"])
    return out_path


def use_library(path: str | None):
    """Point the wrappers at another build of the oracle (None: the default)."""
    global _lib
    _lib = None if path is None else _configure(ctypes.CDLL(path))


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        _lib = _configure(ctypes.CDLL(_SO))
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


@dataclass
class Means:
    """k means, mean-major: per cluster an ascending (term, FP64 value) list."""
    k: int
    d: int
    indptr: np.ndarray   # int64 [k+1]
    indices: np.ndarray  # int32 [nnz]
    values: np.ndarray   # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def dense(self) -> np.ndarray:
        m = np.zeros((self.k, self.d), np.float64)
        for j in range(self.k):
            a, b = int(self.indptr[j]), int(self.indptr[j + 1])
            m[j, self.indices[a:b]] = self.values[a:b]
        return m


@dataclass
class AssignResult:
    assign: np.ndarray   # int32 [n]
    rho: np.ndarray      # float64 [n], rho of the chosen cluster
    rho2: np.ndarray     # float64 [n], best rho among the other clusters
    objective: float
    changed: int
    zero_overlap: int
    mult_adds: int


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def assign(x, means: Means, prev: np.ndarray, threads: int = 0) -> AssignResult:
    """Assignment step (Algorithm 3, assignment part) in FP64."""
    lib = _load()
    n = x.n
    xp, xi, xv = _c(x.indptr, np.int64), _c(x.indices, np.int32), _c(x.values, np.float32)
    mp, mi, mv = _c(means.indptr, np.int64), _c(means.indices, np.int32), _c(means.values,
                                                                             np.float64)
    prev = _c(prev, np.int32)
    out = np.empty(n, np.int32)
    rho = np.empty(n, np.float64)
    rho2 = np.empty(n, np.float64)
    stats = np.zeros(3, np.float64)
    mult = np.zeros(1, np.int64)
    rc = lib.oracle_assign(n, x.d, _p(xp), _p(xi), _p(xv), means.k, _p(mp), _p(mi), _p(mv),
                           _p(prev), _p(out), _p(rho), _p(rho2), _p(stats), _p(mult), threads)
    if rc != 0:
        raise MemoryError("oracle_assign failed")
    return AssignResult(out, rho, rho2, float(stats[0]), int(stats[1]), int(stats[2]),
                        int(mult[0]))


def ivfd_assign(x, means: Means, prev: np.ndarray) -> AssignResult:
    """Assignment step of IVFD (Algorithm 4): the objects inverted, each mean a
    query over them, FP64, single-threaded."""
    lib = _load()
    n = x.n
    xp, xi, xv = _c(x.indptr, np.int64), _c(x.indices, np.int32), _c(x.values, np.float32)
    mp, mi, mv = _c(means.indptr, np.int64), _c(means.indices, np.int32), _c(means.values,
                                                                             np.float64)
    prev = _c(prev, np.int32)
    out = np.empty(n, np.int32)
    rho = np.empty(n, np.float64)
    rho2 = np.empty(n, np.float64)
    stats = np.zeros(3, np.float64)
    mult = np.zeros(1, np.int64)
    rc = lib.oracle_ivfd_assign(n, x.d, _p(xp), _p(xi), _p(xv), means.k, _p(mp), _p(mi),
                                _p(mv), _p(prev), _p(out), _p(rho), _p(rho2), _p(stats),
                                _p(mult))
    if rc != 0:
        raise MemoryError("oracle_ivfd_assign failed")
    return AssignResult(out, rho, rho2, float(stats[0]), int(stats[1]), int(stats[2]),
                        int(mult[0]))


def scores(x, means: Means, objs, clus) -> np.ndarray:
    """rho(x_i, mu_j) for listed pairs, by the same FP64 walk as ``assign``."""
    lib = _load()
    objs = _c(objs, np.int64)
    clus = _c(clus, np.int32)
    out = np.empty(len(objs), np.float64)
    xp, xi, xv = _c(x.indptr, np.int64), _c(x.indices, np.int32), _c(x.values, np.float32)
    mp, mi, mv = _c(means.indptr, np.int64), _c(means.indices, np.int32), _c(means.values,
                                                                             np.float64)
    rc = lib.oracle_scores(len(objs), _p(objs), _p(clus), x.d, _p(xp), _p(xi), _p(xv), means.k,
                           _p(mp), _p(mi), _p(mv), _p(out))
    if rc != 0:
        raise MemoryError("oracle_scores failed")
    return out


def update(x, k: int, assign_vec: np.ndarray, prev: Means | None, threads: int = 0):
    """Update step (Algorithm 3, update part).  Returns (Means, sizes[k])."""
    lib = _load()
    if prev is None:
        prev = Means(k, x.d, np.zeros(k + 1, np.int64), np.zeros(0, np.int32),
                     np.zeros(0, np.float64))
    xp, xi, xv = _c(x.indptr, np.int64), _c(x.indices, np.int32), _c(x.values, np.float32)
    pp, pi, pv = _c(prev.indptr, np.int64), _c(prev.indices, np.int32), _c(prev.values,
                                                                           np.float64)
    a = _c(assign_vec, np.int32)
    cap = int(x.nnz + prev.nnz + 1)
    op = np.empty(k + 1, np.int64)
    oi = np.empty(cap, np.int32)
    ov = np.empty(cap, np.float64)
    sizes = np.empty(k, np.int64)
    nnz = lib.oracle_update(x.n, x.d, _p(xp), _p(xi), _p(xv), k, _p(a), _p(pp), _p(pi), _p(pv),
                            _p(op), _p(oi), _p(ov), cap, _p(sizes), threads)
    if nnz < 0:
        raise MemoryError("oracle_update failed (%d)" % nnz)
    return Means(k, x.d, op, oi[:nnz].copy(), ov[:nnz].copy()), sizes


def term_counts(x, means: Means):
    """(no[t], nc[t]): document and centroid frequency of every term."""
    lib = _load()
    no = np.empty(x.d, np.int64)
    nc = np.empty(x.d, np.int64)
    xp, xi = _c(x.indptr, np.int64), _c(x.indices, np.int32)
    mp, mi = _c(means.indptr, np.int64), _c(means.indices, np.int32)
    lib.oracle_term_counts(x.n, x.d, _p(xp), _p(xi), means.k, _p(mp), _p(mi), _p(no), _p(nc))
    return no, nc


def initial_means(x, seeds) -> Means:
    """Initial state: mean j is object seeds[j] renormalised in FP64, i.e. the
    update step applied to the partition {seeds[j]} -> j."""
    k = len(seeds)
    a = np.full(x.n, -1, np.int32)
    a[np.asarray(seeds, np.int64)] = np.arange(k, dtype=np.int32)
    m, _ = update(x, k, a, None)
    return m


@dataclass
class ChainStep:
    assign: AssignResult
    means_in: Means
    means_out: Means
    sizes: np.ndarray


def chain(x, seeds, iters: int, threads: int = 0, keep_means: bool = True):
    """Lloyd iterations from the seeded initial state; yields one ChainStep per
    iteration (assignment under the previous means, then the update)."""
    k = len(seeds)
    means = initial_means(x, seeds)
    prev = np.full(x.n, -1, np.int32)
    for _ in range(iters):
        ar = assign(x, means, prev, threads)
        new, sizes = update(x, k, ar.assign, means, threads)
        yield ChainStep(ar, means if keep_means else None, new, sizes)
        means = new
        prev = ar.assign
