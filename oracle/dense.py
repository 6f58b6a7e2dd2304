"""Dense brute-force cosine Lloyd for tiny inputs (test infrastructure only).

Spherical k-means (the paper's Algorithm 2) with full k x D means and the
argmax rule of Algorithm 3 (rho_max starts at 0, strict ">", ascending j, so
the lowest j wins among equal maxima; all-zero scores keep the previous
assignment).  Every score is accumulated over ALL D terms in ascending order,
one FP64 multiply and one FP64 add per term: the extra terms contribute an
exact +0.0, so the result is bit-identical to the sparse inverted-file walk
whenever that walk is right.  Independent of ``ivf_oracle.c`` by construction
(numpy, no inverted file, no sparse structure).
"""
from __future__ import annotations

import numpy as np


def to_dense(x) -> np.ndarray:
    out = np.zeros((x.n, x.d), np.float64)
    for i in range(x.n):
        a, b = int(x.indptr[i]), int(x.indptr[i + 1])
        out[i, x.indices[a:b]] = x.values[a:b].astype(np.float64)
    return out


def assign(X: np.ndarray, M: np.ndarray, prev: np.ndarray):
    """Returns (assignment, rho matrix n x k)."""
    n, d = X.shape
    k = M.shape[0]
    rho = np.zeros((n, k), np.float64)
    for t in range(d):
        prod = X[:, t][:, None] * M[:, t][None, :]
        rho = rho + prod
    out = np.array(prev, dtype=np.int32, copy=True)
    for i in range(n):
        best = 0.0
        for j in range(k):
            if rho[i, j] > best:
                best = rho[i, j]
                out[i] = j
    return out, rho


def update(X: np.ndarray, a: np.ndarray, M_prev: np.ndarray):
    """Dense update: member sum in ascending i, divide by |C_j|, divide by the
    2-norm summed over ascending p; an empty cluster keeps its previous mean."""
    n, d = X.shape
    k = M_prev.shape[0]
    W = np.zeros((k, d), np.float64)
    size = np.zeros(k, np.int64)
    for i in range(n):
        if a[i] >= 0:
            W[a[i]] = W[a[i]] + X[i]
            size[a[i]] += 1
    out = M_prev.copy()
    for j in range(k):
        if size[j] == 0:
            continue
        w = W[j] / float(size[j])
        ss = 0.0
        for p in range(d):
            ss = ss + w[p] * w[p]
        out[j] = w / np.sqrt(ss)
    return out, size


def euclid_assign(X: np.ndarray, M: np.ndarray, prev: np.ndarray):
    """Standard Lloyd assignment (the paper's Algorithm 1): squared Euclidean
    distance, d_min starts at the current cluster (+inf when unassigned),
    strict "<" over ascending j.  Returns (assignment, distance matrix)."""
    n = X.shape[0]
    k = M.shape[0]
    dist = np.empty((n, k), np.float64)
    for j in range(k):
        diff = X - M[j][None, :]
        dist[:, j] = np.einsum("ij,ij->i", diff, diff)
    out = np.array(prev, dtype=np.int32, copy=True)
    for i in range(n):
        dmin = dist[i, out[i]] if out[i] >= 0 else np.inf
        for j in range(k):
            if dist[i, j] < dmin:
                dmin = dist[i, j]
                out[i] = j
    return out, dist
