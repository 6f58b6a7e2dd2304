"""Exact-rational checker for tiny inputs (test infrastructure only).

Every FP32 object value and FP64 mean value is a dyadic rational, so inner
products, member sums and squared norms are computed here without any
rounding (``fractions.Fraction``).  The assignment is the exact argmax
(lowest j on exact ties, all-zero scores keep the previous cluster); the
renormalised mean u_p = w_p / ||w|| is irrational in general and is checked
through the exact identity u_p^2 * ||w||^2 = w_p^2.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def exact_scores(x, means) -> list:
    """rho[i][j] as exact rationals."""
    mrows = []
    for j in range(means.k):
        a, b = int(means.indptr[j]), int(means.indptr[j + 1])
        mrows.append({int(t): Fraction(float(v)) for t, v in zip(means.indices[a:b],
                                                                 means.values[a:b])})
    out = []
    for i in range(x.n):
        a, b = int(x.indptr[i]), int(x.indptr[i + 1])
        terms = [(int(t), Fraction(float(v))) for t, v in zip(x.indices[a:b], x.values[a:b])]
        row = []
        for j in range(means.k):
            m = mrows[j]
            row.append(sum((v * m[t] for t, v in terms if t in m), Fraction(0)))
        out.append(row)
    return out


def exact_assign(x, means, prev):
    rho = exact_scores(x, means)
    out = np.array(prev, dtype=np.int32, copy=True)
    for i, row in enumerate(rho):
        best = Fraction(0)
        for j, r in enumerate(row):
            if r > best:
                best = r
                out[i] = j
    return out, rho


def exact_mean_sums(x, k, assign):
    """Per cluster: (size, {term: exact member sum})."""
    sums = [dict() for _ in range(k)]
    size = [0] * k
    for i in range(x.n):
        j = int(assign[i])
        if j < 0:
            continue
        size[j] += 1
        a, b = int(x.indptr[i]), int(x.indptr[i + 1])
        for t, v in zip(x.indices[a:b], x.values[a:b]):
            sums[j][int(t)] = sums[j].get(int(t), Fraction(0)) + Fraction(float(v))
    return size, sums


def mean_rel_error(u_fp: float, w_p: Fraction, sq_norm: Fraction) -> float:
    """|u_fp / (w_p / ||w||) - 1|, from exact rationals (no square root):
    (u_fp / u)^2 = u_fp^2 ||w||^2 / w_p^2."""
    r = Fraction(u_fp) ** 2 * sq_norm / (w_p * w_p)
    # r = (1 + e)^2 -> e ~ (r - 1) / 2 for tiny e
    return abs(float(r - 1)) / 2.0
