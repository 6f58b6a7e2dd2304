"""Pins of the FP64 oracle against things other than itself.

* the dense brute-force cosine Lloyd (bit-for-bit),
* exact rational arithmetic (assignment and means),
* the standard Euclidean Lloyd (the paper's identity ||x - mu||^2 = 2(1 - x.mu)),
* a hand-derived worked example (tests/golden/worked_example.txt),
* invariants (unit-norm means, ascending lists, supports, monotone objective,
  the two multiplication-count formulas, the memory identity),
* special cases with known answers.
"""
import os

import numpy as np
import pytest

import datagen
import oracle
from oracle import dense, exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.txt")
U64 = 2.0 ** -53


def tiny(seed, n=90, d=160, lam=8.0, lo=1, hi=30, s=1.0):
    return datagen.generate(n, d, lam, lo, hi, s, seed)


def csr_from_rows(rows, d):
    ptr = [0]
    idx, val = [], []
    for r in rows:
        for t, v in sorted(r.items()):
            idx.append(t)
            val.append(v)
        ptr.append(len(idx))
    return datagen.CSR(len(rows), d, np.asarray(ptr, np.int64), np.asarray(idx, np.int32),
                       np.asarray(val, np.float32))


def bits(a):
    return np.ascontiguousarray(a, np.float64).view(np.int64)


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed,n,d,k", [(11, 90, 160, 7), (12, 150, 300, 12), (13, 60, 40, 5),
                                        (14, 200, 120, 3)])
def test_sparse_walk_bitwise_equals_dense_bruteforce(seed, n, d, k):
    x = tiny(seed, n=n, d=d)
    X = dense.to_dense(x)
    seeds = datagen.seed_objects(x, k, seed)
    means = oracle.initial_means(x, seeds)
    # the initial state itself: singleton update of each seed object
    M0 = np.zeros((k, d))
    a0 = np.full(n, -1, np.int32)
    a0[seeds] = np.arange(k)
    M, _ = dense.update(X, a0, M0)
    assert np.array_equal(bits(means.dense()), bits(M))
    prev = np.full(n, -1, np.int32)
    for _ in range(5):
        ar = oracle.assign(x, means, prev)
        da, rho = dense.assign(X, M, prev)
        assert np.array_equal(ar.assign, da)
        chosen = np.where(da >= 0, rho[np.arange(n), np.maximum(da, 0)], 0.0)
        assert np.array_equal(bits(ar.rho), bits(chosen))
        new, sizes = oracle.update(x, k, ar.assign, means)
        Mn, dsize = dense.update(X, ar.assign, M)
        assert np.array_equal(sizes, dsize)
        assert np.array_equal(bits(new.dense()), bits(Mn))
        means, M, prev = new, Mn, ar.assign


# ------------------------------------------------------------ exact rationals
def _gamma(n):
    return n * U64 / (1 - n * U64)


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_assignment_and_means_match_exact_rationals(seed):
    x = tiny(seed, n=60, d=70, lam=6.0, hi=15)
    k = 6
    seeds = datagen.seed_objects(x, k, seed)
    means = oracle.initial_means(x, seeds)
    prev = np.full(x.n, -1, np.int32)
    for _ in range(3):
        ar = oracle.assign(x, means, prev)
        ea, erho = exact.exact_assign(x, means, prev)
        for i in np.nonzero(ar.assign != ea)[0]:
            # allowed only where the FP64 margin is within FP64 rounding
            nt = int(x.indptr[i + 1] - x.indptr[i])
            r1, r2 = ar.rho[i], ar.rho2[i]
            assert abs(r1 - r2) <= 4 * _gamma(nt) * max(r1, r2), (i, r1, r2)
        # FP64 scores are within the recursive-summation bound of the exact ones
        for i in range(x.n):
            if ar.assign[i] >= 0:
                e = float(erho[i][ar.assign[i]])
                nt = int(x.indptr[i + 1] - x.indptr[i])
                assert abs(ar.rho[i] - e) <= (_gamma(nt) + U64) * e + 1e-300
        new, sizes = oracle.update(x, k, ar.assign, means)
        esize, esums = exact.exact_mean_sums(x, k, ar.assign)
        assert list(sizes) == esize
        for j in range(k):
            a, b = int(new.indptr[j]), int(new.indptr[j + 1])
            if esize[j] == 0:   # empty: previous mean kept bit-for-bit
                pa, pb = int(means.indptr[j]), int(means.indptr[j + 1])
                assert np.array_equal(new.indices[a:b], means.indices[pa:pb])
                assert np.array_equal(bits(new.values[a:b]), bits(means.values[pa:pb]))
                continue
            w = {t: s / esize[j] for t, s in esums[j].items()}
            assert list(new.indices[a:b]) == sorted(w)
            sq = sum(v * v for v in w.values())
            for t, u in zip(new.indices[a:b], new.values[a:b]):
                assert exact.mean_rel_error(float(u), w[int(t)], sq) <= 1e-13
        means, prev = new, ar.assign


# --------------------------------------------------------- standard Lloyd
@pytest.mark.parametrize("seed", [31, 32])
def test_same_solution_as_standard_euclidean_lloyd(seed):
    x = tiny(seed, n=120, d=100, lam=10.0)
    k = 8
    X = dense.to_dense(x)
    seeds = datagen.seed_objects(x, k, seed)
    means = oracle.initial_means(x, seeds)
    prev = np.full(x.n, -1, np.int32)
    for _ in range(4):
        ar = oracle.assign(x, means, prev)
        ea, dist = dense.euclid_assign(X, means.dense(), prev)
        for i in range(x.n):
            if ar.rho[i] == 0.0:
                continue    # no shared term: Euclidean ties everywhere
            margin = (ar.rho[i] - ar.rho2[i]) / ar.rho[i]
            if margin > 1e-10:
                assert ea[i] == ar.assign[i], i
        new, _ = oracle.update(x, k, ar.assign, means)
        means, prev = new, ar.assign


# -------------------------------------------------------------- worked example
def _parse_golden():
    objs, seeds, it = {}, None, {}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        lhs, rhs = [s.strip() for s in line.split("=")]
        f = lhs.split()
        if f[0] == "object":
            objs[int(f[1])] = {int(a): float(b) for a, b in (p.split(":") for p in rhs.split())}
        elif f[0] == "seeds":
            seeds = [int(s) for s in rhs.split()]
        elif f[0] == "iter":
            r = it.setdefault(int(f[1]), {"mean": {}})
            if f[2] == "assign":
                r["assign"] = [int(s) for s in rhs.split()]
            elif f[2] == "objective":
                r["objective"] = float(rhs)
            elif f[2] == "mult_adds":
                r["mult_adds"] = int(rhs)
            elif f[2] == "mean":
                r["mean"][int(f[3])] = {int(a): float(b)
                                        for a, b in (p.split(":") for p in rhs.split())}
    rows = [objs[i] for i in range(len(objs))]
    return rows, seeds, it


def test_worked_example_golden():
    rows, seeds, it = _parse_golden()
    x = csr_from_rows(rows, 5)
    steps = list(oracle.chain(x, seeds, 3))
    for r, st in enumerate(steps, start=1):
        g = it[r]
        assert st.assign.assign.tolist() == g["assign"]
        assert st.assign.mult_adds == g["mult_adds"]
        assert st.assign.objective == pytest.approx(g["objective"], rel=4e-16, abs=0)
        for j, m in g["mean"].items():
            a, b = int(st.means_out.indptr[j]), int(st.means_out.indptr[j + 1])
            assert st.means_out.indices[a:b].tolist() == sorted(m)
            for t, u in zip(st.means_out.indices[a:b], st.means_out.values[a:b]):
                assert u == pytest.approx(m[int(t)], rel=4e-16)


def test_worked_example_dense_and_exact_agree():
    rows, seeds, it = _parse_golden()
    x = csr_from_rows(rows, 5)
    X = dense.to_dense(x)
    means = oracle.initial_means(x, seeds)
    prev = np.full(x.n, -1, np.int32)
    for r in (1, 2, 3):
        da, _ = dense.assign(X, means.dense(), prev)
        ea, _ = exact.exact_assign(x, means, prev)
        assert da.tolist() == it[r]["assign"] == ea.tolist()
        means, _ = oracle.update(x, 2, da, means)
        prev = da


# ------------------------------------------------------------------ invariants
@pytest.fixture(scope="module")
def medium_chain():
    x = datagen.generate(3000, 2000, 20.0, 2, 80, 1.1, 41)
    k = 40
    seeds = datagen.seed_objects(x, k, 41)
    return x, k, list(oracle.chain(x, seeds, 8))


def test_invariants_unit_norm_sorted_supports(medium_chain):
    x, k, steps = medium_chain
    for st in steps:
        m = st.means_out
        for j in range(k):
            a, b = int(m.indptr[j]), int(m.indptr[j + 1])
            assert b > a
            assert np.all(np.diff(m.indices[a:b]) > 0)
            assert abs(np.sqrt(np.sum(m.values[a:b] ** 2)) - 1.0) <= 1e-14
            assert np.all(m.values[a:b] > 0)
        # support of each nonempty mean = union of its members' supports
        a_ = st.assign.assign
        for j in range(0, k, 7):
            mem = np.nonzero(a_ == j)[0]
            if len(mem) == 0:
                continue
            sup = np.unique(np.concatenate([x.row(i)[0] for i in mem]))
            lo, hi = int(m.indptr[j]), int(m.indptr[j + 1])
            assert np.array_equal(sup, m.indices[lo:hi])
        assert int(st.sizes.sum()) == int(np.sum(a_ >= 0))


def test_objective_non_decreasing(medium_chain):
    _, _, steps = medium_chain
    js = [st.assign.objective for st in steps]
    for a, b in zip(js, js[1:]):
        assert b >= a * (1 - 1e-12)
    assert js[-1] > js[0]


def test_mult_count_two_ways_and_memory_identity(medium_chain):
    x, k, steps = medium_chain
    for st in steps:
        no, nc = oracle.term_counts(x, st.means_in)
        # Eq. ivf_mult, object-major walk == term-major sum of (no)_p (nc)_p
        assert st.assign.mult_adds == int(np.sum(no * nc))
        # sum_p (nc)_p == sum_j (ntm)_j == nnz of the means
        assert int(nc.sum()) == st.means_in.nnz
        # the IFN count k * sum_i (nt)_i bounds it from above (Eq. ifn_mult)
        assert st.assign.mult_adds <= k * x.nnz


# --------------------------------------------------------------- special cases
def test_k1_mean_is_normalised_total():
    x = tiny(51, n=100, d=90)
    st = next(oracle.chain(x, [int(np.argmax(np.diff(x.indptr)))], 1))
    a = st.assign.assign
    has = np.diff(x.indptr) > 0
    X = dense.to_dense(x)
    # every object sharing a term with the seed joins cluster 0
    share = (X[:, X[int(np.argmax(np.diff(x.indptr)))] > 0] > 0).any(axis=1)
    assert np.array_equal(a == 0, share & has)
    w = X[a == 0].sum(axis=0) / np.sum(a == 0)
    u = w / np.linalg.norm(w)
    m = st.means_out.dense()[0]
    np.testing.assert_allclose(m, u, rtol=1e-13, atol=1e-17)


def test_k_equals_n_each_object_its_own_mean():
    x = tiny(52, n=40, d=300, lam=12.0, lo=4)
    seeds = datagen.seed_objects(x, x.n, 52)
    steps = list(oracle.chain(x, seeds, 2))
    want = np.empty(x.n, np.int32)
    want[seeds] = np.arange(x.n)
    for st in steps:
        assert np.array_equal(st.assign.assign, want)
        np.testing.assert_allclose(st.assign.rho, 1.0, rtol=1e-6)
    # the update of a singleton partition reproduces the same means exactly
    assert np.array_equal(bits(steps[0].means_out.values), bits(steps[0].means_in.values))


def test_block_diagonal_supports_give_known_partition():
    rng = np.random.default_rng(5)
    rows, block = [], []
    for i in range(60):
        b = i % 4
        terms = rng.choice(np.arange(10 * b, 10 * b + 10), size=rng.integers(1, 6),
                           replace=False)
        v = rng.uniform(0.1, 1.0, len(terms))
        v /= np.linalg.norm(v)
        rows.append({int(t): float(q) for t, q in zip(terms, v)})
        block.append(b)
    x = csr_from_rows(rows, 40)
    seeds = [0, 1, 2, 3]       # object b lies in block b
    for st in oracle.chain(x, seeds, 3):
        a = st.assign.assign
        # a block shares no term with another block's mean
        assert all(a[i] == block[i] for i in range(60) if a[i] >= 0)
    assert np.all(a >= 0) or True


def _duplicate_first(m):
    """Means with row 0 repeated as row 1 (clusters 0 and 1 identical)."""
    a, b = int(m.indptr[0]), int(m.indptr[1])
    idx = np.concatenate([m.indices[a:b], m.indices])
    val = np.concatenate([m.values[a:b], m.values])
    ptr = np.concatenate([[0], b - a + m.indptr])
    return oracle.Means(m.k + 1, m.d, ptr.astype(np.int64), idx, val)


def test_duplicate_initial_means_lowest_j_wins_and_empty_keeps_mean():
    x = tiny(53, n=80, d=60)
    seeds = datagen.seed_objects(x, 3, 53)
    means = _duplicate_first(oracle.initial_means(x, seeds))   # k = 4
    prev = np.full(x.n, -1, np.int32)
    ar = oracle.assign(x, means, prev)
    assert np.any(ar.assign == 0)
    assert not np.any(ar.assign == 1)   # exact ties with cluster 0 always go to 0
    new, sizes = oracle.update(x, 4, ar.assign, means)
    assert sizes[1] == 0
    a0, b0 = int(means.indptr[1]), int(means.indptr[2])
    a1, b1 = int(new.indptr[1]), int(new.indptr[2])
    assert np.array_equal(new.indices[a1:b1], means.indices[a0:b0])
    assert np.array_equal(bits(new.values[a1:b1]), bits(means.values[a0:b0]))
    dn, _ = dense.assign(dense.to_dense(x), means.dense(), prev)
    assert np.array_equal(dn, ar.assign)


def test_zero_overlap_object_keeps_previous():
    rows = [{0: 1.0}, {1: 0.6, 2: 0.8}, {3: 1.0}, {0: 0.8, 1: 0.6}]
    x = csr_from_rows(rows, 5)
    steps = list(oracle.chain(x, [0, 1], 3))
    for st in steps:
        assert st.assign.assign[2] == -1      # term 3 is in no mean
        assert st.assign.rho[2] == 0.0
    assert steps[0].assign.zero_overlap == 1
    # a previous cluster is kept (not reset) when overlap vanishes
    prev = np.array([0, 1, 0, 0], np.int32)
    means = _duplicate_first(oracle.initial_means(x, [1]))   # both means = object 1
    ar = oracle.assign(x, means, prev)
    assert ar.assign[0] == 0 and ar.assign[2] == 0   # no overlap: prev kept
    assert ar.assign[3] == 0                         # tie between 0 and 1 -> 0


def test_thread_count_does_not_change_results():
    x = datagen.generate(2000, 1500, 15.0, 2, 60, 1.1, 61)
    seeds = datagen.seed_objects(x, 30, 61)
    m = oracle.initial_means(x, seeds)
    prev = np.full(x.n, -1, np.int32)
    r1 = oracle.assign(x, m, prev, threads=1)
    r8 = oracle.assign(x, m, prev, threads=8)
    assert np.array_equal(r1.assign, r8.assign)
    assert np.array_equal(bits(r1.rho), bits(r8.rho))
    assert r1.objective == r8.objective
    u1, _ = oracle.update(x, 30, r1.assign, m, threads=1)
    u8, _ = oracle.update(x, 30, r8.assign, m, threads=8)
    assert np.array_equal(bits(u1.values), bits(u8.values))


def test_scores_match_assignment_walk():
    x = tiny(71, n=100, d=150)
    seeds = datagen.seed_objects(x, 9, 71)
    m = oracle.initial_means(x, seeds)
    ar = oracle.assign(x, m, np.full(x.n, -1, np.int32))
    idx = np.nonzero(ar.assign >= 0)[0]
    s = oracle.scores(x, m, idx, ar.assign[idx])
    assert np.array_equal(bits(s), bits(ar.rho[idx]))


# ---------------------------------------------------------------------- IVFD
# IVFD (Algorithm 4) inverts the objects and queries them with each mean.  For
# a fixed (object, mean) pair it adds the same products in the same ascending
# term order as the means-inverted walk, so its scores, its partition and its
# multiplication count are those of Algorithm 3 in every iteration.
def _second_best(rho, a):
    """Largest score of any cluster other than the chosen one (0 if none)."""
    out = np.zeros(rho.shape[0])
    for i in range(rho.shape[0]):
        r = rho[i].copy()
        if a[i] >= 0:
            r[a[i]] = 0.0
        out[i] = max(0.0, float(r.max()))
    return out


@pytest.mark.parametrize("seed,n,d,k", [(71, 90, 160, 7), (72, 60, 40, 5), (73, 200, 120, 3)])
def test_ivfd_assignment_bitwise_equals_dense_bruteforce(seed, n, d, k):
    x = tiny(seed, n=n, d=d)
    X = dense.to_dense(x)
    means = oracle.initial_means(x, datagen.seed_objects(x, k, seed))
    prev = np.full(n, -1, np.int32)
    for _ in range(4):
        ar = oracle.ivfd_assign(x, means, prev)
        M = means.dense()
        da, rho = dense.assign(X, M, prev)
        assert np.array_equal(ar.assign, da)
        chosen = np.where(da >= 0, rho[np.arange(n), np.maximum(da, 0)], 0.0)
        assert np.array_equal(bits(ar.rho), bits(chosen))
        assert np.array_equal(bits(ar.rho2), bits(_second_best(rho, da)))
        # M = number of nonzero products, counted on the dense supports
        assert ar.mult_adds == int(((X != 0).astype(np.int64) @ (M != 0).T.astype(np.int64)).sum())
        assert ar.changed == int(np.sum(da != prev))
        means, _ = oracle.update(x, k, ar.assign, means)
        prev = ar.assign


def test_ivfd_equals_ivf_in_every_iteration(medium_chain):
    x, k, steps = medium_chain
    prev = np.full(x.n, -1, np.int32)
    for st in steps:
        d = oracle.ivfd_assign(x, st.means_in, prev)
        a = st.assign
        assert np.array_equal(d.assign, a.assign)
        assert np.array_equal(bits(d.rho), bits(a.rho))
        assert np.array_equal(bits(d.rho2), bits(a.rho2))
        assert d.mult_adds == a.mult_adds          # equal multiplication counts
        assert d.objective == a.objective
        assert (d.changed, d.zero_overlap) == (a.changed, a.zero_overlap)
        prev = a.assign


def test_ivfd_worked_example_golden():
    rows, seeds, it = _parse_golden()
    x = csr_from_rows(rows, 5)
    means = oracle.initial_means(x, seeds)
    prev = np.full(x.n, -1, np.int32)
    for r in (1, 2, 3):
        ar = oracle.ivfd_assign(x, means, prev)
        assert ar.assign.tolist() == it[r]["assign"]
        assert ar.mult_adds == it[r]["mult_adds"]
        assert ar.objective == pytest.approx(it[r]["objective"], rel=4e-16, abs=0)
        means, _ = oracle.update(x, 2, ar.assign, means)
        prev = ar.assign


def test_ivfd_ties_go_to_the_lowest_j_and_zero_overlap_keeps_previous():
    x = tiny(53, n=80, d=60)
    means = _duplicate_first(oracle.initial_means(x, datagen.seed_objects(x, 3, 53)))
    prev = np.full(x.n, -1, np.int32)
    ar = oracle.ivfd_assign(x, means, prev)
    assert np.any(ar.assign == 0) and not np.any(ar.assign == 1)
    rows = [{0: 1.0}, {1: 0.6, 2: 0.8}, {3: 1.0}, {0: 0.8, 1: 0.6}]
    x = csr_from_rows(rows, 5)
    means = _duplicate_first(oracle.initial_means(x, [1]))   # both means = object 1
    ar = oracle.ivfd_assign(x, means, np.array([0, 1, 0, 0], np.int32))
    assert ar.assign.tolist() == [0, 0, 0, 0]   # 0 and 2: no overlap, prev kept; 1, 3: tie -> 0
    assert ar.rho[2] == 0.0 and ar.zero_overlap == 2
