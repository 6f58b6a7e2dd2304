"""GPU: the incremental update against the full reduction, bit for bit.

The member sums of every (cluster, term) are exact integers in the update's
fixed point, so the sums of a new assignment equal the stored sums of the
previous one minus the values of the objects that left each cluster plus
those of the objects that joined it.  A handle built with full_update=True
always reduces all object entries; the default handle merges the changed
objects' entries into its stored sums once few objects move.  At every
iteration of the same chain the two must give identical assignments and
bit-identical means, objectives and counts, and the incremental path must
actually run.  The chains also pass through caller-given means (the stored
sums depend only on the assignment), repeated means that leave a cluster
empty, objects without a shared term, and updates from arbitrary
assignments; the FP64 oracle checks the means along the way.
"""
import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2002_09094_amd as ivf  # noqa: E402
from gpu_util import i32, means_to_dev, means_to_host, to_dev  # noqa: E402


def _same_means(a, b):
    pa, ia, va = (t.cpu().numpy() for t in a.get_means())
    pb, ib, vb = (t.cpu().numpy() for t in b.get_means())
    return np.array_equal(pa, pb) and np.array_equal(ia, ib) and np.array_equal(
        va.view(np.uint64), vb.view(np.uint64))


def _lockstep(x, k, iters, opts, seeds=None, means=None):
    """Two handles (incremental default, full reduction) advanced together;
    returns the per-iteration update stats of the incremental one."""
    dx = to_dev(x)
    inc = ivf.IVFKMeans(*dx, x.d, k, **opts)
    full = ivf.IVFKMeans(*dx, x.d, k, full_update=True, **opts)
    for km in (inc, full):
        if seeds is not None:
            km.init_seeds(i32(seeds))
        else:
            km.set_means(*means_to_dev(means))
    a = i32(np.full(x.n, -1, np.int32))
    b = i32(np.full(x.n, -1, np.int32))
    out = []
    for r in range(iters):
        si = inc.assign(a)
        sf = full.assign(b)
        assert torch.equal(a, b), r
        assert si["changed"] == sf["changed"] and si["mult_adds"] == sf["mult_adds"]
        ui = inc.update(a)
        uf = full.update(b)
        assert uf["update_delta_entries"] == -1
        for key in ("nnz_means", "empty_clusters"):
            assert ui[key] == uf[key], (r, key)
        assert ui["objective_exact"] == uf["objective_exact"], r
        assert _same_means(inc, full), r
        print("iter %d: changed %d, delta entries %d, update %.2f ms (full %.2f ms)"
              % (r + 1, si["changed"], ui["update_delta_entries"], ui["update_ms"],
                 uf["update_ms"]), flush=True)
        out.append((si, ui))
    return inc, full, a, out


@pytest.mark.parametrize("shape", [
    (20000, 10000, 50.0, 5, 200, 1.1, 100, 11, {}),
    (9000, 3000, 25.0, 0, 120, 1.05, 700, 12, {"cluster_range": 64}),
    (6000, 4000, 60.0, 10, 400, 1.2, 37, 13, {"objects_per_item": 3, "waves_per_wg": 5}),
    # wide vocabularies: term keys of 17 and 18 bits sort in two 9-bit
    # passes (the inverted file and the incremental update's term order),
    # 19 bits in three 8-bit passes and a copy back
    (15000, 120000, 40.0, 5, 200, 1.1, 80, 14, {}),
    (12000, 262144, 40.0, 5, 200, 1.1, 60, 15, {}),
    (12000, 300000, 40.0, 5, 200, 1.1, 60, 16, {}),
])
def test_incremental_update_equals_the_full_reduction(shape):
    n, d, lam, lo, hi, s, k, seed, opts = shape
    x = datagen.generate(n, d, lam, lo, hi, s, seed)
    seeds = datagen.seed_objects(x, k, seed)
    inc, full, a, out = _lockstep(x, k, 10, opts, seeds=seeds)
    assert any(u["update_delta_entries"] >= 0 for _, u in out)
    # the last means against the oracle's update of the final assignment
    steps = list(oracle.chain(x, seeds, 10))
    assert np.array_equal(a.cpu().numpy(), steps[-1].assign.assign)
    gm = means_to_host(*inc.get_means(), k, d)
    om = steps[-1].means_out
    assert np.array_equal(gm.indptr, om.indptr) and np.array_equal(gm.indices, om.indices)
    np.testing.assert_allclose(gm.values, om.values, rtol=1e-12, atol=0)
    inc.close()
    full.close()


def test_caller_means_repeated_means_and_arbitrary_assignments():
    """Repeated means empty a cluster (it keeps its mean); set_means between
    updates keeps the stored sums valid; updates from arbitrary assignments
    (some objects unassigned, -1) still equal the full reduction."""
    x = datagen.generate(8000, 5000, 30.0, 0, 150, 1.1, 21)
    k = 60
    seeds = datagen.seed_objects(x, k, 21)
    base = oracle.initial_means(x, seeds)
    # mean 7 repeated as mean 41: every tie goes to 7, and 41 empties
    ptr, idx, val = base.indptr, base.indices, base.values
    rows = [(idx[ptr[j]:ptr[j + 1]], val[ptr[j]:ptr[j + 1]]) for j in range(k)]
    rows[41] = rows[7]
    p2 = np.concatenate([[0], np.cumsum([len(r[0]) for r in rows])]).astype(np.int64)
    m0 = oracle.Means(k, x.d, p2, np.concatenate([r[0] for r in rows]),
                      np.concatenate([r[1] for r in rows]))
    inc, full, a, out = _lockstep(x, k, 6, {}, means=m0)
    assert out[0][1]["empty_clusters"] >= 1
    # caller means between updates: the oracle's means of the current state
    cur = means_to_host(*full.get_means(), k, x.d)
    for km in (inc, full):
        km.set_means(*means_to_dev(cur))
    rng = np.random.default_rng(3)
    ga = a.cpu().numpy()
    for r in range(4):
        # move a few hundred objects to random clusters, unassign some
        b = ga.copy()
        mv = rng.choice(x.n, 300, replace=False)
        b[mv] = rng.integers(0, k, 300)
        b[mv[:40]] = -1
        ui = inc.update(i32(b))
        uf = full.update(i32(b))
        assert ui["update_delta_entries"] >= 0, r
        assert ui["nnz_means"] == uf["nnz_means"] and ui["empty_clusters"] == uf["empty_clusters"]
        assert ui["objective_exact"] == uf["objective_exact"]
        assert _same_means(inc, full), r
        new, _ = oracle.update(x, k, b, cur)
        gm = means_to_host(*inc.get_means(), k, x.d)
        assert np.array_equal(gm.indptr, new.indptr) and np.array_equal(gm.indices, new.indices)
        np.testing.assert_allclose(gm.values, new.values, rtol=1e-12, atol=0)
        cur = gm
        for km in (inc, full):
            km.set_means(*means_to_dev(cur))
        ga = b
    inc.close()
    full.close()
