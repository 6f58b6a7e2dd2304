"""GPU parity of IVFD (the paper's Algorithm 4: the objects inverted, each mean
a query over them).

Its partition must be the FP64 oracle's IVFD partition (which the oracle's
pins tie to the dense brute force and to the means-inverted walk), its
multiplication count the oracle's M, and its results those of the handle's
own means-inverted assignment step.  Ranges of 4096 objects make the small
cases span several ranges with a ragged last one.
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


def _check_step(st, ref, got):
    assert np.array_equal(got, ref.assign), np.nonzero(got != ref.assign)[0][:10]
    assert st["mult_adds"] == ref.mult_adds
    assert st["changed"] == ref.changed
    assert st["zero_overlap"] == ref.zero_overlap
    assert st["certified"] + st["rescored"] + st["zero_overlap"] == len(got)
    # certified objects contribute FP32 scores within the stated bound; the
    # FP64 sum over n objects in another order adds at most n * 2^-53 of it
    tol = 2 * st["objective_bound"] + len(got) * 2.0 ** -52
    assert abs(st["objective"] - ref.objective) <= tol * ref.objective


@pytest.mark.parametrize("n,d,lam,lo,hi,k,seed", [
    (10_000, 3000, 25.0, 1, 120, 60, 501),    # 3 ranges, ragged tail
    (9000, 6000, 35.0, 0, 300, 700, 502),     # empty objects, k > range count
])
def test_ivfd_chain_equals_oracle_and_the_means_inverted_step(n, d, lam, lo, hi, k, seed):
    x = datagen.generate(n, d, lam, lo, hi, 1.1, seed)
    seeds = datagen.seed_objects(x, k, seed)
    dx = to_dev(x)
    a = ivf.IVFKMeans(*dx, d, k)      # IVFD
    b = ivf.IVFKMeans(*dx, d, k)      # means inverted
    a.init_seeds(i32(seeds))
    b.init_seeds(i32(seeds))
    ga = i32(np.full(n, -1, np.int32))
    gb = i32(np.full(n, -1, np.int32))
    means = oracle.initial_means(x, seeds)
    prev = np.full(n, -1, np.int32)
    for r in range(4):
        print("iteration", r, flush=True)
        st = a.assign_ivfd(ga, objects_per_range=4096)
        sb = b.assign(gb)
        ref = oracle.ivfd_assign(x, means, prev)
        got = ga.cpu().numpy()
        _check_step(st, ref, got)
        assert np.array_equal(got, gb.cpu().numpy())
        assert st["mult_adds"] == sb["mult_adds"]
        a.update(ga)
        b.update(gb)
        means, _ = oracle.update(x, k, ref.assign, means)
        prev = ref.assign
    ma = means_to_host(*a.get_means(), k, d)
    mb = means_to_host(*b.get_means(), k, d)
    assert np.array_equal(ma.indices, mb.indices) and np.array_equal(ma.values, mb.values)
    a.close()
    b.close()


@pytest.mark.parametrize("n_r", [4096, 8192, 16384])
def test_every_range_size_gives_the_same_partition(n_r):
    n, d, k, seed = 20_000, 5000, 90, 503
    x = datagen.generate(n, d, 30.0, 2, 150, 1.1, seed)
    seeds = datagen.seed_objects(x, k, seed)
    km = ivf.IVFKMeans(*to_dev(x), d, k)
    km.init_seeds(i32(seeds))
    g = i32(np.full(n, -1, np.int32))
    km.assign(g)
    km.update(g)             # second iteration's means: many ties broken by score
    first = next(oracle.chain(x, seeds, 1))
    assert np.array_equal(g.cpu().numpy(), first.assign.assign)
    ref = oracle.ivfd_assign(x, first.means_out, first.assign.assign)
    st = km.assign_ivfd(g, objects_per_range=n_r)
    _check_step(st, ref, g.cpu().numpy())
    km.close()


def test_ties_zero_overlap_and_a_single_partial_range():
    x = datagen.generate(300, 200, 6.0, 0, 12, 1.2, 504)   # few terms: objects without overlap
    k = 6
    base = oracle.initial_means(x, datagen.seed_objects(x, k - 1, 504))
    a, b = int(base.indptr[0]), int(base.indptr[1])         # mean 0 repeated as mean 1
    means = oracle.Means(k, x.d, np.concatenate([[0], b - a + base.indptr]).astype(np.int64),
                         np.concatenate([base.indices[a:b], base.indices]),
                         np.concatenate([base.values[a:b], base.values]))
    prev = np.arange(x.n, dtype=np.int32) % k
    ref = oracle.ivfd_assign(x, means, prev)
    assert ref.zero_overlap > 0 and not np.any(ref.assign[ref.rho > 0] == 1)
    km = ivf.IVFKMeans(*to_dev(x), x.d, k)
    km.set_means(*means_to_dev(means))
    g = i32(prev)
    st = km.assign_ivfd(g)
    _check_step(st, ref, g.cpu().numpy())
    km.close()


def test_k1_and_forced_rescore():
    x = datagen.generate(5000, 1500, 20.0, 1, 80, 1.1, 505)
    for k, opts in ((1, {}), (25, {"force_rescore": 1})):
        seeds = datagen.seed_objects(x, k, 505)
        km = ivf.IVFKMeans(*to_dev(x), x.d, k, **opts)
        km.init_seeds(i32(seeds))
        g = i32(np.full(x.n, -1, np.int32))
        st = km.assign_ivfd(g, objects_per_range=4096)
        ref = oracle.ivfd_assign(x, oracle.initial_means(x, seeds), np.full(x.n, -1, np.int32))
        _check_step(st, ref, g.cpu().numpy())
        if opts:
            assert st["certified"] == 0 and st["rescored"] == x.n - st["zero_overlap"]
            assert st["objective"] == pytest.approx(ref.objective, rel=1e-12)
        km.close()


def test_large_instance_same_partition_as_the_means_inverted_step():
    # a property that holds at any size: IVFD and IVF give one partition and
    # one multiplication count (300,000 objects: 19 ranges of 16,384)
    n, d, k, seed = 300_000, 60_000, 2000, 506
    x = datagen.generate(n, d, 60.0, 3, 400, 1.1, seed)
    seeds = datagen.seed_objects(x, k, seed)
    km = ivf.IVFKMeans(*to_dev(x), d, k)
    km.init_seeds(i32(seeds))
    g = i32(np.full(n, -1, np.int32))
    km.assign(g)
    km.update(g)
    g1 = g.clone()
    s1 = km.assign(g1)
    g2 = g.clone()
    s2 = km.assign_ivfd(g2)
    assert torch.equal(g1, g2)
    assert s1["mult_adds"] == s2["mult_adds"] and s1["changed"] == s2["changed"]
    print("IVF walk ms", s1["walk_ms"], "IVFD walk ms", s2["walk_ms"], flush=True)
    km.close()


def test_ivfd_rejects_what_it_does_not_support():
    x = datagen.generate(500, 300, 10.0, 1, 40, 1.1, 507)
    seeds = datagen.seed_objects(x, 5, 507)
    km = ivf.IVFKMeans(*to_dev(x), x.d, 5, valtype="bf16")
    km.init_seeds(i32(seeds))
    with pytest.raises(ivf.IvfError):
        km.assign_ivfd(i32(np.full(x.n, -1, np.int32)))
    km.close()
    km = ivf.IVFKMeans(*to_dev(x), x.d, 5)
    with pytest.raises(ivf.IvfError):
        km.assign_ivfd(i32(np.full(x.n, -1, np.int32)))          # no means yet
    km.init_seeds(i32(seeds))
    with pytest.raises(ivf.IvfError):
        km.assign_ivfd(i32(np.full(x.n, -1, np.int32)), objects_per_range=1000)
    km.close()


@pytest.mark.parametrize("obj_scale,mean_scale", [(50.0, 1000.0), (1.0, 1e-6), (0.02, 3.0)])
def test_fixed_point_scale_follows_the_norms(obj_scale, mean_scale):
    # objects and caller means of any norm: the fixed-point scale comes from
    # the largest norms (here 2^F = 2^15, 2^51 and 2^31 -ish), so the sums
    # neither overflow nor lose the ranking
    x0 = datagen.generate(6000, 2500, 25.0, 1, 100, 1.1, 508)
    x = datagen.CSR(x0.n, x0.d, x0.indptr, x0.indices,
                    (x0.values.astype(np.float64) * obj_scale).astype(np.float32))
    k = 40
    m0 = oracle.initial_means(x0, datagen.seed_objects(x0, k, 508))
    means = oracle.Means(k, x.d, m0.indptr, m0.indices, m0.values * mean_scale)
    prev = np.full(x.n, -1, np.int32)
    ref = oracle.ivfd_assign(x, means, prev)
    km = ivf.IVFKMeans(*to_dev(x), x.d, k)
    km.set_means(*means_to_dev(means))
    g = i32(prev)
    st = km.assign_ivfd(g, objects_per_range=4096)
    _check_step(st, ref, g.cpu().numpy())
    ga = i32(prev)
    km.assign(ga)
    assert torch.equal(g, ga)
    km.close()
