"""GPU parity of the means-inverted path (ivf_assign + ivf_update) at exact
ties and at adversarial magnitudes, against the FP64 oracle.

Ties: a mean repeated verbatim scores every object identically in FP32 and in
FP64, so the argmax rule (strict ">" from 0 in ascending cluster order: the
lowest id wins) decides, and the repeated cluster is left empty and keeps its
mean.  Repeats sit in the same cluster range and in different ranges (a small
cluster_range), so the rule is exercised in the range merge and in the FP64
re-score, with and without every object forced through the re-score.

Magnitudes: means scaled far below FP32's normal range, and large object
values beside FP16-subnormal mean values, where the certificate's absolute
terms (not its relative part) must send the objects to the FP64 re-score.
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


def _with_repeats(base, repeats):
    """Means with base.k + len(repeats) rows: for (copy, orig) in repeats
    (orig < copy), row copy repeats row orig; the other rows take base's rows
    in order.  Returns the means and the base row behind every row."""
    k = base.k + len(repeats)
    copies = dict(repeats)
    rest = iter(range(base.k))
    rows = []
    for j in range(k):
        rows.append(rows[copies[j]] if j in copies else next(rest))
    ptr = [0]
    idx, val = [], []
    for r in rows:
        a, b = int(base.indptr[r]), int(base.indptr[r + 1])
        idx.append(base.indices[a:b])
        val.append(base.values[a:b])
        ptr.append(ptr[-1] + b - a)
    return oracle.Means(k, base.d, np.asarray(ptr, np.int64), np.concatenate(idx),
                        np.concatenate(val)), rows


def _scale(m, f):
    return oracle.Means(m.k, m.d, m.indptr, m.indices, m.values * f)


def _chain_parity(x, means0, k, iters, opts):
    """The GPU chain from caller means against the oracle chain from the same
    means: assignments, counts and M identical, means within a few ulps."""
    km = ivf.IVFKMeans(*to_dev(x), x.d, k, **opts)
    km.set_means(*means_to_dev(means0))
    a = i32(np.full(x.n, -1, np.int32))
    means = means0
    prev = np.full(x.n, -1, np.int32)
    out = []
    for r in range(iters):
        ref = oracle.assign(x, means, prev)
        st = km.assign(a)
        got = a.cpu().numpy()
        mism = np.nonzero(got != ref.assign)[0]
        assert len(mism) == 0, (r, mism[:10], got[mism[:10]], ref.assign[mism[:10]])
        assert st["mult_adds"] == ref.mult_adds
        assert st["zero_overlap"] == ref.zero_overlap and st["changed"] == ref.changed
        assert st["certified"] + st["rescored"] + st["zero_overlap"] == x.n
        new, sizes = oracle.update(x, k, ref.assign, means)
        su = km.update(a)
        assert su["empty_clusters"] == int(np.sum(sizes == 0))
        gm = means_to_host(*km.get_means(), k, x.d)
        assert np.array_equal(gm.indptr, new.indptr) and np.array_equal(gm.indices, new.indices)
        np.testing.assert_allclose(gm.values, new.values, rtol=1e-12, atol=0)
        out.append((st, ref, sizes))
        means, prev = new, ref.assign
    km.close()
    return out


@pytest.mark.parametrize("force", [False, True])
@pytest.mark.parametrize("cluster_range", [0, 8])
def test_repeated_means_lowest_id_wins_and_the_copy_empties(cluster_range, force):
    x = datagen.generate(3000, 900, 14.0, 1, 60, 1.15, 611)
    base = oracle.initial_means(x, datagen.seed_objects(x, 36, 611))
    # (copy, original): 1 repeats 0 (same range at any width); 17 repeats 3
    # and 38 repeats 20 (other ranges at 8 clusters per range)
    pairs = [(1, 0), (17, 3), (38, 20)]
    means, rows = _with_repeats(base, pairs)
    k = means.k
    assert k == 39 and all(rows[c] == rows[o] for c, o in pairs)
    steps = _chain_parity(x, means, k, 3, {"cluster_range": cluster_range,
                                           "force_rescore": int(force)})
    st, ref, sizes = steps[0]
    # every object scored by an original also scores its copy exactly as high:
    # the copies win nothing and are left empty, keeping their means
    for copy, orig in pairs:
        assert not np.any(ref.assign == copy)
        assert np.any(ref.assign == orig)
        assert sizes[copy] == 0
    assert st["rescored"] > 0          # exact FP32 ties cannot be certified
    if cluster_range:
        p = ivf.plan_shape(k, cluster_range=cluster_range)
        assert p["ranges"] == 5


def test_zero_overlap_objects_keep_their_cluster():
    x = datagen.generate(400, 300, 5.0, 0, 10, 1.3, 612)     # sparse rows, some empty
    base = oracle.initial_means(x, datagen.seed_objects(x, 4, 612))
    means, _ = _with_repeats(base, [(2, 1)])
    steps = _chain_parity(x, means, means.k, 3, {"cluster_range": 2})
    assert steps[0][1].zero_overlap > 0


@pytest.mark.parametrize("valtype,scale", [("f32", 2.0 ** -100), ("f32", 2.0 ** -125),
                                           ("f32", 2.0 ** -140), ("bf16", 2.0 ** -140)])
def test_means_below_the_normal_range(valtype, scale):
    """Mean values scaled by a power of two: the FP64 scores scale exactly, so
    the oracle's partition is that of the unscaled means; the FP32 tile holds
    subnormal products (2^-125, 2^-140) that only the certificate's absolute
    term accounts for."""
    x = datagen.generate(2000, 700, 12.0, 1, 50, 1.1, 613)
    k = 30
    m1 = next(oracle.chain(x, datagen.seed_objects(x, k, 613), 1)).means_out
    ms = _scale(m1, scale)
    prev = np.full(x.n, -1, np.int32)
    ref = oracle.assign(x, ms, prev)
    assert np.array_equal(ref.assign, oracle.assign(x, m1, prev).assign)
    km = ivf.IVFKMeans(*to_dev(x), x.d, k, valtype=valtype)
    km.set_means(*means_to_dev(ms))
    a = i32(prev)
    st = km.assign(a)
    got = a.cpu().numpy()
    assert np.array_equal(got, ref.assign), np.nonzero(got != ref.assign)[0][:10]
    if scale < 2.0 ** -126:
        assert st["rescored"] > 0
    km.close()


def test_large_object_values_beside_fp16_subnormal_means():
    """Objects scaled to values up to ~50 and FP16 mean values below FP16's
    normal range: the absolute term grows with the largest object value."""
    x = datagen.generate(2000, 600, 12.0, 1, 50, 1.1, 614)
    x = datagen.CSR(x.n, x.d, x.indptr, x.indices, (x.values * np.float32(64.0)))
    k = 25
    m = _scale(oracle.initial_means(x, datagen.seed_objects(x, k, 614)), 2.0 ** -16)
    prev = np.full(x.n, -1, np.int32)
    ref = oracle.assign(x, m, prev)
    km = ivf.IVFKMeans(*to_dev(x), x.d, k, valtype="f16")
    km.set_means(*means_to_dev(m))
    a = i32(prev)
    st = km.assign(a)
    assert np.array_equal(a.cpu().numpy(), ref.assign)
    assert st["rescored"] > 0
    km.close()


def test_values_that_could_overflow_fp32_scores_are_rejected():
    x = datagen.generate(500, 300, 8.0, 1, 30, 1.1, 615)
    k = 5
    m = oracle.initial_means(x, datagen.seed_objects(x, k, 615))
    km = ivf.IVFKMeans(*to_dev(x), x.d, k, valtype="f16")
    with pytest.raises(ivf.IvfError) as e:
        km.set_means(*means_to_dev(_scale(m, 1e5)))     # beyond FP16's range
    assert e.value.status == -5
    km.set_means(*means_to_dev(m))                      # the handle stays usable
    a = i32(np.full(x.n, -1, np.int32))
    km.assign(a)
    assert np.array_equal(a.cpu().numpy(), oracle.assign(x, m, np.full(x.n, -1, np.int32)).assign)
    km.close()
    km = ivf.IVFKMeans(*to_dev(x), x.d, k)
    with pytest.raises(ivf.IvfError) as e:
        km.set_means(*means_to_dev(_scale(m, 2.0 ** 125)))
    assert e.value.status == -5
    km.close()
    big = datagen.CSR(x.n, x.d, x.indptr, x.indices, x.values * np.float32(2.0 ** 118))
    with pytest.raises(ivf.IvfError) as e:
        ivf.IVFKMeans(*to_dev(big), x.d, k)
    assert e.value.status == -5
