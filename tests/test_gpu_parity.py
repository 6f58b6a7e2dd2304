"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Contract: given the same means, the assignment is identical to the oracle's
at every iteration; the objective agrees within 1e-6 relative; given the same
assignment, the updated means have identical supports and values within
1e-6 relative (they are in fact within a few FP64 ulps).
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
from gpu_util import DEV, i32, means_to_dev, means_to_host, to_dev  # noqa: E402

REL = 1e-6


def _case(name):
    # (n, d, lam, lo, hi, s, k, seed, options)
    cases = {
        "k40": (3000, 2000, 20.0, 1, 80, 1.1, 40, 101, {}),
        "k300_ranges": (4000, 3000, 25.0, 2, 120, 1.05, 300, 102, {"cluster_range": 64}),
        "k1": (500, 400, 10.0, 1, 40, 1.1, 1, 103, {}),
        "long_rows": (1500, 5000, 150.0, 40, 600, 1.05, 60, 104, {"cluster_range": 16}),
        "ragged": (1237, 997, 12.0, 0, 50, 1.2, 37, 105, {"objects_per_item": 5,
                                                          "waves_per_wg": 3}),
    }
    return cases[name]


def _assert_means_close(gm, om):
    assert np.array_equal(gm.indptr, om.indptr)
    assert np.array_equal(gm.indices, om.indices)
    np.testing.assert_allclose(gm.values, om.values, rtol=REL, atol=0)


@pytest.mark.parametrize("name", ["k40", "k300_ranges", "k1", "long_rows", "ragged"])
def test_assign_and_update_parity_given_oracle_state(name):
    n, d, lam, lo, hi, s, k, seed, opts = _case(name)
    x = datagen.generate(n, d, lam, lo, hi, s, seed)
    seeds = datagen.seed_objects(x, k, seed)
    print("case", name, "n", n, "k", k, "nnz", x.nnz, flush=True)
    dx = to_dev(x)
    km = ivf.IVFKMeans(*dx, d, k, **opts)
    last = np.full(n, -1, np.int32)
    for r, st in enumerate(oracle.chain(x, seeds, 6)):
        km.set_means(*means_to_dev(st.means_in))
        a = i32(last)
        gs = km.assign(a)
        ga = a.cpu().numpy()
        mism = np.nonzero(ga != st.assign.assign)[0]
        assert len(mism) == 0, (name, r, mism[:10])
        assert gs["mult_adds"] == st.assign.mult_adds
        assert gs["zero_overlap"] == st.assign.zero_overlap
        assert gs["changed"] == st.assign.changed
        assert gs["objective"] == pytest.approx(st.assign.objective, rel=REL)
        # update from the oracle's assignment
        us = km.update(i32(st.assign.assign))
        gm = means_to_host(*km.get_means(), k, d)
        _assert_means_close(gm, st.means_out)
        assert us["objective_exact"] == pytest.approx(st.assign.objective, rel=1e-12)
        assert us["empty_clusters"] == int(np.sum(st.sizes == 0))
        last = st.assign.assign
    km.close()


@pytest.mark.parametrize("name", ["k40", "k300_ranges", "ragged"])
def test_chain_parity_gpu_means(name):
    n, d, lam, lo, hi, s, k, seed, opts = _case(name)
    x = datagen.generate(n, d, lam, lo, hi, s, seed)
    seeds = datagen.seed_objects(x, k, seed)
    km = ivf.IVFKMeans(*to_dev(x), d, k, **opts)
    km.init_seeds(i32(seeds))
    gm0 = means_to_host(*km.get_means(), k, d)
    om0 = oracle.initial_means(x, seeds)
    _assert_means_close(gm0, om0)
    a = i32(np.full(n, -1, np.int32))
    steps = list(oracle.chain(x, seeds, 8))
    for r, st in enumerate(steps):
        gs = km.assign(a)
        assert np.array_equal(a.cpu().numpy(), st.assign.assign), (name, r)
        assert gs["objective"] == pytest.approx(st.assign.objective, rel=REL)
        us = km.update(a)
        assert us["objective_exact"] == pytest.approx(st.assign.objective, rel=1e-12)
        _assert_means_close(means_to_host(*km.get_means(), k, d), st.means_out)
    km.close()


@pytest.mark.parametrize("valtype", ["f32", "bf16", "f16"])
def test_wide_ranges_parity(valtype):
    """Ranges wider than one round trip's slab (two ranges of 1,300 and 1,299
    clusters under a 2,048 limit): dense slabs take the looped path and 16-bit
    terms are not paired; assignments, M and the zero-overlap count equal the
    oracle's."""
    n, d, k, seed = 3000, 1500, 2599, 107
    x = datagen.generate(n, d, 40.0, 2, 150, 1.1, seed)
    seeds = datagen.seed_objects(x, k, seed)
    print("wide ranges", valtype, "n", n, "k", k, "nnz", x.nnz, flush=True)
    km = ivf.IVFKMeans(*to_dev(x), d, k, valtype=valtype, cluster_range=2048)
    assert km.plan["k_r"] == 1300 and km.plan["ranges"] == 2
    last = np.full(n, -1, np.int32)
    for r, st in enumerate(oracle.chain(x, seeds, 3)):
        km.set_means(*means_to_dev(st.means_in))
        a = i32(last)
        gs = km.assign(a)
        assert np.array_equal(a.cpu().numpy(), st.assign.assign), (valtype, r)
        assert gs["mult_adds"] == st.assign.mult_adds
        assert gs["zero_overlap"] == st.assign.zero_overlap
        last = st.assign.assign
    km.close()


@pytest.mark.parametrize("valtype", ["bf16", "f16"])
def test_half_precision_values_same_assignments(valtype):
    n, d, lam, lo, hi, s, k, seed, opts = _case("k300_ranges")
    x = datagen.generate(n, d, lam, lo, hi, s, seed)
    seeds = datagen.seed_objects(x, k, seed)
    km = ivf.IVFKMeans(*to_dev(x), d, k, valtype=valtype, **opts)
    last = np.full(n, -1, np.int32)
    for r, st in enumerate(oracle.chain(x, seeds, 5)):
        km.set_means(*means_to_dev(st.means_in))
        a = i32(last)
        gs = km.assign(a)
        assert np.array_equal(a.cpu().numpy(), st.assign.assign), (valtype, r)
        assert gs["certified"] + gs["rescored"] + gs["zero_overlap"] == n
        last = st.assign.assign
    km.close()


def test_forced_rescore_alone_matches():
    n, d, lam, lo, hi, s, k, seed, opts = _case("k300_ranges")
    x = datagen.generate(n, d, lam, lo, hi, s, seed)
    seeds = datagen.seed_objects(x, k, seed)
    km = ivf.IVFKMeans(*to_dev(x), d, k, force_rescore=True, **opts)
    last = np.full(n, -1, np.int32)
    for r, st in enumerate(oracle.chain(x, seeds, 3)):
        km.set_means(*means_to_dev(st.means_in))
        a = i32(last)
        gs = km.assign(a)
        assert gs["certified"] == 0
        assert gs["rescored"] == n - gs["zero_overlap"]
        assert np.array_equal(a.cpu().numpy(), st.assign.assign)
        # the objective is now the FP64 one, summed in another order
        assert gs["objective"] == pytest.approx(st.assign.objective, rel=1e-13)
        last = st.assign.assign
    km.close()


def test_small_workload_full_parity():
    w = datagen.WORKLOADS["small"]
    x = w.generate()
    seeds = w.seeds(x)
    km = ivf.IVFKMeans(*to_dev(x), w.d, w.k)
    last = np.full(x.n, -1, np.int32)
    for r, st in enumerate(oracle.chain(x, seeds, w.iters)):
        km.set_means(*means_to_dev(st.means_in))
        a = i32(last)
        gs = km.assign(a)
        assert np.array_equal(a.cpu().numpy(), st.assign.assign), r
        assert gs["mult_adds"] == st.assign.mult_adds
        assert gs["objective"] == pytest.approx(st.assign.objective, rel=REL)
        last = st.assign.assign
    km.close()
