"""GPU checks of the entry points the parity tests do not drive directly:
ivf_iterate, the per-object flags of ivf_get_scores, the content checks that
run on the device (unsorted or out-of-range term ids, non-finite or
non-positive values, in objects and in caller means), multi-iteration batch
calls and the autotuner's report."""
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


def _data(seed=401, n=2500, d=1800, k=60):
    x = datagen.generate(n, d, 25.0, 1, 120, 1.1, seed)
    return x, datagen.seed_objects(x, k, seed), d, k


def test_iterate_equals_assign_then_update_and_the_oracle_chain():
    x, seeds, d, k = _data()
    dx = to_dev(x)
    a = ivf.IVFKMeans(*dx, d, k)
    b = ivf.IVFKMeans(*dx, d, k)
    a.init_seeds(i32(seeds))
    b.init_seeds(i32(seeds))
    ga = i32(np.full(x.n, -1, np.int32))
    gb = i32(np.full(x.n, -1, np.int32))
    stats = a.iterate(5, ga)
    per = []
    for _ in range(5):
        per.append((b.assign(gb), b.update(gb)))
    assert np.array_equal(ga.cpu().numpy(), gb.cpu().numpy())
    ma = means_to_host(*a.get_means(), k, d)
    mb = means_to_host(*b.get_means(), k, d)
    assert np.array_equal(ma.indptr, mb.indptr) and np.array_equal(ma.indices, mb.indices)
    assert np.array_equal(ma.values, mb.values)
    for st, (sa, su) in zip(stats, per):
        for key in ("changed", "mult_adds", "certified", "rescored", "zero_overlap"):
            assert st[key] == sa[key]
        assert st["objective"] == sa["objective"]
        assert st["objective_exact"] == su["objective_exact"]
        assert st["nnz_means"] == su["nnz_means"]
    # and the chain is the FP64 reference's
    ref = list(oracle.chain(x, seeds, 5))
    assert np.array_equal(ga.cpu().numpy(), ref[-1].assign.assign)
    for st, r in zip(stats, ref):
        assert st["changed"] == r.assign.changed and st["mult_adds"] == r.assign.mult_adds
    a.close()
    b.close()


def test_score_flags_match_the_counts():
    x, seeds, d, k = _data(seed=402)
    km = ivf.IVFKMeans(*to_dev(x), d, k, valtype="bf16")   # BF16: some objects re-scored
    km.init_seeds(i32(seeds))
    a = i32(np.full(x.n, -1, np.int32))
    for _ in range(2):
        st = km.assign(a)
        km.update(a)
    st = km.assign(a)
    best, best_id, second, rho, flags = (t.cpu().numpy() for t in km.get_scores())
    assert int(np.sum(flags & 1)) == st["certified"]
    assert int(np.sum((flags >> 1) & 1)) == st["rescored"]
    assert int(np.sum((flags >> 2) & 1)) == st["zero_overlap"]
    assert st["certified"] + st["rescored"] + st["zero_overlap"] == x.n
    ga = a.cpu().numpy()
    cert = (flags & 1) == 1
    assert np.array_equal(ga[cert], best_id[cert])        # certified: the FP32 winner
    assert np.all(best[cert] > second[cert])
    zero = ((flags >> 2) & 1) == 1
    assert np.all(best_id[zero] == -1) and np.all(rho[zero] == 0.0)
    # the objective is the sum of rho in FP64
    assert st["objective"] == pytest.approx(float(np.sum(rho)), rel=1e-12)
    km.close()


def _bad_objects(kind):
    x, _, d, k = _data(seed=403, n=300, d=200, k=5)
    idx = x.indices.copy()
    val = x.values.copy()
    row = int(np.argmax(np.diff(x.indptr) >= 3))
    a = int(x.indptr[row])
    if kind == "unsorted":
        idx[a], idx[a + 1] = idx[a + 1], idx[a]
    elif kind == "range":
        idx[a + 2] = d + 7
    elif kind == "nan":
        val[a] = np.nan
    elif kind == "negative":
        val[a] = -val[a]
    return x, idx, val, d, k


@pytest.mark.parametrize("kind,status", [("unsorted", "IVF_ERR_UNSORTED"), ("range", "IVF_ERR_UNSORTED"),
                                         ("nan", "IVF_ERR_NONFINITE"),
                                         ("negative", "IVF_ERR_NEGATIVE")])
def test_object_content_errors_are_found_on_the_device(kind, status):
    x, idx, val, d, k = _bad_objects(kind)
    ptr = torch.from_numpy(x.indptr.astype(np.int64)).to(DEV)
    with pytest.raises(ivf.IvfError) as e:
        ivf.IVFKMeans(ptr, torch.from_numpy(idx).to(DEV), torch.from_numpy(val).to(DEV), d, k)
    assert status in str(e.value)


@pytest.mark.parametrize("kind,status", [("unsorted", "IVF_ERR_UNSORTED"), ("nan", "IVF_ERR_NONFINITE")])
def test_mean_content_errors_are_found_on_the_device(kind, status):
    x, seeds, d, k = _data(seed=404, n=400, d=300, k=6)
    means = oracle.initial_means(x, seeds)
    idx = means.indices.copy()
    val = means.values.copy()
    j = int(np.argmax(np.diff(means.indptr) >= 2))       # a mean with at least two terms
    a = int(means.indptr[j])
    if kind == "unsorted":
        idx[a], idx[a + 1] = idx[a + 1], idx[a]
    else:
        val[a] = np.inf
    km = ivf.IVFKMeans(*to_dev(x), d, k)
    bad = oracle.Means(k, d, means.indptr, idx, val)
    with pytest.raises(ivf.IvfError) as e:
        km.set_means(*means_to_dev(bad))
    assert status in str(e.value)
    km.set_means(*means_to_dev(means))          # the handle stays usable
    g = i32(np.full(x.n, -1, np.int32))
    km.assign(g)
    r = oracle.assign(x, means, np.full(x.n, -1, np.int32))
    assert np.array_equal(g.cpu().numpy(), r.assign)
    km.close()


def test_batch_multi_iteration_calls_and_tuning_report():
    sets = [(2000, 1500, 20.0, 1, 80, 1.1, 40, 405), (1500, 900, 15.0, 1, 60, 1.15, 300, 406)]
    inst = []
    for (n, d, lam, lo, hi, s, k, seed) in sets:
        x = datagen.generate(n, d, lam, lo, hi, s, seed)
        inst.append((x, to_dev(x), d, k, datagen.seed_objects(x, k, seed)))
    b = ivf.IVFBatch([(*dx, d) for (_, dx, d, _, _) in inst], [k for (_, _, _, k, _) in inst])
    b.init_seeds([i32(sd) for (_, _, _, _, sd) in inst])
    ba = [i32(np.full(x.n, -1, np.int32)) for (x, _, _, _, _) in inst]
    stats = b.iterate(3, ba) + b.iterate(3, ba)           # eager, tuned, recorded, replayed
    assert len(stats) == 6 and all(len(s) == 2 for s in stats)
    tuning = b.tuning
    assert len(tuning) == 5 and all(ms > 0 for (_, _, ms) in tuning)
    assert b.plan["kr_max"] == min(tuning, key=lambda t: t[2])[0]
    # then the dense-slab threshold on that shape
    thetas = b.threshold_tuning
    assert [round(t, 6) for (t, _) in thetas] == [0.35, 0.45, 0.5, 0.65]
    assert all(ms > 0 for (_, ms) in thetas)
    for i, (x, _, _, _, seeds) in enumerate(inst):
        ref = list(oracle.chain(x, seeds, 6))
        assert np.array_equal(ba[i].cpu().numpy(), ref[-1].assign.assign)
        assert [s[i]["changed"] for s in stats] == [r.assign.changed for r in ref]
    b.close()


def test_batch_threshold_given_by_the_caller_is_not_tuned():
    x = datagen.generate(1500, 900, 15.0, 1, 60, 1.15, 409)
    k = 60
    b = ivf.IVFBatch([(*to_dev(x), 900)], [k], dense_threshold=0.2)
    b.init_seeds([i32(datagen.seed_objects(x, k, 409))])
    a = [i32(np.full(x.n, -1, np.int32))]
    b.iterate(3, a)
    assert len(b.tuning) == 5 and b.threshold_tuning == []
    ref = list(oracle.chain(x, datagen.seed_objects(x, k, 409), 3))
    assert np.array_equal(a[0].cpu().numpy(), ref[-1].assign.assign)
    b.close()


def test_converge_stops_at_the_oracle_fixed_point():
    x, seeds, d, k = _data(seed=408, n=3000, d=2000, k=40)
    ref = list(oracle.chain(x, seeds, 30))
    fixed = next(r for r, st in enumerate(ref) if st.assign.changed == 0)   # 0-based step
    km = ivf.IVFKMeans(*to_dev(x), d, k)
    km.init_seeds(i32(seeds))
    a = i32(np.full(x.n, -1, np.int32))
    stats = km.converge(30, a)
    assert len(stats) == fixed + 1 and stats[-1]["changed"] == 0
    assert [s["changed"] for s in stats] == [st.assign.changed for st in ref[:fixed + 1]]
    assert np.array_equal(a.cpu().numpy(), ref[fixed].assign.assign)
    gm = means_to_host(*km.get_means(), k, d)
    assert np.array_equal(gm.indices, ref[fixed - 1].means_out.indices)   # the fixed point's means
    # a call with a small budget stops there
    km2 = ivf.IVFKMeans(*to_dev(x), d, k)
    km2.init_seeds(i32(seeds))
    a2 = i32(np.full(x.n, -1, np.int32))
    assert len(km2.converge(2, a2)) == 2
    km.close()
    km2.close()
