"""GPU parity of the batched form: many instances of uneven N, D and k (and
restarts of one object set) advanced together, one persistent walk launch per
iteration, the iteration replayed from recorded HIP graphs.

Every instance must compute exactly what one handle of the same options
computes: identical assignments at every iteration and bit-identical means.
Between replays the test does its own eager work (single-handle iterations,
copies to the host, synchronisations), and every replay is checked.  Two
instances are also checked against the FP64 oracle's chain directly.
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
from gpu_util import i32, means_to_host, to_dev  # noqa: E402

# (n, d, lam, lo, hi, s, k, seed, restarts)
SETS = [
    (3000, 2000, 20.0, 1, 80, 1.1, 40, 101, 1),
    (1237, 997, 12.0, 0, 50, 1.2, 37, 105, 1),
    (9000, 6000, 35.0, 3, 300, 1.05, 700, 301, 1),
    (500, 400, 10.0, 1, 40, 1.1, 1, 103, 1),
    (6000, 3000, 60.0, 5, 400, 1.15, 1500, 302, 1),
    (2500, 1500, 30.0, 2, 100, 1.1, 120, 201, 4),   # one object set, four restarts
]


def _instances():
    out = []
    for (n, d, lam, lo, hi, s, k, seed, reps) in SETS:
        x = datagen.generate(n, d, lam, lo, hi, s, seed)
        dx = to_dev(x)
        for r in range(reps):
            out.append((x, dx, d, k, datagen.seed_objects(x, k, seed + 1000 * r)))
    return out


def _same_fp32_stats(bs, ss, n, exact):
    """Statistics read from the FP32 tile scores.  With the same plan (range
    width and slab threshold) the batch computes every score as the single
    handle does, bit for bit.  Across plans, the FP32 register walk adds an
    object's dense-slab and sparse-slice products in two sums, and which
    slices are dense depends on the plan, so scores may differ in the last
    bits: the objective then agrees within both bounds, and the counts still
    partition the objects."""
    if exact:
        for key in ("certified", "rescored"):
            assert bs[key] == ss[key], key
        assert bs["objective"] == ss["objective"]
        return
    for st in (bs, ss):
        assert st["certified"] + st["rescored"] + st["zero_overlap"] == n
    tol = bs["objective_bound"] + ss["objective_bound"]
    assert abs(bs["objective"] - ss["objective"]) <= tol * ss["objective"] + 1e-300


def _run_against_singles(inst, iters, batch_opts, single_opts, slack=None, exact_fp32=True):
    b = ivf.IVFBatch([(dx[0], dx[1], dx[2], d) for (_, dx, d, _, _) in inst],
                     [k for (_, _, _, k, _) in inst], **batch_opts)
    if slack is not None:
        b.set_slack(*slack)
    singles = []
    for (x, dx, d, k, seeds) in inst:
        km = ivf.IVFKMeans(*dx, d, k, **single_opts)
        km.init_seeds(i32(seeds))
        singles.append(km)
    b.init_seeds([i32(sd) for (_, _, _, _, sd) in inst])
    ba = [i32(np.full(x.n, -1, np.int32)) for (x, _, _, _, _) in inst]
    sa = [i32(np.full(x.n, -1, np.int32)) for (x, _, _, _, _) in inst]
    plans = []
    for r in range(iters):
        bst = b.iterate(1, ba)[0]
        plans.append(b.plan)
        for i, km in enumerate(singles):
            s1 = km.assign(sa[i])
            s2 = km.update(sa[i])
            ga, gs = ba[i].cpu().numpy(), sa[i].cpu().numpy()
            mism = np.nonzero(ga != gs)[0]
            assert len(mism) == 0, ("iteration", r, "instance", i, mism[:10])
            for key in ("changed", "mult_adds", "zero_overlap"):
                assert bst[i][key] == s1[key], (r, i, key, bst[i][key], s1[key])
            _same_fp32_stats(bst[i], s1, ga.shape[0], exact_fp32)
            assert bst[i]["objective_exact"] == s2["objective_exact"]
            assert bst[i]["empty_clusters"] == s2["empty_clusters"]
            assert bst[i]["nnz_means"] == s2["nnz_means"]
        torch.cuda.synchronize()
    for i, km in enumerate(singles):
        bp, bi, bv = (t.cpu().numpy() for t in b.get_means(i))
        sp, si, sv = (t.cpu().numpy() for t in km.get_means())
        assert np.array_equal(bp, sp) and np.array_equal(bi, si)
        assert np.array_equal(bv, sv)           # bit-identical FP64 means
        km.close()
    plan = b.plan
    b.close()
    return plans, plan


def test_batch_equals_single_handles_with_autotuned_tiles():
    # the tuner picks the batch's tiles and slab threshold, the single handles
    # keep their defaults: FP32 statistics agree within the bound
    inst = _instances()
    print("instances", len(inst), flush=True)
    plans, plan = _run_against_singles(inst, 7, {}, {}, exact_fp32=False)
    print("plan", plan, flush=True)
    assert plans[0]["graphs"] == 0 and plans[1]["tuned"] == 1
    assert plans[2]["graphs"] == 1 and plan["captures"] >= 1
    assert plan["kr_max"] in (1024, 1280, 2560, 5120)


def test_batch_overflow_recovery_and_fixed_tiles():
    # no slack: the first replays outgrow the fixed buffers; every overflow is
    # redone eagerly and the graphs recorded again, with identical results
    inst = _instances()
    opts = {"cluster_range": 64, "waves_per_wg": 3}
    plans, plan = _run_against_singles(inst, 7, opts, opts, slack=(0.0, 0))
    print("plan", plan, flush=True)
    assert plan["tuned"] == 0 and plan["kr_max"] == 64 and plan["waves"] == 3
    assert plan["recoveries"] >= 1 and plan["captures"] >= 2


def test_batch_mixed_tile_kinds_equal_single_handles():
    # 2,560-wide tiles: instances whose ranges fit 1,024 clusters take the
    # FP32 register walk, the others the LDS-tile walk, in one launch; with
    # the same plan every statistic equals the single handle's bit for bit
    inst = _instances()
    opts = {"cluster_range": 2560, "waves_per_wg": 4, "dense_threshold": 0.35}
    plans, plan = _run_against_singles(inst, 4, opts, opts)
    assert plan["kr_max"] == 2560 and plan["tuned"] == 0
    assert any(k > 1024 for (_, _, _, k, _) in inst) and any(k <= 1024 for (_, _, _, k, _) in inst)


@pytest.mark.parametrize("valtype", ["bf16", "f16"])
def test_batch_low_precision_values(valtype):
    inst = _instances()[:5]
    _run_against_singles(inst, 4, {"valtype": valtype}, {"valtype": valtype})


def test_batch_chain_against_oracle():
    inst = [v for v in _instances() if v[3] in (40, 37)]
    b = ivf.IVFBatch([(dx[0], dx[1], dx[2], d) for (_, dx, d, _, _) in inst],
                     [k for (_, _, _, k, _) in inst])
    b.init_seeds([i32(sd) for (_, _, _, _, sd) in inst])
    ba = [i32(np.full(x.n, -1, np.int32)) for (x, _, _, _, _) in inst]
    chains = [oracle.chain(x, seeds, 6) for (x, _, _, _, seeds) in inst]
    for r in range(6):
        bst = b.iterate(1, ba)[0]
        for i, ch in enumerate(chains):
            st = next(ch)
            assert np.array_equal(ba[i].cpu().numpy(), st.assign.assign), (r, i)
            assert bst[i]["mult_adds"] == st.assign.mult_adds
            assert bst[i]["objective"] == pytest.approx(st.assign.objective, rel=1e-6)
            x, _, d, k, _ = inst[i]
            gm = means_to_host(*b.get_means(i), k, d)
            assert np.array_equal(gm.indptr, st.means_out.indptr)
            assert np.array_equal(gm.indices, st.means_out.indices)
            np.testing.assert_allclose(gm.values, st.means_out.values, rtol=1e-6, atol=0)
    b.close()


def test_batch_rejects_bad_arguments():
    x = datagen.generate(300, 200, 10.0, 1, 30, 1.1, 7)
    dx = to_dev(x)
    with pytest.raises(ivf.IvfError):
        ivf.IVFBatch([(dx[0], dx[1], dx[2], 200)], [301])        # k > n
    b = ivf.IVFBatch([(dx[0], dx[1], dx[2], 200)], [5])
    with pytest.raises(ivf.IvfError):
        b.iterate(1, [i32(np.full(300, -1, np.int32))])          # no means yet
    with pytest.raises(ivf.IvfError):
        b.set_slack(-1.0, 0)
    b.close()


def test_batch_at_the_many_instance_workload_scale():
    """24 instances of the 96-instance workload (uneven N up to 400,000, k up
    to the workload's largest, one object set's 8 restarts) for 5 iterations:
    2 eager, then graph replays.  Every instance's assignment vector and
    counters at every iteration, and its final means, equal a single
    handle's bit for bit; at every iteration each single handle's FP64
    re-scored objects are re-assigned identically by the oracle from the
    same means, so the batch's are too."""
    from gpu_util import digest, oracle_check
    allinst = datagen.batched_instances()
    distinct = [i for i, (w, r) in enumerate(allinst) if w.name < "batch48"]
    restarted_sets = sorted({w.name for w, r in allinst if w.name >= "batch48"},
                            key=lambda nm: -[w.k for w, _ in allinst if w.name == nm][0])
    chosen = [i for i, (w, r) in enumerate(allinst) if w.name == restarted_sets[0]]
    by_k = sorted(distinct, key=lambda i: allinst[i][0].k)
    chosen.append(by_k[-1])                                   # the largest k
    rest = by_k[:-1]
    chosen += [rest[int(round(q * (len(rest) - 1) / 14))] for q in range(15)]
    assert len(set(chosen)) == 24
    inst = [allinst[i] for i in chosen]
    data = {}
    for w, _ in inst:
        if w.name not in data:
            x = w.generate()
            data[w.name] = (x, to_dev(x))
    print("instances", [(w.name, w.n, w.k, r) for w, r in inst], flush=True)
    b = ivf.IVFBatch([(*data[w.name][1], w.d) for w, _ in inst], [w.k for w, _ in inst])
    seeds = [w.seeds(data[w.name][0], restart=r) for w, r in inst]
    b.init_seeds([i32(s) for s in seeds])
    ba = [i32(np.full(w.n, -1, np.int32)) for w, _ in inst]
    iters = 5
    hist = []
    for r in range(iters):
        bst = b.iterate(1, ba)[0]
        hist.append([(digest(ba[i].cpu().numpy()), bst[i]) for i in range(len(inst))])
        print("batch iteration", r + 1, "plan", b.plan, flush=True)
        torch.cuda.synchronize()
    assert b.plan["graphs"] == 1 and b.plan["captures"] >= 1
    final = [tuple(t.cpu().numpy() for t in b.get_means(i)) for i in range(len(inst))]
    b.close()
    checked = 0
    for i, (w, rs) in enumerate(inst):
        x, dx = data[w.name]
        km = ivf.IVFKMeans(*dx, w.d, w.k)
        km.init_seeds(i32(seeds[i]))
        sa = i32(np.full(w.n, -1, np.int32))
        prev = np.full(w.n, -1, np.int32)
        for r in range(iters):
            means = means_to_host(*km.get_means(), w.k, w.d)
            s1 = km.assign(sa)
            got = sa.cpu().numpy()
            h, bs = hist[r][i]
            assert digest(got) == h, (w.name, rs, r)
            for key in ("changed", "mult_adds", "zero_overlap"):
                assert bs[key] == s1[key], (w.name, rs, r, key)
            # the batch's plan (tuned tiles and threshold) is not the single
            # handle's default
            _same_fp32_stats(bs, s1, w.n, False)
            flags = km.get_scores()[4].cpu().numpy()
            resc = np.nonzero(flags & 2)[0]
            if len(resc):
                _, mism = oracle_check(x, means, prev, got, resc)
                assert len(mism) == 0, (w.name, rs, r, mism[:10])
                checked += len(resc)
            s2 = km.update(sa)
            for key in ("objective_exact", "empty_clusters", "nnz_means"):
                assert bs[key] == s2[key], (w.name, rs, r, key)
            prev = got
        sp, si, sv = (t.cpu().numpy() for t in km.get_means())
        bp, bi, bv = final[i]
        assert np.array_equal(bp, sp) and np.array_equal(bi, si) and np.array_equal(bv, sv)
        km.close()
    print("re-scored objects checked against the oracle:", checked, flush=True)
    assert checked > 0
