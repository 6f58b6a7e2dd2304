"""GPU parity at the benchmark sizes, on sampled outputs the oracle computes
one by one, plus properties of the GPU's own chain that hold at any size.

The means handed to both sides come from the oracle: its update step applied
to a seeded random partition (the shape of steady-state means on this
structureless data).  The GPU walk then assigns all objects in the launch
configuration bench.py times; the oracle assigns a seeded sample of them.
"""
import json
import os

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2002_09094_amd as ivf  # noqa: E402
from gpu_util import DEV, i32, means_to_dev, to_dev  # noqa: E402

# measured numbers are also written as JSON files into $IVF_REPORT_DIR, if set
REPORT_DIR = os.environ.get("IVF_REPORT_DIR", "")


def _report(name, payload):
    print(name, json.dumps(payload), flush=True)
    if REPORT_DIR and os.path.isdir(REPORT_DIR):
        with open(os.path.join(REPORT_DIR, name + ".json"), "w") as f:
            json.dump(payload, f, indent=1)


def _partition_means(x, k, seed):
    labels = datagen.uniform_labels(x.n, k, seed, stream=11)
    means, _ = oracle.update(x, k, labels, None)
    return means


def _sample(n, m, seed):
    return np.sort(datagen.perm_prefix(n, m, seed, stream=7))


@pytest.fixture(scope="module")
def pubmed():
    w = datagen.WORKLOADS["pubmed_8m"]
    print("generating pubmed_8m", flush=True)
    x = w.generate()
    means = _partition_means(x, w.k, w.seed)
    return w, x, means


def test_pubmed_8m_sampled_parity_and_exact_count(pubmed):
    w, x, means = pubmed
    km = ivf.IVFKMeans(*to_dev(x), w.d, w.k)
    km.set_means(*means_to_dev(means))
    a = i32(np.full(x.n, -1, np.int32))
    st = km.assign(a)
    ga = a.cpu().numpy()
    no, nc = oracle.term_counts(x, means)
    assert st["mult_adds"] == int(np.sum(no * nc))          # Eq. ivf_mult, exact
    idx = _sample(x.n, 3000, 31)
    xs = x.subset(idx)
    ar = oracle.assign(xs, means, np.full(len(idx), -1, np.int32))
    assert np.array_equal(ga[idx], ar.assign)
    best, best_id, second, rho, flags = km.get_scores()
    rho = rho.cpu().numpy()[idx]
    np.testing.assert_allclose(rho, ar.rho, rtol=1e-5)        # FP32 scores of the winners
    _report("pubmed_8m_sampled_parity", {
        "sample": len(idx), "identical": int(np.sum(ga[idx] == ar.assign)),
        "certified": st["certified"], "rescored": st["rescored"], "mult_adds": st["mult_adds"],
        "walk_ms": st["walk_ms"],
        "max_rel_err_winner": float(np.max(np.abs(rho - ar.rho) / ar.rho))})
    km.close()


def test_pubmed_8m_gpu_chain_properties(pubmed):
    w, x, _ = pubmed
    km = ivf.IVFKMeans(*to_dev(x), w.d, w.k)
    km.init_seeds(i32(w.seeds(x)))
    a = i32(np.full(x.n, -1, np.int32))
    objs = []
    for r in range(3):
        sa = km.assign(a)
        su = km.update(a)
        assert su["objective_exact"] == pytest.approx(sa["objective"], rel=sa["objective_bound"])
        objs.append(su["objective_exact"])
        assert sa["certified"] + sa["rescored"] + sa["zero_overlap"] == x.n
    assert objs == sorted(objs)                           # non-decreasing objective
    ptr, idx, val = (t.cpu().numpy() for t in km.get_means())
    ga = a.cpu().numpy()
    rng = np.random.default_rng(5)
    for j in rng.choice(w.k, 20, replace=False):
        lo, hi = int(ptr[j]), int(ptr[j + 1])
        assert abs(np.sqrt(np.sum(val[lo:hi] ** 2)) - 1.0) < 1e-13
        assert np.all(np.diff(idx[lo:hi]) > 0)
        mem = np.nonzero(ga == j)[0]
        if len(mem):
            sup = np.unique(np.concatenate([x.row(i)[0] for i in mem]))
            assert np.array_equal(sup, idx[lo:hi])
            # the mean is the normalised member sum (member sum in FP64 here)
            s = np.zeros(w.d)
            for i in mem:
                t, v = x.row(i)
                s[t] += v.astype(np.float64)
            u = s / np.linalg.norm(s)
            np.testing.assert_allclose(val[lo:hi], u[idx[lo:hi]], rtol=1e-12)
    km.close()


@pytest.mark.parametrize("valtype", ["f32", "bf16", "f16"])
def test_precision_workload_sampled(valtype):
    w = datagen.WORKLOADS["precision"]
    x = _precision_data()
    means = _precision_means()
    km = ivf.IVFKMeans(*to_dev(x), w.d, w.k, valtype=valtype)
    km.set_means(*means_to_dev(means))
    a = i32(np.full(x.n, -1, np.int32))
    st = km.assign(a)
    ga = a.cpu().numpy()
    best, best_id, second, rho, flags = (t.cpu().numpy() for t in km.get_scores())
    idx = _sample(x.n, 2000, 41)
    xs = x.subset(idx)
    ar = oracle.assign(xs, means, np.full(len(idx), -1, np.int32))
    assert np.array_equal(ga[idx], ar.assign)
    # tile-score error against the FP64 scores of the same clusters
    bi = best_id[idx]
    ok = bi >= 0
    r64 = oracle.scores(x, means, idx[ok], bi[ok])
    err1 = np.abs(best[idx][ok].astype(np.float64) - r64) / r64
    c, _, g = ivf.cert_bound(valtype, int(np.max(np.diff(x.indptr))))
    assert np.all(err1 <= c)
    # top-2: where the tile's winner is the FP64 winner, the tile's best other
    # score and the oracle's are maxima over the same clusters, so they agree
    # within the same bound (plus the FP64 reference's own rounding)
    same = (bi == ar.assign) & (ar.rho2 > 0)
    err2 = np.abs(second[idx][same].astype(np.float64) - ar.rho2[same]) / ar.rho2[same]
    assert same.sum() > 0.9 * len(idx) and np.all(err2 <= c + 2 * g)
    _report("precision_%s" % valtype, {
        "valtype": valtype, "n": x.n, "k": w.k, "sample": len(idx),
        "identical_sample": int(np.sum(ga[idx] == ar.assign)),
        "certified_fraction": st["certified"] / x.n, "rescored": st["rescored"],
        "zero_overlap": st["zero_overlap"], "walk_ms": st["walk_ms"],
        "assign_ms": st["assign_ms"], "mult_adds": st["mult_adds"],
        "max_rel_err_top1_sample": float(err1.max()),
        "max_rel_err_top2_sample": float(err2.max()),
        "max_rel_err_rescored_winners": st["max_rel_err"], "plan": km.plan})
    km.close()


_PREC = {}


def _precision_data():
    if "x" not in _PREC:
        _PREC["x"] = datagen.WORKLOADS["precision"].generate()
    return _PREC["x"]


def _precision_means():
    if "m" not in _PREC:
        w = datagen.WORKLOADS["precision"]
        _PREC["m"] = _partition_means(_precision_data(), w.k, w.seed)
    return _PREC["m"]
