"""GPU parity at the benchmark sizes: the GPU's own Lloyd chain from the
seeded initial state, in the launch configuration bench.py times, checked
against the FP64 oracle at every iteration.

Per iteration the means the GPU assigned with are copied to the host, and the
oracle assigns, from the same previous assignment,
  - every object the GPU re-scored in FP64 (its FP32 margin was inside the
    certification bound),
  - the objects with the smallest FP32 margin (best - second) / best,
  - a seeded sample;
the GPU's assignment must be identical on all of them.  Every other object
was certified: its FP32 winner is provably the oracle's argmax.  The same
chain with BF16 and FP16 mean values must give the identical assignment
vector (SHA-256) at every iteration, re-scoring some objects in FP64.  The
multiplication count M must equal sum_t (no)_t (nc)_t exactly (Eq. ivf_mult).

Workloads: 8M documents x 140k terms at k = 10,000 (the benchmark's), and the
precision workload, 2M documents x 200k terms at k = 50,000 (40+ cluster
ranges).  Measured numbers are also written as JSON into $IVF_REPORT_DIR.
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
from gpu_util import (digest, i32, means_to_host, oracle_check, score_errors,  # noqa: E402
                      to_dev, uncertain_objects)

REPORT_DIR = os.environ.get("IVF_REPORT_DIR", "")
VALTYPES = ("f32", "bf16", "f16")


def _report(name, payload):
    print(name, json.dumps(payload), flush=True)
    if REPORT_DIR and os.path.isdir(REPORT_DIR):
        with open(os.path.join(REPORT_DIR, name + ".json"), "w") as f:
            json.dump(payload, f, indent=1)


def _chains_against_oracle(w, x, iters, n_margin, n_sample):
    """FP32, BF16 and FP16 handles advanced in lockstep from the seeds; the FP32
    chain's uncertain objects and a sample checked against the oracle at every
    iteration, the 16-bit chains' assignments compared with FP32's."""
    dx = to_dev(x)
    kms = {vt: ivf.IVFKMeans(*dx, w.d, w.k, valtype=vt) for vt in VALTYPES}
    seeds = i32(w.seeds(x))
    for km in kms.values():
        km.init_seeds(seeds)
    a = {vt: i32(np.full(x.n, -1, np.int32)) for vt in VALTYPES}
    prev = np.full(x.n, -1, np.int32)
    vmax = float(x.values.max())
    nmax = int(np.max(np.diff(x.indptr)))
    rows, objs_hist = [], []
    for r in range(iters):
        means = means_to_host(*kms["f32"].get_means(), w.k, w.d)
        no, nc = oracle.term_counts(x, means)
        m_exact = int(np.sum(no * nc))
        st, got, sc = {}, {}, {}
        for vt in VALTYPES:
            st[vt] = kms[vt].assign(a[vt])
            got[vt] = a[vt].cpu().numpy()
            sc[vt] = [t.cpu().numpy() for t in kms[vt].get_scores()]
        best, best_id, second, _, flags = sc["f32"]
        resc, low = uncertain_objects(best, second, flags, n_margin)
        samp = np.sort(datagen.perm_prefix(x.n, n_sample, w.seed + 17 * r, stream=7))
        objs = np.unique(np.concatenate([resc, low, samp]))
        print("iteration %d: oracle on %d objects (%d re-scored, %d lowest margins, %d sampled)"
              % (r + 1, len(objs), len(resc), len(low), len(samp)), flush=True)
        ar, mism = oracle_check(x, means, prev, got["f32"], objs)
        assert len(mism) == 0, (r, mism[:10])
        row = {"iter": r + 1, "oracle_objects": int(len(objs)), "mult_adds": m_exact,
               "nnz_means": means.nnz, "assign_sha256": digest(got["f32"])}
        # the sample's rows of the oracle result, for the score errors
        pos = np.searchsorted(objs, samp)
        ar_s = oracle.AssignResult(ar.assign[pos], ar.rho[pos], ar.rho2[pos], 0.0, 0, 0, 0)
        for vt in VALTYPES:
            s = st[vt]
            assert s["mult_adds"] == m_exact
            assert s["certified"] + s["rescored"] + s["zero_overlap"] == x.n
            assert digest(got[vt]) == row["assign_sha256"], (vt, r)
            b, bi, s2, _, fl = sc[vt]
            c, ab, g = ivf.cert_bound(vt, nmax, vmax)
            e1, e2, n1, n2, held = score_errors(x, means, samp, ar_s, b, bi, s2, (c, ab, g))
            assert held, (vt, r, e1, e2, c)
            row[vt] = {"certified_fraction": s["certified"] / x.n, "rescored": s["rescored"],
                       "changed": s["changed"], "walk_ms": s["walk_ms"],
                       "max_rel_err_top1_sample": e1, "max_rel_err_top2_sample": e2,
                       "sample_top1": n1, "sample_top2": n2,
                       "max_rel_err_rescored": s["max_rel_err_rescored"], "bound_c": c}
        rows.append(row)
        objs_hist.append(objs)
        for vt in VALTYPES:
            su = kms[vt].update(a[vt])
            assert su["objective_exact"] == pytest.approx(
                st[vt]["objective"], rel=max(st[vt]["objective_bound"], 1e-12))
            row[vt]["objective_exact"] = su["objective_exact"]
        prev = got["f32"]
    return kms, a, rows


@pytest.fixture(scope="module")
def pubmed():
    w = datagen.WORKLOADS["pubmed_8m"]
    print("generating pubmed_8m", flush=True)
    return w, w.generate()


def test_pubmed_8m_chain_matches_oracle_on_every_uncertain_object(pubmed):
    w, x = pubmed
    kms, a, rows = _chains_against_oracle(w, x, 3, 20_000, 50_000)
    objs = [r["f32"]["objective_exact"] for r in rows]
    assert objs == sorted(objs)                           # non-decreasing objective
    for vt in ("bf16", "f16"):
        assert sum(r[vt]["rescored"] for r in rows) > 0
    # the means: unit norm, supports = union of the members', values = the
    # normalised member sums
    ptr, idx, val = (t.cpu().numpy() for t in kms["f32"].get_means())
    ga = a["f32"].cpu().numpy()
    rng = np.random.default_rng(5)
    for j in rng.choice(w.k, 20, replace=False):
        lo, hi = int(ptr[j]), int(ptr[j + 1])
        assert abs(np.sqrt(np.sum(val[lo:hi] ** 2)) - 1.0) < 1e-13
        assert np.all(np.diff(idx[lo:hi]) > 0)
        mem = np.nonzero(ga == j)[0]
        if len(mem):
            sup = np.unique(np.concatenate([x.row(i)[0] for i in mem]))
            assert np.array_equal(sup, idx[lo:hi])
            s = np.zeros(w.d)
            for i in mem:
                t, v = x.row(i)
                s[t] += v.astype(np.float64)
            u = s / np.linalg.norm(s)
            np.testing.assert_allclose(val[lo:hi], u[idx[lo:hi]], rtol=1e-12)
    for km in kms.values():
        km.close()
    _report("pubmed_8m_chain_parity", {"workload": w.name, "n": x.n, "k": w.k, "iters": rows})


def test_precision_workload_chain_matches_oracle():
    w = datagen.WORKLOADS["precision"]
    print("generating precision", flush=True)
    x = w.generate()
    kms, a, rows = _chains_against_oracle(w, x, 3, 20_000, 20_000)
    assert kms["f32"].plan["ranges"] >= 40
    for vt in ("bf16", "f16"):
        assert sum(r[vt]["rescored"] for r in rows) > 0
    for km in kms.values():
        km.close()
    _report("precision_chain_parity", {"workload": w.name, "n": x.n, "k": w.k, "iters": rows})
