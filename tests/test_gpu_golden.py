"""The GPU's own Lloyd chain against the oracle's stored chains:
  - nyt_like: 300,000 documents x 100,000 terms, k = 10,000, 20 iterations
    (NYT-like density; this chain reaches a fixed point at iteration 2);
  - pubmed_1m: 1,000,000 documents x 140,000 terms, k = 10,000, 10 iterations
    (the paper's 1M-document PubMed sample shape; hundreds of thousands of
    objects still move after the first iterations, so every iteration checks
    a new state).

tests/golden/<workload>_chain.json was written by make_chain_golden.py, which
calls only the input generator and the FP64 oracle.  Per iteration the GPU
chain (its own means, no injection) must give the identical assignment vector
(SHA-256), the same mult-add count (Eq. ivf_mult), change count, zero-overlap
count and new-means size, and the objective within 1e-6 relative.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2002_09094_amd as ivf  # noqa: E402
from gpu_util import i32, to_dev  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("workload", ["nyt_like", "pubmed_1m"])
def test_chain_matches_oracle_golden(workload):
    g = json.load(open(os.path.join(GOLDEN, workload + "_chain.json")))
    w = datagen.WORKLOADS[g["workload"]]
    print("generating", w.name, flush=True)
    x = w.generate()
    assert x.nnz == g["nnz"]
    seeds = w.seeds(x)
    assert hashlib.sha256(seeds.astype(np.int64).tobytes()).hexdigest() == g["seeds_sha256"]
    km = ivf.IVFKMeans(*to_dev(x), w.d, w.k)
    km.init_seeds(i32(seeds))
    a = i32(np.full(x.n, -1, np.int32))
    for step in g["steps"]:
        sa = km.assign(a)
        su = km.update(a)
        got = hashlib.sha256(a.cpu().numpy().astype(np.int32).tobytes()).hexdigest()
        print("iter", step["iter"], "changed", sa["changed"], "walk_ms", round(sa["walk_ms"], 2),
              flush=True)
        assert got == step["assign_sha256"], step["iter"]
        assert sa["mult_adds"] == step["mult_adds"]
        assert sa["changed"] == step["changed"]
        assert sa["zero_overlap"] == step["zero_overlap"]
        assert su["nnz_means"] == step["nnz_means_out"]
        assert su["empty_clusters"] == step["empty_clusters"]
        assert sa["objective"] == pytest.approx(step["objective"], rel=1e-6)
    km.close()
