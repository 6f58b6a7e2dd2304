"""Writes tests/golden/<workload>_chain.json: the FP64 oracle's Lloyd chain on a
seeded synthetic workload (per iteration: SHA-256 of the assignment vector,
objective, mult-add count, changes, objects without a shared term, nnz of the
new means).  Calls only the oracle and the input generator.

    python tests/golden/make_chain_golden.py nyt_like [iters]
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import datagen  # noqa: E402
import oracle  # noqa: E402


def main():
    name = sys.argv[1]
    w = datagen.WORKLOADS[name]
    iters = int(sys.argv[2]) if len(sys.argv) > 2 else w.iters
    x = w.generate()
    seeds = w.seeds(x)
    out = {"workload": name, "n": w.n, "d": w.d, "k": w.k, "nnz": x.nnz, "seed": w.seed,
           "iters": iters, "seeds_sha256": hashlib.sha256(seeds.astype(np.int64).tobytes()).hexdigest(),
           "steps": []}
    t0 = time.time()
    for r, st in enumerate(oracle.chain(x, seeds, iters, keep_means=False)):
        a = st.assign
        out["steps"].append({
            "iter": r + 1,
            "assign_sha256": hashlib.sha256(a.assign.astype(np.int32).tobytes()).hexdigest(),
            "objective": a.objective, "mult_adds": a.mult_adds, "changed": a.changed,
            "zero_overlap": a.zero_overlap, "nnz_means_out": st.means_out.nnz,
            "empty_clusters": int(np.sum(st.sizes == 0))})
        print("iter %d: J=%.10g M=%d changed=%d (%.0fs)" % (r + 1, a.objective, a.mult_adds,
                                                           a.changed, time.time() - t0), flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "%s_chain.json" % name),
              "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
