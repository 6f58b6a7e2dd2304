"""GPU: the FP32 walk's two tile kinds against each other and the oracle.

With FP32 values, ranges of up to 1,024 clusters take the register walk (the
dense slabs' products summed in registers, the sparse slices' in the wave's
LDS tile, the two sums added once); wider ranges take the LDS-tile walk (every
product in ascending term order).  Both are certified by the same bound and
re-scored in FP64 where it does not decide, so every plan (range width, slab
threshold) must give the oracle's assignment.  The FP32 scores of two plans
may differ in their last bits, each within the bound of the FP64 score; the
scores of one plan are reproducible bit for bit.
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
from gpu_util import i32, means_to_dev, to_dev  # noqa: E402

PLANS = [
    {"cluster_range": 1000},                          # register walk, 3 ranges of 700
    {"cluster_range": 1000, "dense_threshold": 0.2},  # register walk, more slabs
    {"cluster_range": 1000, "dense_threshold": 2.0},  # register walk, no slab at all
    {"cluster_range": 600},                           # register walk, 4 ranges of 525
    {"cluster_range": 1050},                          # LDS-tile walk, 2 ranges of 1,050
    {"cluster_range": 2100, "dense_threshold": 0.45}, # LDS-tile walk, one range
]


def test_every_plan_gives_the_oracle_assignment_and_bounded_scores():
    # the third iteration of a chain: 735 objects change cluster
    n, d, k = 30000, 6000, 2100
    x = datagen.generate(n, d, 40.0, 2, 200, 1.1, 77)
    seeds = datagen.seed_objects(x, k, 77)
    steps = list(oracle.chain(x, seeds, 3))
    means, prev, want = steps[2].means_in, steps[1].assign.assign, steps[2].assign
    assert want.changed > 500
    dx = to_dev(x)
    nnz = np.diff(x.indptr)
    vmax = float(x.values.max())
    seen = {}
    for opts in PLANS:
        runs = []
        for _ in range(2):   # two handles of the same plan
            km = ivf.IVFKMeans(*dx, d, k, **opts)
            km.set_means(*means_to_dev(means))
            a = i32(prev.copy())
            st = km.assign(a)
            got = a.cpu().numpy()
            assert np.array_equal(got, want.assign), opts
            assert st["mult_adds"] == want.mult_adds and st["changed"] == want.changed
            best, bid, second, _, _ = (t.cpu().numpy() for t in km.get_scores())
            runs.append((best, bid, second))
            km.close()
        # one plan: bit for bit
        assert all(np.array_equal(u.view(np.uint32), v.view(np.uint32))
                   for u, v in zip(runs[0][::2], runs[1][::2])), opts
        assert np.array_equal(runs[0][1], runs[1][1]), opts
        best, bid, _ = runs[0]
        # every FP32 winner's score within the bound of its FP64 score
        objs = np.nonzero(bid >= 0)[0]
        rho = oracle.scores(x, means, objs, bid[objs])
        for i, r, b in zip(objs[::7], rho[::7], best[objs][::7]):
            c, a_abs, g64 = ivf.cert_bound("f32", int(nnz[i]), vmax)
            assert abs(float(b) - r) <= (c + g64) * r * 1.0001 + a_abs, (opts, i, float(b), r)
        seen[str(opts)] = (best, bid)
    # two plans' scores of the same winner are no farther apart than both bounds
    cs = {}
    for nt in np.unique(nnz):
        c, a_abs, g64 = ivf.cert_bound("f32", int(nt), vmax)
        cs[int(nt)] = (c + g64, a_abs)
    tol_rel = np.array([cs[int(t)][0] for t in nnz])
    tol_abs = np.array([cs[int(t)][1] for t in nnz])
    ref, ref_id = seen[str(PLANS[0])]
    for key, (best, bid) in seen.items():
        both = np.nonzero((ref_id >= 0) & (bid == ref_id))[0]
        assert len(both) > 0.99 * n, key
        diff = np.abs(best[both].astype(np.float64) - ref[both].astype(np.float64))
        lim = 2.0002 * tol_rel[both] * ref[both] + 2 * tol_abs[both]
        assert np.all(diff <= lim), (key, float((diff / lim).max()))
