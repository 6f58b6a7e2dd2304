"""GPU: ivf_assign_static (the assignment step with its scratch in the
library's fixed per-device array, no device allocation) against ivf_assign on
the same handle state, bit for bit: assignments, per-object scores and flags,
counters and objective.  Two calls in a row on one GPU, the second on a
smaller object set (the array keeps the first call's contents), each after an
update so the means move; the FP64 re-score runs on every object of one
call.  A step needing more than the array is refused before any launch.
"""
import numpy as np
import pytest

import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2002_09094_amd as ivf  # noqa: E402
from gpu_util import i32, to_dev  # noqa: E402

EXACT = ("changed", "certified", "rescored", "zero_overlap", "mult_adds", "objective",
         "objective_bound", "max_rel_err_rescored")


def _compare(km, prev):
    a = i32(prev)
    b = i32(prev)
    sa = km.assign(a)
    ref = [t.cpu().numpy() for t in km.get_scores()]
    sb = km.assign_static(b)
    got = [t.cpu().numpy() for t in km.get_scores()]
    assert torch.equal(a, b)
    for key in EXACT:
        assert sa[key] == sb[key], key
    for x, y in zip(ref, got):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
    return a.cpu().numpy(), sa


@pytest.mark.parametrize("force", [False, True])
def test_static_scratch_assign_equals_assign_on_two_calls(force):
    shapes = [(30000, 8000, 40.0, 3, 200, 1.1, 300, 31, {}),
              (7000, 3000, 25.0, 0, 120, 1.05, 90, 32, {"cluster_range": 32})]
    prev_n = None
    for n, d, lam, lo, hi, s, k, seed, opts in shapes:
        assert prev_n is None or n < prev_n      # the second call is the smaller input
        prev_n = n
        x = datagen.generate(n, d, lam, lo, hi, s, seed)
        km = ivf.IVFKMeans(*to_dev(x), d, k, force_rescore=force, **opts)
        km.init_seeds(i32(datagen.seed_objects(x, k, seed)))
        prev = np.full(n, -1, np.int32)
        for r in range(2):
            got, st = _compare(km, prev)
            if force:
                assert st["rescored"] + st["zero_overlap"] == n
            km.update(i32(got))
            prev = got
        km.close()


def test_static_scratch_refuses_steps_beyond_its_size():
    # 40,000 objects x 125 ranges x 16 B of records > 64 MiB
    x = datagen.generate(40000, 3000, 10.0, 1, 40, 1.1, 33)
    km = ivf.IVFKMeans(*to_dev(x), x.d, 2000, cluster_range=16)
    km.init_seeds(i32(datagen.seed_objects(x, 2000, 33)))
    a = i32(np.full(x.n, -1, np.int32))
    with pytest.raises(ivf.IvfError) as e:
        km.assign_static(a)
    assert e.value.status == -5 and "fixed" in str(e.value)
    assert torch.equal(a, i32(np.full(x.n, -1, np.int32)))   # nothing ran
    km.assign(a)                                               # the handle still works
    km.close()
