"""Seeded input generator: determinism and the stated recipe's structure."""
import hashlib
import os
import subprocess
import sys

import numpy as np

import datagen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _digest(x):
    h = hashlib.sha256()
    for a in (x.indptr, x.indices, x.values):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_deterministic_and_thread_count_independent():
    x = datagen.generate(5000, 3000, 30.0, 3, 200, 1.1, 7)
    y = datagen.generate(5000, 3000, 30.0, 3, 200, 1.1, 7)
    assert _digest(x) == _digest(y)
    code = ("import datagen,hashlib,numpy as np;x=datagen.generate(5000,3000,30.0,3,200,1.1,7);"
            "h=hashlib.sha256();[h.update(np.ascontiguousarray(a).tobytes()) for a in "
            "(x.indptr,x.indices,x.values)];print(h.hexdigest())")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.check_output([sys.executable, "-c", code], cwd=ROOT, env=env, text=True)
    assert out.strip() == _digest(x)
    z = datagen.generate(5000, 3000, 30.0, 3, 200, 1.1, 8)
    assert _digest(z) != _digest(x)


def test_structure():
    n, d, lam, lo, hi = 20000, 10000, 50.0, 5, 200
    x = datagen.generate(n, d, lam, lo, hi, 1.1, 1)
    lens = np.diff(x.indptr)
    assert lens.max() <= hi
    assert abs(lens.mean() - lam) < 0.02 * lam           # Poisson(lambda) mean
    assert np.all(x.indices >= 0) and np.all(x.indices < d)
    assert np.all(np.isfinite(x.values)) and np.all(x.values > 0)
    for i in range(0, n, 97):
        t, _ = x.row(i)
        assert np.all(np.diff(t) > 0)
    nrm = np.sqrt(np.add.reduceat(x.values.astype(np.float64) ** 2, x.indptr[:-1]))
    assert np.all(np.abs(nrm - 1.0) < 1e-6)               # FP32-rounded unit rows
    # Zipf: the document frequency of the r-th most common term decays roughly
    # like a power law; the head terms appear in most documents
    df = np.bincount(x.indices, minlength=d)
    top = np.sort(df)[::-1]
    assert top[0] > 0.5 * n
    assert top[10] > top[100] > top[1000] > 0


def test_seed_objects_distinct_nonempty():
    x = datagen.generate(3000, 2000, 10.0, 1, 40, 1.1, 9)
    s = datagen.seed_objects(x, 200, 9)
    assert len(set(s.tolist())) == 200
    rows = {(x.row(i)[0].tobytes(), x.row(i)[1].tobytes()) for i in s}
    assert len(rows) == 200
    assert np.all(np.diff(x.indptr)[s] > 0)
    assert np.array_equal(s, datagen.seed_objects(x, 200, 9))


def test_batched_instance_parameters():
    inst = datagen.batched_instances()
    assert len(inst) == 96
    for w, r in inst:
        assert 5000 <= w.n <= 400000 and 20000 <= w.d <= 150000
        assert 1 <= w.k <= max(1, w.n // 4) and w.k <= 8192
        assert 30.0 <= w.lam <= 250.0 and 1.0 <= w.s <= 1.2
    assert sum(1 for _, r in inst if r > 0) == 6 * 7
