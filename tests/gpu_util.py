"""Helpers shared by the GPU tests: host arrays -> device tensors, and calls
through the library's C ABI (via the package binding)."""
import numpy as np
import torch

import datagen
import oracle

DEV = "cuda:0"


def to_dev(x: datagen.CSR):
    return (torch.from_numpy(np.ascontiguousarray(x.indptr, np.int64)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(x.indices, np.int32)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(x.values, np.float32)).to(DEV))


def means_to_dev(m: oracle.Means):
    return (torch.from_numpy(np.ascontiguousarray(m.indptr, np.int64)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(m.indices, np.int32)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(m.values, np.float64)).to(DEV))


def means_to_host(ptr, idx, val, k, d):
    return oracle.Means(k, d, ptr.cpu().numpy(), idx.cpu().numpy(), val.cpu().numpy())


def i32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).to(DEV)


def digest(a):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a, np.int32).tobytes()).hexdigest()


def uncertain_objects(best, second, flags, n_margin):
    """Objects re-scored in FP64 (flag bit 1) and the n_margin objects with the
    smallest FP32 margin (best - second) / best among those with a score."""
    resc = np.nonzero(flags & 2)[0]
    margin = np.full(len(best), np.inf)
    pos = best > 0
    margin[pos] = (best[pos] - second[pos]) / best[pos]
    m = min(n_margin, int(pos.sum()))
    low = np.argpartition(margin, m - 1)[:m] if m > 0 else np.zeros(0, np.int64)
    return resc, np.sort(low)


def oracle_check(x, means, prev, got, objs):
    """The FP64 oracle's assignment step for the objects `objs` (sorted) under
    `means` from the previous assignment `prev`: returns its AssignResult and
    the objects on which `got` differs (must be none)."""
    ar = oracle.assign(x.subset(objs), means, prev[objs])
    return ar, objs[ar.assign != got[objs]]


def score_errors(x, means, objs, ar, best, best_id, second, bound):
    """Largest relative error of the FP32 tile scores against the FP64 oracle on
    `objs` (ar: the oracle's assignment of exactly these objects): top-1 is
    the tile's winner score against that cluster's FP64 score; top-2 the
    tile's best other score against the oracle's, where the two winners agree
    (both are then maxima over the same other clusters).  bound = (c, a, g) of
    the certificate: every error must be within (c + 2 g) rho64 + a.  Returns
    (max top-1 error, max top-2 error, pairs, pairs, bound held)."""
    c, a, g = bound
    b, bi, s2 = best[objs].astype(np.float64), best_id[objs], second[objs].astype(np.float64)
    ok = bi >= 0
    r64 = oracle.scores(x, means, objs[ok], bi[ok])
    pos = r64 > 0
    d1 = np.abs(b[ok][pos] - r64[pos])
    e1 = d1 / r64[pos]
    same = ok & (bi == ar.assign) & (ar.rho2 > 0)
    d2 = np.abs(s2[same] - ar.rho2[same])
    e2 = d2 / ar.rho2[same]
    held = bool(np.all(d1 <= (c + 2 * g) * r64[pos] + a) and
                np.all(d2 <= (c + 2 * g) * ar.rho2[same] + a))
    return (float(e1.max()) if len(e1) else 0.0, float(e2.max()) if len(e2) else 0.0,
            int(len(e1)), int(same.sum()), held)
