"""Inverted-file spherical k-means on MI355X (gfx950).

The product is the C-ABI library ``libivf.so`` (include/ivf.h) built from the
HIP sources in ``csrc/``.  This package is its thin Python binding: PyTorch
supplies device memory and streams; every step of the Lloyd iteration runs in
the library's kernels.  There is no CPU fallback: without the built library or
a GPU, the calls fail.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import IVF_VAL_BF16, IVF_VAL_F16, IVF_VAL_F32, IvfError, check


def library():
    """Load libivf.so (ImportError if it has not been built)."""
    return _lib.get()

VALTYPES = {"f32": IVF_VAL_F32, "bf16": IVF_VAL_BF16, "f16": IVF_VAL_F16}

__all__ = ["IVFKMeans", "IVFBatch", "IvfError", "VALTYPES", "plan_shape", "cert_bound",
           "cert_bound_fixed", "read_ceiling"]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need_cuda(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s tensor" % (name, dtype))
    return t


def _options(valtype="f32", certify=True, cluster_range=0, waves_per_wg=0, objects_per_item=0,
             force_rescore=False, dense_threshold=0.0, stream=None, full_update=False):
    o = _lib.ivf_options()
    _lib.get().ivf_default_options(ctypes.byref(o))
    o.valtype = VALTYPES[valtype] if isinstance(valtype, str) else int(valtype)
    o.certify = 1 if certify else 0
    o.cluster_range = int(cluster_range)
    o.waves_per_wg = int(waves_per_wg)
    o.objects_per_item = int(objects_per_item)
    o.force_rescore = 1 if force_rescore else 0
    o.dense_threshold = float(dense_threshold)
    o.stream = ctypes.c_void_p(stream) if stream else None
    o.full_update = 1 if full_update else 0
    return o


def plan_shape(k, **opts):
    """Launch plan the library would pick for k clusters (host only)."""
    o = _options(**opts)
    plan = (ctypes.c_int32 * 7)()
    check(_lib.get().ivf_plan_shape(int(k), ctypes.byref(o), plan))
    keys = ("k_r", "ranges", "waves", "chunk", "rescore_k_r", "rescore_ranges", "lds_bytes")
    return dict(zip(keys, list(plan)))


def cert_bound(valtype, nt, vmax=1.0):
    """(c, a, g64) certification constants for an object of nt nonzeros, all
    object values <= vmax."""
    c = (ctypes.c_double * 3)()
    vt = VALTYPES[valtype] if isinstance(valtype, str) else int(valtype)
    check(_lib.get().ivf_cert_bound(vt, int(nt), float(vmax), c))
    return tuple(c)


def cert_bound_fixed(nt, scale, vmax=1.0):
    """(c, a, g64) constants of IVFD's fixed-point scores (products scaled by
    `scale` and rounded to integers) for an object of nt nonzeros, all object
    values <= vmax."""
    c = (ctypes.c_double * 3)()
    check(_lib.get().ivf_cert_bound_fixed(int(nt), float(scale), float(vmax), c))
    return tuple(c)


def read_ceiling(buf, mode, passes, unroll=4, wgs_per_cu=8, stream=None):
    """Read bandwidth (GB/s) of a plain streaming read of the CUDA tensor `buf`
    (mode 0: every workgroup reads all of it; mode 1: split and swept
    `passes` times; `unroll` loads per lane in flight, `wgs_per_cu`
    workgroups per compute unit): the measured roofs of the walk's traffic."""
    import torch
    if not isinstance(buf, torch.Tensor) or not buf.is_cuda or not buf.is_contiguous():
        raise TypeError("buf must be a contiguous CUDA tensor")
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    out = ctypes.c_double()
    check(_lib.get().ivf_read_ceiling(_ptr(buf), buf.numel() * buf.element_size(), int(mode),
                                      int(passes), int(unroll), int(wgs_per_cu),
                                      ctypes.c_void_p(stream) if stream else None,
                                      ctypes.byref(out)))
    return out.value


class IVFKMeans:
    """One clustering instance on the current HIP device.

    indptr (int64 [n+1]), indices (int32 [nnz]), values (float32 [nnz]) are CUDA
    tensors holding the object set in CSR form; they are borrowed and must
    outlive the instance.
    """

    def __init__(self, indptr, indices, values, d, k, *, valtype="f32", certify=True,
                 cluster_range=0, waves_per_wg=0, objects_per_item=0, force_rescore=False,
                 dense_threshold=0.0, stream=None, full_update=False):
        import torch
        _need_cuda(indptr, torch.int64, "indptr")
        _need_cuda(indices, torch.int32, "indices")
        _need_cuda(values, torch.float32, "values")
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self._keep = (indptr, indices, values)
        self.n = indptr.numel() - 1
        self.d = int(d)
        self.k = int(k)
        self.nnz = indices.numel()
        x = _lib.ivf_csr(self.n, self.d, self.nnz, _ptr(indptr), _ptr(indices), _ptr(values))
        o = _options(valtype, certify, cluster_range, waves_per_wg, objects_per_item,
                     force_rescore, dense_threshold, stream, full_update)
        h = ctypes.c_void_p()
        check(_lib.get().ivf_build(ctypes.byref(x), self.k, ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    # -- state -------------------------------------------------------------
    def set_means(self, indptr, indices, values):
        import torch
        _need_cuda(indptr, torch.int64, "indptr")
        _need_cuda(indices, torch.int32, "indices")
        _need_cuda(values, torch.float64, "values")
        m = _lib.ivf_means(self.k, self.d, indices.numel(), _ptr(indptr), _ptr(indices),
                           _ptr(values))
        check(_lib.get().ivf_set_means(self._h, ctypes.byref(m)), self._h)

    def init_seeds(self, seeds):
        import torch
        _need_cuda(seeds, torch.int32, "seeds")
        if seeds.numel() != self.k:
            raise ValueError("need k seeds")
        check(_lib.get().ivf_init_seeds(self._h, _ptr(seeds)), self._h)

    def get_means(self):
        import torch
        m = _lib.ivf_means()
        check(_lib.get().ivf_get_means(self._h, ctypes.byref(m)), self._h)
        nnz = m.nnz
        dev = self._keep[0].device
        ptr = torch.empty(self.k + 1, dtype=torch.int64, device=dev)
        idx = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        val = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)
        m2 = _lib.ivf_means(self.k, self.d, nnz, _ptr(ptr), _ptr(idx), _ptr(val))
        check(_lib.get().ivf_get_means(self._h, ctypes.byref(m2)), self._h)
        return ptr, idx[:nnz], val[:nnz]

    def get_scores(self):
        """(best FP32, best cluster, second FP32, rho FP64, flags) per object."""
        import torch
        dev = self._keep[0].device
        best = torch.empty(self.n, dtype=torch.float32, device=dev)
        best_id = torch.empty(self.n, dtype=torch.int32, device=dev)
        second = torch.empty(self.n, dtype=torch.float32, device=dev)
        rho = torch.empty(self.n, dtype=torch.float64, device=dev)
        flags = torch.empty(self.n, dtype=torch.uint8, device=dev)
        check(_lib.get().ivf_get_scores(self._h, _ptr(best), _ptr(best_id), _ptr(second),
                                        _ptr(rho), _ptr(flags)), self._h)
        return best, best_id, second, rho, flags

    @property
    def plan(self):
        plan = (ctypes.c_int32 * 7)()
        check(_lib.get().ivf_get_plan(self._h, plan), self._h)
        keys = ("k_r", "ranges", "waves", "chunk", "rescore_k_r", "rescore_ranges", "lds_bytes")
        return dict(zip(keys, list(plan)))

    # -- steps -------------------------------------------------------------
    def assign(self, assign, stats=True):
        import torch
        _need_cuda(assign, torch.int32, "assign")
        st = _lib.ivf_stats() if stats else None
        check(_lib.get().ivf_assign(self._h, _ptr(assign), ctypes.byref(st) if stats else None),
              self._h)
        return st.to_dict() if stats else None

    def assign_static(self, assign, stats=True):
        """``assign`` with its per-call scratch in the library's fixed per-device
        array (no device allocation); the same results bit for bit.  Calls on one
        GPU must not overlap."""
        import torch
        _need_cuda(assign, torch.int32, "assign")
        st = _lib.ivf_stats() if stats else None
        check(_lib.get().ivf_assign_static(self._h, _ptr(assign),
                                           ctypes.byref(st) if stats else None), self._h)
        return st.to_dict() if stats else None

    def assign_ivfd(self, assign, objects_per_range=0, stats=True):
        """The assignment step of IVFD (the objects inverted, each mean a
        query): the same partition as ``assign``; FP32 handles only."""
        import torch
        _need_cuda(assign, torch.int32, "assign")
        st = _lib.ivf_stats() if stats else None
        check(_lib.get().ivf_assign_ivfd(self._h, int(objects_per_range), _ptr(assign),
                                         ctypes.byref(st) if stats else None), self._h)
        return st.to_dict() if stats else None

    def update(self, assign, stats=True):
        import torch
        _need_cuda(assign, torch.int32, "assign")
        st = _lib.ivf_stats() if stats else None
        check(_lib.get().ivf_update(self._h, _ptr(assign), ctypes.byref(st) if stats else None),
              self._h)
        return st.to_dict() if stats else None

    def iterate(self, iters, assign, stats=True):
        import torch
        _need_cuda(assign, torch.int32, "assign")
        arr = (_lib.ivf_stats * max(int(iters), 1))() if stats else None
        check(_lib.get().ivf_iterate(self._h, int(iters), _ptr(assign), arr), self._h)
        return [arr[i].to_dict() for i in range(int(iters))] if stats else None

    def converge(self, max_iters, assign, stats=True):
        """Iterate until an assignment step changes nothing (or max_iters steps);
        returns the per-step stats (the last step's update is skipped)."""
        import torch
        _need_cuda(assign, torch.int32, "assign")
        arr = (_lib.ivf_stats * max(int(max_iters), 1))()
        done = ctypes.c_int32()
        check(_lib.get().ivf_converge(self._h, int(max_iters), _ptr(assign), arr,
                                      ctypes.byref(done)), self._h)
        return [arr[i].to_dict() for i in range(done.value)]

    def close(self):
        if getattr(self, "_h", None):
            _lib.get().ivf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class IVFBatch:
    """Many clustering instances advanced together (one persistent walk launch
    per iteration for all of them, the iteration replayed as HIP graphs).

    sets: list of (indptr, indices, values, d) CUDA tensor tuples, one per
    instance (instances may share one tuple: restarts of one object set);
    ks: clusters of each instance.  Options as IVFKMeans, applied to all.
    """

    def __init__(self, sets, ks, *, valtype="f32", certify=True, cluster_range=0,
                 waves_per_wg=0, dense_threshold=0.0):
        import torch
        if len(sets) != len(ks) or not sets:
            raise ValueError("need one k per object set")
        self.count = len(sets)
        xs = (_lib.ivf_csr * self.count)()
        self._keep = []
        self.n, self.k, self.d = [], [int(k) for k in ks], []
        for i, (indptr, indices, values, d) in enumerate(sets):
            _need_cuda(indptr, torch.int64, "indptr")
            _need_cuda(indices, torch.int32, "indices")
            _need_cuda(values, torch.float32, "values")
            self._keep.append((indptr, indices, values))
            self.n.append(indptr.numel() - 1)
            self.d.append(int(d))
            xs[i] = _lib.ivf_csr(indptr.numel() - 1, int(d), indices.numel(), _ptr(indptr),
                                 _ptr(indices), _ptr(values))
        karr = (ctypes.c_int32 * self.count)(*self.k)
        # the batch creates and owns its stream (graphs cannot record the null stream)
        o = _options(valtype, certify, cluster_range, waves_per_wg, 0, False, dense_threshold,
                     None)
        b = ctypes.c_void_p()
        _lib.check_batch(_lib.get().ivf_batch_build(self.count, xs, karr, ctypes.byref(o),
                                                    ctypes.byref(b)))
        self._b = b
        self._device = sets[0][0].device

    def _ptrs(self, tensors, dtype, sizes, name):
        import torch
        if len(tensors) != self.count:
            raise ValueError("need one %s per instance" % name)
        arr = (ctypes.c_void_p * self.count)()
        for i, t in enumerate(tensors):
            _need_cuda(t, dtype, name)
            if t.numel() != sizes[i]:
                raise ValueError("%s[%d] has %d entries, expected %d" % (name, i, t.numel(),
                                                                         sizes[i]))
            arr[i] = t.data_ptr()
        return arr

    def init_seeds(self, seeds):
        import torch
        torch.cuda.synchronize()
        arr = self._ptrs(seeds, torch.int32, self.k, "seeds")
        _lib.check_batch(_lib.get().ivf_batch_init_seeds(self._b, arr), self._b)

    def set_means(self, inst, indptr, indices, values):
        import torch
        _need_cuda(indptr, torch.int64, "indptr")
        _need_cuda(indices, torch.int32, "indices")
        _need_cuda(values, torch.float64, "values")
        torch.cuda.synchronize()
        m = _lib.ivf_means(self.k[inst], self.d[inst], indices.numel(), _ptr(indptr),
                           _ptr(indices), _ptr(values))
        _lib.check_batch(_lib.get().ivf_batch_set_means(self._b, int(inst), ctypes.byref(m)),
                         self._b)

    def iterate(self, iters, assigns, stats=True):
        """Run iters iterations; assigns: one int32 [n_i] CUDA tensor per instance.
        Returns per-iteration lists of per-instance stats dicts (or None)."""
        import torch
        arr = self._ptrs(assigns, torch.int32, self.n, "assign")
        torch.cuda.synchronize()   # the batch's stream does not wait for torch's
        iters = int(iters)
        st = (_lib.ivf_stats * max(iters * self.count, 1))() if stats else None
        _lib.check_batch(_lib.get().ivf_batch_iterate(self._b, iters, arr, st), self._b)
        if not stats:
            return None
        return [[st[r * self.count + i].to_dict() for i in range(self.count)]
                for r in range(iters)]

    def get_means(self, inst):
        import torch
        m = _lib.ivf_means()
        _lib.check_batch(_lib.get().ivf_batch_get_means(self._b, int(inst), ctypes.byref(m)),
                         self._b)
        nnz = m.nnz
        ptr = torch.empty(self.k[inst] + 1, dtype=torch.int64, device=self._device)
        idx = torch.empty(max(nnz, 1), dtype=torch.int32, device=self._device)
        val = torch.empty(max(nnz, 1), dtype=torch.float64, device=self._device)
        m2 = _lib.ivf_means(self.k[inst], self.d[inst], nnz, _ptr(ptr), _ptr(idx), _ptr(val))
        _lib.check_batch(_lib.get().ivf_batch_get_means(self._b, int(inst), ctypes.byref(m2)),
                         self._b)
        return ptr, idx[:nnz], val[:nnz]

    def set_slack(self, frac, abs_entries):
        """Fixed capacities = need * (1 + frac) + abs_entries (defaults 0.5, 1024)."""
        _lib.check_batch(_lib.get().ivf_batch_set_slack(self._b, float(frac),
                                                        int(abs_entries)), self._b)

    @property
    def plan(self):
        plan = (ctypes.c_int32 * 8)()
        _lib.check_batch(_lib.get().ivf_batch_get_plan(self._b, plan), self._b)
        keys = ("kr_max", "waves", "tile_stride", "grid", "graphs", "tuned", "captures",
                "recoveries")
        return dict(zip(keys, list(plan)))

    @property
    def tuning(self):
        """[(clusters per tile, waves, walk ms)] the autotuner measured."""
        cap = 16
        shapes = (ctypes.c_int32 * (2 * cap))()
        ms = (ctypes.c_float * cap)()
        n = ctypes.c_int32()
        _lib.check_batch(_lib.get().ivf_batch_get_tuning(self._b, cap, shapes, ms,
                                                         ctypes.byref(n)), self._b)
        return [(shapes[2 * i], shapes[2 * i + 1], ms[i]) for i in range(min(n.value, cap))]

    @property
    def threshold_tuning(self):
        """[(dense-slab threshold, walk ms)] the autotuner measured on its shape."""
        cap = 16
        thetas = (ctypes.c_float * cap)()
        ms = (ctypes.c_float * cap)()
        n = ctypes.c_int32()
        _lib.check_batch(_lib.get().ivf_batch_get_threshold_tuning(self._b, cap, thetas, ms,
                                                                   ctypes.byref(n)), self._b)
        return [(thetas[i], ms[i]) for i in range(min(n.value, cap))]

    def close(self):
        if getattr(self, "_b", None):
            _lib.get().ivf_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
