"""ctypes binding of libivf.so: the C ABI of include/ivf.h, same names.

Argument marshalling only; every step of the method runs in the library's
HIP kernels.  Importing this module fails loudly when the library is absent.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libivf.so")

c_int32, c_int64, c_double, c_float, c_void_p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                 ctypes.c_float, ctypes.c_void_p)

IVF_OK = 0
IVF_VAL_F32, IVF_VAL_BF16, IVF_VAL_F16 = 0, 1, 2
STATUS = {0: "IVF_OK", -1: "IVF_ERR_ARG", -2: "IVF_ERR_UNSORTED", -3: "IVF_ERR_NONFINITE",
          -4: "IVF_ERR_NEGATIVE", -5: "IVF_ERR_CAPACITY", -6: "IVF_ERR_OOM", -7: "IVF_ERR_HIP",
          -8: "IVF_ERR_STATE"}


class ivf_csr(ctypes.Structure):
    _fields_ = [("n", c_int64), ("d", c_int64), ("nnz", c_int64), ("indptr", c_void_p),
                ("indices", c_void_p), ("values", c_void_p)]


class ivf_means(ctypes.Structure):
    _fields_ = [("k", c_int32), ("d", c_int64), ("nnz", c_int64), ("indptr", c_void_p),
                ("indices", c_void_p), ("values", c_void_p)]


class ivf_options(ctypes.Structure):
    _fields_ = [("valtype", c_int32), ("certify", c_int32), ("cluster_range", c_int32),
                ("waves_per_wg", c_int32), ("objects_per_item", c_int32),
                ("force_rescore", c_int32), ("dense_threshold", c_float),
                ("stream", c_void_p), ("full_update", c_int32)]


class ivf_stats(ctypes.Structure):
    _fields_ = [("objective", c_double), ("objective_bound", c_double), ("changed", c_int64),
                ("certified", c_int64), ("rescored", c_int64), ("zero_overlap", c_int64),
                ("mult_adds", c_int64), ("max_rel_err_rescored", c_double),
                ("assign_ms", c_float), ("walk_ms", c_float),
                ("objective_exact", c_double), ("empty_clusters", c_int64),
                ("nnz_means", c_int64), ("inexact_terms", c_int64), ("update_ms", c_float),
                ("update_delta_entries", c_int64)]

    def to_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# name -> (restype, argtypes); mirrors include/ivf.h
SIGNATURES = {
    "ivf_default_options": (None, [ctypes.POINTER(ivf_options)]),
    "ivf_build": (c_int32, [ctypes.POINTER(ivf_csr), c_int32, ctypes.POINTER(ivf_options),
                            ctypes.POINTER(c_void_p)]),
    "ivf_set_means": (c_int32, [c_void_p, ctypes.POINTER(ivf_means)]),
    "ivf_init_seeds": (c_int32, [c_void_p, c_void_p]),
    "ivf_assign": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(ivf_stats)]),
    "ivf_assign_static": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(ivf_stats)]),
    "ivf_update": (c_int32, [c_void_p, c_void_p, ctypes.POINTER(ivf_stats)]),
    "ivf_iterate": (c_int32, [c_void_p, c_int32, c_void_p, ctypes.POINTER(ivf_stats)]),
    "ivf_converge": (c_int32, [c_void_p, c_int32, c_void_p, ctypes.POINTER(ivf_stats),
                               ctypes.POINTER(c_int32)]),
    "ivf_assign_ivfd": (c_int32, [c_void_p, c_int32, c_void_p, ctypes.POINTER(ivf_stats)]),
    "ivf_get_means": (c_int32, [c_void_p, ctypes.POINTER(ivf_means)]),
    "ivf_get_scores": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ivf_get_plan": (c_int32, [c_void_p, ctypes.POINTER(c_int32)]),
    "ivf_plan_shape": (c_int32, [c_int32, ctypes.POINTER(ivf_options), ctypes.POINTER(c_int32)]),
    "ivf_cert_bound": (c_int32, [c_int32, c_int64, c_double, ctypes.POINTER(c_double)]),
    "ivf_cert_bound_fixed": (c_int32, [c_int64, c_double, c_double,
                                       ctypes.POINTER(c_double)]),
    "ivf_read_ceiling": (c_int32, [c_void_p, c_int64, c_int32, c_int32, c_int32, c_int32,
                                   c_void_p, ctypes.POINTER(c_double)]),
    "ivf_destroy": (None, [c_void_p]),
    "ivf_last_error": (ctypes.c_char_p, [c_void_p]),
    "ivf_status_str": (ctypes.c_char_p, [c_int32]),
    # batches
    "ivf_batch_build": (c_int32, [c_int32, ctypes.POINTER(ivf_csr), ctypes.POINTER(c_int32),
                                  ctypes.POINTER(ivf_options), ctypes.POINTER(c_void_p)]),
    "ivf_batch_init_seeds": (c_int32, [c_void_p, ctypes.POINTER(c_void_p)]),
    "ivf_batch_set_means": (c_int32, [c_void_p, c_int32, ctypes.POINTER(ivf_means)]),
    "ivf_batch_iterate": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_void_p),
                                    ctypes.POINTER(ivf_stats)]),
    "ivf_batch_get_means": (c_int32, [c_void_p, c_int32, ctypes.POINTER(ivf_means)]),
    "ivf_batch_set_slack": (c_int32, [c_void_p, c_double, c_int64]),
    "ivf_batch_get_plan": (c_int32, [c_void_p, ctypes.POINTER(c_int32)]),
    "ivf_batch_get_tuning": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_int32),
                                       ctypes.POINTER(c_float), ctypes.POINTER(c_int32)]),
    "ivf_batch_get_threshold_tuning": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_float),
                                                 ctypes.POINTER(c_float),
                                                 ctypes.POINTER(c_int32)]),
    "ivf_batch_destroy": (None, [c_void_p]),
    "ivf_batch_last_error": (ctypes.c_char_p, [c_void_p]),
}


def load(path: str = LIB_PATH):
    # PyTorch supplies the device memory and streams the library works on, and
    # its HIP runtime must be the process's only one: loaded first, it also
    # serves the library; loading the library first would start the system's
    # runtime beside it, whose calls then find no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise ImportError("libivf.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2002_09094_amd.build): " + path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = None


def get():
    """The loaded library (loaded on first use; raises ImportError if not built)."""
    global _lib
    if _lib is None:
        _lib = load()
    return _lib


class IvfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


def check(status, handle=None):
    if status != IVF_OK:
        msg = get().ivf_last_error(handle)
        raise IvfError(status, msg.decode() if msg else "")
    return status


def check_batch(status, batch=None):
    if status != IVF_OK:
        msg = get().ivf_batch_last_error(batch)
        raise IvfError(status, msg.decode() if msg else "")
    return status
