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
