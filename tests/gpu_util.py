"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np


def to_device_u64(arr):
    import torch
    a = np.ascontiguousarray(arr, np.uint64)
    t = torch.from_numpy(a.view(np.int64).copy()).cuda()
    torch.cuda.synchronize()      # the library's stream does not wait for torch's
    return t


def from_device_u64(t):
    return t.cpu().numpy().view(np.uint64)


def brev(x, bits):
    return int(format(x, f"0{bits}b")[::-1], 2)
