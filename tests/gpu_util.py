"""Helpers for the GPU tests: numpy <-> device tensors (16/32-bit samples
travel in int16/int32 storage), and the banner each GPU step prints first."""
import sys

import numpy as np

_STORE = {np.dtype(np.uint8): np.uint8, np.dtype(np.uint16): np.int16, np.dtype(np.uint32): np.int32}
_BACK = {1: np.uint8, 2: np.uint16, 4: np.uint32}


def to_dev(a):
    import torch
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view(_STORE[a.dtype])).cuda()


def to_host(t, width_bytes=None):
    a = t.cpu().numpy()
    wb = width_bytes or a.dtype.itemsize
    return a.view(_BACK[wb])


def banner(*parts):
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()
