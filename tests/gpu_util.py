"""Helpers of the GPU tests: moving uint64 oracle arrays to device word
tensors and back, and building contexts from oracle keys."""
import numpy as np
import torch

import paper_2510_15413_amd as fs


def to_dev(p, a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
    if p.q == 32:
        return torch.from_numpy(a.astype(np.uint32).view(np.int32)).cuda()
    return torch.from_numpy(a.view(np.int64)).cuda()


def from_dev(p, t):
    a = t.detach().cpu().contiguous().numpy()
    if p.q == 32:
        return a.view(np.uint32).astype(np.uint64)
    return a.view(np.uint64).copy()


def context(p, keys):
    return fs.Context(p, keys.bsk, keys.ksk)


def empty(p, *shape):
    return torch.empty(shape, dtype=torch.int32 if p.q == 32 else torch.int64, device="cuda")
