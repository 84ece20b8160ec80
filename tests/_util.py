"""Helpers for the GPU tests: host <-> device conversions of pattern arrays."""
import numpy as np


def dev_u32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.uint64).astype(np.uint32)).view(np.int32)).cuda()


def dev_u64(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.uint64)).view(np.int64)).cuda()


def host_u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32).astype(np.uint64)


def host_u64(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def host_rank(t) -> np.ndarray:
    """Device ranks (int32 storage) as int64 with MBR_NOT_FOUND mapped to -1."""
    r = t.cpu().numpy().view(np.uint32).astype(np.int64)
    r[r == 0xFFFFFFFF] = -1
    return r


def say(*a):
    print(*a, flush=True)
