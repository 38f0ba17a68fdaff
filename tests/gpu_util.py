"""Helpers for the GPU tests: host<->device copies of unsigned arrays and
property checks that hold at any size.  No sorting arithmetic here."""
import numpy as np

_SIGNED = {np.dtype(np.uint32): np.int32, np.dtype(np.uint64): np.int64}


def to_dev(a):
    import torch
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view(_SIGNED[a.dtype])).cuda()


def to_host(t, dtype):
    return t.cpu().numpy().view(dtype)


def _mix64(z):
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def multiset_hash(a, chunk=1 << 24):
    """Sum of a 64-bit mix of every element, mod 2^64: equal for any two
    arrays holding the same multiset (independent of order)."""
    h = np.uint64(0)
    with np.errstate(over="ignore"):
        for s in range(0, a.size, chunk):
            z = a[s:s + chunk].astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
            h = h + np.add.reduce(_mix64(z), dtype=np.uint64)
    return int(h)


def first_mismatch(a, b):
    d = np.nonzero(a != b)[0]
    return None if d.size == 0 else int(d[0])
