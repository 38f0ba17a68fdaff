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


def _lsr(z, k):
    """Logical right shift of an int64 tensor holding uint64 bit patterns."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def _s64(u):
    return u - (1 << 64) if u >= (1 << 63) else u


def mix64_dev(z):
    """The same 64-bit mix as _mix64, on an int64 torch tensor holding
    uint64 bit patterns (products wrap modulo 2^64)."""
    z = (z ^ _lsr(z, 30)) * _s64(0xBF58476D1CE4E5B9)
    z = (z ^ _lsr(z, 27)) * _s64(0x94D049BB133111EB)
    return z ^ _lsr(z, 31)


def multiset_hash_rows_dev(t2d):
    """Per-row multiset hash (the sum of mix64(x + golden) mod 2^64, as
    multiset_hash) of a 2-D int32/int64 torch tensor of unsigned keys: one
    int64 per row, equal for rows that hold the same multiset."""
    import torch
    z = t2d.to(torch.int64)
    if t2d.dtype == torch.int32:
        z = z & 0xFFFFFFFF
    return mix64_dev(z + _s64(0x9E3779B97F4A7C15)).sum(dim=1)


def segment_hashes_dev(t, seg_ids, num_segments, chunk=1 << 27):
    """Per-segment multiset hash of a 1-D int32 tensor of uint32 keys whose
    element i belongs to segment seg_ids[i]: int64 tensor of num_segments."""
    import torch
    h = torch.zeros(num_segments, dtype=torch.int64, device=t.device)
    for a in range(0, t.numel(), chunk):
        b = min(t.numel(), a + chunk)
        z = (t[a:b].to(torch.int64) & 0xFFFFFFFF) + _s64(0x9E3779B97F4A7C15)
        h.index_add_(0, seg_ids[a:b], mix64_dev(z))
        del z
    return h


def first_mismatch(a, b):
    d = np.nonzero(a != b)[0]
    return None if d.size == 0 else int(d[0])


def _ordered(t):
    """Device tensor holding uint32/uint64 bit patterns (as int32/int64) mapped
    to int64 values with the same order as the unsigned keys."""
    import torch
    if t.dtype == torch.int32:
        return t.to(torch.int64) & 0xFFFFFFFF
    return t ^ torch.iinfo(torch.int64).min


def is_sorted_dev(t):
    """True when the unsigned keys in device tensor t are non-decreasing."""
    o = _ordered(t)
    return bool((o[1:] >= o[:-1]).all()) if t.numel() > 1 else True


def stable_index_kv_ok(keys_in, ko, vo):
    """For a key-value sort whose input values are 0..n-1 (the original
    index): true when ko is non-decreasing, vo is a permutation of 0..n-1,
    ko[i] == keys_in[vo[i]] and equal keys keep increasing indexes.  These
    four facts determine the stable sort's output uniquely."""
    import torch
    n = keys_in.numel()
    if n == 0:
        return True
    idx = vo.to(torch.int64)
    if int(idx.min()) < 0 or int(idx.max()) >= n:
        return False
    seen = torch.zeros(n, dtype=torch.bool, device=vo.device)
    seen[idx] = True
    if not bool(seen.all()):
        return False
    del seen
    if not torch.equal(keys_in[idx], ko):
        return False
    o = _ordered(ko)
    if n > 1 and not bool(((o[1:] > o[:-1]) | ((o[1:] == o[:-1]) & (idx[1:] > idx[:-1]))).all()):
        return False
    return True


def ranks_ok(host_in, host_out, positions):
    """The sorted position of a key is fixed by the number of smaller and
    equal keys in the input: check below <= i < below + equal at each i."""
    for i in positions:
        k = host_out[i]
        below = int(np.count_nonzero(host_in < k))
        equal = int(np.count_nonzero(host_in == k))
        if not (below <= i < below + equal):
            return False
    return True
