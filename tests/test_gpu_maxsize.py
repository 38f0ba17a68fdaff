"""The largest sizes the LSD rounds plan for: 64-bit look-back words (2^30
keys and up) and 64-bit destinations (2^31 keys and up).  The checks run on
the device, in chunks, and hold at any size: sorted order; the same multiset
(a 65,536-bin histogram of the top 16 bits, the sum and the sum of squares
of the keys modulo 2^64); and, at sampled output positions q,
#{input < out[q]} <= q < #{input <= out[q]}, which fixes out[q] as the q-th
smallest key."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CHUNK = 1 << 27


@pytest.fixture(scope="module")
def rs():
    import paper_1708_09495_amd as rs
    rs.lib()
    return rs


def _u(t):
    """int64 values with the order of the unsigned keys in t (uint32 values,
    or uint64 bit patterns with the sign bit flipped)."""
    import torch
    if t.dtype == torch.int32:
        return t.to(torch.int64) & 0xFFFFFFFF
    return t ^ torch.iinfo(torch.int64).min


def _chunks(n):
    return [(s, min(n, s + CHUNK)) for s in range(0, n, CHUNK)]


def _sorted(out):
    n = out.numel()
    for s, e in _chunks(n):
        o = _u(out[max(0, s - 1):e])
        if not bool((o[1:] >= o[:-1]).all()):
            return False
    return True


def _fingerprint(t, kbits):
    import torch
    h = torch.zeros(65536, dtype=torch.int64, device=t.device)
    s1 = torch.zeros((), dtype=torch.int64, device=t.device)
    s2 = torch.zeros((), dtype=torch.int64, device=t.device)
    for s, e in _chunks(t.numel()):
        u = _u(t[s:e])
        h += torch.bincount((u >> (kbits - 16)) & 0xFFFF, minlength=65536)
        v = t[s:e].to(torch.int64)
        s1 += v.sum()          # int64 sums wrap: modulo 2^64
        s2 += (v * v).sum()
    return h, int(s1), int(s2)


def _rank_bounds(a, key):
    lt = le = 0
    for s, e in _chunks(a.numel()):
        u = _u(a[s:e])
        lt += int((u < key).sum())
        le += int((u <= key).sum())
    return lt, le


@pytest.mark.parametrize("kb,n", [(8, (1 << 30) + 777), (4, (1 << 31) + 12_345)])
def test_largest_plans(rs, kb, n):
    import gen
    import torch
    print("case max size kb=%d n=%d" % (kb, n), flush=True)
    a = torch.empty(n, dtype=torch.int32 if kb == 4 else torch.int64, device="cuda")
    (gen.uniform_u32_dev if kb == 4 else gen.uniform_u64_dev)(gen.S0 + 41, a)
    sort = rs.rs_sort_u32 if kb == 4 else rs.rs_sort_u64
    out = sort(a, algo=rs.RS_ALGO_LSD)
    st = rs.rs_get_stats()
    assert st.device_error == 0 and st.passes == kb
    assert _sorted(out)
    ha, s1a, s2a = _fingerprint(a, 8 * kb)
    ho, s1o, s2o = _fingerprint(out, 8 * kb)
    assert torch.equal(ha, ho) and s1a == s1o and s2a == s2o
    for q in [0, n - 1] + [int(x) for x in np.random.default_rng(41).integers(0, n, 8)]:
        lt, le = _rank_bounds(a, _u(out[q:q + 1])[0])
        assert lt <= q < le, q
    del a, out
    torch.cuda.empty_cache()


def test_largest_kv_plan(rs):
    """Key-value at 2^31 + 4,321 uint32 keys with the index as uint32 payload:
    keys sorted, payload a permutation of 0..n-1, out key == in key at the
    payload, payload increasing inside each run of equal keys -- together the
    stable sort."""
    import gen
    import torch
    n = (1 << 31) + 4_321
    print("case max size kv n=%d" % n, flush=True)
    k = torch.empty(n, dtype=torch.int32, device="cuda")
    gen.uniform_u32_dev(gen.S0 + 42, k)
    k &= 0x00FFFFFF                       # many equal keys, so tie order matters
    v = torch.empty(n, dtype=torch.int32, device="cuda")
    gen.iota_dev(v)
    ko, vo = rs.rs_sort_kv(k, v, algo=rs.RS_ALGO_LSD)
    st = rs.rs_get_stats()
    assert st.device_error == 0
    assert _sorted(ko)
    seen = torch.zeros(n, dtype=torch.bool, device="cuda")
    for s, e in _chunks(n):
        idx = vo[s:e].to(torch.int64) & 0xFFFFFFFF
        seen[idx] = True
        assert torch.equal(k[idx], ko[s:e])
        e2 = min(n, e + 1)
        kk, vv = _u(ko[s:e2]), vo[s:e2].to(torch.int64) & 0xFFFFFFFF
        tie = kk[1:] == kk[:-1]
        assert bool((vv[1:][tie] > vv[:-1][tie]).all())
    assert bool(seen.all())
    del k, v, ko, vo, seen
    torch.cuda.empty_cache()


def test_largest_segments(rs):
    """Segmented sort at the edge of the shared device-wide rounds: a segment
    of 2^30 - 1 keys (the longest they take: look-back words and
    destinations counted from the segment's start fit 30 and 31 bits), a
    short one, and one of 2^30 + 5 keys (sorted by one workgroup's own
    rounds, with 64-bit loop bounds).  Per segment: sorted, the same
    multiset, and sampled ranks."""
    import gen
    import torch
    lens = [(1 << 30) - 1, 7, (1 << 30) + 5]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    n = int(off[-1])
    print("case max segments n=%d lens=%s" % (n, lens), flush=True)
    a = torch.empty(n, dtype=torch.int32, device="cuda")
    gen.uniform_u32_dev(gen.S0 + 43, a)
    out = rs.rs_sort_segmented(a, torch.from_numpy(off).cuda())
    assert rs.rs_get_stats().device_error == 0
    rng = np.random.default_rng(43)
    for s in range(len(lens)):
        b, e = int(off[s]), int(off[s + 1])
        sa, so = a[b:e], out[b:e]
        assert _sorted(so), s
        ha, s1a, s2a = _fingerprint(sa, 32)
        ho, s1o, s2o = _fingerprint(so, 32)
        assert torch.equal(ha, ho) and s1a == s1o and s2a == s2o, s
        L = e - b
        for q in [0, L - 1] + [int(x) for x in rng.integers(0, L, 3)]:
            lt, le = _rank_bounds(sa, _u(so[q:q + 1])[0])
            assert lt <= q < le, (s, q)
    del a, out
    torch.cuda.empty_cache()
