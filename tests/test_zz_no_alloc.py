"""The sort that allocates nothing (rs_sort_u32_noalloc, scratch in a
static device array of the library) against the workspace entry point
rs_sort_u32 and the oracle: two calls in a row, the second smaller, so the
second runs on scratch the first left behind; radix 2^8 and 2^11, AUTO, in
place; sizes over the limit refused before any device work."""
import numpy as np
import pytest

from gpu_util import first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import paper_1708_09495_amd as rs
    rs.lib()
    return rs


def _check(out, ref, what):
    i = first_mismatch(out, ref)
    assert i is None, "%s: first mismatch at %d: got %d want %d" % (what, i, out[i], ref[i])


@pytest.mark.parametrize("bits,algo", [(8, 1), (11, 1), (8, 0)])
def test_noalloc_matches_workspace_entry(rs, orc, bits, algo):
    import gen
    for n in (3_000_017, 100_003):   # second call smaller: stale scratch from the first
        print("case noalloc n=%d bits=%d algo=%d" % (n, bits, algo), flush=True)
        a = gen.uniform_u32(gen.S0 + 60 + n, n)
        if algo == 0:
            a &= np.uint32(0x00FFFFFF)              # a round to skip
        d = to_dev(a)
        got = rs.rs_sort_u32_noalloc(d, radix_bits=bits, algo=algo)
        st = rs.rs_get_stats()
        assert st.device_error == 0
        want = rs.rs_sort_u32(d, radix_bits=bits, algo=algo)
        g, w = to_host(got, np.uint32), to_host(want, np.uint32)
        _check(g, w, "noalloc vs rs_sort_u32 n=%d" % n)
        _check(g, orc.lsd(a, bits), "noalloc vs oracle n=%d" % n)


def test_noalloc_in_place_and_limits(rs, orc):
    import gen
    import torch
    n = rs.RS_NOALLOC_MAX_KEYS
    a = gen.uniform_u32(gen.S0 + 61, n)
    t = to_dev(a)
    rs.rs_sort_u32_noalloc(t, t, radix_bits=11)     # 3 rounds in place: ends with a copy back
    assert rs.rs_get_stats().device_error == 0
    _check(to_host(t, np.uint32), orc.lsd(a, 11), "noalloc in place n=%d" % n)
    big = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    for kw in (dict(), dict(radix_bits=16)):
        x = big if not kw else big[:1000]
        with pytest.raises(rs.RsError) as e:
            rs.rs_sort_u32_noalloc(x, **kw)
        assert e.value.code == rs.RS_ERR_UNSUPPORTED
    with pytest.raises(rs.RsError) as e:
        rs.rs_sort_u32_noalloc(big[:1000], algo=rs.RS_ALGO_BTN)
    assert e.value.code == rs.RS_ERR_UNSUPPORTED
