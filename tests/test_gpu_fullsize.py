"""The full-size workloads in the launch configuration the benchmark times:
2^28 keys.  The oracle cannot sort these in a test's time, so the checks are
the properties that fix the answer at any size: sorted order, the key
multiset (a 64-bit order-free hash) and sampled ranks for keys-only sorts;
for key-value sorts with the original index as payload, sortedness, the
permutation, key/value agreement and tie order, which together determine
the stable sort uniquely."""
import numpy as np
import pytest

from gpu_util import is_sorted_dev, multiset_hash, ranks_ok, stable_index_kv_ok, to_dev, to_host

pytestmark = pytest.mark.gpu

N = 1 << 28


@pytest.fixture(scope="module")
def rs():
    import paper_1708_09495_amd as rs
    rs.lib()
    return rs


def _keys_dev(kb, seed):
    import gen
    import torch
    t = torch.empty(N, dtype=torch.int32 if kb == 4 else torch.int64, device="cuda")
    (gen.uniform_u32_dev if kb == 4 else gen.uniform_u64_dev)(seed, t)
    return t


@pytest.mark.parametrize("kb,bits", [(4, 8), (4, 11), (4, 16), (8, 8)])
def test_keys_only(rs, kb, bits):
    import gen
    import torch
    print("case full keys kb=%d bits=%d n=%d" % (kb, bits, N), flush=True)
    a = _keys_dev(kb, gen.S0 + 2)
    sort = rs.rs_sort_u32 if kb == 4 else rs.rs_sort_u64
    out = sort(a, radix_bits=bits, algo=rs.RS_ALGO_LSD)
    st = rs.rs_get_stats()
    assert st.device_error == 0 and st.passes == -(-8 * kb // bits)
    assert is_sorted_dev(out)
    dt = np.uint32 if kb == 4 else np.uint64
    ha, ho = to_host(a, dt), to_host(out, dt)
    del a, out
    torch.cuda.empty_cache()
    assert multiset_hash(ha) == multiset_hash(ho)
    pos = np.random.default_rng(31 + bits).integers(0, N, 12)
    assert ranks_ok(ha, ho, list(pos) + [0, N - 1])


@pytest.mark.parametrize("kb,vb,bits", [(4, 4, 8), (4, 4, 16), (8, 8, 8)])
def test_kv_index_payload(rs, kb, vb, bits):
    import gen
    import torch
    print("case full kv kb=%d vb=%d bits=%d n=%d" % (kb, vb, bits, N), flush=True)
    keys = _keys_dev(kb, gen.S0 + 2)
    vals = torch.arange(N, dtype=torch.int32 if vb == 4 else torch.int64, device="cuda")
    ko, vo = rs.rs_sort_kv(keys, vals, radix_bits=bits, algo=rs.RS_ALGO_LSD)
    del vals
    assert rs.rs_get_stats().device_error == 0
    assert stable_index_kv_ok(keys, ko, vo)


@pytest.mark.parametrize("dist", ["zipf", "lognormal", "mixture"])
def test_learned_kv_index_payload(rs, dist):
    """The learned-bucket workload: 2^28 uint64 keys from each distribution,
    uint64 payload = original index."""
    import gen
    import torch
    print("case full learned %s n=%d" % (dist, N), flush=True)
    seed = gen.S0 + 5
    host = {"zipf": gen.zipf_u64, "lognormal": gen.lognormal_u64,
            "mixture": gen.gauss_mix_u64}[dist](seed, N)
    keys = to_dev(host)
    del host
    vals = torch.arange(N, dtype=torch.int64, device="cuda")
    ko, vo = rs.rs_sort_kv(keys, vals, algo=rs.RS_ALGO_LEARNED)
    del vals
    st = rs.rs_get_stats()
    print("  fallback=%d overflowed buckets=%d keys=%d" % (st.fallback, st.buckets_overflowed,
                                                          st.keys_overflowed), flush=True)
    assert st.device_error == 0
    assert stable_index_kv_ok(keys, ko, vo)
