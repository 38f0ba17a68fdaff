"""GPU parity of the wide-digit count-sort rounds (radix 2^12 .. 2^16, the
paper's PR2 point of Section 3) through the C ABI, bit for bit against the
oracle: several tiles, several sub-tiles per tile and ragged tails, runs of
equal digits longer than a sub-tile, key-value stability, odd round counts in
place."""
import numpy as np
import pytest

from gpu_util import first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu

# 4096-key sub-tiles, at most 512 tiles: 2^21 + 12_345 keys gives tiles of two
# sub-tiles, 5_000_001 of three with a short last tile
SIZES = [0, 1, 2, 4095, 4096, 4097, 65_537, 1 << 20, (1 << 21) + 12_345, 5_000_001]


@pytest.fixture(scope="module")
def rs():
    import paper_1708_09495_amd as rs
    rs.lib()
    return rs


def _check(out, ref, what):
    i = first_mismatch(out, ref)
    assert i is None, "%s: first mismatch at %d: got %d want %d" % (what, i, out[i], ref[i])


@pytest.mark.parametrize("bits", [16, 12, 13, 14])
def test_u32_uniform(rs, orc, bits):
    import gen
    for n in SIZES:
        print("case wide u32 n=%d bits=%d" % (n, bits), flush=True)
        a = gen.uniform_u32(gen.S0 + 21 + n, n)
        out = to_host(rs.rs_sort_u32(to_dev(a), radix_bits=bits, algo=rs.RS_ALGO_LSD), np.uint32)
        _check(out, orc.lsd(a, bits), "u32 n=%d b=%d" % (n, bits))
        st = rs.rs_get_stats()
        assert st.device_error == 0
        assert st.passes == -(-32 // bits) and st.radix_bits == bits


@pytest.mark.parametrize("case", ["equal", "sorted", "reverse", "high", "low", "few", "zipf"])
def test_u32_structured(rs, orc, case):
    import gen
    rng = np.random.default_rng(17)
    n = 3_000_001
    a = {
        "equal": np.full(n, 0xDEADBEEF, np.uint32),
        "sorted": np.sort(rng.integers(0, 2**32, n, dtype=np.uint64)).astype(np.uint32),
        "reverse": np.sort(rng.integers(0, 2**32, n, dtype=np.uint64))[::-1].astype(np.uint32),
        "high": (rng.integers(0, 65536, n).astype(np.uint32) << np.uint32(16)),
        "low": rng.integers(0, 300, n).astype(np.uint32),
        "few": rng.choice(np.array([3, 2**31, 77, 2**32 - 1], np.uint32), n),
        "zipf": (gen.zipf_u64(gen.S0 + 23, n) & 0xFFFFFFFF).astype(np.uint32),
    }[case]
    print("case wide structured %s n=%d" % (case, n), flush=True)
    out = to_host(rs.rs_sort_u32(to_dev(a), radix_bits=16, algo=rs.RS_ALGO_LSD), np.uint32)
    _check(out, orc.lsd(a, 16), case)
    assert rs.rs_get_stats().device_error == 0


@pytest.mark.parametrize("bits", [16, 13])
def test_u64_uniform(rs, orc, bits):
    import gen
    for n in [1, 4097, 100_000, (1 << 21) + 3]:
        print("case wide u64 n=%d bits=%d" % (n, bits), flush=True)
        a = gen.uniform_u64(gen.S0 + 22 + n, n)
        out = to_host(rs.rs_sort_u64(to_dev(a), radix_bits=bits, algo=rs.RS_ALGO_LSD), np.uint64)
        _check(out, orc.lsd(a, bits), "u64 n=%d b=%d" % (n, bits))
        assert rs.rs_get_stats().passes == -(-64 // bits)


@pytest.mark.parametrize("kdt,vdt", [(np.uint32, np.uint32), (np.uint32, np.uint64),
                                     (np.uint64, np.uint32), (np.uint64, np.uint64)])
def test_kv_stable(rs, orc, kdt, vdt):
    rng = np.random.default_rng(19)
    for n in [1, 1000, 8193, 2_500_000]:
        print("case wide kv %s/%s n=%d" % (np.dtype(kdt).name, np.dtype(vdt).name, n), flush=True)
        keys = rng.integers(0, 1000, n).astype(kdt)            # many ties
        keys[::7] = rng.integers(0, np.iinfo(kdt).max, keys[::7].size, dtype=kdt)
        vals = np.arange(n, dtype=vdt)
        ko, vo = rs.rs_sort_kv(to_dev(keys), to_dev(vals), radix_bits=16, algo=rs.RS_ALGO_LSD)
        ko, vo = to_host(ko, kdt), to_host(vo, vdt)
        rk, rv = orc.lsd(keys, 16, vals=vals)
        _check(ko, rk, "kv keys n=%d" % n)
        _check(vo, rv, "kv vals n=%d" % n)
        assert orc.check_stable_kv(keys, ko, vo) == 0


@pytest.mark.parametrize("bits", [16, 12])
def test_in_place(rs, orc, bits):
    import gen
    n = 1_200_003
    print("case wide in place bits=%d" % bits, flush=True)
    a = gen.uniform_u32(gen.S0 + 24, n)
    t = to_dev(a)
    rs.rs_sort_u32(t, t, radix_bits=bits, algo=rs.RS_ALGO_LSD)   # 2 rounds, or 3 and a copy back
    _check(to_host(t, np.uint32), orc.lsd(a, bits), "in place")
    keys = np.random.default_rng(5).integers(0, 5000, n).astype(np.uint32)
    vals = np.arange(n, dtype=np.uint32)
    kt, vt = to_dev(keys), to_dev(vals)
    rs.rs_sort_kv(kt, vt, kt, vt, radix_bits=bits, algo=rs.RS_ALGO_LSD)
    rk, rv = orc.lsd(keys, bits, vals=vals)
    _check(to_host(kt, np.uint32), rk, "kv in place keys")
    _check(to_host(vt, np.uint32), rv, "kv in place vals")

