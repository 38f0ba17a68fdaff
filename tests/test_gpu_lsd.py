"""GPU parity of the LSD radix sort (count-sort rounds of Section 3) through
the C ABI: every output is compared bit for bit with the oracle on the same
seeded input, including the order of equal keys in key-value sorts."""
import numpy as np
import pytest

from gpu_util import first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 2, 63, 64, 65, 4095, 4096, 4097, 8191, 8192, 8193, 100_000, 1 << 20,
         (1 << 20) + 12_345]


@pytest.fixture(scope="module")
def rs():
    import paper_1708_09495_amd as rs
    rs.lib()
    return rs


def _u32(seed, n):
    import gen
    return gen.uniform_u32(seed, n)


def _check(out, ref, what):
    i = first_mismatch(out, ref)
    assert i is None, "%s: first mismatch at %d: got %d want %d" % (what, i, out[i], ref[i])


@pytest.mark.parametrize("bits", [8, 11, 4, 1])
def test_u32_uniform(rs, orc, bits):
    import gen
    sizes = SIZES if bits >= 4 else [0, 1, 65, 8193, 100_000]
    for n in sizes:
        print("case u32 n=%d bits=%d" % (n, bits), flush=True)
        a = _u32(gen.S0 + 1 + n, n)
        out = to_host(rs.rs_sort_u32(to_dev(a), radix_bits=bits, algo=rs.RS_ALGO_LSD), np.uint32)
        _check(out, orc.lsd(a, bits), "u32 n=%d b=%d" % (n, bits))
        assert rs.rs_get_stats().device_error == 0
        assert rs.rs_get_stats().passes == -(-32 // bits)


@pytest.mark.parametrize("case", ["equal", "sorted", "reverse", "high", "low", "max", "few"])
@pytest.mark.parametrize("bits", [8, 11])
def test_u32_structured(rs, orc, case, bits):
    rng = np.random.default_rng(7)
    n = 300_001
    a = {
        "equal": np.full(n, 0xDEADBEEF, np.uint32),
        "sorted": np.sort(rng.integers(0, 2**32, n, dtype=np.uint64)).astype(np.uint32),
        "reverse": np.sort(rng.integers(0, 2**32, n, dtype=np.uint64))[::-1].astype(np.uint32),
        "high": (rng.integers(0, 256, n).astype(np.uint32) << np.uint32(24)),
        "low": rng.integers(0, 256, n).astype(np.uint32),
        "max": np.where(rng.random(n) < 0.5, 2**32 - 1, rng.integers(0, 2**32, n)).astype(np.uint32),
        "few": rng.choice(np.array([3, 2**31, 77, 2**32 - 1], np.uint32), n),
    }[case]
    out = to_host(rs.rs_sort_u32(to_dev(a), radix_bits=bits, algo=rs.RS_ALGO_LSD), np.uint32)
    _check(out, orc.lsd(a, bits), case)


@pytest.mark.parametrize("bits", [8, 11, 4])
def test_skewed_histograms(rs, orc, bits):
    """Digits shared by many lanes of a wave (radix 2^8: several lanes on
    one LDS counter column; other radices: one add per wave for the lanes
    on lane 0's digit): Zipf keys (the high bytes mostly zero, the low ones
    crowded), keys 90% equal to one value and keys all equal; every round
    run (LSD) and with the identity rounds skipped (AUTO)."""
    import gen
    rng = np.random.default_rng(11)
    n = (1 << 20) + 4099
    z = gen.zipf_u64(gen.S0 + 44, n)
    m = np.where(rng.random(n) < 0.9, 0x12345678, rng.integers(0, 2**32, n)).astype(np.uint32)
    zref, mref = orc.lsd(z, bits), orc.lsd(m, bits)
    e = np.full(n, 0x9ABCDEF0, dtype=np.uint32)
    out = to_host(rs.rs_sort_u32(to_dev(e), radix_bits=bits, algo=rs.RS_ALGO_LSD), np.uint32)
    assert rs.rs_get_stats().device_error == 0
    _check(out, e, "all equal b=%d" % bits)
    for algo in (rs.RS_ALGO_LSD, rs.RS_ALGO_AUTO):
        print("case skewed bits=%d algo=%d" % (bits, algo), flush=True)
        out = to_host(rs.rs_sort_u64(to_dev(z), radix_bits=bits, algo=algo), np.uint64)
        assert rs.rs_get_stats().device_error == 0
        _check(out, zref, "zipf b=%d algo=%d" % (bits, algo))
        out = to_host(rs.rs_sort_u32(to_dev(m), radix_bits=bits, algo=algo), np.uint32)
        assert rs.rs_get_stats().device_error == 0
        _check(out, mref, "90%% one value b=%d algo=%d" % (bits, algo))


@pytest.mark.parametrize("bits", [8, 11])
def test_u64_uniform(rs, orc, bits):
    import gen
    for n in [1, 65, 4097, 100_000, (1 << 20) + 3]:
        a = gen.uniform_u64(gen.S0 + 2 + n, n)
        out = to_host(rs.rs_sort_u64(to_dev(a), radix_bits=bits, algo=rs.RS_ALGO_LSD), np.uint64)
        _check(out, orc.lsd(a, bits), "u64 n=%d" % n)


@pytest.mark.parametrize("kdt,vdt", [(np.uint32, np.uint32), (np.uint32, np.uint64),
                                     (np.uint64, np.uint32), (np.uint64, np.uint64)])
@pytest.mark.parametrize("bits", [8, 11])
def test_kv_stable(rs, orc, kdt, vdt, bits):
    rng = np.random.default_rng(11)
    for n in [1, 1000, 8193, 250_000]:
        keys = rng.integers(0, 1000, n).astype(kdt)            # many ties
        keys[::7] = rng.integers(0, np.iinfo(kdt).max, keys[::7].size, dtype=kdt)
        vals = np.arange(n, dtype=vdt)
        ko, vo = rs.rs_sort_kv(to_dev(keys), to_dev(vals), radix_bits=bits, algo=rs.RS_ALGO_LSD)
        ko, vo = to_host(ko, kdt), to_host(vo, vdt)
        rk, rv = orc.lsd(keys, bits, vals=vals)
        _check(ko, rk, "kv keys n=%d" % n)
        _check(vo, rv, "kv vals n=%d" % n)
        assert orc.check_stable_kv(keys, ko, vo) == 0


@pytest.mark.parametrize("bits", [8, 11])
def test_in_place(rs, orc, bits):
    import gen
    n = 200_003
    a = _u32(gen.S0 + 9, n)
    t = to_dev(a)
    rs.rs_sort_u32(t, t, radix_bits=bits, algo=rs.RS_ALGO_LSD)
    _check(to_host(t, np.uint32), orc.lsd(a, bits), "in place")
    keys = np.random.default_rng(3).integers(0, 50, n).astype(np.uint32)
    vals = np.arange(n, dtype=np.uint32)
    kt, vt = to_dev(keys), to_dev(vals)
    rs.rs_sort_kv(kt, vt, kt, vt, radix_bits=bits, algo=rs.RS_ALGO_LSD)
    rk, rv = orc.lsd(keys, bits, vals=vals)
    _check(to_host(kt, np.uint32), rk, "kv in place keys")
    _check(to_host(vt, np.uint32), rv, "kv in place vals")


def test_repeat_runs_identical(rs):
    import gen
    import torch
    a = to_dev(_u32(gen.S0 + 10, 1 << 20))
    ref = rs.rs_sort_u32(a, radix_bits=8, algo=rs.RS_ALGO_LSD)
    ws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_SORT, a.numel(), 4, 0, 8), dtype=torch.uint8,
                     device="cuda")
    out = torch.empty_like(a)
    for _ in range(100):
        rs.rs_sort_u32(a, out, radix_bits=8, algo=rs.RS_ALGO_LSD, ws=ws)
        assert torch.equal(out, ref)
    assert rs.rs_get_stats().device_error == 0
    # key-value with many equal keys: the order of equal keys (the values)
    # must come out the same every time too
    k = to_dev((_u32(gen.S0 + 11, 1 << 20) & np.uint32(0xFF)).astype(np.uint32))
    v = to_dev(np.arange(1 << 20, dtype=np.uint32))
    rk, rv = rs.rs_sort_kv(k, v, radix_bits=8, algo=rs.RS_ALGO_LSD)
    for _ in range(100):
        ok, ov = rs.rs_sort_kv(k, v, radix_bits=8, algo=rs.RS_ALGO_LSD)
        assert torch.equal(ok, rk) and torch.equal(ov, rv)
    assert rs.rs_get_stats().device_error == 0


def test_argument_errors(rs):
    import ctypes
    import torch
    L = rs.lib()
    a = torch.zeros(100, dtype=torch.int32, device="cuda")
    ws = torch.empty(rs.rs_workspace_bytes(rs.RS_OP_SORT, 100, 4, 0, 8), dtype=torch.uint8,
                     device="cuda")
    p = ctypes.c_void_p
    s = p(torch.cuda.current_stream().cuda_stream)
    assert L.rs_sort_u32(None, p(a.data_ptr()), 100, 8, 1, p(ws.data_ptr()), ws.numel(), s) == rs.RS_ERR_INVALID
    assert L.rs_sort_u32(p(a.data_ptr()), p(a.data_ptr() + 4), 100, 8, 1, p(ws.data_ptr()), ws.numel(), s) == rs.RS_ERR_INVALID
    assert L.rs_sort_u32(p(a.data_ptr()), p(a.data_ptr()), 100, 17, 1, p(ws.data_ptr()), ws.numel(), s) == rs.RS_ERR_INVALID
    assert L.rs_sort_u32(p(a.data_ptr()), p(a.data_ptr()), 100, 8, 1, p(ws.data_ptr()), 16, s) == rs.RS_ERR_WORKSPACE
    assert L.rs_sort_u32(p(a.data_ptr()), p(a.data_ptr()), 100, 8, 1, None, 0, s) == rs.RS_ERR_WORKSPACE
    assert L.rs_sort_kv(p(a.data_ptr()), None, p(a.data_ptr()), None, 100, 4, 3, 8, 1, p(ws.data_ptr()), ws.numel(), s) == rs.RS_ERR_INVALID
    assert L.rs_sort_u32(None, None, 0, 8, 1, None, 0, s) == rs.RS_OK


@pytest.mark.parametrize("log2n,extra", [(23, 1237), (28, 0)])
def test_headline_tiles_bit_exact(rs, orc, log2n, extra):
    """uint32 keys at radix 2^8 from 2^23 keys up take the large tiles (28
    keys per thread), the launch configuration the benchmark times; here
    every key is compared with the oracle, at 2^23 + 1,237 keys (a ragged
    last tile) and at the benchmark's own 2^28 keys and seed."""
    import gen
    n = (1 << log2n) + extra
    seed = gen.S0 + 2 if extra == 0 else gen.S0 + 21
    print("case headline tiles n=%d" % n, flush=True)
    import torch
    a = gen.uniform_u32(seed, n)
    d = torch.empty(n, dtype=torch.int32, device="cuda")
    gen.uniform_u32_dev(seed, d)          # the benchmark's own input path
    _check(to_host(d, np.uint32), a, "device generator against the host one")
    out = rs.rs_sort_u32(d, radix_bits=8, algo=rs.RS_ALGO_LSD)
    st = rs.rs_get_stats()
    assert st.device_error == 0 and st.passes == 4 and st.tile_keys == 512 * 28
    out = to_host(out, np.uint32)
    _check(out, orc.lsd(a, 8), "u32 n=%d b=8" % n)


@pytest.mark.parametrize("kdt", [np.uint32, np.uint64])
def test_kv_in_place_odd_rounds(rs, orc, kdt):
    """Key-value sorts in place whose executed round count is odd, so the
    rounds end in the workspace and copy back: radix 2^11 for uint32 keys (3
    rounds) and 2^10 for uint64 keys (7 rounds) with every round run, and AUTO at radix 2^8 on keys whose
    top byte is zero (uint32: 3 of 4 rounds run; uint64 keys below 2^40:
    5 of 8), each compared with the oracle's stable sort."""
    rng = np.random.default_rng(21)
    n = 300_007
    below = 2**24 if kdt == np.uint32 else 2**40
    odd_bits = 11 if kdt == np.uint32 else 10       # 3 rounds / 7 rounds
    cases = [(odd_bits, rs.RS_ALGO_LSD, rng.integers(0, 2**32, n, dtype=np.uint64).astype(kdt)),
             (8, rs.RS_ALGO_AUTO, rng.integers(0, below, n, dtype=np.uint64).astype(kdt))]
    for bits, algo, keys in cases:
        keys[::5] = keys[3]                       # ties
        vals = np.arange(n, dtype=np.uint32)
        print("case kv in place %s bits=%d algo=%d" % (np.dtype(kdt).name, bits, algo), flush=True)
        kt, vt = to_dev(keys), to_dev(vals)
        rs.rs_sort_kv(kt, vt, kt, vt, radix_bits=bits, algo=algo)
        st = rs.rs_get_stats()
        assert st.device_error == 0
        assert (st.passes - st.passes_skipped) % 2 == 1
        rk, rv = orc.lsd(keys, bits, vals=vals)
        _check(to_host(kt, kdt), rk, "kv in place keys")
        _check(to_host(vt, np.uint32), rv, "kv in place vals")


def test_kv_mixed_in_place_refused(rs):
    """Keys in place but values not (or the reverse) is refused on the host."""
    import torch
    k = torch.zeros(1000, dtype=torch.int32, device="cuda")
    v = torch.zeros(1000, dtype=torch.int32, device="cuda")
    v2 = torch.zeros(1000, dtype=torch.int32, device="cuda")
    for kw in (dict(keys_out=k, vals_out=v2), dict(keys_out=torch.empty_like(k), vals_out=v)):
        with pytest.raises(rs.RsError) as e:
            rs.rs_sort_kv(k, v, radix_bits=11, algo=rs.RS_ALGO_LSD, **kw)
        assert e.value.code == rs.RS_ERR_INVALID


def test_stream_copy(rs):
    """The bench's copy kernel copies exactly, aligned or not, any length."""
    import torch
    src = torch.randint(0, 255, ((1 << 22) + 77,), dtype=torch.uint8, device="cuda")
    for off, n in ((0, 1 << 22), (0, (1 << 22) + 77), (3, 100_003), (16, 17), (1, 0)):
        a = src[off:off + n]
        b = torch.zeros(n + 5, dtype=torch.uint8, device="cuda")[5:]
        rs.rs_stream_copy(a, b)
        assert torch.equal(a, b), (off, n)


@pytest.mark.parametrize("items", [8, 16, 28])
def test_tile_choices_bit_exact(rs, orc, items):
    """Every tile the tuning table can pick for uint32 keys at radix 2^8 (8,
    16 or 28 keys per thread), forced through the table, sorts exactly,
    every round run and with rounds skipped."""
    import gen
    old = rs.rs_tune_get()
    try:
        rs.rs_tune_set([(c, 0, 0, 8, items, 0) for c in (13 + 2, 17, 21)])
        for n in ((1 << 17) - 5, (1 << 21) - 1001):
            a = gen.uniform_u32(gen.S0 + 90 + items, n)
            for algo in (rs.RS_ALGO_LSD, rs.RS_ALGO_AUTO):
                x = a if algo == rs.RS_ALGO_LSD else a & np.uint32(0x00FFFFFF)
                out = to_host(rs.rs_sort_u32(to_dev(x), radix_bits=0, algo=algo), np.uint32)
                st = rs.rs_get_stats()
                assert st.device_error == 0 and st.tile_keys == 512 * items, (n, st.tile_keys)
                _check(out, orc.lsd(x, 8), "tile %d n=%d algo=%d" % (items, n, algo))
    finally:
        rs.rs_tune_set(old)


@pytest.mark.parametrize("kdt,offset", [(np.uint32, 1), (np.uint32, 2), (np.uint32, 3), (np.uint64, 1)])
def test_unaligned_views(rs, orc, kdt, offset):
    """Key arrays that start off a 16-byte boundary (a view into a larger
    tensor): the histogram reads the aligned body with 16-byte loads and
    the keys before and after it one by one."""
    import gen
    for n in [1, 3, 5, 4099, (1 << 20) + 7]:
        print("case unaligned %s offset=%d n=%d" % (np.dtype(kdt).name, offset, n), flush=True)
        a = (gen.uniform_u32 if kdt == np.uint32 else gen.uniform_u64)(gen.S0 + 70 + n, n + offset)
        base = to_dev(a)
        view = base[offset:]
        sort = rs.rs_sort_u32 if kdt == np.uint32 else rs.rs_sort_u64
        out = to_host(sort(view, radix_bits=8, algo=rs.RS_ALGO_LSD), kdt)
        assert rs.rs_get_stats().device_error == 0
        _check(out, orc.lsd(a[offset:], 8), "unaligned offset=%d n=%d" % (offset, n))


_SINGLE_COUNTER = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np, torch
import paper_1708_09495_amd as rs, gen, oracle
n = (1 << 24) + 1237  # 1,171 tiles: the XCD order would be on
keys = gen.uniform_u32(gen.S0 + 44, n)
out = rs.rs_sort_u32(torch.from_numpy(keys.view(np.int32)).cuda(), algo=rs.RS_ALGO_LSD)
kv = gen.uniform_u32(gen.S0 + 45, 1 << 20)
vals = np.arange(1 << 20, dtype=np.uint32)
ko, vo = rs.rs_sort_kv(torch.from_numpy(kv.view(np.int32)).cuda(), torch.from_numpy(vals.view(np.int32)).cuda(),
                       algo=rs.RS_ALGO_LSD)
ok = np.array_equal(out.cpu().numpy().view(np.uint32), oracle.lsd(keys, 8))
rk, rv = oracle.lsd(kv, 8, vals=vals)
ok = ok and np.array_equal(ko.cpu().numpy().view(np.uint32), rk) and np.array_equal(vo.cpu().numpy().view(np.uint32), rv)
ok = ok and rs.rs_get_stats().device_error == 0
print("single-counter order matches the oracle" if ok else "MISMATCH", flush=True)
sys.exit(0 if ok else 1)
"""


def test_single_counter_tile_order():
    """The rounds' other tile order (one arrival counter, on parts that are
    not 256 compute units in 8 XCDs, or with RS_XCD_ORDER=0), which the
    process-wide setting keeps from the rest of this run: a child process
    with RS_XCD_ORDER=0 sorts keys and key-value pairs, bit-exact against
    the oracle."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, RS_XCD_ORDER="0")
    print("case single-counter tile order (child process)", flush=True)
    r = subprocess.run([sys.executable, "-c", _SINGLE_COUNTER, root], env=env, capture_output=True, text=True,
                       timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0


def test_stats_survive_later_allocations(rs):
    """rs_get_stats reads the status word in the last call's workspace: a
    workspace the binding allocated itself stays alive until the thread's
    next call, so allocations in between (which the caching allocator would
    serve from freed memory) do not change what the stats report."""
    import gen
    import torch
    for n, sort in ((8_389_383, lambda t: rs.rs_sort_u32(t, algo=rs.RS_ALGO_LSD)),
                    (8_389_383, lambda t: rs.rs_sort_blocks_u32(t, algo=rs.RS_ALGO_BTN, p=64))):
        t = torch.empty(n, dtype=torch.int32, device="cuda")
        gen.uniform_u32_dev(gen.S0 + 46, t)
        out = sort(t)
        junk = [torch.full((m,), -1, dtype=torch.int32, device="cuda") for m in (n // 4, n // 2, n, 2 * n)]
        torch.cuda.synchronize()
        assert rs.rs_get_stats().device_error == 0
        assert bool(torch.equal(torch.sort(t.to(torch.int64) & 0xFFFFFFFF).values, out.to(torch.int64) & 0xFFFFFFFF))
        del t, out, junk
