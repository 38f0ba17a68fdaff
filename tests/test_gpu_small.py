"""GPU parity of the one-workgroup sorts: BTN and OET (the block networks of
Section 2 and Eq. Tb / Eq. To) and the LDS radix sort, through the C ABI.

Each instance is compared bit for bit with the oracle's block network for
the same p (or the oracle's LSD sort for the LDS radix sort); the 0-1
principle is checked exhaustively on the GPU kernels themselves for n <= 16.
"""
import numpy as np
import pytest

from gpu_util import first_mismatch, multiset_hash, multiset_hash_rows_dev, to_dev, to_host

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 17, 63, 64, 65, 100, 255, 256, 1000, 1024, 4095, 4096, 8192, 10_000, 16_384]


@pytest.fixture(scope="module")
def rs():
    import paper_1708_09495_amd as rs
    rs.lib()
    return rs


def _valid_ps(n):
    npad = 1
    while npad < n:
        npad <<= 1
    return [p for p in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024) if p <= npad and npad // p <= 64]


def _instances(seed, n, count):
    import gen
    return gen.instances_u32(seed, n, count)


@pytest.mark.parametrize("algo", ["BTN", "OET"])
def test_networks_all_p(rs, orc, algo):
    code = getattr(rs, "RS_ALGO_" + algo)
    for n in SIZES:
        ps = _valid_ps(n)
        for p in ps:
            print("case %s n=%d p=%d" % (algo, n, p), flush=True)
            count = 5
            a = _instances(1000 + n, n, count)
            out = to_host(rs.rs_sort_batch_u32(to_dev(a.ravel()), n, count, algo=code, p=p),
                          np.uint32).reshape(count, n)
            st = rs.rs_get_stats()
            lg = p.bit_length() - 1
            assert st.runs_p == p
            assert st.network_stages == (lg * (lg + 1) // 2 if algo == "BTN" else p)
            for i in range(count):
                ref = (orc.bitonic_block(a[i], p) if algo == "BTN" else orc.oet_block(a[i], p))[0]
                j = first_mismatch(out[i], ref)
                assert j is None, "%s n=%d p=%d inst %d pos %d" % (algo, n, p, i, j)


def test_lds_radix(rs, orc):
    for n in SIZES:
        print("case LDS_RADIX n=%d" % n, flush=True)
        count = 7
        a = _instances(2000 + n, n, count)
        out = to_host(rs.rs_sort_batch_u32(to_dev(a.ravel()), n, count, algo=rs.RS_ALGO_LDS_RADIX),
                      np.uint32).reshape(count, n)
        for i in range(count):
            assert first_mismatch(out[i], orc.lsd(a[i], 8)) is None, (n, i)


@pytest.mark.parametrize("algo", ["BTN", "OET", "LDS_RADIX"])
def test_zero_one_exhaustive_on_gpu(rs, algo):
    """All 2^n binary inputs, n <= 16, as 2^n instances of one launch."""
    code = getattr(rs, "RS_ALGO_" + algo)
    for n in (2, 3, 5, 8, 13, 16):
        i = np.arange(1 << n, dtype=np.uint64)[:, None]
        ins = ((i >> np.arange(n, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.uint32)
        ps = _valid_ps(n) if algo != "LDS_RADIX" else [0]
        for p in ps:
            out = to_host(rs.rs_sort_batch_u32(to_dev(ins.ravel()), n, ins.shape[0], algo=code, p=p),
                          np.uint32).reshape(ins.shape)
            zeros = n - ins.sum(axis=1)
            ok = np.array([(not out[r, :zeros[r]].any()) and out[r, zeros[r]:].all()
                           for r in range(ins.shape[0])])
            assert ok.all(), "%s n=%d p=%d first bad input %s" % (algo, n, p, ins[~ok][0])


@pytest.mark.parametrize("algo", ["BTN", "OET", "LDS_RADIX"])
def test_pad_value_and_duplicates(rs, orc, algo):
    code = getattr(rs, "RS_ALGO_" + algo)
    rng = np.random.default_rng(5)
    for n in (5, 100, 1000, 16_384):
        a = rng.choice(np.array([0, 7, 2**32 - 1], dtype=np.uint32), (3, n))
        out = to_host(rs.rs_sort_batch_u32(to_dev(a.ravel()), n, 3, algo=code), np.uint32).reshape(3, n)
        for i in range(3):
            assert first_mismatch(out[i], np.sort(a[i])) is None


@pytest.mark.parametrize("n", [64, 256, 1024, 4096, 8192, 16384])
def test_full_config_10000_instances(rs, orc, n):
    """The full small-n workload: 10,000 seeded instances per size in one
    launch per algorithm; 40 sampled instances against the oracle, every
    instance checked sorted and holding the multiset of its own input (a
    per-instance 64-bit multiset hash, so a key swapped between two
    instances that both stay sorted is caught)."""
    import gen
    count = 10_000
    a = gen.instances_u32(gen.S0 + 3, n, count)
    dev = to_dev(a.ravel())
    h_in = multiset_hash_rows_dev(dev.view(count, n))
    rng = np.random.default_rng(n)
    sample = rng.choice(count, 40, replace=False)
    for algo in ("BTN", "OET", "LDS_RADIX"):
        print("case full %s n=%d" % (algo, n), flush=True)
        outd = rs.rs_sort_batch_u32(dev, n, count, algo=getattr(rs, "RS_ALGO_" + algo))
        h_out = multiset_hash_rows_dev(outd.view(count, n))
        bad = (h_out != h_in).nonzero()
        assert bad.numel() == 0, "%s n=%d: instance %d changed its multiset" % (algo, n, int(bad[0]))
        out = to_host(outd, np.uint32).reshape(count, n)
        assert (np.diff(out.astype(np.int64), axis=1) >= 0).all()
        assert multiset_hash(out.ravel()) == multiset_hash(a.ravel())
        for i in sample:
            assert first_mismatch(out[i], orc.lsd(a[i], 8)) is None, (algo, n, i)


def test_single_array_through_sort_u32(rs, orc):
    rng = np.random.default_rng(9)
    for algo in ("BTN", "OET", "LDS_RADIX"):
        for n in (1, 1000, 16_384):
            a = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
            out = to_host(rs.rs_sort_u32(to_dev(a), algo=getattr(rs, "RS_ALGO_" + algo)), np.uint32)
            assert first_mismatch(out, orc.lsd(a, 8)) is None


def test_small_errors(rs):
    import torch
    a = torch.zeros(20000, dtype=torch.int32, device="cuda")
    with pytest.raises(rs.RsError) as e:
        rs.rs_sort_batch_u32(a, 20000, 1, algo=rs.RS_ALGO_BTN)
    assert e.value.code == rs.RS_ERR_UNSUPPORTED
    b = torch.zeros(1000, dtype=torch.int32, device="cuda")
    with pytest.raises(rs.RsError) as e:
        rs.rs_sort_batch_u32(b, 1000, 1, algo=rs.RS_ALGO_BTN, p=3)     # not a power of two
    assert e.value.code == rs.RS_ERR_INVALID
    with pytest.raises(rs.RsError) as e:
        rs.rs_sort_batch_u32(b, 1000, 1, algo=rs.RS_ALGO_BTN, p=4)     # runs of 256 > 64
    assert e.value.code == rs.RS_ERR_INVALID


def test_autotuner_installs_fastest_and_stays_correct(rs, orc):
    old = rs.rs_tune_get()
    try:
        res = rs.rs_tune_run(instances=256)
        table = {e[0]: e[1:] for e in rs.rs_tune_get()}
        for c in range(1, 15):
            rows = [r for r in res if r["size_log2"] == c and r["algo"] != rs.RS_ALGO_LSD]
            assert rows and all(r["us_per_array"] > 0 for r in rows)
            best = min(rows, key=lambda r: r["us_per_array"])
            assert best["chosen"] == 1
            assert table[c][0] == best["algo"]
            assert any(r["algo"] == rs.RS_ALGO_LSD for r in res if r["size_log2"] == c)
        # the tuned AUTO path still sorts exactly
        rng = np.random.default_rng(1)
        for n in (3, 100, 5000, 16384):
            a = rng.integers(0, 2**32, (4, n), dtype=np.uint64).astype(np.uint32)
            out = to_host(rs.rs_sort_batch_u32(to_dev(a.ravel()), n, 4), np.uint32).reshape(4, n)
            for i in range(4):
                assert first_mismatch(out[i], orc.lsd(a[i], 8)) is None
    finally:
        rs.rs_tune_set(old)
