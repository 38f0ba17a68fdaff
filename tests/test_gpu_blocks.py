"""GPU parity of the block networks at device scale (Section 2; Section 3,
Eqs. Tb and To): p runs of ceil(n/p) keys in device memory, each sorted by
one workgroup, then BTN's lg p (lg p + 1)/2 or OET's p merge-split stages.
Outputs are compared bit for bit with the oracle's block network for the
same p; the stage counts with their closed forms."""
import numpy as np
import pytest

from gpu_util import first_mismatch, multiset_hash, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import paper_1708_09495_amd as rs
    rs.lib()
    return rs


def _check(out, ref, what):
    i = first_mismatch(out, ref)
    assert i is None, "%s: first mismatch at %d: got %d want %d" % (what, i, out[i], ref[i])


def _stages(algo, p):
    lg = p.bit_length() - 1
    return lg * (lg + 1) // 2 if algo == "BTN" else p


@pytest.mark.parametrize("algo,ps", [("BTN", [2, 4, 64, 256, 1024]), ("OET", [2, 3, 7, 16, 33])])
def test_against_oracle(rs, orc, algo, ps):
    import gen
    code = getattr(rs, "RS_ALGO_" + algo)
    # several chunks per pair, ragged last runs, runs of padding only
    for n in [2, 1000, 16_385, 100_003, (1 << 20) + 7]:
        a = gen.uniform_u32(gen.S0 + 31 + n, n)
        for p in ps:
            if p > n:
                continue
            print("case blocks %s n=%d p=%d" % (algo, n, p), flush=True)
            out = to_host(rs.rs_sort_blocks_u32(to_dev(a), algo=code, p=p), np.uint32)
            st = rs.rs_get_stats()
            assert st.device_error == 0
            assert st.runs_p == p and st.network_stages == _stages(algo, p)
            ref = (orc.bitonic_block(a, p) if algo == "BTN" else orc.oet_block(a, p))[0]
            _check(out, ref, "%s n=%d p=%d" % (algo, n, p))


@pytest.mark.parametrize("case", ["equal", "sorted", "reverse", "few", "max", "low"])
def test_structured(rs, orc, case):
    rng = np.random.default_rng(23)
    n = 300_001
    a = {
        "equal": np.full(n, 0x5EED, np.uint32),
        "sorted": np.sort(rng.integers(0, 2**32, n, dtype=np.uint64)).astype(np.uint32),
        "reverse": np.sort(rng.integers(0, 2**32, n, dtype=np.uint64))[::-1].astype(np.uint32),
        "few": rng.choice(np.array([7, 2**31, 9, 2**32 - 2], np.uint32), n),
        # keys equal to the padding value mix with the padding
        "max": rng.choice(np.array([0, 2**32 - 1], np.uint32), n),
        "low": rng.integers(0, 50, n).astype(np.uint32),
    }[case]
    for algo, p in (("BTN", 128), ("OET", 12)):
        print("case blocks structured %s %s p=%d" % (case, algo, p), flush=True)
        out = to_host(rs.rs_sort_blocks_u32(to_dev(a), algo=getattr(rs, "RS_ALGO_" + algo), p=p),
                      np.uint32)
        ref = (orc.bitonic_block(a, p) if algo == "BTN" else orc.oet_block(a, p))[0]
        _check(out, ref, "%s %s" % (case, algo))


@pytest.mark.parametrize("n", [500_000, (1 << 23) + 5])
def test_default_p_and_sort_entry(rs, orc, n):
    """p = 0 takes the MBSP model's p (OET's is not a power of two here)."""
    import gen
    a = gen.uniform_u32(gen.S0 + 33, n)
    ref = orc.lsd(a, 8)
    for algo in ("BTN", "OET"):
        code = getattr(rs, "RS_ALGO_" + algo)
        p = rs.rs_blocks_default_p(n, code)
        assert 2 <= p <= 4096
        print("case blocks default p %s n=%d p=%d" % (algo, n, p), flush=True)
        out = to_host(rs.rs_sort_blocks_u32(to_dev(a), algo=code), np.uint32)
        assert rs.rs_get_stats().runs_p == p
        _check(out, ref, "blocks default " + algo)
        # rs_sort_u32 with BTN / OET above one workgroup's capacity
        out = to_host(rs.rs_sort_u32(to_dev(a), algo=code), np.uint32)
        st = rs.rs_get_stats()
        assert st.runs_p == p and st.network_stages == _stages(algo, p)
        assert st.device_error == 0
        _check(out, ref, "sort_u32 " + algo)


def test_in_place(rs, orc):
    import gen
    n = 123_457
    a = gen.uniform_u32(gen.S0 + 34, n)
    for algo, p in (("BTN", 64), ("OET", 9)):
        print("case blocks in place %s" % algo, flush=True)
        t = to_dev(a)
        rs.rs_sort_blocks_u32(t, t, algo=getattr(rs, "RS_ALGO_" + algo), p=p)
        _check(to_host(t, np.uint32), orc.lsd(a, 8), "in place " + algo)


def test_bench_sizes(rs, orc):
    """At the sizes the bench times (2^23 and 2^25 keys, p = 256), against the
    oracle's sort: a keys-only sort has one correct output for every p."""
    import gen
    for lg in (23, 25):
        n = 1 << lg
        a = gen.uniform_u32(gen.S0 + 35 + lg, n)
        ref = orc.lsd(a, 8)
        for algo in ("BTN", "OET"):
            print("case blocks bench size 2^%d %s" % (lg, algo), flush=True)
            out = to_host(rs.rs_sort_blocks_u32(to_dev(a), algo=getattr(rs, "RS_ALGO_" + algo), p=256),
                          np.uint32)
            assert rs.rs_get_stats().device_error == 0
            _check(out, ref, "2^%d %s" % (lg, algo))
            assert multiset_hash(out) == multiset_hash(a)


def test_bench_configuration(rs, orc):
    """The launch configuration the bench times: 2^27 keys at the MBSP
    model's p (BTN and OET), every output key against the oracle's sort."""
    import gen
    n = 1 << 27
    a = gen.uniform_u32(gen.S0 + 2, n)
    ref = orc.lsd(a, 8)
    for algo in ("BTN", "OET"):
        code = getattr(rs, "RS_ALGO_" + algo)
        p = rs.rs_blocks_default_p(n, code)
        print("case blocks bench configuration %s n=2^27 p=%d" % (algo, p), flush=True)
        out = to_host(rs.rs_sort_blocks_u32(to_dev(a), algo=code), np.uint32)
        st = rs.rs_get_stats()
        assert st.device_error == 0 and st.runs_p == p and st.network_stages == _stages(algo, p)
        _check(out, ref, "2^27 %s p=%d" % (algo, p))
