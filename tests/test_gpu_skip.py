"""GPU parity of the LSD sort that skips identity rounds (RS_ALGO_AUTO): a
round whose digit is the same for every key moves nothing, so the output
must equal the oracle's full LSD sort bit for bit, and the number of rounds
skipped must equal the number of the oracle's per-round histograms that
have a single non-empty bin.  Skipped rounds at the start, the middle, the
end, all of them, odd and even counts of rounds run, in place and not,
keys only and key-value."""
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


def _single_bin_rounds(orc, a, bits):
    _, hist, _ = orc.lsd(a, bits, want_hist=True)
    return int(np.sum(hist.max(axis=1) == a.size)) if a.size else 0


def _cases(rng, n):
    r32 = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    r64 = rng.integers(0, 2**63, n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n).astype(np.uint64)
    return {
        "u64_below_2p32": r64 & np.uint64(0xFFFFFFFF),                        # top 4 rounds
        "u64_fixed_top": (r64 & np.uint64(0xFFFFFFFFFFFF)) | np.uint64(0xABCD << 48),  # top 2
        "u32_fixed_top": (r32 & np.uint32(0x00FFFFFF)) | np.uint32(0x5A000000),  # 1 of 4: odd
        "u32_fixed_mid": (r32 & np.uint32(0xFFFF00FF)) | np.uint32(0x3700),   # a middle round
        "u32_fixed_low": (r32 & np.uint32(0xFFFFFF00)) | np.uint32(0x11),     # the first round
        "u32_two_low": (r32 & np.uint32(0xFFFF0000)) | np.uint32(0x2211),     # two, even count
        "u32_equal": np.full(n, 0xC0FFEE, np.uint32),                         # every round
        "u32_uniform": r32,                                                   # none
    }


@pytest.mark.parametrize("n", [1, 4097, 300_001])
def test_keys(rs, orc, n):
    rng = np.random.default_rng(41 + n)
    for name, a in _cases(rng, n).items():
        for inplace in (False, True):
            print("case skip keys %s n=%d inplace=%d" % (name, n, inplace), flush=True)
            f = rs.rs_sort_u32 if a.dtype == np.uint32 else rs.rs_sort_u64
            t = to_dev(a)
            out = f(t, t, algo=rs.RS_ALGO_AUTO) if inplace else f(t, algo=rs.RS_ALGO_AUTO)
            st = rs.rs_get_stats()
            assert st.device_error == 0
            _check(to_host(out, a.dtype), orc.lsd(a, 8), "%s n=%d inplace=%d" % (name, n, inplace))
            assert st.passes_skipped == _single_bin_rounds(orc, a, 8), name
            if not inplace:
                _check(to_host(t, a.dtype), a, "%s: input untouched" % name)


def test_keys_at_xcd_order_sizes(rs, orc):
    """Skipped rounds where the rounds take their tiles in the XCD-aware
    order (from 1,024 tiles: 2^24 + 3 keys are 1,171 tiles of uint32 keys
    and 1,821 of uint64): skips at the start, the middle and the top, and
    an odd count of rounds run, against the oracle."""
    n = (1 << 24) + 3
    rng = np.random.default_rng(47)
    cases = _cases(rng, n)
    for name in ("u64_below_2p32", "u32_fixed_top", "u32_fixed_mid", "u32_fixed_low"):
        a = cases[name]
        print("case skip keys %s n=%d" % (name, n), flush=True)
        f = rs.rs_sort_u32 if a.dtype == np.uint32 else rs.rs_sort_u64
        out = f(to_dev(a), algo=rs.RS_ALGO_AUTO)
        st = rs.rs_get_stats()
        assert st.device_error == 0
        _check(to_host(out, a.dtype), orc.lsd(a, 8), "%s n=%d" % (name, n))
        assert st.passes_skipped == _single_bin_rounds(orc, a, 8), name


@pytest.mark.parametrize("bits", [8, 11])
def test_kv(rs, orc, bits):
    rng = np.random.default_rng(43 + bits)
    n = 250_003
    for name, a in _cases(rng, n).items():
        for vdt in (np.uint32, np.uint64):
            for inplace in (False, True):
                print("case skip kv %s b=%d v=%s inplace=%d" % (name, bits, np.dtype(vdt).name, inplace),
                      flush=True)
                vals = np.arange(n, dtype=vdt)
                kt, vt = to_dev(a), to_dev(vals)
                if inplace:
                    rs.rs_sort_kv(kt, vt, kt, vt, radix_bits=bits, algo=rs.RS_ALGO_AUTO)
                    ko, vo = kt, vt
                else:
                    ko, vo = rs.rs_sort_kv(kt, vt, radix_bits=bits, algo=rs.RS_ALGO_AUTO)
                st = rs.rs_get_stats()
                rk, rv = orc.lsd(a, bits, vals=vals)
                _check(to_host(ko, a.dtype), rk, "kv keys %s" % name)
                _check(to_host(vo, vdt), rv, "kv vals %s" % name)
                assert st.passes_skipped == _single_bin_rounds(orc, a, bits), name


def test_lsd_runs_every_round(rs, orc):
    # RS_ALGO_LSD is the paper's sort as stated: every round runs
    a = np.full(10_000, 7, np.uint64)
    out = to_host(rs.rs_sort_u64(to_dev(a), algo=rs.RS_ALGO_LSD), np.uint64)
    st = rs.rs_get_stats()
    assert st.passes == 8 and st.passes_skipped == 0
    _check(out, a, "equal keys")
