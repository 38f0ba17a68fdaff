"""Pins for the oracle's count-sort rounds and LSD radix sort (Section 3,
"Serial radix-r radix-sort", Eq. Ts).

What pins it, since the paper prints no worked example:
  * brute force over every short array of a small alphabet, against Python's
    own sort (a comparison sort, no shared code);
  * random tiny arrays against numpy's sort;
  * the stable key-value sort against Python's stable sort on (key, index);
  * the round count ceil(w/b) of Section 3 (32/lg r for 32-bit keys);
  * per-round histograms against numpy.bincount and their sum n.
"""
import ctypes
import itertools

import numpy as np
import pytest

RADIXES = [1, 3, 8, 11, 16]


def test_brute_force_u32_all_short_arrays(orc):
    alphabet = [0, 1, 2, 2**32 - 1]
    L = orc.lib()
    for b in RADIXES:
        maxlen = 7 if b == 8 else 5
        for n in range(0, maxlen + 1):
            buf = np.zeros(max(n, 1), dtype=np.uint32)
            out = np.zeros(max(n, 1), dtype=np.uint32)
            pin, pout = buf.ctypes.data, out.ctypes.data
            for combo in itertools.product(alphabet, repeat=n):
                buf[:n] = combo
                assert L.o_lsd(pin, pout, None, None, n, 4, 0, b, None, None) == 0
                assert list(out[:n]) == sorted(combo), (b, combo)


def test_brute_force_u64_all_short_arrays(orc):
    alphabet = [0, 1, 2**32, 2**63, 2**64 - 1]
    L = orc.lib()
    for b in [8, 11, 16]:
        for n in range(0, 6):
            buf = np.zeros(max(n, 1), dtype=np.uint64)
            out = np.zeros(max(n, 1), dtype=np.uint64)
            for combo in itertools.product(alphabet, repeat=n):
                buf[:n] = combo
                assert L.o_lsd(buf.ctypes.data, out.ctypes.data, None, None, n, 8, 0, b, None,
                               None) == 0
                assert [int(x) for x in out[:n]] == sorted(combo), (b, combo)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_random_tiny_against_numpy(orc, dtype):
    rng = np.random.default_rng(1234)
    info = np.iinfo(dtype)
    for trial in range(3000):
        n = int(rng.integers(0, 65))
        b = RADIXES[trial % len(RADIXES)]
        if trial % 3 == 0:   # many duplicates
            a = rng.integers(0, 5, n).astype(dtype)
        else:
            a = rng.integers(0, info.max, n, dtype=dtype, endpoint=True)
        np.testing.assert_array_equal(orc.lsd(a, b), np.sort(a, kind="stable"))


@pytest.mark.parametrize("kdt,vdt", [(np.uint32, np.uint32), (np.uint32, np.uint64),
                                     (np.uint64, np.uint32), (np.uint64, np.uint64)])
def test_stable_kv_against_python_stable_sort(orc, kdt, vdt):
    rng = np.random.default_rng(99)
    for trial in range(300):
        n = int(rng.integers(0, 300))
        keys = rng.integers(0, 1 + int(rng.integers(1, 50)), n).astype(kdt)
        if trial % 4 == 0:
            keys = (keys.astype(np.uint64) << np.uint64(8 * keys.itemsize - 8)).astype(kdt)
        vals = np.arange(n, dtype=vdt)
        b = RADIXES[trial % len(RADIXES)]
        ko, vo = orc.lsd(keys, b, vals=vals)
        order = sorted(range(n), key=lambda i: int(keys[i]))   # Python's sort is stable
        np.testing.assert_array_equal(vo, np.array(order, dtype=vdt))
        np.testing.assert_array_equal(ko, keys[order])
        assert orc.check_stable_kv(keys, ko, vo) == 0


@pytest.mark.parametrize("kb,b,rounds", [(4, 8, 4), (4, 11, 3), (4, 16, 2), (4, 3, 11),
                                         (4, 1, 32), (8, 8, 8), (8, 11, 6), (8, 16, 4)])
def test_round_count_closed_form(orc, kb, b, rounds):
    # Section 3: 32/lg r rounds of count-sort for 32-bit keys; ceil(w/b) in general.
    dt = np.uint32 if kb == 4 else np.uint64
    a = np.random.default_rng(3).integers(0, np.iinfo(dt).max, 257, dtype=dt, endpoint=True)
    (out), hist, cnt = orc.lsd(a, b, want_hist=True)
    assert cnt.rounds == rounds == orc.lsd_rounds(kb, b)
    assert hist.shape == (rounds, 1 << b)


@pytest.mark.parametrize("b", [8, 11])
def test_round_histograms(orc, b):
    rng = np.random.default_rng(5)
    a = rng.integers(0, 2**32, 5000, dtype=np.uint64).astype(np.uint32)
    out, hist, cnt = orc.lsd(a, b, want_hist=True)
    # digit histograms do not depend on the order the keys are in
    for j in range(cnt.rounds):
        d = (a.astype(np.uint64) >> np.uint64(j * b)) & np.uint64((1 << b) - 1)
        np.testing.assert_array_equal(hist[j], np.bincount(d.astype(np.int64), minlength=1 << b))
        assert int(hist[j].sum()) == a.size


def test_single_round_is_stable_by_digit(orc):
    rng = np.random.default_rng(8)
    keys = rng.integers(0, 2**16, 2000).astype(np.uint64)
    idx = np.arange(keys.size, dtype=np.uint64)
    ko, vo, h = orc.count_round(keys, 4, 4, vals=idx)
    dig = (keys >> np.uint64(4)) & np.uint64(15)
    order = sorted(range(keys.size), key=lambda i: int(dig[i]))
    np.testing.assert_array_equal(vo, np.array(order, dtype=np.uint64))
    np.testing.assert_array_equal(h, np.bincount(dig.astype(np.int64), minlength=16))


@pytest.mark.parametrize("case", ["empty", "one", "two", "equal", "sorted", "reverse", "high",
                                  "low", "max"])
def test_special_cases(orc, case):
    rng = np.random.default_rng(11)
    n = 5000
    a = {
        "empty": np.zeros(0, np.uint32),
        "one": np.array([7], np.uint32),
        "two": np.array([9, 3], np.uint32),
        "equal": np.full(n, 12345, np.uint32),
        "sorted": np.arange(n, dtype=np.uint32) * 977,
        "reverse": (np.arange(n, dtype=np.uint32) * 977)[::-1].copy(),
        "high": (rng.integers(0, 256, n).astype(np.uint32) << np.uint32(24)),
        "low": rng.integers(0, 256, n).astype(np.uint32),
        "max": np.where(rng.random(n) < 0.5, 2**32 - 1, rng.integers(0, 2**32, n)).astype(np.uint32),
    }[case]
    for b in RADIXES:
        np.testing.assert_array_equal(orc.lsd(a, b), np.sort(a))


def test_checker_catches_planted_mistakes(orc):
    rng = np.random.default_rng(21)
    n = 1000
    keys = rng.integers(0, 20, n).astype(np.uint32)
    ko, vo = orc.lsd(keys, 8, vals=np.arange(n, dtype=np.uint32))
    assert orc.check_stable_kv(keys, ko, vo) == 0
    # 1: order broken
    bad = ko.copy(); bad[[10, 900]] = bad[[900, 10]]
    assert orc.check_stable_kv(keys, bad, vo) == 1
    # 2: payload not a permutation
    badv = vo.copy(); badv[5] = badv[6]
    assert orc.check_stable_kv(keys, ko, badv) == 2
    # 3: payload does not point at its key
    badv3 = vo.copy(); i0 = 0; i1 = int(np.nonzero(ko != ko[0])[0][0])
    badv3[[i0, i1]] = badv3[[i1, i0]]
    assert orc.check_stable_kv(keys, ko, badv3) == 3
    # 4: ties out of input order
    run = np.nonzero(ko == ko[0])[0]
    badv4 = vo.copy(); badv4[[run[0], run[1]]] = badv4[[run[1], run[0]]]
    assert orc.check_stable_kv(keys, ko, badv4) == 4
