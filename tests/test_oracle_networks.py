"""Pins for the oracle's merge-split, block bitonic (BTN) and block odd-even
transposition (OET) sorts (Section 2, the BTN and OET paragraphs; Section 3,
Eq. To and Eq. Tb).

What pins them:
  * merge-split against Python's sort of the union, split in halves;
  * the 0-1 principle: every binary input of every length n <= 16 through
    the textbook networks, and every binary input of every block shape
    (p, N) with p N <= 16 through the block networks (merge-split and the
    local sort commute with monotone maps, so the principle carries over);
  * the stage counts lg p (lg p + 1)/2 (BTN) and p (OET) and the number of
    merge-splits per stage;
  * random inputs of every size against numpy's sort, including n not a
    multiple of p and keys equal to the pad value.
"""
import ctypes
import itertools

import numpy as np
import pytest


def _binary_inputs(n):
    """All 2^n binary vectors of length n as a (2^n, n) uint32 array."""
    i = np.arange(1 << n, dtype=np.uint64)[:, None]
    return ((i >> np.arange(n, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.uint32)


def test_merge_split_against_sorted_union(orc):
    rng = np.random.default_rng(2)
    for trial in range(2000):
        N = int(rng.integers(1, 12))
        A = np.sort(rng.integers(0, 6, N)).astype(np.uint64)
        B = np.sort(rng.integers(0, 6, N)).astype(np.uint64)
        lo, hi = orc.merge_split(A, B)
        u = sorted(list(A) + list(B))
        assert list(lo) == u[:N] and list(hi) == u[N:]


def _run_all(fn_name, n, extra_args):
    fn = getattr(__import__("oracle").lib(), fn_name)
    ins = _binary_inputs(n)
    out = np.zeros(max(n, 1), dtype=np.uint32)
    buf = np.zeros(max(n, 1), dtype=np.uint32)
    zeros_needed = n - ins.sum(axis=1)
    for row, z in zip(ins, zeros_needed):
        buf[:n] = row
        assert fn(buf.ctypes.data, out.ctypes.data, n, 4, *extra_args) == 0
        # sorted binary output: z zeros then ones
        if out[:z].any() or not out[z:n].all():
            return row
    return None


@pytest.mark.parametrize("n", list(range(1, 17)))
def test_zero_one_textbook_bitonic(orc, n):
    assert _run_all("o_bitonic", n, [None]) is None


@pytest.mark.parametrize("n", list(range(1, 17)))
@pytest.mark.parametrize("parity", [0, 1])
def test_zero_one_textbook_oet(orc, n, parity):
    assert _run_all("o_oet", n, [parity, None]) is None


def _block_shapes(pow2_only):
    for p in range(1, 17):
        if pow2_only and p & (p - 1):
            continue
        for N in range(1, 17):
            if p * N <= 16:
                yield p, N


@pytest.mark.parametrize("p,N", list(_block_shapes(True)))
def test_zero_one_block_bitonic(orc, p, N):
    assert _run_all("o_bitonic_block", p * N, [p, None]) is None


@pytest.mark.parametrize("p,N", list(_block_shapes(False)))
@pytest.mark.parametrize("parity", [0, 1])
def test_zero_one_block_oet(orc, p, N, parity):
    assert _run_all("o_oet_block", p * N, [p, parity, None]) is None


def test_zero_one_catches_a_planted_wrong_direction(orc):
    # A network with the direction rule flipped in one stage must fail the
    # exhaustive 0-1 check: the check has teeth.  (Planted in a Python copy
    # of the textbook network, never in the library.)
    def bad_bitonic(a):
        a = list(a)
        m = len(a)
        k = 2
        while k <= m:
            j = k // 2
            while j >= 1:
                for i in range(m):
                    l = i ^ j
                    if l > i:
                        asc = (i & k) == 0
                        if k == m and j == 1:
                            asc = not asc            # the planted mistake
                        if (asc and a[i] > a[l]) or (not asc and a[i] < a[l]):
                            a[i], a[l] = a[l], a[i]
                j //= 2
            k *= 2
        return a
    ins = _binary_inputs(8)
    assert any(bad_bitonic(r) != sorted(r) for r in ins.tolist())


@pytest.mark.parametrize("p", [1, 2, 4, 8, 16, 32, 64])
def test_bitonic_stage_count(orc, p):
    a = np.random.default_rng(p).integers(0, 2**32, 1000, dtype=np.uint64).astype(np.uint32)
    out, cnt = orc.bitonic_block(a, p)
    lg = p.bit_length() - 1
    assert cnt.stages == lg * (lg + 1) // 2          # Section 2: lg p (lg p + 1)/2 stages
    assert cnt.merge_splits == cnt.stages * (p // 2)
    assert cnt.local_sorts == p
    np.testing.assert_array_equal(out, np.sort(a))


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8, 13, 16])
@pytest.mark.parametrize("parity", [0, 1])
def test_oet_round_count(orc, p, parity):
    a = np.random.default_rng(p).integers(0, 2**32, 999, dtype=np.uint64).astype(np.uint32)
    out, cnt = orc.oet_block(a, p, parity)
    assert cnt.stages == p                            # Section 2: p rounds
    expect = sum(len(range((t + parity) % 2, p - 1, 2)) for t in range(p))
    assert cnt.merge_splits == expect
    np.testing.assert_array_equal(out, np.sort(a))


def test_textbook_counts(orc):
    a = np.random.default_rng(0).integers(0, 2**32, 64, dtype=np.uint64).astype(np.uint32)
    out, cnt = orc.bitonic(a)
    assert cnt.stages == 6 * 7 // 2 and cnt.merge_splits == 21 * 32
    out2, cnt2 = orc.oet(a)
    assert cnt2.stages == 64
    np.testing.assert_array_equal(out, np.sort(a))
    np.testing.assert_array_equal(out2, np.sort(a))


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_block_networks_random(orc, dtype):
    rng = np.random.default_rng(17)
    mx = np.iinfo(dtype).max
    for n in [1, 2, 3, 7, 64, 100, 255, 256, 1000, 4097]:
        for p in [1, 2, 4, 8, 64]:
            a = rng.integers(0, mx, n, dtype=dtype, endpoint=True)
            a[rng.random(n) < 0.1] = mx                   # keys equal to the pad value
            ref = np.sort(a)
            np.testing.assert_array_equal(orc.bitonic_block(a, p)[0], ref)
            np.testing.assert_array_equal(orc.oet_block(a, p, 0)[0], ref)
            np.testing.assert_array_equal(orc.oet_block(a, p + 1, 1)[0], ref)
        if n <= 1000:
            np.testing.assert_array_equal(orc.bitonic(a)[0], np.sort(a))
            np.testing.assert_array_equal(orc.oet(a)[0], np.sort(a))


def test_block_with_one_key_per_run_equals_textbook(orc):
    rng = np.random.default_rng(4)
    for n in [2, 8, 32, 128]:
        a = rng.integers(0, 50, n).astype(np.uint32)
        np.testing.assert_array_equal(orc.bitonic_block(a, n)[0], orc.bitonic(a)[0])
        np.testing.assert_array_equal(orc.oet_block(a, n, 1)[0], orc.oet(a, 1)[0])


def test_segmented(orc):
    rng = np.random.default_rng(6)
    lens = rng.integers(0, 300, 50)
    lens[[3, 17]] = 0
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    a = rng.integers(0, 2**32, off[-1], dtype=np.uint64).astype(np.uint32)
    out = orc.segmented(a, off)
    for s in range(lens.size):
        np.testing.assert_array_equal(out[off[s]:off[s + 1]], np.sort(a[off[s]:off[s + 1]]))
