"""Pins the oracle's structure counters to numbers the paper prints: the cost
coefficients of Section 3 (Eqs. TsG, Tp4, Tp2, ToG, TbG, MBSP model with
g = 5G).  Each coefficient is rebuilt from what the oracle actually ran --
its count-sort rounds, bitonic stages and odd-even transposition rounds --
and the per-round access counts the paper charges (3N main-memory accesses
and 2N count-array accesses per serial round, 4N and 2N plus 2pr per
parallel round, 4N/p per network stage), so a wrong round or stage count in
the oracle shows up as a coefficient that differs from the printed one."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mbsp_coefficients.txt")
g = 5  # g = 5G (Section 3)


def _golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = int(v)
    return out


def _rounds(orc, b):
    keys = np.arange(1000, dtype=np.uint32)[::-1].copy()
    _, _, cnt = orc.lsd(keys, b, want_hist=True)
    return cnt.rounds


def test_serial_radix_coefficient(orc):
    want = _golden()
    rounds = _rounds(orc, 8)
    assert rounds * (3 * g + 2) == want["Ts_r8_N"]


@pytest.mark.parametrize("b,tag", [(8, "Tp4"), (16, "Tp2")])
def test_parallel_radix_coefficients(orc, b, tag):
    want = _golden()
    rounds = _rounds(orc, b)
    assert rounds * (4 * g + 2) == want[tag + "_n_over_p"]
    assert rounds * 2 * (1 << b) * g == want[tag + "_p"]


@pytest.mark.parametrize("p", [2, 4, 8, 16])
def test_oet_coefficients(orc, p):
    want = _golden()
    n = 64 * p
    keys = np.random.default_rng(p).integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    out, cnt = orc.oet_block(keys, p)
    assert (out == np.sort(keys)).all()
    # local sorts: T_s(n/p); then cnt.stages rounds of 4 (n/p) g each
    assert _rounds(orc, 8) * (3 * g + 2) == want["To_n_over_p"]
    assert cnt.stages * 4 * g == want["To_n"] * p


@pytest.mark.parametrize("p", [2, 4, 8, 16])
def test_bitonic_coefficients(orc, p):
    want = _golden()
    n = 64 * p
    keys = np.random.default_rng(p).integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    out, cnt = orc.bitonic_block(keys, p)
    assert (out == np.sort(keys)).all()
    lg = p.bit_length() - 1
    assert _rounds(orc, 8) * (3 * g + 2) == want["Tb_n_over_p"]
    # stages of 4 (n/p) g: coefficient of n lg p (lg p + 1) / p
    assert cnt.stages * 4 * g == want["Tb_n_lgp_lgp1_over_p"] * lg * (lg + 1)
