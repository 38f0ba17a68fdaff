"""GPU parity of the batched segmented sort (one persistent launch) through
the C ABI: every segment must equal the oracle's sort of that segment."""
import numpy as np
import pytest

from gpu_util import first_mismatch, segment_hashes_dev, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rs():
    import paper_1708_09495_amd as rs
    rs.lib()
    return rs


def _offsets(lens):
    return np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)


def _run(rs, keys, off, algo=0, inplace=False):
    import torch
    k = to_dev(keys)
    o = torch.from_numpy(off).cuda()
    out = k if inplace else None
    res = rs.rs_sort_segmented(k, o, keys_out=out, algo=algo)
    return to_host(res, np.uint32)


# (segments of 10,241 .. 14,336 keys and above 16,384 keys are sorted by the
# onesweep rounds shared by all workgroups, in tiles of 14,336 keys: the
# lengths on either side of 10,240 / 10,241, 14,336 / 14,337 and 16,384 /
# 16,385, and whole / ragged tile counts, sit on either side of those edges)
MIXED = [0, 1, 2, 3, 15, 16, 17, 63, 64, 65, 100, 255, 256, 1000, 4095, 4096, 8192, 8193, 10_240,
         10_241, 14_336, 14_337, 16383, 16384, 16385, 20000, 40000, 65_535, 65_536, 71_680, 71_681,
         100_000, 262_144, 0, 1]


@pytest.mark.parametrize("algo", ["AUTO", "BTN", "OET", "LDS_RADIX", "LSD"])
def test_mixed_lengths(rs, orc, algo):
    import gen
    lens = np.array(MIXED, dtype=np.int64)
    off = _offsets(lens)
    keys = gen.uniform_u32(gen.S0 + 4, int(off[-1]))
    out = _run(rs, keys, off, getattr(rs, "RS_ALGO_" + algo))
    ref = orc.segmented(keys, off)
    i = first_mismatch(out, ref)
    assert i is None, "first mismatch at %d (segment %d)" % (i, np.searchsorted(off, i, "right") - 1)
    assert rs.rs_get_stats().device_error == 0


def test_random_lengths_and_duplicates(rs, orc):
    rng = np.random.default_rng(3)
    lens = np.floor(2.0 ** rng.uniform(0, 17, 300)).astype(np.int64)
    lens[::17] = 0
    off = _offsets(lens)
    keys = rng.integers(0, 5, int(off[-1])).astype(np.uint32)          # heavy ties
    keys[::3] = rng.integers(0, 2**32, keys[::3].size, dtype=np.uint64).astype(np.uint32)
    out = _run(rs, keys, off)
    assert first_mismatch(out, orc.segmented(keys, off)) is None


def test_in_place_and_single_segment(rs, orc):
    import gen
    for lens in ([1 << 20], [5], [0, 0, 0], [16384, 1 << 18]):
        off = _offsets(np.array(lens, dtype=np.int64))
        keys = gen.uniform_u32(gen.S0 + 40, int(off[-1]))
        out = _run(rs, keys, off, inplace=True)
        assert first_mismatch(out, orc.segmented(keys, off)) is None, lens


def test_shared_rounds_only_without_lsd(rs, orc):
    # AUTO sorts a segment of 2^17 keys by the four shared device-wide
    # rounds; LSD by one workgroup's own rounds (no shared round launched)
    import gen, torch
    n = (1 << 17) + 3
    keys = gen.uniform_u32(gen.S0 + 41, n)
    off = np.array([0, n], dtype=np.int64)
    ref = orc.segmented(keys, off)
    for algo, rounds in ((rs.RS_ALGO_AUTO, 4), (rs.RS_ALGO_LSD, 0)):
        rs.rs_profile_read()
        rs.rs_profile_enable(True)
        out = _run(rs, keys, off, algo)
        torch.cuda.synchronize()
        rs.rs_profile_enable(False)
        prof = rs.rs_profile_read()
        assert first_mismatch(out, ref) is None, algo
        assert rs.rs_get_stats().device_error == 0
        assert prof.get("seg_round", (0, 0.0))[0] == rounds, (algo, prof)


def test_invalid_offsets_reported(rs):
    import torch
    keys = torch.zeros(100, dtype=torch.int32, device="cuda")
    off = torch.tensor([0, 50, 40, 100], dtype=torch.int64, device="cuda")   # decreasing
    rs.rs_sort_segmented(keys, off)
    assert rs.rs_get_stats().device_error & 2
    # segments long enough for the shared device-wide rounds: one that ends
    # past the keys, and two valid ones that overlap (around an invalid one)
    # by more tiles than the rounds' tables hold; both are reported, and no
    # kernel touches memory outside the keys and the workspace
    n = (1 << 17) + 1000
    keys = torch.zeros(n, dtype=torch.int32, device="cuda")
    for o in ([0, n + 4096], [0, 1 << 17, 0, n]):
        rs.rs_sort_segmented(keys, torch.tensor(o, dtype=torch.int64, device="cuda"))
        assert rs.rs_get_stats().device_error & 2, o


def test_tuning_table_round_trip(rs, orc):
    import gen
    old = rs.rs_tune_get()
    try:
        rs.rs_tune_set([(c, rs.RS_ALGO_OET, max(1, (1 << c) // 32)) for c in range(1, 15)])
        assert all(e[1] == rs.RS_ALGO_OET for e in rs.rs_tune_get()[1:15])
        lens = np.array([3, 700, 9000, 16384], dtype=np.int64)
        off = _offsets(lens)
        keys = gen.uniform_u32(gen.S0 + 41, int(off[-1]))
        assert first_mismatch(_run(rs, keys, off), orc.segmented(keys, off)) is None
        with pytest.raises(rs.RsError):
            rs.rs_tune_set([(20, rs.RS_ALGO_BTN, 4)])
    finally:
        rs.rs_tune_set(old)


def test_full_config_65536_segments(rs, orc):
    """The batched workload: 65,536 segments with lengths log-uniform in
    [16, 2^20), about 6.2e9 uint32 keys, sorted in one persistent launch.
    Checked: 48 sampled segments bit for bit against the oracle; every
    segment sorted; every segment's multiset unchanged (a per-segment 64-bit
    multiset hash: keys moved between segments, or {1, 3} turned into
    {2, 2}, would show)."""
    import torch

    import gen
    S = 65536
    lens = gen.loguniform_lengths(gen.S0 + 4, S, 4.0, 20.0)
    off = _offsets(lens)
    total = int(off[-1])
    keys = torch.empty(total, dtype=torch.int32, device="cuda")
    gen.uniform_u32_dev(gen.S0 + 4, keys)
    offd = torch.from_numpy(off).cuda()
    out = torch.empty_like(keys)
    rs.rs_sort_segmented(keys, offd, keys_out=out)
    torch.cuda.synchronize()
    assert rs.rs_get_stats().device_error == 0
    # every segment sorted: a descent may only occur across a segment start
    starts = torch.zeros(total, dtype=torch.bool, device="cuda")
    starts[offd[1:-1]] = True
    bad = 0
    chunk = 1 << 28
    for a in range(0, total - 1, chunk):
        b = min(total, a + chunk + 1)
        x = out[a:b].to(torch.int64) & 0xFFFFFFFF
        desc = x[1:] < x[:-1]
        desc &= ~starts[a + 1:b]
        bad += int(desc.sum())
        del x, desc
    assert bad == 0
    # per-segment multisets unchanged
    segid = torch.repeat_interleave(torch.arange(S, device="cuda"), torch.from_numpy(lens).cuda())
    h_in = segment_hashes_dev(keys, segid, S)
    h_out = segment_hashes_dev(out, segid, S)
    bad = (h_in != h_out).nonzero()
    assert bad.numel() == 0, "segment %d changed its multiset" % int(bad[0])
    del segid, starts
    rng = np.random.default_rng(7)
    for s in np.concatenate([rng.choice(S, 40, replace=False), np.argsort(lens)[-4:], np.argsort(lens)[:4]]):
        a, b = int(off[s]), int(off[s + 1])
        seg_in = keys[a:b].cpu().numpy().view(np.uint32)
        seg_out = out[a:b].cpu().numpy().view(np.uint32)
        assert first_mismatch(seg_out, orc.lsd(seg_in, 8)) is None, (s, b - a)
