"""Host checks of the test helpers' multiset hashes: the torch form (used on
the device for the full-size workloads) gives the same bits as the numpy
form, and a per-row hash tells apart multisets that per-row sums do not."""
import numpy as np

from gpu_util import _mix64, mix64_dev, multiset_hash, multiset_hash_rows_dev, segment_hashes_dev


def test_torch_mix_matches_numpy():
    import torch
    rng = np.random.default_rng(1)
    u = rng.integers(0, 2**63, 5000, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 5000).astype(np.uint64)
    t = torch.from_numpy(u.view(np.int64).copy())
    with np.errstate(over="ignore"):
        ref = _mix64(u)
    assert np.array_equal(mix64_dev(t).numpy().view(np.uint64), ref)


def test_row_and_segment_hashes():
    import torch
    rng = np.random.default_rng(2)
    a = rng.integers(0, 2**32, (6, 100), dtype=np.uint64).astype(np.uint32)
    t = torch.from_numpy(a.view(np.int32).copy())
    rows = multiset_hash_rows_dev(t).numpy().view(np.uint64)
    for r in range(6):
        assert int(rows[r]) == multiset_hash(a[r])
        assert int(rows[r]) == int(multiset_hash_rows_dev(torch.from_numpy(
            rng.permutation(a[r]).view(np.int32).copy())[None, :])[0].numpy().view(np.uint64))
    # {1, 3} and {2, 2}: equal sums, different multisets
    x = torch.tensor([[1, 3], [2, 2]], dtype=torch.int32)
    h = multiset_hash_rows_dev(x)
    assert int(h[0]) != int(h[1])
    seg = torch.tensor([0, 0, 1, 1])
    hs = segment_hashes_dev(torch.tensor([1, 3, 2, 2], dtype=torch.int32), seg, 2, chunk=3)
    assert torch.equal(hs, h)
