"""CPU checks of the test-side property helpers used at full sizes: each
rejects the mistake it exists to catch."""
import numpy as np
import torch

from gpucheck import fingerprint, segment_fingerprints


def test_segment_fingerprints_catch_a_key_moved_between_segments():
    rng = np.random.default_rng(0)
    lens = np.array([5, 0, 9, 3, 12])
    keys = torch.from_numpy(rng.integers(0, 1 << 31, size=int(lens.sum())).astype(np.int32))
    seg_id = torch.repeat_interleave(torch.arange(lens.size), torch.from_numpy(lens))
    ref = segment_fingerprints(keys, seg_id, lens.size)
    assert ref[:, 0].tolist() == lens.tolist()
    # a permutation inside every segment keeps every row
    perm = torch.cat([torch.randperm(int(L)) + int(o) for L, o in zip(lens, np.r_[0, np.cumsum(lens)[:-1]])])
    assert torch.equal(segment_fingerprints(keys[perm], seg_id, lens.size), ref)
    # swapping two keys across a segment boundary keeps the global multiset
    # but changes the rows of both segments
    moved = keys.clone()
    moved[4], moved[5] = keys[5].item(), keys[4].item()
    assert fingerprint(moved) == fingerprint(keys)
    got = segment_fingerprints(moved, seg_id, lens.size)
    assert not torch.equal(got[0], ref[0]) and not torch.equal(got[2], ref[2])
    assert torch.equal(got[3:], ref[3:])
