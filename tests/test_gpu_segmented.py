"""GPU parity of ak_segmented_sort against the oracle's per-segment sort."""
import zlib

import numpy as np
import pytest
import torch

import oracle
import paper_2507_16710_amd as ak
import synth
from gpucheck import fingerprint, segment_fingerprints, signed_order_key, to_gpu, to_host
from pools import DTYPES, bits, from_image, prefix_groups, random_keys

pytestmark = pytest.mark.gpu


def _seg(k: np.ndarray, off: np.ndarray, dt: str) -> np.ndarray:
    t = to_gpu(k, dt)
    o = torch.from_numpy(off.astype(np.int64)).cuda()
    ak.segmented_sort_(t, o, dtype=dt)
    torch.cuda.synchronize()
    return to_host(t, dt)


def _offsets(lengths) -> np.ndarray:
    return np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)


@pytest.mark.parametrize("dt", DTYPES)
def test_class_boundaries(dt):
    """Lengths at and around the short / medium / long class limits (with
    every tuning: 128/256 short, 2048/4096/8192 medium), empties and ones."""
    rng = np.random.default_rng(zlib.crc32(dt.encode()))
    lens = [0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 255, 256, 257, 0, 2047, 2048, 2049,
            4095, 4096, 4097, 8191, 8192, 8193, 12289, 70_001, 1, 0]
    lens = lens + list(rng.integers(0, 600, size=200))
    k = random_keys(dt, int(np.sum(lens)), rng, "mixed")
    off = _offsets(lens)
    assert np.array_equal(bits(_seg(k, off, dt)), bits(oracle.segsort(k, off)))


@pytest.mark.parametrize("dt", ["u32", "f64", "i64"])
def test_single_segment_equals_sort(dt):
    rng = np.random.default_rng(3)
    for n in [5, 4096, 100_000]:
        k = random_keys(dt, n, rng, "mixed")
        assert np.array_equal(bits(_seg(k, np.array([0, n]), dt)), bits(oracle.sort(k)))


def test_outside_range_untouched_and_repeated_calls():
    rng = np.random.default_rng(5)
    k = random_keys("u32", 50_000, rng, "uniform")
    off = np.array([1000, 1000, 5000, 20_000, 30_000], dtype=np.int64)
    got = _seg(k, off, "u32")
    assert np.array_equal(got[:1000], k[:1000]) and np.array_equal(got[30_000:], k[30_000:])
    assert np.array_equal(got, oracle.segsort(k, off))
    # replays of the captured graph with new pointers and new data
    for seed in range(3):
        k2 = random_keys("u32", 50_000, np.random.default_rng(100 + seed), "mixed")
        assert np.array_equal(_seg(k2, off, "u32"), oracle.segsort(k2, off))


def test_bad_offsets_reported():
    k = torch.zeros(100, dtype=torch.int32, device="cuda")
    off = torch.tensor([0, 50, 40, 100], dtype=torch.int64, device="cuda")
    ak.segmented_sort_(k, off, dtype="u32", check=False)
    with pytest.raises(ak.AKError):
        ak.check_device_error()
    ak.check_device_error()        # the flag was cleared
    lib = ak.load_library()
    assert lib.ak_segmented_sort(k.data_ptr(), off.data_ptr(), -1, 3, None) == 1
    bad_end = torch.tensor([10, 5], dtype=torch.int64, device="cuda")
    assert lib.ak_segmented_sort(k.data_ptr(), bad_end.data_ptr(), 1, 3, None) == 1


def test_workload4_scaled():
    """Lognormal segment sizes (clip [16, 2**20], mean 5000), uniform uint32
    keys: 4,000 segments."""
    keys, off = synth.workload4(nseg=4000, seed=2)
    k = keys.numpy().view(np.uint32)
    assert np.array_equal(_seg(k, off.numpy(), "u32"), oracle.segsort(k, off.numpy()))


def test_segmented_sort_returns_before_the_device_finishes():
    """The segmented sort never waits for the device (ak_segmented_sort_n:
    the batch's ends are read on the device): right after the call on the
    100,000-segment batch the stream still has work, and the result is
    every segment sorted with its own multiset."""
    keys, off = synth.workload4(device="cuda")
    nseg = off.numel() - 1
    seg_id = torch.repeat_interleave(torch.arange(nseg, device="cuda"), off[1:] - off[:-1])
    seg_fp = segment_fingerprints(keys, seg_id, nseg)
    work = keys.clone()
    ak.segmented_sort_(work, off, dtype="u32")        # scratch and graph ready
    work.copy_(keys)
    torch.cuda.synchronize()
    ak.segmented_sort_(work, off, dtype="u32", check=False)
    busy = not torch.cuda.current_stream().query()
    torch.cuda.synchronize()
    ak.check_device_error()
    assert busy, "the call waited for the device"
    assert torch.equal(segment_fingerprints(work, seg_id, nseg), seg_fp)
    k = signed_order_key(work, "u32")
    same = seg_id[1:] == seg_id[:-1]
    assert bool((k[1:][same] >= k[:-1][same]).all())


def test_workload4_full_size():
    """100,000 segments, ~5e8 keys: every segment sorted (GPU check), the
    multiset kept, and a sample of segments equal to the oracle's."""
    keys, off = synth.workload4(device="cuda")
    orig = keys.clone()
    fp = fingerprint(keys)
    nseg = off.numel() - 1
    seg_id = torch.repeat_interleave(torch.arange(nseg, device="cuda"), off[1:] - off[:-1])
    seg_fp = segment_fingerprints(keys, seg_id, nseg)
    ak.segmented_sort_(keys, off, dtype="u32")
    torch.cuda.synchronize()
    assert fingerprint(keys) == fp
    # every segment keeps its own multiset (a key moved between segments
    # would change two rows)
    assert torch.equal(segment_fingerprints(keys, seg_id, nseg), seg_fp)
    k = signed_order_key(keys, "u32")
    same = seg_id[1:] == seg_id[:-1]
    assert bool((k[1:][same] >= k[:-1][same]).all())
    offh = off.cpu().numpy()
    lens = np.diff(offh)
    pick = list(np.argsort(lens)[-3:]) + list(np.random.default_rng(0).integers(0, lens.size, 50))
    for s in pick:
        a, b = int(offh[s]), int(offh[s + 1])
        src = to_host(orig[a:b], "u32")
        assert np.array_equal(to_host(keys[a:b], "u32"), oracle.sort(src)), s


@pytest.mark.parametrize("dt", ["u32", "f64", "i64"])
def test_huge_segments_under_tunings(dt):
    """Segments above the many-workgroup threshold (several thresholds),
    including constant ones and ones where only the lowest byte varies
    (one active pass: the result ends in the scratch copy)."""
    rng = np.random.default_rng(17)
    lens = [40_000, 100_000, 5_000, 70_000, 65_536, 9000, 0, 33_000]
    parts = []
    for i, L in enumerate(lens):
        if i == 3:
            parts.append(np.full(L, random_keys(dt, 1, rng, "uniform")[0]))
        elif i == 4:
            parts.append((rng.integers(0, 200, size=L)).astype(bits(random_keys(dt, 1, rng)).dtype)
                         .view(random_keys(dt, 1, rng).dtype))
        else:
            parts.append(random_keys(dt, L, rng, "mixed"))
    k = np.concatenate(parts)
    off = _offsets(lens)
    kb = 32 if dt in ("u32", "i32", "f32") else 64
    try:
        for xl in (4096, 32768, 1 << 20):
            ak.seg_set_tuning(kb, 4, 16, 4, 0, xl)
            assert np.array_equal(bits(_seg(k, off, dt)), bits(oracle.segsort(k, off))), xl
    finally:
        ak.seg_set_tuning(kb, 4, 16, 4, 0, 32768)


@pytest.mark.parametrize("dt", DTYPES)
def test_on_chip_prefix_groups(dt):
    """On-chip classes (short, medium, big): segments whose keys spread
    over every bit, shaped in image bits so that after ordering by the top
    8 (segments of up to 256 keys) or 16 varying bits the groups of equal
    prefix hold at most 16 keys (each key placed by comparisons inside its
    group), or one group holds 17 (the segment then takes the passes over
    every varying bit), with equal keys inside groups."""
    rng = np.random.default_rng(zlib.crc32(b"groups" + dt.encode()))
    w = 32 if dt in ("i32", "u32", "f32") else 64
    lens, parts = [], []
    for L in [40, 200, 256, 257, 1000, 2048, 2049, 4096, 4097, 8192, 12_000, 16_384]:
        t = 8 if L <= 256 else 16
        for long_group in (0, 17, 16 * 3):
            lens.append(L)
            parts.append(from_image(prefix_groups(L, w, t, 16, rng, long_group), dt))
        lens.append(L)
        parts.append(random_keys(dt, L, rng, "uniform"))
    k = np.concatenate(parts)
    off = _offsets(lens)
    assert np.array_equal(bits(_seg(k, off, dt)), bits(oracle.segsort(k, off)))


@pytest.mark.parametrize("dt", DTYPES)
def test_huge_segments_shaped_keys(dt):
    """Huge segments (above 16384 keys) shaped in image bits: uniform keys,
    one top-byte bucket of exactly 8192 keys and one of 8193, keys below
    2^20 (the top byte constant: its place is skipped), a segment one key
    above the class limit, and keys repeated 60 times."""
    rng = np.random.default_rng(zlib.crc32(b"hugeshaped" + dt.encode()))
    w = 32 if dt in ("i32", "u32", "f32") else 64
    ub = np.uint32 if w == 32 else np.uint64
    top = np.uint64(w - 8)

    def img_uniform(n, bits_=w):
        v = rng.integers(0, 1 << min(bits_, 63), size=n, dtype=np.uint64)
        if bits_ == 64:
            v ^= rng.integers(0, 2, size=n, dtype=np.uint64) << np.uint64(63)
        return v.astype(ub)

    def img_bucket(n, big):
        v = img_uniform(n)
        v[:big] = (v[:big] & ub((1 << (w - 8)) - 1)) | (ub(0x80) << ub(top))
        rest = v[big:]
        hit = (rest >> ub(top)) == ub(0x80)
        rest[hit] ^= ub(1) << ub(top)       # no other key in that bucket
        rng.shuffle(v)
        return v

    segs = [img_uniform(40_000), img_uniform(300_000), img_bucket(40_000, 8192), img_bucket(40_000, 8193),
            img_uniform(70_000, 20), img_uniform(16_385), np.repeat(img_uniform(500), 60)]
    lens = [int(x.size) for x in segs]
    k = np.concatenate([from_image(x, dt) for x in segs])
    off = _offsets(lens)
    assert np.array_equal(bits(_seg(k, off, dt)), bits(oracle.segsort(k, off)))
