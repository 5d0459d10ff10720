"""GPU checks of the caller-owned scratch arena (ak_set_workspace): every
path sorts bit-exactly from an arena of ak_temp_bytes, a too-small arena is
refused before anything is launched (the keys stay as they were), and the
library's own scratch works again after unbinding."""
import zlib

import numpy as np
import pytest
import torch

import oracle
import paper_2507_16710_amd as ak
from gpucheck import to_gpu, to_host
from pools import bits, random_keys

pytestmark = pytest.mark.gpu


def _offsets(lengths) -> np.ndarray:
    return np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)


@pytest.mark.parametrize("dt", ["u64", "f32"])
def test_arena_paths_bit_exact(dt):
    rng = np.random.default_rng(zlib.crc32(f"arena{dt}".encode()))

    def segments(n):
        # segment lengths summing to n: tiny, empty, one-workgroup and huge ones
        lens = [5, n // 4, 0, 3000, n // 2, 1]
        return _offsets(lens + [n - sum(lens)])

    n = 300_001
    nseg = len(segments(n)) - 1
    need = max(ak.temp_bytes("sort", n, dt), ak.temp_bytes("sortperm", n, dt),
               ak.temp_bytes_segmented(n, nseg, dt), ak.temp_bytes("learned", n, dt),
               ak.temp_bytes("sort_by_key", n, dt), ak.temp_bytes("sortperm_lowmem", n, dt))
    arena = torch.empty(need, dtype=torch.uint8, device="cuda")
    ak.set_workspace(arena)
    try:
        for it in range(2):   # the second round reuses the arena's carving
            off = segments(n)
            assert int(off[-1]) == n
            k = random_keys(dt, n, rng, "mixed")
            print(f"arena dt={dt} round={it} sort", flush=True)
            t = to_gpu(k, dt)
            ak.sort_(t, dtype=dt)
            assert np.array_equal(bits(to_host(t, dt)), bits(oracle.sort(k)))
            print(f"arena dt={dt} round={it} sortperm", flush=True)
            t = to_gpu(k, dt)
            p = ak.sortperm(t, dtype=dt)
            assert np.array_equal(p.cpu().numpy().view(np.uint32), oracle.sortperm(k))
            print(f"arena dt={dt} round={it} sortperm_lowmem", flush=True)
            p = ak.sortperm_lowmem(t, dtype=dt)
            assert np.array_equal(p.cpu().numpy().view(np.uint32), oracle.sortperm(k))
            print(f"arena dt={dt} round={it} sort_by_key", flush=True)
            t = to_gpu(k, dt)
            v = torch.arange(k.size, dtype=torch.int64, device="cuda") * 3 - 7
            ak.sort_by_key_(t, v, dtype=dt)
            rk, rv = oracle.sort_by_key(k, (np.arange(k.size, dtype=np.int64) * 3 - 7))
            assert np.array_equal(bits(to_host(t, dt)), bits(rk)) and np.array_equal(v.cpu().numpy(), rv)
            print(f"arena dt={dt} round={it} segmented", flush=True)
            t = to_gpu(k, dt)
            ak.segmented_sort_(t, torch.from_numpy(off).cuda(), dtype=dt)
            assert np.array_equal(bits(to_host(t, dt)), bits(oracle.segsort(k, off)))
            print(f"arena dt={dt} round={it} learned", flush=True)
            t = to_gpu(k, dt)
            ak.sort_learned_(t, dtype=dt)
            assert np.array_equal(bits(to_host(t, dt)), bits(oracle.sort(k)))
            n = n // 3   # smaller second round
        torch.cuda.synchronize()
        # too small: refused before any launch, keys untouched
        small = torch.empty(8192, dtype=torch.uint8, device="cuda")
        ak.set_workspace(small)
        k = random_keys(dt, 100_000, rng, "mixed")
        t = to_gpu(k, dt)
        with pytest.raises(ak.AKError) as e:
            ak.sort_(t, dtype=dt)
        assert e.value.status == 3
        torch.cuda.synchronize()
        assert np.array_equal(bits(to_host(t, dt)), bits(k))
        with pytest.raises(ak.AKError):
            ak.sort_learned_(t, dtype=dt)
        assert np.array_equal(bits(to_host(t, dt)), bits(k))
    finally:
        ak.set_workspace(None)
    # library-owned scratch again
    t = to_gpu(k, dt)
    ak.sort_(t, dtype=dt)
    assert np.array_equal(bits(to_host(t, dt)), bits(oracle.sort(k)))


def test_segment_offsets_beyond_keys_are_refused():
    """Offsets that run past the key array (or start below 0) are found on
    the device against the key count the call is given: the error word is
    set and no key is touched."""
    t = torch.arange(1000, 0, -1, dtype=torch.int64, device="cuda")
    before = t.clone()
    off = torch.tensor([0, 500, 2000], dtype=torch.int64, device="cuda")
    with pytest.raises(ak.AKError):
        ak.segmented_sort_(t, off, dtype="i64")
    off = torch.tensor([-1, 500], dtype=torch.int64, device="cuda")
    with pytest.raises(ak.AKError):
        ak.segmented_sort_(t, off, dtype="i64")
    assert torch.equal(t, before)
    ak.check_device_error()                      # cleared by the raise


def test_arena_prefix_route_exact_size():
    """Key-only sorts above 2**22 keys take the prefix route with the
    segmented fallback, whose run lists and scratch come from the arena too:
    an arena of exactly ak_temp_bytes("sort", n) suffices, with and without
    fallback runs."""
    rng = np.random.default_rng(41)
    n = (1 << 22) + 777
    need = ak.temp_bytes("sort", n, "u64")
    arena = torch.empty(need, dtype=torch.uint8, device="cuda")
    ak.set_workspace(arena)
    try:
        for heavy_frac in (0.0, 0.002):
            k = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
            if heavy_frac:
                h = rng.random(n) < heavy_frac
                k[h] = (np.uint64(0x7777) << np.uint64(48)) | (k[h] & np.uint64((1 << 48) - 1))
            print(f"arena prefix heavy={heavy_frac}", flush=True)
            t = to_gpu(k, "u64")
            ak.sort_(t, dtype="u64")
            route = ak.sort_route()
            assert route["prefix_places"] >= 2, route
            if heavy_frac:
                assert route["fallback_runs"] >= 1, route
            assert np.array_equal(to_host(t, "u64"), oracle.sort(k))
    finally:
        ak.set_workspace(None)


def test_arena_accumulate_exact_size():
    """Prefix sums take their chunk totals from the arena: exactly
    ak_temp_bytes("accumulate", n) suffices, and one byte less than a
    256-byte block is refused before any launch."""
    rng = np.random.default_rng(43)
    n = 3 * 4096 * 1000 + 11
    need = ak.temp_bytes("accumulate", n, "i64")
    assert need >= ((n + 4095) // 4096) * 8
    x = rng.integers(-(1 << 40), 1 << 40, size=n, dtype=np.int64)
    arena = torch.empty(need, dtype=torch.uint8, device="cuda")
    ak.set_workspace(arena)
    try:
        print(f"arena accumulate n={n} bytes={need}", flush=True)
        got = ak.accumulate(to_gpu(x, "i64"), True, dtype="i64")
        assert np.array_equal(to_host(got, "i64"), oracle.accumulate(x, True))
    finally:
        ak.set_workspace(None)
    small = torch.empty(max(4096, need - 256), dtype=torch.uint8, device="cuda")
    ak.set_workspace(small)
    try:
        with pytest.raises(ak.AKError):
            ak.accumulate(to_gpu(x, "i64"), True, dtype="i64")
    finally:
        ak.set_workspace(None)


def test_arena_lookback_words_reused_then_refilled():
    """In a bound arena the radix passes' look-back words are zero-filled
    only when their bytes last held other data: back-to-back sorts reuse
    them (earlier runs' words carry older epochs), and after a segmented
    sort has carved its own buffers over them the next sort fills them
    again.  Every result is bit-exact."""
    rng = np.random.default_rng(47)
    n = 1_000_003
    need = max(ak.temp_bytes("sort", n, "u64"), ak.temp_bytes_segmented(n, 3, "u64"))
    arena = torch.empty(need, dtype=torch.uint8, device="cuda")
    ak.set_workspace(arena)
    try:
        for it in range(6):
            k = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
            if it % 2:
                k >>= np.uint64(rng.integers(8, 40))      # fewer active places
            t = to_gpu(k, "u64")
            print(f"arena look-back reuse it={it}", flush=True)
            ak.sort_(t, dtype="u64")
            assert np.array_equal(to_host(t, "u64"), oracle.sort(k)), it
            if it == 2:
                off = _offsets([n // 3, n // 3, n - 2 * (n // 3)])
                s = to_gpu(k, "u64")
                ak.segmented_sort_(s, torch.from_numpy(off).cuda(), dtype="u64")
                assert np.array_equal(to_host(s, "u64"), oracle.segsort(k, off))
    finally:
        ak.set_workspace(None)
