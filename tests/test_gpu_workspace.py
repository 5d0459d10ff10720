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
    n = 300_001
    lens = [5, 70_000, 0, 3000, 150_000, 1, 77_000 - 5]
    off = _offsets(lens)
    nseg = len(lens)
    need = max(ak.temp_bytes("sort", n, dt), ak.temp_bytes("sortperm", n, dt),
               ak.temp_bytes_segmented(int(off[-1]), nseg, dt), ak.temp_bytes("learned", n, dt))
    arena = torch.empty(need, dtype=torch.uint8, device="cuda")
    ak.set_workspace(arena)
    try:
        for it in range(2):   # the second round reuses the arena's carving
            k = random_keys(dt, n, rng, "mixed")
            print(f"arena dt={dt} round={it} sort", flush=True)
            t = to_gpu(k, dt)
            ak.sort_(t, dtype=dt)
            assert np.array_equal(bits(to_host(t, dt)), bits(oracle.sort(k)))
            print(f"arena dt={dt} round={it} sortperm", flush=True)
            t = to_gpu(k, dt)
            p = ak.sortperm(t, dtype=dt)
            assert np.array_equal(p.cpu().numpy().view(np.uint32), oracle.sortperm(k))
            print(f"arena dt={dt} round={it} segmented", flush=True)
            ks = k[: int(off[-1])]
            t = to_gpu(ks, dt)
            ak.segmented_sort_(t, torch.from_numpy(off).cuda(), dtype=dt)
            assert np.array_equal(bits(to_host(t, dt)), bits(oracle.segsort(ks, off)))
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
