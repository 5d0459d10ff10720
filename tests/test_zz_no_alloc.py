"""ak_sort_noalloc (scratch in a static device array, no allocation) against
ak_sort, through the C ABI: bit-exact on two calls in a row, the second on
fewer keys, for every dtype; the size limit is refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2507_16710_amd as ak
from gpucheck import to_gpu, to_host
from pools import DTYPES, bits, random_keys

pytestmark = pytest.mark.gpu

MAX_BYTES = 1 << 24


def _run(fn, k: np.ndarray, dt: str) -> np.ndarray:
    lib = ak.load_library()
    t = to_gpu(k, dt)
    st = getattr(lib, fn)(t.data_ptr(), t.numel(), ak.DTYPE_CODE[dt], torch.cuda.current_stream().cuda_stream)
    assert st == 0, (fn, st, lib.ak_last_error())
    torch.cuda.synchronize()
    return to_host(t, dt)


@pytest.mark.parametrize("dt", DTYPES)
def test_noalloc_matches_sort_two_calls(dt):
    rng = np.random.default_rng(21)
    kb = 8 if dt in ("i64", "u64", "f64") else 4
    n_max = MAX_BYTES // kb
    for n, kind in [(n_max, "mixed"), (300_001, "ties"), (4097, "uniform"), (777, "mixed"), (n_max - 1, "uniform")]:
        k = random_keys(dt, n, rng, kind)
        got = _run("ak_sort_noalloc", k, dt)
        ref = _run("ak_sort", k, dt)
        assert np.array_equal(bits(got), bits(ref)), (dt, n, kind)
    # a small case against the oracle too
    k = random_keys(dt, 50_000, rng, "mixed")
    assert np.array_equal(bits(_run("ak_sort_noalloc", k, dt)), bits(oracle.sort(k)))


def test_noalloc_limit_refused():
    lib = ak.load_library()
    t = torch.zeros(4, dtype=torch.int64, device="cuda")
    before = t.clone()
    assert lib.ak_sort_noalloc(t.data_ptr(), MAX_BYTES // 8 + 1, 2, None) == 1
    assert lib.ak_sort_noalloc(t.data_ptr(), MAX_BYTES // 4 + 1, 3, None) == 1
    assert b"at most" in lib.ak_last_error()
    assert lib.ak_sort_noalloc(t.data_ptr(), 0, 2, None) == 0
    torch.cuda.synchronize()
    assert torch.equal(t, before)


def test_noalloc_interleaved_with_workspace_calls():
    """The static array and the per-stream workspaces are independent:
    interleaved calls of both entry points on one stream stay bit-exact."""
    rng = np.random.default_rng(5)
    for i in range(3):
        k = random_keys("u64", 1_000_000 - 1000 * i, rng, "mixed")
        a = _run("ak_sort_noalloc", k, "u64")
        b = _run("ak_sort", k, "u64")
        assert np.array_equal(a, b)
