"""GPU parity of ak_sort / ak_sortperm against the oracle (bit-exact).

Sizes cover the single-workgroup path (<= 4096 keys), several one-sweep tiles
with ragged tails, and the workload shapes; full-size workloads are checked
through sampled ranks and properties that hold at any size.
"""
import zlib

import numpy as np
import pytest
import torch

import oracle
import paper_2507_16710_amd as ak
import synth
from gpucheck import (check_perm_sorts_stably, fingerprint, is_sorted, rank_checks, to_gpu, to_host)
from pools import DTYPES, bits, random_keys

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 64, 1000, 4095, 4096, 4097, 3071, 3073, 12289, 65536 + 7, 300_001]


def _run_sort(k: np.ndarray, dt: str) -> np.ndarray:
    t = to_gpu(k, dt)
    ak.sort_(t, dtype=dt)
    torch.cuda.synchronize()
    return to_host(t, dt)


def _run_perm(k: np.ndarray, dt: str) -> np.ndarray:
    t = to_gpu(k, dt)
    before = to_host(t, dt).copy()
    p = ak.sortperm(t, dtype=dt)
    torch.cuda.synchronize()
    assert np.array_equal(bits(to_host(t, dt)), bits(before)), "sortperm modified its keys"
    return p.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("kind", ["mixed", "uniform", "ties"])
def test_sort_bit_exact(dt, kind):
    rng = np.random.default_rng(zlib.crc32(f"{dt}{kind}s".encode()))
    for n in SIZES:
        k = random_keys(dt, n, rng, kind)
        print(f"sort dt={dt} kind={kind} n={n}", flush=True)
        got = _run_sort(k, dt)
        assert np.array_equal(bits(got), bits(oracle.sort(k))), (dt, kind, n)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("kind", ["mixed", "ties"])
def test_sortperm_exact(dt, kind):
    rng = np.random.default_rng(zlib.crc32(f"{dt}{kind}p".encode()))
    for n in SIZES:
        k = random_keys(dt, n, rng, kind)
        print(f"sortperm dt={dt} kind={kind} n={n}", flush=True)
        assert np.array_equal(_run_perm(k, dt), oracle.sortperm(k)), (dt, kind, n)


@pytest.mark.parametrize("dt", ["i64", "f32", "u32"])
def test_degenerate_inputs(dt):
    rng = np.random.default_rng(1)
    for n in [5000, 70_000]:
        base = random_keys(dt, 3, rng, "uniform")
        const = np.full(n, base[0])
        assert np.array_equal(bits(_run_sort(const, dt)), bits(const))
        assert np.array_equal(_run_perm(const, dt), np.arange(n, dtype=np.uint32))
        srt = oracle.sort(random_keys(dt, n, rng, "mixed"))
        assert np.array_equal(bits(_run_sort(srt, dt)), bits(srt))
        rev = srt[::-1].copy()
        assert np.array_equal(_run_perm(rev, dt), oracle.sortperm(rev))
        # only the lowest byte varies: one active pass, odd count -> copy back
        lowbyte = (np.arange(n) % 7).astype(np.int64).astype(bits(const).dtype).view(const.dtype)
        assert np.array_equal(bits(_run_sort(lowbyte, dt)), bits(oracle.sort(lowbyte)))
    # n == 0: nothing launched, no error
    t = torch.empty(0, dtype=torch.int64, device="cuda")
    ak.sort_(t, dtype="i64")
    assert ak.sortperm(t, dtype="i64").numel() == 0


def test_argument_errors():
    t = torch.zeros(10, dtype=torch.int64, device="cuda")
    lib = ak.load_library()
    assert lib.ak_sort(t.data_ptr(), -1, 2, None) == 1
    assert lib.ak_sort(None, 10, 2, None) == 1
    assert lib.ak_sort(t.data_ptr(), 10, 99, None) == 2
    assert lib.ak_sort(t.data_ptr(), 1 << 32, 2, None) == 1
    assert lib.ak_sortperm(t.data_ptr(), t.data_ptr(), 10, 2, None) == 1     # overlap
    assert lib.ak_sortperm(t.data_ptr(), None, 10, 2, None) == 1
    assert lib.ak_sort(t.data_ptr(), 0, 2, None) == 0
    with pytest.raises(ak.AKError):
        ak._check(lib.ak_sort(t.data_ptr(), -5, 2, None), "ak_sort")
    with pytest.raises(TypeError):
        ak.sort_(t, dtype="f32")         # 8-byte elements declared as f32


def test_workload1_full():
    """1,000,000 uniform int64 keys: sort and sortperm, full size."""
    k = synth.as_numpy(synth.workload1(), "i64")
    assert np.array_equal(_run_sort(k, "i64"), oracle.sort(k))
    assert np.array_equal(_run_perm(k, "i64"), oracle.sortperm(k))


def test_workload2_scaled():
    """float32 N(0,1e3) with NaN / signed zero / Inf injections, 2**22 keys."""
    k = synth.as_numpy(synth.workload2(n=1 << 22), "f32")
    assert np.array_equal(bits(_run_sort(k, "f32")), bits(oracle.sort(k)))
    assert np.array_equal(_run_perm(k, "f32"), oracle.sortperm(k))


@pytest.mark.parametrize("variant", ["uniform", "zipf", "lognormal"])
def test_workload3_scaled(variant):
    k = synth.as_numpy(synth.workload3(variant, n=1 << 22), "i64")
    assert np.array_equal(_run_sort(k, "i64"), oracle.sort(k))
    assert np.array_equal(_run_perm(k, "i64"), oracle.sortperm(k))


def test_workload2_full_size_properties():
    """2**28 float32 keys with specials, in the benchmark's launch shape."""
    t = synth.workload2(device="cuda")
    fp = fingerprint(t)
    keys = t.clone()
    perm = ak.sortperm(keys, dtype="f32")
    ak.sort_(t, dtype="f32")
    torch.cuda.synchronize()
    assert is_sorted(t, "f32") and fingerprint(t) == fp
    assert torch.equal(torch.isnan(t[-(t.numel() // 1000):]).all(), torch.tensor(True, device="cuda"))
    check_perm_sorts_stably(keys, perm, "f32")
    assert torch.equal(keys[perm.to(torch.int64) & 0xFFFFFFFF].view(torch.int32), t.view(torch.int32))
    rank_checks(keys, t, "f32", samples=16)


@pytest.mark.parametrize("variant", ["uniform", "zipf", "lognormal"])
def test_workload3_full_size_properties(variant):
    """One GPU's share: 2**30 int64 keys (8 GiB)."""
    t = synth.workload3(variant, device="cuda")
    keys = t.clone()
    fp = fingerprint(t)
    ak.sort_(t, dtype="i64")
    torch.cuda.synchronize()
    assert is_sorted(t, "i64") and fingerprint(t) == fp
    rank_checks(keys, t, "i64", samples=8)
    # the sorted sample equals the oracle's sort of the same sample
    idx = torch.arange(0, keys.numel(), 4099, device="cuda")
    sub = to_host(keys[idx], "i64")
    del keys
    t2 = to_gpu(sub, "i64")
    ak.sort_(t2, dtype="i64")
    assert np.array_equal(to_host(t2, "i64"), oracle.sort(sub))


def test_repeat_determinism():
    rng = np.random.default_rng(4)
    k = random_keys("f32", 200_000, rng, "mixed")
    first = _run_perm(k, "f32")
    for _ in range(5):
        assert np.array_equal(_run_perm(k, "f32"), first)


@pytest.mark.parametrize("dt", ["u32", "i32", "u64", "i64"])
def test_active_pass_counts(dt):
    """Keys whose images vary in exactly the q lowest bytes, for every q:
    the device skips the other places, and an odd number of active passes
    ends in the caller's buffer through the second scratch buffer (one pass:
    through the copy back).  Both the graph-replayed size range and the
    direct launch (n > 2**22) are covered."""
    kb = 4 if dt in ("u32", "i32") else 8
    rng = np.random.default_rng(zlib.crc32(f"{dt}q".encode()))
    np_dt = {"u32": np.uint32, "i32": np.int32, "u64": np.uint64, "i64": np.int64}[dt]
    for q in range(1, kb + 1):
        for n in (12289, 300_001, (1 << 22) + 5):
            hi = 1 << (8 * q)
            if q == kb:
                k = rng.integers(np.iinfo(np_dt).min, np.iinfo(np_dt).max, size=n, dtype=np_dt, endpoint=True)
            else:
                k = rng.integers(0, hi, size=n, dtype=np.uint64).astype(np_dt)
            print(f"active places dt={dt} q={q} n={n}", flush=True)
            got = _run_sort(k, dt)
            assert np.array_equal(bits(got), bits(oracle.sort(k))), (dt, q, n)
            if n == 300_001 and q in (1, 3):
                assert np.array_equal(_run_perm(k, dt), oracle.sortperm(k)), (dt, q, n)


@pytest.mark.parametrize("dt", ["u32", "u64"])
def test_histogram_folds_on_skewed_keys(dt):
    """Sizes at which every histogram workgroup folds its 16-bit LDS counts
    into registers several times (above 2**28 64-bit and 2**29 32-bit keys
    at one workgroup per CU), on keys whose top bytes are constant and whose
    lowest byte is 0x55 for half of them: one bin of each constant place
    takes every count, so a wrapped count would show as wrong digit offsets
    or a constant place taken for active.  Exactly the three low places
    run."""
    kb = 4 if dt == "u32" else 8
    n = (5 << 28) + 12345 if kb == 4 else (5 << 27) + 12345
    g = torch.Generator(device="cuda").manual_seed(77)
    low = torch.randint(0, 1 << 24, (n,), generator=g, device="cuda", dtype=torch.int64)
    half = torch.rand(n, generator=g, device="cuda") < 0.5
    low = torch.where(half, (low & ~0xFF) | 0x55, low)
    if kb == 4:
        t = (low | (0xAB << 24)).to(torch.int32)
    else:
        t = low | (0x123456789A << 24)
    del low, half
    fp = fingerprint(t)
    print(f"histogram folds dt={dt} n={n}", flush=True)
    ak.sort_(t, dtype=dt)
    route = ak.sort_route()
    assert route["passes"] == 3 and route["prefix_places"] == 0, route
    assert is_sorted(t, dt) and fingerprint(t) == fp
