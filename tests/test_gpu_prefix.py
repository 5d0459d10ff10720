"""GPU parity of the prefix-partitioned radix sort (bit-exact vs the oracle).

A key-only sort of more than 2**16 keys whose top digit places spread the
keys takes passes over those places only; each run of equal prefix is then
sorted on chip, and runs longer than a chunk by the segmented sort (above
2**22 keys) or by one workgroup each (at the sizes replayed from a captured
graph).  The route is read back with ak_sort_route, so every case checks
both the order and the route it expects.
"""
import zlib

import numpy as np
import pytest
import torch

import oracle
import paper_2507_16710_amd as ak
from gpucheck import fingerprint, is_sorted, rank_checks, to_gpu, to_host
from pools import bits, random_keys

pytestmark = pytest.mark.gpu

N0 = (1 << 22) + 777  # just above the sizes that replay a captured graph
CHUNK = 2048          # keys one on-chip chunk sort holds


def _sort_route(k: np.ndarray, dt: str):
    t = to_gpu(k, dt)
    ak.sort_(t, dtype=dt)
    route = ak.sort_route()
    return to_host(t, dt), route


def _check(k, dt, tag):
    print(f"prefix {tag} dt={dt} n={k.size}", flush=True)
    got, route = _sort_route(k, dt)
    assert np.array_equal(bits(got), bits(oracle.sort(k))), (tag, dt, k.size)
    return route


@pytest.mark.parametrize("dt", ["u64", "i64", "f64", "u32", "i32", "f32"])
def test_uniform_keys_take_prefix_route(dt):
    """Random bits in every place: two prefix places leave runs of about
    n / 2**16 keys, so two passes and the chunk sorts finish the sort."""
    rng = np.random.default_rng(zlib.crc32(f"pfx{dt}".encode()))
    for n in (N0, (1 << 23) + 12345):
        k = random_keys(dt, n, rng, "uniform")
        route = _check(k, dt, "uniform")
        assert route["prefix_places"] == 2 and route["passes"] == 2, route
        assert route["chunks"] > 0, route


def test_heavy_prefix_goes_to_fallback():
    """0.1% of the keys share one 16-bit prefix: the per-place counts look
    uniform (prefix chosen), but that run exceeds a chunk and is sorted by
    the segmented sort."""
    rng = np.random.default_rng(11)
    n = (1 << 22) + 4321
    k = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    heavy = rng.random(n) < 0.001
    k[heavy] = (np.uint64(0xA5C3) << np.uint64(48)) | (k[heavy] & np.uint64((1 << 48) - 1))
    route = _check(k, "u64", "heavy")
    assert route["prefix_places"] == 2, route
    assert route["fallback_runs"] >= 1 and route["fallback_keys"] > CHUNK, route


def test_constant_place_inside_prefix():
    """Byte 6 is constant: the prefix spans bytes 6..7 (two places, one of
    them inactive), so one pass plus the chunk sorts."""
    rng = np.random.default_rng(12)
    n = N0
    k = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    k = (k & ~np.uint64(0xFF << 48)) | np.uint64(0x5A << 48)
    route = _check(k, "u64", "inactive")
    assert route["prefix_places"] >= 2 and route["passes"] == route["prefix_places"] - 1, route


def test_skewed_and_small_keys_take_plain_passes():
    """Keys whose top places are mostly zero (80% below 2**20, the rest
    random bits) and keys with few distinct values keep every active pass."""
    rng = np.random.default_rng(13)
    k = rng.integers(0, 1 << 64, size=N0, dtype=np.uint64).view(np.int64)
    small = rng.random(N0) < 0.8
    k[small] = rng.integers(0, 1 << 20, size=int(small.sum()), dtype=np.int64)
    route = _check(k, "i64", "skewed")
    assert route["prefix_places"] == 0 and route["passes"] == 8, route
    k = random_keys("f64", N0, rng, "mixed")
    route = _check(k, "f64", "mixed")
    assert route["prefix_places"] == 0, route
    k = np.full(N0, 77, dtype=np.uint64)
    route = _check(k, "u64", "constant")
    assert route == {"prefix_places": 0, "passes": 0, "chunks": 0, "fallback_runs": 0, "fallback_keys": 0}, route


def test_sortperm_never_takes_prefix_route():
    rng = np.random.default_rng(14)
    k = random_keys("u64", N0, rng, "uniform")
    t = to_gpu(k, "u64")
    p = ak.sortperm(t, dtype="u64")
    route = ak.sort_route()
    assert route["prefix_places"] == 0 and route["passes"] == 8, route
    assert np.array_equal(p.cpu().numpy().view(np.uint32), oracle.sortperm(k))


def test_prefix_route_repeats():
    """Back-to-back sorts of different inputs on one workspace (the prefix
    scratch and the fallback's cached launch sequence are reused)."""
    rng = np.random.default_rng(15)
    for i in range(3):
        k = rng.integers(0, 1 << 64, size=N0 + 1000 * i, dtype=np.uint64)
        if i == 1:
            heavy = rng.random(k.size) < 0.002
            k[heavy] = np.uint64(0x1234) << np.uint64(48) | (k[heavy] & np.uint64(0xFFFF))
        _check(k, "u64", f"repeat{i}")
    torch.cuda.synchronize()


def test_repeated_keys_take_in_chunk_fallback():
    """Every value repeated 100 times: the per-place counts still look
    uniform (prefix route), but each chunk's top-digit buckets hold about
    100 keys, more than the comparison finish takes, so those chunks run the
    LSD passes on chip; ties keep their order (identical keys)."""
    rng = np.random.default_rng(16)
    vals = rng.integers(0, 1 << 64, size=N0 // 100 + 1, dtype=np.uint64)
    k = np.repeat(vals, 100)[:N0]
    rng.shuffle(k)
    route = _check(k, "u64", "repeated")
    assert route["prefix_places"] >= 2 and route["chunks"] > 0, route
    # float keys with repeated values and both zeros
    f = np.repeat(rng.standard_normal(N0 // 50 + 1), 50)[:N0]
    f[rng.random(N0) < 0.01] = -0.0
    f[rng.random(N0) < 0.01] = 0.0
    rng.shuffle(f)
    _check(f.astype(np.float64), "f64", "repeated-float")


@pytest.mark.parametrize("reps", [16, 17])
def test_repeats_at_the_group_limit(reps):
    """Every value repeated 16 or 17 times: a chunk's groups of equal top
    16 bits are the repeats (one group per value).  At 16 each key is
    placed by comparisons inside its group; at 17 every chunk exceeds the
    limit and takes the passes over all its varying bits."""
    rng = np.random.default_rng(100 + reps)
    vals = rng.integers(0, 1 << 64, size=N0 // reps + 1, dtype=np.uint64)
    k = np.repeat(vals, reps)[:N0]
    rng.shuffle(k)
    route = _check(k, "u64", f"repeats{reps}")
    assert route["prefix_places"] >= 2 and route["chunks"] > 0, route


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_prefix_route_with_nan_payloads_and_zeros(dt):
    """Raw random bits: NaNs with every payload and sign (all tie, so they
    keep input order), both zeros and infinities.  The NaN run exceeds a
    chunk and goes to the segmented fallback, which must keep it stable."""
    rng = np.random.default_rng(zlib.crc32(f"pfxnan{dt}".encode()))
    n = N0
    w = 32 if dt == "f32" else 64
    raw = rng.integers(0, 1 << w, size=n, dtype=np.uint64).astype(np.uint32 if w == 32 else np.uint64)
    k = raw.view(np.float32 if w == 32 else np.float64).copy()
    pos = rng.choice(n, size=3000, replace=False)
    k[pos[:1000]] = -0.0
    k[pos[1000:2000]] = 0.0
    k[pos[2000:2500]] = np.inf
    k[pos[2500:]] = -np.inf
    route = _check(k, dt, "nan-payloads")
    assert route["prefix_places"] >= 2, route
    if dt == "f32":
        assert route["fallback_runs"] >= 1, route   # about n/256 NaNs in one run


SMALL_SIZES = [(1 << 16) + 1, 300_001, 1_000_000, 1 << 22]


@pytest.mark.parametrize("dt", ["u64", "i64", "f64", "u32", "i32", "f32"])
def test_small_runs_take_prefix_route(dt):
    """Sizes whose launch sequence is replayed from a captured graph
    (2**16 < n <= 2**22) take the prefix route too, with fixed launches
    only; a second input of the same size replays the same graph."""
    rng = np.random.default_rng(zlib.crc32(f"pfxsmall{dt}".encode()))
    for n in SMALL_SIZES:
        for rep in range(2):
            k = random_keys(dt, n, rng, "uniform")
            route = _check(k, dt, f"small-uniform{rep}")
            assert route["prefix_places"] == 2 and route["passes"] == 2, route
            assert route["chunks"] > 0, route


@pytest.mark.parametrize("n,frac", [(300_001, 0.01), (1 << 22, 0.001)])
def test_small_heavy_prefix_sorted_by_fallback_kernel(n, frac):
    """A fraction of the keys share one 16-bit prefix (small enough that the
    per-place counts still choose two prefix places): that run exceeds a
    chunk and one workgroup sorts it (LSD through the scratch copy); the rest
    finish in chunks."""
    rng = np.random.default_rng(n)
    k = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    heavy = rng.random(n) < frac
    k[heavy] = (np.uint64(0x5A5A) << np.uint64(48)) | (k[heavy] & np.uint64((1 << 48) - 1))
    route = _check(k, "u64", "small-heavy")
    assert route["prefix_places"] == 2, route
    assert route["fallback_runs"] >= 1 and route["fallback_keys"] > CHUNK, route


def test_small_runs_nan_payloads_repeated_and_constant_place():
    """At graph-replayed sizes: float32 raw bits (a run of about n/256 NaNs
    of every payload, which must keep input order), keys repeated 100 times,
    and a constant byte inside the prefix."""
    rng = np.random.default_rng(19)
    n = 1_000_000
    k = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32).view(np.float32).copy()
    k[rng.choice(n, size=2000, replace=False)] = -0.0
    route = _check(k, "f32", "small-nan")
    assert route["prefix_places"] >= 2 and route["fallback_runs"] >= 1, route
    vals = rng.integers(0, 1 << 64, size=n // 100 + 1, dtype=np.uint64)
    r = np.repeat(vals, 100)[:n]
    rng.shuffle(r)
    route = _check(r, "u64", "small-repeated")
    assert route["prefix_places"] >= 2, route
    c = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    c = (c & ~np.uint64(0xFF << 48)) | np.uint64(0x3C << 48)
    route = _check(c, "u64", "small-inactive")
    assert route["prefix_places"] >= 2 and route["passes"] == route["prefix_places"] - 1, route


def test_prefix_route_full_size_2p31():
    """2**31 uniform uint64 keys (17 GiB, about a million chunks): the prefix
    route at the largest size; sorted, same multiset, sampled ranks, and the
    oracle's sort of a strided sample equals the sorted sample."""
    g = torch.Generator(device="cuda").manual_seed(2031)
    keys = torch.randint(-(1 << 63), (1 << 63) - 1, (1 << 31,), generator=g, device="cuda", dtype=torch.int64)
    fp = fingerprint(keys)
    t = keys.clone()
    ak.sort_(t, dtype="u64")
    route = ak.sort_route()
    print(route, flush=True)
    assert route["prefix_places"] == 3 and route["passes"] == 3, route
    assert is_sorted(t, "u64") and fingerprint(t) == fp
    rank_checks(keys, t, "u64", samples=8)
    idx = torch.arange(0, keys.numel(), 65537, device="cuda")
    sub = to_host(keys[idx], "u64")
    del keys, t
    torch.cuda.empty_cache()
    t2 = to_gpu(sub, "u64")
    ak.sort_(t2, dtype="u64")
    assert np.array_equal(to_host(t2, "u64"), oracle.sort(sub))
