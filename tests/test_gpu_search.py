"""GPU parity of ak_searchsortedfirst / ak_searchsortedlast (Sec. II-B
binary search) against the oracle's bisection, element by element (int64,
bit-exact).

Haystacks are sorted by the oracle (small sizes) or by ak_sort (large
sizes, whose order the sort tests establish); they span fewer elements than
the staged splitters, exactly that many, and many gaps; needles are
haystack members, float specials (NaN payloads, signed zeros, infinities)
and random keys.
"""
import zlib

import numpy as np
import pytest
import torch

import oracle
import paper_2507_16710_amd as ak
from gpucheck import NP, to_gpu, to_host
from pools import random_keys, special_bits

pytestmark = pytest.mark.gpu

DTYPES = ["i32", "i64", "u32", "u64", "f32", "f64"]
# haystack elements staged per workgroup: 64 KB of key images
SPLIT = {"i32": 16384, "u32": 16384, "f32": 16384, "i64": 8192, "u64": 8192, "f64": 8192}


def _search_both(v: np.ndarray, x: np.ndarray, dt: str):
    tv, tx = to_gpu(v, dt), to_gpu(x, dt)
    first = ak.searchsortedfirst(tv, tx, dtype=dt).cpu().numpy()
    last = ak.searchsortedlast(tv, tx, dtype=dt).cpu().numpy()
    return first, last


@pytest.mark.parametrize("dt", DTYPES)
def test_search_matches_oracle(dt):
    rng = np.random.default_rng(zlib.crc32(f"gpusearch{dt}".encode()))
    sp = SPLIT[dt]
    for n in [0, 1, 7, 2049, sp - 1, sp, sp + 1, 3 * sp + 5, 100003]:
        for kind in ("ties", "mixed"):
            v = oracle.sort(random_keys(dt, n, rng, kind))
            members = v[rng.integers(0, n, size=min(n, 5000))] if n else v
            x = np.concatenate([members, special_bits(dt).view(NP[dt]), random_keys(dt, 3001, rng, "mixed")])
            print(f"search dt={dt} n={n} kind={kind} m={x.size}", flush=True)
            first, last = _search_both(v, x, dt)
            assert np.array_equal(first, oracle.searchsorted(v, x, False)), (dt, n, kind)
            assert np.array_equal(last, oracle.searchsorted(v, x, True)), (dt, n, kind)


def test_search_empty_queries_and_out_argument():
    v = to_gpu(np.arange(10, dtype=np.int64), "i64")
    x = torch.empty(0, dtype=torch.int64, device="cuda")
    assert ak.searchsortedfirst(v, x, dtype="i64").numel() == 0
    out = torch.full((3,), 77, dtype=torch.int64, device="cuda")
    q = to_gpu(np.array([-5, 4, 100], dtype=np.int64), "i64")
    ak.searchsortedlast(v, q, dtype="i64", out=out)
    assert out.cpu().tolist() == [-1, 4, 9]


@pytest.mark.parametrize("dt", ["i64", "f32"])
def test_search_large_haystack_sorted_on_gpu(dt):
    """2^26 + 12345 keys sorted by ak_sort, 2^20 + 3 needles (half members):
    every result against the oracle's bisection over the same sorted keys."""
    rng = np.random.default_rng(zlib.crc32(f"gpusearchL{dt}".encode()))
    n, m = (1 << 26) + 12345, (1 << 20) + 3
    k = random_keys(dt, n, rng, "mixed")
    t = to_gpu(k, dt)
    ak.sort_(t, dtype=dt)
    v = to_host(t, dt)
    x = np.concatenate([v[rng.integers(0, n, size=m // 2)], random_keys(dt, m - m // 2, rng, "mixed")])
    print(f"search large dt={dt} n={n} m={m}", flush=True)
    tx = to_gpu(x, dt)
    first = ak.searchsortedfirst(t, tx, dtype=dt).cpu().numpy()
    last = ak.searchsortedlast(t, tx, dtype=dt).cpu().numpy()
    assert np.array_equal(first, oracle.searchsorted(v, x, False))
    assert np.array_equal(last, oracle.searchsorted(v, x, True))


def test_search_bench_configuration_sampled():
    """The timed configuration: 2^24 int64 keys (half haystack members, half
    random) in 2^28 sorted uniform int64 keys; a strided sample of 2^16
    results of each search against the oracle's bisection."""
    import synth
    k = synth.workload3("uniform", n=1 << 28, device="cuda")
    ak.sort_(k, dtype="i64")
    g = torch.Generator(device="cuda").manual_seed(28)
    m = 1 << 24
    idx = torch.randint(0, k.numel(), (m // 2,), generator=g, device="cuda")
    q = torch.cat([k[idx], torch.randint(-(1 << 62), 1 << 62, (m - m // 2,), generator=g, device="cuda")])
    print(f"search bench configuration n={k.numel()} m={m}", flush=True)
    first = ak.searchsortedfirst(k, q, dtype="i64")
    last = ak.searchsortedlast(k, q, dtype="i64")
    pick = torch.arange(0, m, m >> 16, device="cuda")
    v = to_host(k, "i64")
    x = to_host(q[pick].contiguous(), "i64")
    assert np.array_equal(first[pick].cpu().numpy(), oracle.searchsorted(v, x, False))
    assert np.array_equal(last[pick].cpu().numpy(), oracle.searchsorted(v, x, True))
