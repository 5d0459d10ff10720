"""Seeded synthetic inputs for the sort path.

This module only draws inputs; it holds none of the sort method's
arithmetic, and both the HIP path and the oracle consume the arrays it makes.
The paper's sorting runs are synthetic arrays of machine numbers by dtype and
size per rank (Sec. IV-C); the five workloads below keep those dtypes and
give them the shapes, sizes and value distributions of the workloads this
library is measured on:

  1. uniform int64 over the full range                    (1,000,000 keys)
  2. float32 N(0, sd=1e3) with 0.1% NaN, 0.1% +-0.0 and 0.1% +-Inf at disjoint
     random positions                                     (2**28 keys)
  3. one GPU's share of a distributed sort, int64, three variants
     (uniform / Zipf(s=1.2) over 1e6 ranks / floor(lognormal(20, 2)))
                                                          (2**30 keys)
  4. 100,000 segments, lognormal sizes clipped to [16, 2**20] with mean
     about 5,000, uniform uint32 keys, int64 CSR offsets
  5. uint64 mixture in blocks of 4096: 50% lognormal(30, 3), 30% Zipf(s=1.1)
     over 1e7 ranks, 20% presorted runs of uniform keys    (2**31 keys)

Every array is drawn with ``torch`` on the requested device from a generator
seeded with (seed, workload, variant); the same seed gives the same bytes on
the same device type.  Integer keys are returned as torch integer tensors
(uint32 / uint64 data held in int32 / int64 storage); ``DTYPE`` says what the
bits mean.
"""
from __future__ import annotations

import math

import numpy as np
import torch

# what each returned key tensor's bits mean
DTYPE = {1: "i64", 2: "f32", 3: "i64", 4: "u32", 5: "u64"}

N_DEFAULT = {1: 1_000_000, 2: 1 << 28, 3: 1 << 30, 5: 1 << 31}


def _gen(device, seed: int, workload: int, variant: int, stream: int) -> torch.Generator:
    g = torch.Generator(device=device)
    # one 63-bit seed per (seed, workload, variant, stream)
    mix = (seed * 1_000_003 + workload * 10_007 + variant * 101 + stream) & ((1 << 63) - 1)
    g.manual_seed(mix)
    return g


def _u64_bits(g, n, device) -> torch.Tensor:
    """n uniform 64-bit patterns (int64 storage)."""
    hi = torch.randint(0, 1 << 32, (n,), generator=g, device=device, dtype=torch.int64)
    lo = torch.randint(0, 1 << 32, (n,), generator=g, device=device, dtype=torch.int64)
    return (hi << 32) | lo


def _f64_to_u64_sat(v: torch.Tensor) -> torch.Tensor:
    """floor(v) for v >= 0 as uint64 bits in int64 storage, saturating at
    2**64 - 1."""
    v = torch.floor(v)
    two63 = float(1 << 63)
    big = v >= two63
    sat = v >= float(1 << 64)
    low = torch.where(big, v - two63, v).clamp(max=two63 - 1024).to(torch.int64)
    out = torch.where(big, low | torch.tensor(-(1 << 63), device=v.device, dtype=torch.int64), low)
    return torch.where(sat, torch.full_like(out, -1), out)


_ZIPF_CACHE: dict = {}


def _zipf_cdf(s: float, K: int, device) -> torch.Tensor:
    key = (s, K, str(device))
    if key not in _ZIPF_CACHE:
        k = np.arange(1, K + 1, dtype=np.float64)
        w = k ** (-s)
        c = np.cumsum(w)
        c /= c[-1]
        _ZIPF_CACHE[key] = torch.from_numpy(c).to(device)
    return _ZIPF_CACHE[key]


def zipf(g, n: int, s: float, K: int, device) -> torch.Tensor:
    """Bounded Zipf on ranks 1..K, P(k) ~ k**-s, by inverse CDF; the key is
    the rank (int64)."""
    cdf = _zipf_cdf(s, K, device)
    u = torch.rand(n, generator=g, device=device, dtype=torch.float64)
    idx = torch.searchsorted(cdf, u, right=True)
    return (idx.clamp(max=K - 1) + 1).to(torch.int64)


def lognormal_int(g, n: int, mu: float, sigma: float, device) -> torch.Tensor:
    """floor(exp(mu + sigma*z)) in float64, saturated at 2**64-1 (uint64
    bits in int64 storage)."""
    z = torch.randn(n, generator=g, device=device, dtype=torch.float64)
    return _f64_to_u64_sat(torch.exp(mu + sigma * z))


# ---------------------------------------------------------------- workloads
def workload1(n: int = N_DEFAULT[1], seed: int = 0, device="cpu") -> torch.Tensor:
    """Uniform int64 over the whole int64 range."""
    return _u64_bits(_gen(device, seed, 1, 0, 0), n, device)


def workload2(n: int = N_DEFAULT[2], seed: int = 0, device="cpu") -> torch.Tensor:
    """float32 N(0, sd=1e3) rounded from float64; k = floor(0.001 n) NaNs
    (0x7FC00000), k signed zeros and k signed infinities (fair-coin sign) at
    disjoint random positions."""
    g = _gen(device, seed, 2, 0, 0)
    v = (torch.randn(n, generator=g, device=device, dtype=torch.float64) * 1e3).to(torch.float32)
    k = n // 1000
    if k:
        pos = torch.randperm(n, generator=g, device=device)[: 3 * k]
        sign = torch.randint(0, 2, (2 * k,), generator=g, device=device).to(torch.float32) * 2 - 1
        v[pos[:k]] = float("nan")
        v[pos[k:2 * k]] = torch.where(sign[:k] > 0, 0.0, -0.0).to(torch.float32)
        v[pos[2 * k:3 * k]] = sign[k:] * float("inf")
    return v


def workload3(variant: str = "uniform", n: int = N_DEFAULT[3], seed: int = 0, device="cpu") -> torch.Tensor:
    """int64 keys; variant 'uniform' (full range), 'zipf' (s=1.2 over 1e6
    ranks; key = rank) or 'lognormal' (floor(exp(20 + 2z)))."""
    vid = {"uniform": 0, "zipf": 1, "lognormal": 2}[variant]
    g = _gen(device, seed, 3, vid, 0)
    if variant == "uniform":
        return _u64_bits(g, n, device)
    if variant == "zipf":
        return zipf(g, n, 1.2, 1_000_000, device)
    return lognormal_int(g, n, 20.0, 2.0, device)


def _clipped_lognormal_mean(mu: float, sigma: float, a: float, b: float) -> float:
    Phi = lambda t: 0.5 * (1.0 + math.erf(t / math.sqrt(2.0)))
    al = (math.log(a) - mu) / sigma
    be = (math.log(b) - mu) / sigma
    return (a * Phi(al) + b * (1 - Phi(be))
            + math.exp(mu + sigma * sigma / 2) * (Phi(be - sigma) - Phi(al - sigma)))


def segment_mu(mean: float = 5000.0, sigma: float = 2.0, a: float = 16.0, b: float = float(1 << 20)) -> float:
    """mu such that E[clip(lognormal(mu, sigma), a, b)] = mean (bisection)."""
    lo, hi = 0.0, 14.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _clipped_lognormal_mean(mid, sigma, a, b) < mean:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def workload4_sizes(nseg: int = 100_000, seed: int = 0, device="cpu",
                    lo: int = 16, hi: int = 1 << 20, mean: float = 5000.0) -> torch.Tensor:
    """Segment lengths: round(clip(lognormal(mu, 2), lo, hi)), mu solved so
    the clipped mean is `mean`."""
    mu = segment_mu(mean, 2.0, float(lo), float(hi))
    g = _gen(device, seed, 4, 0, 0)
    z = torch.randn(nseg, generator=g, device=device, dtype=torch.float64)
    s = torch.exp(mu + 2.0 * z).clamp(float(lo), float(hi))
    return torch.round(s).to(torch.int64)


def workload4(nseg: int = 100_000, seed: int = 0, device="cpu", **kw):
    """(keys uint32 bits in int32 storage, offsets int64[nseg+1])."""
    sizes = workload4_sizes(nseg, seed, device, **kw)
    off = torch.zeros(nseg + 1, dtype=torch.int64, device=device)
    off[1:] = torch.cumsum(sizes, 0)
    n = int(off[-1])
    g = _gen(device, seed, 4, 0, 1)
    keys = torch.randint(0, 1 << 32, (n,), generator=g, device=device, dtype=torch.int64)
    return keys.to(torch.int32), off


def sorted_uniform_runs(g, nruns: int, run: int, device) -> torch.Tensor:
    """nruns ascending runs of `run` uniform 64-bit keys each, drawn as order
    statistics: normalised partial sums of exponential spacings."""
    e = -torch.log1p(-torch.rand(nruns, run + 1, generator=g, device=device, dtype=torch.float64))
    c = torch.cumsum(e, dim=1)
    u = c[:, :run] / c[:, run:run + 1]
    return _f64_to_u64_sat(u * float(1 << 64)).reshape(-1)


def workload5(n: int = N_DEFAULT[5], seed: int = 0, device="cpu", block: int = 4096) -> torch.Tensor:
    """uint64 mixture (int64 storage): n/block blocks, each one component
    drawn with probabilities 0.5 / 0.3 / 0.2: lognormal(30, 3) saturated,
    Zipf(s=1.1) over 1e7 ranks, or one presorted run of uniform keys."""
    assert n % block == 0, "n must be a multiple of the block length"
    nb = n // block
    g = _gen(device, seed, 5, 0, 0)
    u = torch.rand(nb, generator=g, device=device, dtype=torch.float64)
    comp = (u >= 0.5).to(torch.int64) + (u >= 0.8).to(torch.int64)   # 0,1,2
    out = torch.empty(n, dtype=torch.int64, device=device)
    view = out.view(nb, block)
    for c in range(3):
        idx = torch.nonzero(comp == c).flatten()
        cnt = int(idx.numel())
        if cnt == 0:
            continue
        gc = _gen(device, seed, 5, 0, 1 + c)
        if c == 0:
            vals = lognormal_int(gc, cnt * block, 30.0, 3.0, device)
        elif c == 1:
            vals = zipf(gc, cnt * block, 1.1, 10_000_000, device)
        else:
            vals = sorted_uniform_runs(gc, cnt, block, device)
        view[idx] = vals.view(cnt, block)
    return out


def as_numpy(t: torch.Tensor, dtype: str) -> np.ndarray:
    """Host copy viewed with the meaning of its bits."""
    a = t.detach().cpu().contiguous().numpy()
    return a.view({"i32": np.int32, "u32": np.uint32, "i64": np.int64,
                   "u64": np.uint64, "f32": np.float32, "f64": np.float64}[dtype])
