"""Test-side helpers for GPU parity checks (inputs, copies, properties).

Property checks here run on the GPU with plain torch comparisons so that
full-size outputs (too large for the oracle to sort in seconds) can still be
checked: order, multiset fingerprint, permutation validity and stability.
They implement the order's definition directly, not the library's method.
"""
from __future__ import annotations

import numpy as np
import torch

NP = {"i32": np.int32, "i64": np.int64, "u32": np.uint32, "u64": np.uint64,
      "f32": np.float32, "f64": np.float64}
STORAGE = {"i32": torch.int32, "u32": torch.int32, "f32": torch.float32,
           "i64": torch.int64, "u64": torch.int64, "f64": torch.float64}


def to_gpu(a: np.ndarray, dt: str) -> torch.Tensor:
    """Device tensor holding exactly the bits of `a`."""
    st = STORAGE[dt]
    view = a.view({torch.int32: np.int32, torch.int64: np.int64,
                   torch.float32: np.float32, torch.float64: np.float64}[st])
    return torch.from_numpy(np.ascontiguousarray(view)).to("cuda")


def to_host(t: torch.Tensor, dt: str) -> np.ndarray:
    return t.detach().cpu().numpy().view(NP[dt])


def signed_order_key(t: torch.Tensor, dt: str) -> torch.Tensor:
    """int64 tensor whose signed order is the total order of the keys
    (NaNs all equal and above +Inf; -0.0 below +0.0)."""
    if dt in ("i32", "u32", "f32"):
        b = t.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        if dt == "i32":
            return t.to(torch.int64)
        if dt == "u32":
            return b
        neg = (b & 0x80000000) != 0
        img = torch.where(neg, (~b) & 0xFFFFFFFF, b | 0x80000000)
        img = torch.where(torch.isnan(t), torch.full_like(img, 0xFFFFFFFF), img)
        return img
    b = t.view(torch.int64)
    if dt == "i64":
        return b.clone()
    sign = torch.tensor(-(1 << 63), dtype=torch.int64, device=t.device)
    if dt == "u64":
        return b ^ sign
    # f64: image = (negative ? ~b : b | sign); NaN -> all ones; then ^ sign
    img = torch.where(b < 0, ~b, b | sign)
    img = torch.where(torch.isnan(t), torch.full_like(img, -1), img)
    return img ^ sign


def is_sorted(t: torch.Tensor, dt: str) -> bool:
    k = signed_order_key(t, dt)
    return bool((k[1:] >= k[:-1]).all()) if k.numel() > 1 else True


def fingerprint(t: torch.Tensor) -> tuple:
    """Order-independent multiset fingerprint of the raw bits: count plus two
    wrapping sums of a 64-bit mix of every element."""
    b = t.view(torch.int32).to(torch.int64) if t.element_size() == 4 else t.view(torch.int64)
    z = b * -7046029254386353131                      # 0x9E3779B97F4A7C15, wraps
    z = (z ^ ((z >> 31) & ((1 << 33) - 1))) * -4658895280553007687
    z = z ^ ((z >> 29) & ((1 << 35) - 1))
    return int(t.numel()), int(z.sum()), int((z * z).sum())


def _mix(t: torch.Tensor) -> torch.Tensor:
    b = t.view(torch.int32).to(torch.int64) if t.element_size() == 4 else t.view(torch.int64)
    z = b * -7046029254386353131
    z = (z ^ ((z >> 31) & ((1 << 33) - 1))) * -4658895280553007687
    return z ^ ((z >> 29) & ((1 << 35) - 1))


def segment_fingerprints(t: torch.Tensor, seg_id: torch.Tensor, nseg: int) -> torch.Tensor:
    """Per-segment multiset fingerprints: for every segment the count and
    two wrapping sums of a 64-bit mix of its elements' bits ([nseg, 3]).  A
    key that moved into another segment changes two rows."""
    z = _mix(t)
    cols = []
    for v in (torch.ones_like(z), z, z * z):
        c = torch.zeros(nseg, dtype=torch.int64, device=t.device)
        c.index_add_(0, seg_id, v)
        cols.append(c)
    return torch.stack(cols, dim=1)


def check_perm_sorts_stably(keys: torch.Tensor, perm: torch.Tensor, dt: str) -> None:
    n = keys.numel()
    p = perm.to(torch.int64) & 0xFFFFFFFF
    assert p.numel() == n
    seen = torch.zeros(n, dtype=torch.int32, device=keys.device)
    seen.index_add_(0, p, torch.ones_like(p, dtype=torch.int32))
    assert bool((seen == 1).all()), "perm is not a permutation"
    k = signed_order_key(keys, dt)[p]
    assert bool((k[1:] >= k[:-1]).all()), "keys[perm] not sorted"
    tie = k[1:] == k[:-1]
    assert bool((p[1:][tie] > p[:-1][tie]).all()), "ties not in index order"


def rank_checks(keys: torch.Tensor, out: torch.Tensor, dt: str, samples: int = 64, seed: int = 0) -> None:
    """Sampled outputs computed one by one: for position i holding x,
    #{keys < x} <= i < #{keys <= x}."""
    k = signed_order_key(keys, dt)
    o = signed_order_key(out, dt)
    g = torch.Generator(device="cpu").manual_seed(seed)
    idx = torch.randint(0, out.numel(), (samples,), generator=g).tolist()
    idx += [0, out.numel() - 1]
    for i in idx:
        x = o[i]
        lt = int((k < x).sum())
        le = int((k <= x).sum())
        assert lt <= i < le, (i, lt, le)
