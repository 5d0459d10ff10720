"""Brute-force checkers that pin the oracle: TEST INFRASTRUCTURE ONLY.

Written separately from ``sort_oracle.c`` so that a mistake in one does not
hide in the other.  The comparator is Julia Base ``isless`` restated from its
definition (the paper's library dispatches onto the Base function names,
Sec. II): NaN is above every non-NaN and equal to any NaN; -0.0 is below
+0.0; otherwise numeric order.  Pure Python, for small inputs only.
"""
from __future__ import annotations

import math

import numpy as np


def isless(a, b) -> bool:
    """Julia ``isless`` on Python numbers (ints or floats)."""
    if isinstance(a, float) or isinstance(b, float):
        a, b = float(a), float(b)
        if math.isnan(a):
            return False          # NaN is never below anything
        if math.isnan(b):
            return True           # every non-NaN is below NaN
        if a != b:
            return a < b
        # equal values: only the signed zeros are told apart
        return math.copysign(1.0, a) < 0 and math.copysign(1.0, b) > 0
    return a < b


def wide_ints(rows: np.ndarray, signed: bool) -> list:
    """(n, 2) uint64 rows (low word, high word) -> Python ints: the value
    lo + hi * 2**64, minus 2**128 when signed and the top bit is set."""
    out = []
    for lo, hi in rows.tolist():
        v = int(lo) + (int(hi) << 64)
        if signed and v >= 1 << 127:
            v -= 1 << 128
        out.append(v)
    return out


def _py(keys: np.ndarray, dtype: str | None = None) -> list:
    if dtype in ("i128", "u128"):
        return wide_ints(keys, dtype == "i128")
    if keys.dtype.kind == "f":
        return [float(v) for v in keys.tolist()]
    return [int(v) for v in keys.tolist()]


def insertion_sortperm(keys: np.ndarray, dtype: str | None = None) -> np.ndarray:
    """Stable insertion sort of indices: an element moves left only past
    strictly greater keys, so equal keys keep their input order."""
    vals = _py(keys, dtype)
    idx = list(range(len(vals)))
    for i in range(1, len(idx)):
        cur = idx[i]
        j = i - 1
        while j >= 0 and isless(vals[cur], vals[idx[j]]):
            idx[j + 1] = idx[j]
            j -= 1
        idx[j + 1] = cur
    return np.asarray(idx, dtype=np.uint32)


def insertion_sort(keys: np.ndarray, dtype: str | None = None) -> np.ndarray:
    return keys[insertion_sortperm(keys, dtype)]


# ---------------------------------------------------------------- invariants
def is_nondecreasing(out: np.ndarray) -> bool:
    """No adjacent pair is strictly decreasing under ``isless``."""
    v = _py(out)
    return all(not isless(v[i + 1], v[i]) for i in range(len(v) - 1))


def same_multiset(a: np.ndarray, b: np.ndarray) -> bool:
    """Bitwise multiset equality (keys compared as raw bit patterns)."""
    if a.size != b.size or a.dtype != b.dtype:
        return False
    ua = a.view(np.uint32 if a.itemsize == 4 else np.uint64)
    ub = b.view(np.uint32 if b.itemsize == 4 else np.uint64)
    va, ca = np.unique(ua, return_counts=True)
    vb, cb = np.unique(ub, return_counts=True)
    return np.array_equal(va, vb) and np.array_equal(ca, cb)


def is_permutation(perm: np.ndarray, n: int) -> bool:
    if perm.size != n:
        return False
    seen = np.zeros(n, dtype=bool)
    p = perm.astype(np.int64)
    if n and (p.min() < 0 or p.max() >= n):
        return False
    seen[p] = True
    return bool(seen.all())


def perm_is_stable_sort(keys: np.ndarray, perm: np.ndarray) -> bool:
    """perm sorts keys and, within keys equal under the order, indices rise."""
    if not is_permutation(perm, keys.size):
        return False
    v = _py(keys)
    p = perm.tolist()
    for i in range(len(p) - 1):
        a, b = v[p[i]], v[p[i + 1]]
        if isless(b, a):
            return False
        if not isless(a, b) and p[i + 1] < p[i]:   # tie: index must rise
            return False
    return True


def count_search(v: np.ndarray, x: np.ndarray, last: bool) -> np.ndarray:
    """searchsortedfirst / searchsortedlast (0-based) by counting, without
    using that ``v`` is sorted: first = number of elements below x; last =
    number of elements not above x, minus one."""
    vs, xs = _py(v), _py(x)
    if last:
        return np.asarray([sum(1 for a in vs if not isless(b, a)) - 1 for b in xs], dtype=np.int64)
    return np.asarray([sum(1 for a in vs if isless(a, b)) for b in xs], dtype=np.int64)
