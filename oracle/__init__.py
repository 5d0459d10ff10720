"""Sort oracle: TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct CPU implementations of everything the GPU sort
path computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package.  It shares no code with
the HIP library ``paper_2507_16710_amd`` and never imports it.

Contents
  * ``sort`` / ``sortperm`` / ``segsort`` / ``sort_mt`` -- ctypes wrappers of
    the C merge sort in ``sort_oracle.c`` (paper Sec. II-B: ``merge_sort``,
    ``sortperm``; Julia Base order, Sec. II), for 16- to 128-bit integer
    and 32- / 64-bit float keys.
  * ``sort_by_key`` -- Sec. II-B ``merge_sort_by_key``: keys and payloads
    gathered through the stable sortperm (``sortperm`` is also the result of
    ``sortperm_lowmem``).
  * ``searchsorted`` -- the C bisection of Sec. II-B (searchsortedfirst /
    searchsortedlast) under the same order.
  * ``accumulate`` -- the C left-to-right prefix sum of Sec. II-B.
  * ``rmi`` -- the learned-CDF model (sampling, fitting, loss, gradients,
    bucket codes) in float64 / IEEE float32 numpy.
  * ``brute`` -- independent brute-force checkers (insertion sort with a
    separately written comparator, invariant checks) that pin the above.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sort_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# dtype codes of the oracle's C API (its own numbering)
_DT = {np.dtype(np.int32): 1, np.dtype(np.int64): 2, np.dtype(np.uint32): 3,
       np.dtype(np.uint64): 4, np.dtype(np.float32): 5, np.dtype(np.float64): 6,
       np.dtype(np.int16): 7, np.dtype(np.uint16): 8}
# 128-bit integer keys (numpy has no such dtype): (n, 2) uint64 arrays, the
# low word in column 0, the high word in column 1 (the little-endian layout
# of one 16-byte integer per row), named by an explicit dtype
WIDE = {"i128": 9, "u128": 10}


def build(force: bool = False) -> str:
    """Compile ``sort_oracle.c`` with gcc into ``liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        lib.oracle_sort.argtypes = [i32, vp, i64]
        lib.oracle_sortperm.argtypes = [i32, vp, vp, i64]
        lib.oracle_segsort.argtypes = [i32, vp, vp, i64]
        lib.oracle_sort_mt.argtypes = [i32, vp, i64, i32]
        lib.oracle_searchsorted.argtypes = [i32, vp, i64, vp, i64, i32, vp]
        lib.oracle_accumulate.argtypes = [i32, vp, i64, i32, vp]
        for f in (lib.oracle_sort, lib.oracle_sortperm, lib.oracle_segsort, lib.oracle_sort_mt,
                  lib.oracle_searchsorted, lib.oracle_accumulate):
            f.restype = i32
        _lib = lib
    return _lib


def _code(a: np.ndarray, dtype: str | None = None) -> int:
    if dtype is not None:
        if dtype not in WIDE:
            raise TypeError(f"oracle: unknown explicit dtype {dtype}")
        if a.dtype != np.uint64 or a.ndim != 2 or a.shape[1] != 2:
            raise TypeError("oracle: 128-bit keys are (n, 2) uint64 arrays (low word first)")
        return WIDE[dtype]
    try:
        return _DT[a.dtype]
    except KeyError:
        raise TypeError(f"oracle: unsupported dtype {a.dtype}") from None


def _count(a: np.ndarray, dtype: str | None) -> int:
    return a.shape[0] if dtype in WIDE else a.size


def sort(keys: np.ndarray, dtype: str | None = None) -> np.ndarray:
    """Stable ascending sort under the total order; returns a new array.
    ``dtype`` names 128-bit keys ("i128" / "u128", (n, 2) uint64 rows)."""
    out = np.ascontiguousarray(keys).copy()
    if _load().oracle_sort(_code(out, dtype), out.ctypes.data, _count(out, dtype)) != 0:
        raise RuntimeError("oracle_sort failed")
    return out


def sort_mt(keys: np.ndarray, threads: int) -> np.ndarray:
    """Same result as :func:`sort`, on ``threads`` POSIX threads."""
    out = np.ascontiguousarray(keys).copy()
    if _load().oracle_sort_mt(_code(out), out.ctypes.data, out.size, int(threads)) != 0:
        raise RuntimeError("oracle_sort_mt failed")
    return out


def sortperm(keys: np.ndarray, dtype: str | None = None) -> np.ndarray:
    """0-based stable index permutation (uint32) that sorts ``keys``.  This
    is also the result of the paper's sortperm_lowmem (Sec. II-B), which
    computes the same permutation with less temporary memory."""
    k = np.ascontiguousarray(keys)
    n = _count(k, dtype)
    perm = np.empty(n, dtype=np.uint32)
    if _load().oracle_sortperm(_code(k, dtype), k.ctypes.data, perm.ctypes.data, n) != 0:
        raise RuntimeError("oracle_sortperm failed")
    return perm


def sort_by_key(keys: np.ndarray, vals: np.ndarray, dtype: str | None = None):
    """Sec. II-B merge_sort_by_key: keys and their payloads (a separate
    array, one row per key) reordered together by the stable sort of the
    keys, i.e. both gathered through the stable sortperm of the keys.
    Returns (sorted keys, payloads in the same order)."""
    perm = sortperm(keys, dtype).astype(np.int64)
    v = np.ascontiguousarray(vals)
    if v.shape[0] != perm.size:
        raise ValueError("one payload row per key")
    return np.ascontiguousarray(keys)[perm].copy(), v[perm].copy()


def searchsorted(v: np.ndarray, x: np.ndarray, last: bool) -> np.ndarray:
    """Sec. II-B binary search over ``v`` (sorted under the total order),
    0-based, int64: ``last=False`` gives searchsortedfirst (index of the
    first element not below x; len(v) if none), ``last=True``
    searchsortedlast (index of the last element not above x; -1 if none)."""
    vv = np.ascontiguousarray(v)
    xx = np.ascontiguousarray(x, dtype=vv.dtype)
    out = np.empty(xx.size, dtype=np.int64)
    if _load().oracle_searchsorted(_code(vv), vv.ctypes.data, vv.size, xx.ctypes.data, xx.size,
                                   1 if last else 0, out.ctypes.data) != 0:
        raise RuntimeError("oracle_searchsorted failed")
    return out


def accumulate(x: np.ndarray, inclusive: bool = True) -> np.ndarray:
    """Sec. II-B accumulate with +, left to right.  Integer input: same
    dtype, sums wrap around in its width.  Float input: float64 prefixes of
    a running sum carried wider than the input (its error is far below one
    unit in the last place of the input type)."""
    xx = np.ascontiguousarray(x)
    out = np.empty(xx.size, dtype=np.float64 if xx.dtype.kind == "f" else xx.dtype)
    if _load().oracle_accumulate(_code(xx), xx.ctypes.data, xx.size, 1 if inclusive else 0,
                                 out.ctypes.data) != 0:
        raise RuntimeError("oracle_accumulate failed")
    return out


def segsort(keys: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """Each segment [offsets[s], offsets[s+1]) sorted independently."""
    out = np.ascontiguousarray(keys).copy()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    nseg = off.size - 1
    if nseg < 0:
        raise ValueError("offsets must hold nseg+1 entries")
    if nseg > 0 and off[-1] > out.size:
        raise ValueError("offsets exceed the key array")
    if _load().oracle_segsort(_code(out), out.ctypes.data, off.ctypes.data, nseg) != 0:
        raise RuntimeError("oracle_segsort failed")
    return out


from . import brute, rmi  # noqa: E402,F401
