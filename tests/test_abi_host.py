"""Host-side checks of the C ABI (no GPU needed): libak.so loads, exports
every function include/ak.h declares, and rejects bad arguments before any
device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ak.h")


def _lib():
    import paper_2507_16710_amd as ak
    if not os.path.exists(ak.LIB_PATH):
        from paper_2507_16710_amd import build
        build.build()
    return ak.load_library()


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ak_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    lib = _lib()
    names = declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_errors_without_device_work():
    lib = _lib()
    vp = ctypes.c_void_p
    fake = vp(0x1000)     # never dereferenced: rejected before any launch
    assert lib.ak_sort(fake, -1, 2, None) == 1
    assert lib.ak_sort(None, 10, 2, None) == 1
    assert lib.ak_sort(fake, 10, 0, None) == 2
    assert lib.ak_sort(fake, 10, 11, None) == 2
    assert lib.ak_sort(fake, 1 << 32, 2, None) == 1
    # the accepted range ends at 2^31 keys (32-bit indices and grid-stride
    # loops): one key more is refused before any launch by every entry point
    over = (1 << 31) + 1
    assert lib.ak_sort(fake, over, 2, None) == 1
    assert lib.ak_sortperm(fake, vp(0x10000000000), over, 2, None) == 1
    assert lib.ak_sort_learned(fake, over, 4, None, None, None) == 1
    assert lib.ak_rmi_codes(fake, over, 4, fake, 12, vp(0x10000000000), None) == 1
    assert lib.ak_learned_sample(fake, over, 4, 0, 16, vp(0x10000000000), None) == 1
    assert lib.ak_learned_sample(fake, 100, 4, 0, over, vp(0x10000000000), None) == 1
    assert b"2^31" in lib.ak_last_error() or b"sample" in lib.ak_last_error()
    assert lib.ak_sort(fake, 0, 2, None) == 0           # n == 0: no launch
    assert lib.ak_sortperm(fake, None, 10, 2, None) == 1
    assert lib.ak_sortperm(fake, fake, 10, 2, None) == 1  # keys and perm overlap
    assert lib.ak_segmented_sort(fake, fake, -1, 3, None) == 1
    assert lib.ak_segmented_sort(fake, fake, 0, 3, None) == 0
    assert lib.ak_segmented_sort(None, fake, 5, 3, None) == 1
    # the asynchronous form takes the key count: checked before any launch
    assert lib.ak_segmented_sort_n(fake, -1, fake, 3, 3, None) == 1
    assert lib.ak_segmented_sort_n(fake, (1 << 31) + 1, fake, 3, 3, None) == 1
    assert lib.ak_segmented_sort_n(fake, 100, fake, -1, 3, None) == 1
    assert lib.ak_segmented_sort_n(None, 100, fake, 3, 3, None) == 1
    assert lib.ak_segmented_sort_n(fake, 100, None, 3, 3, None) == 1
    assert lib.ak_segmented_sort_n(fake, 100, fake, 3, 9, None) == 2
    assert lib.ak_segmented_sort_n(fake, 100, fake, 0, 3, None) == 0
    assert lib.ak_segmented_sort_n(fake, 0, fake, 3, 3, None) == 0
    bad = (ctypes.c_int32 * 8)(4095, 12, 0, 0, 0, 0, 0, 0)   # leaves not a power of two
    assert lib.ak_sort_learned(fake, 10, 4, bad, None, None) == 1
    assert lib.ak_rmi_codes(fake, 10, 4, fake, 25, fake, None) == 1
    assert lib.ak_learned_sample(fake, 10, 4, 0, -1, fake, None) == 1
    assert lib.ak_seg_set_tuning(32, 3, 16, 4, 0, 32768) == 1
    assert lib.ak_seg_set_tuning(64, 4, 32, 4, 0, 32768) == 1   # 32 keys/lane: 32-bit only
    msg = lib.ak_last_error()
    assert msg and b"tuning" in msg
    assert lib.ak_set_workspace(None, 4096, None) == 1        # NULL with bytes
    assert lib.ak_set_workspace(vp(0x1008), 1 << 20, None) == 1   # not 256-byte aligned
    assert lib.ak_set_workspace(vp(0x1000), 1024, None) == 1      # smaller than 4096 bytes
    assert lib.ak_status_string(3) == b"out of device memory"
    # the entry point that allocates nothing: its size limit (16 MiB of keys)
    # and argument errors are refused before any device call
    assert lib.ak_sort_noalloc(fake, (1 << 21) + 1, 2, None) == 1
    assert lib.ak_sort_noalloc(fake, (1 << 22) + 1, 5, None) == 1
    assert b"at most" in lib.ak_last_error()
    assert lib.ak_sort_noalloc(None, 10, 2, None) == 1
    assert lib.ak_sort_noalloc(fake, -1, 2, None) == 1
    assert lib.ak_sort_noalloc(fake, 10, 0, None) == 2
    assert lib.ak_sort_noalloc(fake, 0, 2, None) == 0


def test_new_sort_family_argument_errors():
    """Sort by key, the low-memory sortperm and the 16/128-bit key types:
    bad arguments refused before any launch; the calls that take only the
    six 32/64-bit types refuse the others."""
    lib = _lib()
    vp = ctypes.c_void_p
    k, v = vp(0x1000), vp(0x10000000)
    for dt in (2, 7, 10):
        assert lib.ak_sort_by_key(k, v, 10, dt, 3, None) == 1            # val_bytes not 4 or 8
        assert lib.ak_sort_by_key(k, None, 10, dt, 4, None) == 1         # vals NULL
        assert lib.ak_sort_by_key(k, vp(0x1004), 10, dt, 8, None) == 1   # vals overlaps keys
        assert lib.ak_sort_by_key(k, v, (1 << 31) + 1, dt, 4, None) == 1
        assert lib.ak_sort_by_key(k, v, 0, dt, 4, None) == 0
        assert lib.ak_sortperm_lowmem(k, None, 10, dt, None) == 1
        assert lib.ak_sortperm_lowmem(k, vp(0x1004), 10, dt, None) == 1
        assert lib.ak_sortperm_lowmem(k, v, 0, dt, None) == 0
    assert lib.ak_sort_by_key(k, v, 10, 11, 4, None) == 2
    assert lib.ak_sortperm_lowmem(k, v, 10, 0, None) == 2
    # 16- and 128-bit keys: sort family only
    for dt in (7, 8, 9, 10):
        assert lib.ak_segmented_sort(k, v, 3, dt, None) == 2
        assert lib.ak_sort_learned(k, 100, dt, None, None, None) == 2
        assert lib.ak_accumulate(k, v, 100, dt, 1, None) == 2
        assert lib.ak_searchsortedfirst(k, 100, v, 10, dt, vp(0x20000000), None) == 2
        assert lib.ak_rmi_codes(k, 100, dt, v, 12, vp(0x20000000), None) == 2
        assert lib.ak_temp_bytes(2, 1 << 20, dt) == 0
    # scratch: sort by key holds two payload buffers more than sort; the
    # low-memory sortperm only the indices (and per-tile words)
    n = 1 << 24
    for dt, kb in ((5, 4), (2, 8), (7, 2), (9, 16)):
        s_ = lib.ak_temp_bytes(0, n, dt)
        kv = lib.ak_temp_bytes(5, n, dt)
        low = lib.ak_temp_bytes(6, n, dt)
        full = lib.ak_temp_bytes(1, n, dt)
        assert kv >= 2 * n * kb + 2 * n * 8
        # indices plus one look-back word per (tile, digit)
        assert 4 * n <= low <= 4 * n * 1.5 + (1 << 22) and low < full, (dt, low, full)
        assert kb < 4 or low * 2 < full
        assert s_ >= 2 * n * kb


def test_temp_bytes_predictable():
    """Scratch sizes are known from n alone (paper Sec. II-B: temporaries
    are exposed and predictable)."""
    lib = _lib()
    for dt in (1, 2, 3, 4, 5, 6):
        kb = 8 if dt in (2, 4, 6) else 4
        assert lib.ak_temp_bytes(0, 100, dt) == 0                 # on-chip path
        n = 10_000_000
        s = lib.ak_temp_bytes(0, n, dt)
        p = lib.ak_temp_bytes(1, n, dt)
        # two ping-pong buffers + look-back, and above 2**22 keys the prefix
        # finish's segmented fallback scratch (its huge-segment tables scale
        # with n / the tuned huge-segment threshold)
        assert 2 * n * kb <= s <= n * kb * 2.3
        assert p >= 2 * n * kb + n * 4
        assert lib.ak_temp_bytes(2, n, dt) >= n * kb
        assert lib.ak_temp_bytes(3, n, dt) >= s
        # segmented: the bound assumes nseg <= n; more segments need more
        assert lib.ak_temp_bytes(2, n, dt) == lib.ak_temp_bytes_segmented(n, n, dt)
        assert lib.ak_temp_bytes_segmented(n, 10, dt) < lib.ak_temp_bytes_segmented(n, 2 * n, dt)
        assert lib.ak_temp_bytes_segmented(n, 0, dt) == 0
    assert lib.ak_rmi_model_floats(4096) == 8 + 4 * (4096 + 1)


def test_sort_route_argument_error():
    lib = _lib()
    assert lib.ak_sort_route(None, None) == 1  # info NULL, checked before any device call


def test_searchsorted_argument_errors():
    """Bad arguments of ak_searchsortedfirst / ak_searchsortedlast are
    rejected before any launch; m == 0 launches nothing."""
    lib = _lib()
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    for name in ("ak_searchsortedfirst", "ak_searchsortedlast"):
        f = getattr(lib, name)
        f.argtypes = [vp, i64, vp, i64, ctypes.c_int32, vp, vp]
        v, x, out = vp(0x1000), vp(0x100000), vp(0x200000)
        assert f(v, -1, x, 4, 2, out, None) == 1               # n < 0
        assert f(v, 4, x, -1, 2, out, None) == 1               # m < 0
        assert f(v, 1 << 40, x, 4, 2, out, None) == 1          # n too large
        assert f(v, 4, x, 4, 9, out, None) == 2                # unknown dtype
        assert f(v, 4, None, 4, 2, out, None) == 1             # keys NULL
        assert f(v, 4, x, 4, 2, None, None) == 1               # out NULL
        assert f(None, 4, x, 4, 2, out, None) == 1             # sorted NULL with n > 0
        assert f(v, 4, x, 4, 2, vp(0x100010), None) == 1       # out overlaps keys
        assert f(v, 4, x, 0, 2, out, None) == 0                # m == 0: nothing to do


def test_accumulate_argument_errors():
    lib = _lib()
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    f = lib.ak_accumulate
    f.argtypes = [vp, vp, i64, ctypes.c_int32, ctypes.c_int32, vp]
    a = vp(0x1000)
    assert f(a, vp(0x100000), -1, 2, 1, None) == 1          # n < 0
    assert f(a, vp(0x100000), 1 << 32, 2, 1, None) == 1     # too many keys
    assert f(a, vp(0x100000000), (1 << 31) + 1, 2, 1, None) == 1   # one above AK_MAX_KEYS
    assert f(a, None, 8, 2, 1, None) == 1                   # out NULL
    assert f(None, vp(0x100000), 8, 2, 1, None) == 1        # in NULL
    assert f(a, vp(0x1008), 8, 2, 1, None) == 1             # partial overlap
    assert f(a, vp(0x100000), 8, 9, 1, None) == 2           # unknown dtype
    assert f(a, a, 0, 2, 1, None) == 0                      # n == 0
    assert lib.ak_temp_bytes(4, 4096, 2) == 0               # one chunk: no scratch
    assert lib.ak_temp_bytes(4, 4097, 2) == 256
