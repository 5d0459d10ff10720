"""Adversarial small-input pools shared by the tests (inputs only)."""
from __future__ import annotations

import numpy as np

DTYPES = ["i32", "i64", "u32", "u64", "f32", "f64"]
NP = {"i32": np.int32, "i64": np.int64, "u32": np.uint32, "u64": np.uint64,
      "f32": np.float32, "f64": np.float64}


def special_bits(dt: str) -> np.ndarray:
    """Bit patterns that stress the total order of each dtype."""
    if dt == "f32":
        b = [0x7FC00000, 0xFFC00000, 0x7F800001, 0xFFFFFFFF, 0x7FBFFFFF,  # NaNs
             0x7F800000, 0xFF800000, 0x00000000, 0x80000000,              # +-Inf, +-0
             0x00000001, 0x80000001, 0x7F7FFFFF, 0xFF7FFFFF,              # denormals, max
             0x3F800000, 0xBF800000, 0x00800000, 0x80800000]
        return np.array(b, dtype=np.uint32).view(np.float32)
    if dt == "f64":
        b = [0x7FF8000000000000, 0xFFF8000000000000, 0x7FF0000000000001,
             0xFFFFFFFFFFFFFFFF, 0x7FF0000000000000, 0xFFF0000000000000,
             0x0000000000000000, 0x8000000000000000, 0x0000000000000001,
             0x8000000000000001, 0x7FEFFFFFFFFFFFFF, 0xFFEFFFFFFFFFFFFF,
             0x3FF0000000000000, 0xBFF0000000000000]
        return np.array(b, dtype=np.uint64).view(np.float64)
    info = np.iinfo(NP[dt])
    vals = [info.min, info.min + 1, -1 if info.min < 0 else 1, 0, 1, 2,
            info.max - 1, info.max, 255, 256, 65535, 65536]
    return np.array([v for v in vals if info.min <= v <= info.max], dtype=NP[dt])


def random_keys(dt: str, n: int, rng: np.random.Generator, kind: str = "mixed") -> np.ndarray:
    """n keys: 'uniform' random bits, 'ties' (few distinct values) or
    'mixed' (random bits, specials and repeated values interleaved)."""
    w = np.dtype(NP[dt]).itemsize
    ubits = np.uint32 if w == 4 else np.uint64
    rand = rng.integers(0, 1 << (8 * w), size=n, dtype=np.uint64).astype(ubits).view(NP[dt])
    if kind == "uniform":
        out = rand
        if dt.startswith("f"):
            out = np.where(np.isnan(out), NP[dt](1.5), out).astype(NP[dt])
        return out
    sp = special_bits(dt)
    few = rand[: max(1, min(n, 5))]
    pool = np.concatenate([sp, few])
    if kind == "ties":
        return pool[rng.integers(0, pool.size, size=n)]
    pick = rng.integers(0, 3, size=n)
    out = rand.copy()
    out[pick == 1] = sp[rng.integers(0, sp.size, size=int((pick == 1).sum()))]
    out[pick == 2] = few[rng.integers(0, few.size, size=int((pick == 2).sum()))]
    return out


def bits(a: np.ndarray) -> np.ndarray:
    return a.view(np.uint32 if a.itemsize == 4 else np.uint64)


# 16-bit and 128-bit integer keys (the paper's benchmarks sort Int16 up to
# Int128).  128-bit keys are (n, 2) uint64 rows, low word first.
WIDE_DTYPES = ["i16", "u16", "i128", "u128"]
NP16 = {"i16": np.int16, "u16": np.uint16}
M64 = (1 << 64) - 1


def rows128(vals) -> np.ndarray:
    """Python ints (two's complement for negatives) -> (n, 2) uint64 rows."""
    out = np.empty((len(vals), 2), dtype=np.uint64)
    for i, v in enumerate(vals):
        v &= (1 << 128) - 1
        out[i, 0], out[i, 1] = v & M64, v >> 64
    return out


def special128(signed: bool) -> np.ndarray:
    top = 1 << 127
    vals = [0, 1, 2, M64, 1 << 64, (1 << 64) + 1, (5 << 64) | (1 << 63), (5 << 64) | ((1 << 63) - 1),
            (1 << 127) - 1, (1 << 127) - 2]
    if signed:
        vals += [-1, -2, -top, -top + 1, -(1 << 64), -(1 << 64) - 1, -(5 << 64)]
    else:
        vals += [(1 << 128) - 1, (1 << 128) - 2, top, top + 1, top | M64]
    return rows128(vals)


def wide_keys(dt: str, n: int, rng: np.random.Generator, kind: str = "mixed") -> np.ndarray:
    """n keys of a 16- or 128-bit dtype: 'uniform' random bits, 'ties' (few
    distinct values) or 'mixed' (random bits, specials, repeats)."""
    if dt in NP16:
        T = NP16[dt]
        rand = rng.integers(0, 1 << 16, size=n, dtype=np.uint32).astype(np.uint16).view(T)
        info = np.iinfo(T)
        sp = np.array([v for v in [info.min, info.min + 1, -1, 0, 1, 255, 256, info.max - 1, info.max]
                       if info.min <= v <= info.max], dtype=T)
    else:
        rand = rng.integers(0, 1 << 64, size=(n, 2), dtype=np.uint64)
        sp = special128(dt == "i128")
    if kind == "uniform":
        return rand
    few = rand[: max(1, min(n, 5))]
    pool = np.concatenate([sp, few])
    if kind == "ties":
        return pool[rng.integers(0, pool.shape[0], size=n)]
    pick = rng.integers(0, 3, size=n)
    out = rand.copy()
    out[pick == 1] = sp[rng.integers(0, sp.shape[0], size=int((pick == 1).sum()))]
    out[pick == 2] = few[rng.integers(0, few.shape[0], size=int((pick == 2).sum()))]
    return out


def wide_arg(dt: str):
    """The oracle's explicit dtype argument (128-bit keys only)."""
    return dt if dt in ("i128", "u128") else None


def from_image(img: np.ndarray, dt: str) -> np.ndarray:
    """Keys whose order-preserving image (the unsigned integer whose order is
    the keys' total order) is `img`: the inverse of that map, written out
    for tests that shape inputs in image bits (signed integers: the sign
    bit flipped; floats: images with the top bit set are the non-negative
    values with that bit cleared, the others are bit-complemented negative
    values)."""
    w = np.dtype(NP[dt]).itemsize * 8
    ub = np.uint32 if w == 32 else np.uint64
    img = np.asarray(img).astype(ub)
    top = ub(1) << ub(w - 1)
    if dt.startswith("u"):
        b = img
    elif dt.startswith("i"):
        b = img ^ top
    else:
        b = np.where((img & top) != 0, img ^ top, ~img).astype(ub)
    return b.view(NP[dt])


def prefix_groups(n: int, w: int, t: int, gmax: int, rng: np.random.Generator,
                  long_group: int = 0) -> np.ndarray:
    """n w-bit images whose top t bits form groups of equal prefix of at
    most `gmax` images each (plus one group of `long_group` images when it
    is nonzero); prefixes 0 and 2^t - 1 both occur, so the top bit varies,
    and every group holds some equal images.  Shuffled."""
    ub = np.uint32 if w == 32 else np.uint64
    sizes = []
    left = n
    if long_group:
        sizes.append(min(long_group, n))
        left -= sizes[-1]
    while left > 0:
        sizes.append(min(gmax, left))
        left -= sizes[-1]
    g = len(sizes)
    assert g <= (1 << t)
    inner = rng.choice(np.arange(1, (1 << t) - 1, dtype=np.uint64), size=max(g - 2, 0), replace=False)
    pref = np.concatenate([np.array([0, (1 << t) - 1], dtype=np.uint64)[:g], inner])
    lowbits = w - t
    out = []
    for p, s in zip(pref, sizes):
        low = rng.integers(0, 1 << lowbits, size=s, dtype=np.uint64)
        if s >= 3:
            low[1] = low[0]            # equal images inside the group
        low[0] |= np.uint64(1)        # the lowest bit varies
        out.append((np.uint64(p) << np.uint64(lowbits)) | low)
    a = np.concatenate(out).astype(ub)
    rng.shuffle(a)
    return a
