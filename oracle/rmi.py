"""Learned-CDF model oracle: TEST INFRASTRUCTURE ONLY.

The paper's library sorts with a merge sort (Sec. II-B); it has no learned
model.  The learned partition sort this package checks is defined by the
build's own design (a two-level recursive model index, RMI, with linear
leaves), so this module follows that definition step by step:

  1. draw m sample positions with a counter-based SplitMix64 stream
     (Steele, Lea & Flood, OOPSLA 2014; Vigna's reference splitmix64.c):
     pos_j = floor(splitmix64(seed, j) * n / 2**64);
  2. sort the sampled keys (the oracle sort);
  3. root: a monotone linear map of a log-like feature of the key (the bits
     of its float32 value), spanning the sample's feature range in L equal
     widths, routes every key to one of L leaves;
  4. leaves: per leaf, a monotone linear map of the key fitted by least
     squares to the empirical CDF j/m, clamped to the leaf's nested CDF range
     [st/m, en/m];
  5. inference: F(key) in [0,1]; code = floor(F * 2**CB).

Everything that turns floating point into an integer (leaf routing, codes,
float conversion of keys) is done in IEEE float32 with the same operation
order as the GPU kernels (multiply, then add; no fused multiply-add), because
both sides must reach the same integer.  Fitting and loss / gradient values
are float64: the GPU computes them in float32 and is compared with a
tolerance.

Parity: pinned by closed forms (least squares on exactly linear data, finite
differences of the loss, monotonicity, published SplitMix64 outputs).
"""
from __future__ import annotations

import numpy as np

U64 = np.uint64
M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


# ------------------------------------------------------------------ sampling
def splitmix64(seed: int, idx: np.ndarray) -> np.ndarray:
    """Output idx (0-based) of a SplitMix64 generator started at state seed:
    state_{j+1} = state_j + GOLDEN; output = mix(state_{j+1})."""
    with np.errstate(over="ignore"):
        z = (U64(seed & M64) + (idx.astype(U64) + U64(1)) * U64(GOLDEN))
        z = (z ^ (z >> U64(30))) * U64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> U64(27))) * U64(0x94D049BB133111EB)
        return z ^ (z >> U64(31))


def mulhi64(a: np.ndarray, n: int) -> np.ndarray:
    """floor(a * n / 2**64) for uint64 a and 0 <= n < 2**64, exactly."""
    a = a.astype(U64)
    n = int(n)
    a_lo, a_hi = a & U64(0xFFFFFFFF), a >> U64(32)
    n_lo, n_hi = U64(n & 0xFFFFFFFF), U64(n >> 32)
    with np.errstate(over="ignore"):
        ll = a_lo * n_lo
        lh = a_lo * n_hi
        hl = a_hi * n_lo
        hh = a_hi * n_hi
        mid = (ll >> U64(32)) + (lh & U64(0xFFFFFFFF)) + (hl & U64(0xFFFFFFFF))
        return hh + (lh >> U64(32)) + (hl >> U64(32)) + (mid >> U64(32))


def sample_positions(seed: int, n: int, m: int) -> np.ndarray:
    return mulhi64(splitmix64(seed, np.arange(m, dtype=np.int64)), n).astype(np.int64)


def sample_count(n: int, frac: float = 0.01, floor_m: int = 4096) -> int:
    """m = floor(frac * n), but at least min(n, floor_m) so small inputs still
    give every leaf a few samples."""
    return int(min(n, max(int(n * frac), floor_m)))


# -------------------------------------------------------------- key features
def key_image(keys: np.ndarray) -> np.ndarray:
    """Order-preserving unsigned image of the keys (uint64), from the total
    order's definition: unsigned as is; signed shifted by 2**(w-1); floats:
    NaN above +Inf, negatives reversed below -0.0 < +0.0."""
    k = np.ascontiguousarray(keys)
    w = k.dtype.itemsize * 8
    top = U64(1) << U64(w - 1)
    allones = U64((1 << w) - 1)
    if k.dtype.kind == "u":
        return k.astype(U64)
    if k.dtype.kind == "i":
        return k.view(np.uint32 if w == 32 else np.uint64).astype(U64) ^ top
    bits = k.view(np.uint32 if w == 32 else np.uint64).astype(U64)
    out = np.where(bits & top, (~bits) & allones, bits | top)
    return np.where(np.isnan(k), allones, out).astype(U64)


def _bit_length(t: np.ndarray) -> np.ndarray:
    bl = np.zeros(t.shape, dtype=np.int64)
    v = t.copy()
    for s in (32, 16, 8, 4, 2, 1):
        big = (v >> U64(s)) != 0
        bl = np.where(big, bl + s, bl)
        v = np.where(big, v >> U64(s), v)
    return bl + (v != 0)


def to_f32_rne(t: np.ndarray) -> np.ndarray:
    """uint64 -> float32, round to nearest, ties to even (IEEE default)."""
    t = t.astype(U64)
    bl = _bit_length(t)
    shift = np.maximum(bl - 24, 0).astype(U64)
    q = t >> shift
    rem = t - (q << shift)
    half = np.where(shift > 0, U64(1) << (shift - U64(1)), U64(0))
    up = (shift > 0) & ((rem > half) | ((rem == half) & ((q & U64(1)) == 1)))
    q = q + up.astype(U64)
    # q may reach 2**24: still exact in float32 (even significand)
    return (q.astype(np.float64) * np.exp2(shift.astype(np.float64))).astype(np.float32)


def features(keys: np.ndarray):
    """x = float32(image(key)); r = float32(bits of x as an unsigned int)."""
    x = to_f32_rne(key_image(keys))
    r = x.view(np.uint32).astype(np.float32)      # < 2**31, RNE, monotone
    return x, r


# ------------------------------------------------------------------- model
class Model:
    """RMI parameters, all float32 (the dtype the GPU evaluates in).  The
    upper clamp of leaf i is the lower clamp of leaf i+1 (1 for the last
    leaf), so the leaves' output ranges nest by construction."""

    def __init__(self, L: int):
        self.L = int(L)
        self.rc = np.float32(0)
        self.ra = np.float32(0)
        self.rb = np.float32(0)
        self.a = np.zeros(L, np.float32)
        self.b = np.zeros(L, np.float32)
        self.x0 = np.zeros(L, np.float32)
        self.lo = np.zeros(L, np.float32)

    @property
    def hi(self) -> np.ndarray:
        return np.concatenate([self.lo[1:], [np.float32(1)]]).astype(np.float32)

    def as_array(self) -> np.ndarray:
        """Device layout: [rc, ra, rb, L, 0 x4], then L+1 records
        (a, b, x0, lo), the last a sentinel with lo = 1."""
        head = np.array([self.rc, self.ra, self.rb, np.float32(self.L), 0, 0, 0, 0], np.float32)
        leaves = np.zeros((self.L + 1, 4), np.float32)
        leaves[:self.L, 0], leaves[:self.L, 1], leaves[:self.L, 2] = self.a, self.b, self.x0
        leaves[:self.L, 3] = self.lo
        leaves[self.L] = (0, 1, 0, 1)
        return np.concatenate([head, leaves.ravel()])

    @staticmethod
    def from_array(arr: np.ndarray) -> "Model":
        arr = np.asarray(arr, np.float32)
        L = int(arr[3])
        m = Model(L)
        m.rc, m.ra, m.rb = arr[0], arr[1], arr[2]
        lv = arr[8:8 + 4 * (L + 1)].reshape(L + 1, 4)
        m.a, m.b, m.x0, m.lo = (lv[:L, i].copy() for i in range(4))
        return m


def route(model: Model, r: np.ndarray) -> np.ndarray:
    """Leaf index in float32: clamp(floor(ra*(r-rc) + rb), 0, L-1)."""
    f32 = np.float32
    u = (r.astype(f32) - f32(model.rc)).astype(f32)
    p = ((f32(model.ra) * u).astype(f32) + f32(model.rb)).astype(f32)
    p = np.minimum(np.maximum(p, f32(0)), f32(model.L - 1))
    return p.astype(np.int64)


def cdf(model: Model, keys: np.ndarray) -> np.ndarray:
    """F(key) in float32: the leaf's clamp(a*(x-x0) + b, lo, hi)."""
    f32 = np.float32
    x, r = features(keys)
    leaf = route(model, r)
    dx = (x - model.x0[leaf]).astype(f32)
    F = ((model.a[leaf] * dx).astype(f32) + model.b[leaf]).astype(f32)
    return np.minimum(np.maximum(F, model.lo[leaf]), model.hi[leaf])   # hi = next leaf's lo


def codes(model: Model, keys: np.ndarray, cb: int) -> np.ndarray:
    """code = min(floor(F * 2**cb), 2**cb - 1) as uint32."""
    F = cdf(model, keys)
    c = (F * np.float32(2.0 ** cb)).astype(np.float32)
    return np.minimum(c.astype(np.int64), (1 << cb) - 1).astype(np.uint32)


def code_bits(n: int) -> int:
    """CB = clamp(ceil(log2 n) - 7, 12, 24): about 128 keys per code."""
    lg = max(int(n - 1).bit_length(), 1) if n > 1 else 1
    return int(min(24, max(12, lg - 7)))


# ----------------------------------------------------------- fit (float64)
def _ls(u: np.ndarray, y: np.ndarray):
    """Least squares y ~ a*u + b with a >= 0 (float64); (a, b)."""
    cnt = u.size
    su, sy = u.sum(), y.sum()
    suu, suy = (u * u).sum(), (u * y).sum()
    det = cnt * suu - su * su
    if cnt == 0:
        return 0.0, 0.0
    if det <= 0:
        return 0.0, sy / cnt
    a = (cnt * suy - su * sy) / det
    if a < 0:
        return 0.0, sy / cnt
    return a, (sy - a * su) / cnt


def fit_root(model: Model, sorted_keys: np.ndarray) -> None:
    """Root: equal-width leaves over the sample's log-like feature range,
    ra = L / (r_last - r_first), rc = r_first, rb = 0, all in float32 (the
    routing it feeds is an integer decision, so both sides compute these
    three numbers with the same float32 operations)."""
    _, r = features(sorted_keys)
    f32 = np.float32
    model.rc = f32(r[0])
    width = f32(r[-1] - r[0])
    model.ra = f32(f32(model.L) / width) if width > 0 else f32(0)
    model.rb = f32(0)


def leaf_ranges(model: Model, sorted_keys: np.ndarray):
    """[st_i, en_i): the contiguous sample range routed to leaf i."""
    _, r = features(sorted_keys)
    leaf = route(model, r)
    cnt = np.bincount(leaf, minlength=model.L)
    st = np.concatenate([[0], np.cumsum(cnt)[:-1]]).astype(np.int64)
    return st, st + cnt, leaf


def fit_leaves(model: Model, sorted_keys: np.ndarray) -> None:
    """Per-leaf least squares of j/m against dx = x - x0 (float64), with
    x0 the leaf's middle sample and the output range [st/m, en/m]."""
    m = sorted_keys.size
    x, _ = features(sorted_keys)
    st, en, _ = leaf_ranges(model, sorted_keys)
    f32 = np.float32
    for i in range(model.L):
        s, e = int(st[i]), int(en[i])
        model.lo[i] = f32(f32(s) / f32(m))     # the upper clamp is lo[i+1] = en/m
        if e == s:
            model.a[i], model.b[i], model.x0[i] = 0, model.lo[i], 0
            continue
        x0 = x[s + (e - s - 1) // 2]
        dx = (x[s:e] - x0).astype(f32).astype(np.float64)
        y = np.arange(s, e, dtype=np.float64) / m
        a, b = _ls(dx, y)
        model.a[i], model.b[i], model.x0[i] = f32(a), f32(b), x0


def fit(sorted_keys: np.ndarray, L: int) -> Model:
    mdl = Model(L)
    fit_root(mdl, sorted_keys)
    fit_leaves(mdl, sorted_keys)
    return mdl


def untrained(keys_min, keys_max, L: int) -> Model:
    """The method without training: equal-width key ranges, F linear between
    the smallest and largest key; every key in leaf 0."""
    mdl = Model(L)
    x = to_f32_rne(key_image(np.array([keys_min, keys_max])))
    width = np.float32(x[1] - x[0])
    mdl.x0[0] = x[0]
    mdl.a[0] = np.float32(np.float32(1.0) / np.float32(width)) if width > 0 else np.float32(0)
    mdl.lo[0] = 0
    mdl.lo[1:] = 1          # unused leaves; leaf 0 clamps to [0, 1]
    mdl.b[1:] = 1
    return mdl


# ------------------------------------------------ loss and gradient (float64)
def leaf_loss_grad(model: Model, sorted_keys: np.ndarray):
    """For every leaf i with its samples j in [st_i, en_i):
       loss_i = sum (a_i*dx_j + b_i - j/m)^2,
       grad_i = (d loss/d a_i, d loss/d b_i) = 2*sum res*(dx, 1),
       hess_i = 2*(sum dx^2, sum dx, count)   (Gauss-Newton = exact here).
    dx_j = float32(x_j - x0_i) as in the kernels; sums in float64."""
    m = sorted_keys.size
    x, _ = features(sorted_keys)
    st, en, _ = leaf_ranges(model, sorted_keys)
    L = model.L
    loss = np.zeros(L)
    grad = np.zeros((L, 2))
    hess = np.zeros((L, 3))
    for i in range(L):
        s, e = int(st[i]), int(en[i])
        if e == s:
            continue
        dx = (x[s:e] - model.x0[i]).astype(np.float32).astype(np.float64)
        y = np.arange(s, e, dtype=np.float64) / m
        res = np.float64(model.a[i]) * dx + np.float64(model.b[i]) - y
        loss[i] = (res * res).sum()
        grad[i] = 2 * (res * dx).sum(), 2 * res.sum()
        hess[i] = 2 * (dx * dx).sum(), 2 * dx.sum(), 2 * (e - s)
    return loss, grad, hess


def leaf_scales(model: Model, sorted_keys: np.ndarray) -> np.ndarray:
    """Per-leaf power-of-two scale s = 2**-e, 2**e <= max|x - x0| < 2**(e+1)
    over the leaf's first and last sample (1 for an empty or flat leaf); the
    kernels fit the slope in the scaled coordinate dx*s so that sums of
    dx**2 stay inside the float32 range."""
    x, _ = features(sorted_keys)
    st, en, _ = leaf_ranges(model, sorted_keys)
    out = np.ones(model.L, np.float32)
    for i in range(model.L):
        s, e = int(st[i]), int(en[i])
        if e == s:
            continue
        dm = max(abs(np.float32(x[s] - model.x0[i])), abs(np.float32(x[e - 1] - model.x0[i])))
        if dm > 0:
            _, ex = np.frexp(np.float64(dm))
            out[i] = np.float32(np.ldexp(1.0, -(int(ex) - 1)))
    return out


def leaf_grad_scaled(model: Model, sorted_keys: np.ndarray) -> np.ndarray:
    """(L, 7): loss, dL/da', dL/db, 2*sum dx'^2, 2*sum dx', 2*count, s, with
    a' = a/s and dx' = dx*s -- the quantities the backward kernel reports."""
    loss, grad, hess = leaf_loss_grad(model, sorted_keys)
    s = leaf_scales(model, sorted_keys).astype(np.float64)
    out = np.zeros((model.L, 7))
    out[:, 0] = loss
    out[:, 1] = grad[:, 0] * s      # a = a'*s, so dL/da' = s * dL/da
    out[:, 2] = grad[:, 1]
    out[:, 3] = hess[:, 0] * s * s
    out[:, 4] = hess[:, 1] * s
    out[:, 5] = hess[:, 2]
    out[:, 6] = s
    return out


def fallback_stats(keys: np.ndarray, code: np.ndarray, cap: int):
    """Runs of one code longer than ``cap`` keys: once the keys are ordered
    by code, all keys of one code form one run, and a run that does not fit
    one on-chip chunk of ``cap`` keys goes to the radix fallback.  Returns
    (number of such runs, keys in them, keys in those of them that hold one
    repeated bit pattern)."""
    code = np.asarray(code, np.int64)
    vals, counts = np.unique(code, return_counts=True)
    long_codes = vals[counts > cap]
    runs = int(long_codes.size)
    fkeys = int(counts[counts > cap].sum())
    kb = np.ascontiguousarray(keys).view(np.uint32 if keys.dtype.itemsize == 4 else np.uint64)
    ckeys = 0
    for c in long_codes.tolist():
        sel = kb[code == c]
        if np.all(sel == sel[0]):
            ckeys += int(sel.size)
    return runs, fkeys, ckeys


def bucket_stats(code: np.ndarray, cb: int, buckets: int = 4096):
    """Histogram of the top log2(buckets) bits of every code, and
    max bucket / ideal bucket."""
    shift = cb - int(np.log2(buckets))
    h = np.bincount((code >> np.uint32(shift)).astype(np.int64), minlength=buckets)
    ideal = code.size / buckets
    return h, (h.max() / ideal if code.size else 0.0)
