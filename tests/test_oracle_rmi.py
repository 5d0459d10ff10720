"""Pins of the learned-CDF model oracle (oracle/rmi.py).

Checked against published generator outputs, exact integer arithmetic, the
definition of round-to-nearest-even, closed-form least squares on exactly
linear data, finite differences, and monotonicity.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import rmi


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_hex(name):
    vals = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if line:
            vals.append(int(line.split()[0], 16))
    return vals


def test_splitmix64_published_outputs():
    expect = _golden_hex("splitmix64_seed0.txt")
    got = rmi.splitmix64(0, np.arange(len(expect)))
    assert [int(v) for v in got] == expect


def test_mulhi64_exact():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 1 << 64, size=2000, dtype=np.uint64)
    for n in [1, 3, 1000, (1 << 31), (1 << 40) + 12345, (1 << 64) - 1]:
        got = rmi.mulhi64(a, n)
        ref = [(int(x) * n) >> 64 for x in a]
        assert [int(g) for g in got] == ref
    pos = rmi.sample_positions(0, 1000, 5000)
    assert pos.min() >= 0 and pos.max() < 1000


def test_f32_round_nearest_even_definition():
    """The result is a float32 nearest to t; on a tie its significand is even."""
    rng = np.random.default_rng(2)
    t = np.concatenate([
        rng.integers(0, 1 << 64, size=3000, dtype=np.uint64),
        rng.integers(0, 1 << 30, size=500, dtype=np.uint64),
        np.array([0, 1, (1 << 24) + 1, (1 << 24) + 3, (1 << 25) + 2, (1 << 64) - 1,
                  (1 << 63) + (1 << 39), (1 << 63) + (1 << 39) + 1, (1 << 63) + 3 * (1 << 39)],
                 dtype=np.uint64)])
    r = rmi.to_f32_rne(t)
    for ti, ri in zip(t.tolist(), r.tolist()):
        ri32 = np.float32(ri)
        up = np.nextafter(ri32, np.float32(np.inf))
        dn = np.nextafter(ri32, np.float32(0))
        d = abs(int(ri) - ti)
        if np.isfinite(up):
            assert d <= abs(int(up) - ti)
        assert d <= abs(int(dn) - ti)
        if np.isfinite(up) and (d == abs(int(up) - ti) or d == abs(int(dn) - ti)) and d:
            assert (ri32.view(np.uint32) & 1) == 0      # tie -> even
    # agrees with the library conversion where that is a single rounding
    small = rng.integers(0, 1 << 53, size=5000, dtype=np.uint64)
    assert np.array_equal(rmi.to_f32_rne(small), small.astype(np.float64).astype(np.float32))


def test_features_monotone():
    rng = np.random.default_rng(3)
    k = np.sort(rng.integers(0, 1 << 64, size=20000, dtype=np.uint64))
    x, r = rmi.features(k)
    assert np.all(np.diff(x.astype(np.float64)) >= 0)
    assert np.all(np.diff(r.astype(np.float64)) >= 0)


def test_least_squares_closed_form_on_linear_data():
    """Keys in arithmetic progression: the CDF is exactly linear in the key,
    so one leaf recovers slope 1/(d*m) and the loss is ~0."""
    m, d, c = 4096, 1000, 5_000_000
    keys = (c + d * np.arange(m)).astype(np.uint64)      # exact in float32
    mdl = rmi.Model(1)
    rmi.fit_root(mdl, keys)
    rmi.fit_leaves(mdl, keys)
    x0 = np.float64(mdl.x0[0])
    assert abs(mdl.a[0] * d * m - 1) < 1e-6
    j0 = (x0 - c) / d
    assert abs(mdl.b[0] - j0 / m) < 1e-6
    loss, grad, hess = rmi.leaf_loss_grad(mdl, keys)
    assert loss[0] < 1e-9
    # the Newton step the gradient implies is at float32 rounding level
    assert abs(grad[0, 0] / hess[0, 0]) < 1e-6 * abs(float(mdl.a[0]))
    assert abs(grad[0, 1] / hess[0, 2]) < 1e-6


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    keys = np.sort(rng.lognormal(20, 2, size=6000).astype(np.uint64))
    mdl = rmi.fit(keys, 16)
    mdl.a = (mdl.a * np.float32(1.01)).astype(np.float32)    # move off the optimum
    mdl.b = (mdl.b + np.float32(1e-3)).astype(np.float32)
    loss, grad, hess = rmi.leaf_loss_grad(mdl, keys)
    st, en, _ = rmi.leaf_ranges(mdl, keys)
    x, _ = rmi.features(keys)
    for i in range(16):
        s, e = st[i], en[i]
        if e - s < 2:
            continue
        dx = (x[s:e] - mdl.x0[i]).astype(np.float32).astype(np.float64)
        y = np.arange(s, e) / keys.size
        f = lambda a, b: ((a * dx + b - y) ** 2).sum()
        a0, b0 = float(mdl.a[i]), float(mdl.b[i])
        ha, hb = max(abs(a0), 1e-12) * 1e-5, 1e-7
        ga = (f(a0 + ha, b0) - f(a0 - ha, b0)) / (2 * ha)
        gb = (f(a0, b0 + hb) - f(a0, b0 - hb)) / (2 * hb)
        assert np.isclose(grad[i, 0], ga, rtol=1e-5, atol=1e-9 * abs(ga) + 1e-12)
        assert np.isclose(grad[i, 1], gb, rtol=1e-5, atol=1e-9)
        assert np.isclose(hess[i, 2], 2 * (e - s))
    # at the least-squares optimum the gradient vanishes
    opt = rmi.fit(keys, 16)
    _, g2, h2 = rmi.leaf_loss_grad(opt, keys)
    assert np.all(np.abs(g2[:, 1]) <= 1e-4 * (h2[:, 2] + 1))


def test_root_routes_monotone_equal_width():
    rng = np.random.default_rng(6)
    keys = np.sort(rng.integers(0, 1 << 62, size=5000, dtype=np.uint64))
    mdl = rmi.Model(64)
    rmi.fit_root(mdl, keys)
    _, r = rmi.features(keys)
    leaf = rmi.route(mdl, r)
    assert leaf[0] == 0 and leaf[-1] == 63
    assert np.all(np.diff(leaf) >= 0)
    # equal widths: the leaf of a feature at fraction f of the range is ~ f*L
    f = (r.astype(np.float64) - r[0]) / (float(r[-1]) - float(r[0]))
    assert np.all(np.abs(leaf - np.minimum(np.floor(f * 64), 63)) <= 1)


def test_scaled_gradient_finite_differences():
    """The kernels report the gradient in each leaf's scaled coordinate
    (a' = a/s, dx' = dx*s); check it against finite differences in a'."""
    rng = np.random.default_rng(12)
    keys = np.sort(rng.lognormal(30, 3, size=8000).astype(np.uint64))
    mdl = rmi.fit(keys, 32)
    mdl.a = (mdl.a * np.float32(1.03)).astype(np.float32)
    out = rmi.leaf_grad_scaled(mdl, keys)
    st, en, _ = rmi.leaf_ranges(mdl, keys)
    x, _ = rmi.features(keys)
    checked = 0
    for i in range(32):
        s, e = st[i], en[i]
        if e - s < 3:
            continue
        sc = float(out[i, 6])
        dxs = (x[s:e] - mdl.x0[i]).astype(np.float32).astype(np.float64) * sc
        y = np.arange(s, e) / keys.size
        f = lambda ap, b: ((ap * dxs + b - y) ** 2).sum()
        ap0, b0 = float(mdl.a[i]) / sc, float(mdl.b[i])
        h = max(abs(ap0), 1e-9) * 1e-6
        fd = (f(ap0 + h, b0) - f(ap0 - h, b0)) / (2 * h)
        assert np.isclose(out[i, 1], fd, rtol=1e-5, atol=1e-10), (i, out[i, 1], fd)
        assert np.isclose(out[i, 3], 2 * (dxs ** 2).sum(), rtol=1e-12)
        assert 1.0 <= np.abs(dxs).max() < 2.0          # the scale brings max|dx'| into [1, 2)
        checked += 1
    assert checked >= 10


@pytest.mark.parametrize("dist", ["uniform", "lognormal", "zipf", "f32"])
def test_codes_monotone_and_balanced(dist):
    rng = np.random.default_rng(8)
    n = 400_000
    if dist == "uniform":
        keys = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    elif dist == "lognormal":
        keys = np.floor(rng.lognormal(30, 3, size=n)).clip(0, 2.0 ** 63).astype(np.uint64)
    elif dist == "zipf":
        keys = rng.zipf(1.1, size=n).clip(1, 10_000_000).astype(np.int64)
    else:
        keys = rng.normal(0, 1e3, size=n).astype(np.float32)
        keys[:100] = np.nan
        keys[100:200] = -0.0
    m = rmi.sample_count(n, 0.05)
    pos = rmi.sample_positions(123, n, m)
    sample = oracle.sort(keys[pos])
    mdl = rmi.fit(sample, 256)
    cb = rmi.code_bits(n)
    srt = oracle.sort(keys)
    c = rmi.codes(mdl, srt, cb)
    assert np.all(np.diff(c.astype(np.int64)) >= 0)          # monotone in the key
    h, imb = rmi.bucket_stats(c, cb, 256)
    assert h.sum() == n
    if dist in ("uniform", "lognormal"):
        # statistical pin: a bucket's relative sampling error is about
        # sqrt(B/m); the largest of B such deviations stays below ~4.5 sigma
        assert imb < 1 + 4.5 * np.sqrt(256 / m), imb
    # the untrained model (equal-width key ranges) is much worse on skewed keys
    if dist == "lognormal":
        un = rmi.untrained(srt[0], srt[-1], 256)
        _, imb_u = rmi.bucket_stats(rmi.codes(un, srt, cb), cb, 256)
        assert imb_u > 10 * imb


def test_code_bits_closed_forms():
    """cb = clamp(ceil(log2 n) - 7, 12, 24): about 128 keys per code, at
    least 2**12 codes (the 4096 buckets) and at most 2**24 (three 8-bit
    passes)."""
    cases = {1: 12, 2: 12, 1 << 12: 12, 1 << 19: 12, (1 << 19) + 1: 13, 1 << 20: 13,
             (1 << 20) + 1: 14, 10 ** 6: 13, 1 << 30: 23, (1 << 30) + 1: 24, 1 << 31: 24, 1 << 40: 24}
    for n, cb in cases.items():
        assert rmi.code_bits(n) == cb, n
    # between the clamps, n / 2**cb lies in (64, 128]
    for n in [(1 << 19) + 1, 3 << 20, 10 ** 7, 2_147_000_000, 1 << 31]:
        cb = rmi.code_bits(n)
        assert 64 < n / 2 ** cb <= 128, n


def test_sample_count_closed_forms():
    """m = floor(frac * n), at least min(n, 4096); the library takes frac as
    a float32, so the pins use that value too."""
    f = float(np.float32(0.01))
    assert f == 10737418 / 2 ** 30                       # float32(0.01), exactly
    # floor(n * 10737418 / 2**30): just below n/100 when n/100 is whole
    assert rmi.sample_count(10 ** 6, f) == 9_999
    assert rmi.sample_count(10 ** 6, 0.01) == 10_000
    assert rmi.sample_count(100_000, f) == 4096          # the 4096 floor
    assert rmi.sample_count(1000, f) == 1000             # never more than n
    assert rmi.sample_count(4096 * 300, f) == 12_287
    for n in [5000, 409_601, 10 ** 7 + 3, 123_456_789]:
        assert rmi.sample_count(n, f) == min(n, max(n * 10737418 // 2 ** 30, 4096)), n
    # float32(0.01) = 10737418 * 2**-30, so at n = 2**31 the product is the
    # integer 2 * 10737418 exactly
    assert rmi.sample_count(1 << 31, f) == 21_474_836
    assert rmi.sample_count(1 << 31, 0.01) == 21_474_836
    assert rmi.sample_count(1 << 20, 1.0) == 1 << 20


def _round_f32(q):
    """Fraction -> nearest float32 (ties to even), written from the IEEE
    definition with exact rational arithmetic (subnormals included)."""
    from fractions import Fraction
    if q == 0:
        return 0.0
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, -126)
    quantum = Fraction(2) ** (e - 23)
    mq = a / quantum
    fl = mq.numerator // mq.denominator
    rem = mq - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return float((1 if q > 0 else -1) * fl * quantum)


def _code_exact(model, key: int, cb: int):
    """The model code of one uint64 key, every float32 operation rounded once
    from its exact rational value, in the order the definition states."""
    import struct
    from fractions import Fraction as Fr

    def rnd(q):  # exact result of one operation -> float32, as a Fraction
        return Fr(_round_f32(q))

    def f(v):
        return Fr(float(v))
    x = rnd(Fr(key))                                          # float(t), t = key
    rbits = struct.unpack("<I", struct.pack("<f", float(x)))[0]
    r = rnd(Fr(rbits))
    u = rnd(r - f(model.rc))
    p = rnd(rnd(f(model.ra) * u) + f(model.rb))
    p = min(max(p, Fr(0)), Fr(model.L - 1))
    leaf = int(p)
    dx = rnd(x - f(model.x0[leaf]))
    F = rnd(rnd(f(model.a[leaf]) * dx) + f(model.b[leaf]))
    hi = f(model.lo[leaf + 1]) if leaf + 1 < model.L else Fr(1)
    F = min(max(F, f(model.lo[leaf])), hi)
    c = rnd(F * Fr(2 ** cb))
    return leaf, float(F), min(int(c), (1 << cb) - 1)


def test_codes_match_exact_rational_evaluation():
    """route / cdf / codes use float32 arithmetic with one rounding per
    operation and no fused multiply-add: each key's leaf, CDF value and code
    equal an exact-rational evaluation rounded after every operation (a
    float64 evaluation rounded once at the end, or a fused product, would
    differ on some of these keys)."""
    rng = np.random.default_rng(21)
    sample = np.sort(np.concatenate([
        np.floor(rng.lognormal(30, 3, size=3000)).clip(0, 2.0 ** 63).astype(np.uint64),
        rng.integers(0, 1 << 64, size=1000, dtype=np.uint64),
        rng.integers(1, 10_000_000, size=1000).astype(np.uint64)]))
    mdl = rmi.fit(sample, 64)
    keys = np.concatenate([
        rng.choice(sample, 600),
        np.floor(rng.lognormal(30, 3, size=600)).clip(0, 2.0 ** 63).astype(np.uint64),
        rng.integers(0, 1 << 64, size=300, dtype=np.uint64),
        np.array([0, 1, (1 << 24) + 1, (1 << 63) + (1 << 39), (1 << 64) - 1], dtype=np.uint64)])
    # keys whose leaf a float64 evaluation of the route would change (within
    # one float32 rounding of a leaf boundary), found by scanning keys spread
    # evenly over the log-like feature
    scan = np.exp2(rng.uniform(0, 63.9, size=1 << 21)).astype(np.uint64)
    _, rs = rmi.features(scan)
    p64 = np.float64(mdl.ra) * (rs.astype(np.float64) - np.float64(mdl.rc)) + np.float64(mdl.rb)
    near = scan[np.minimum(np.maximum(p64, 0), mdl.L - 1).astype(np.int64) != rmi.route(mdl, rs)]
    assert near.size > 0
    keys = np.concatenate([keys, near[:200]])
    _, r = rmi.features(keys)
    leaf = rmi.route(mdl, r)
    F = rmi.cdf(mdl, keys)
    for cb in (12, 24):
        c = rmi.codes(mdl, keys, cb)
        for i, kv in enumerate(keys.tolist()):
            lx, fx, cx = _code_exact(mdl, kv, cb)
            assert (leaf[i], float(F[i]), int(c[i])) == (lx, fx, cx), (kv, cb)


def test_bucket_and_fallback_stats_closed_forms():
    cb = 14
    # every code once: each of the 4096 buckets holds 2**(cb-12) codes
    code = np.arange(1 << cb, dtype=np.uint32)
    h, imb = rmi.bucket_stats(code, cb, 4096)
    assert np.all(h == 4) and imb == 1.0
    # all keys in code 0: one bucket holds everything
    h, imb = rmi.bucket_stats(np.zeros(1000, np.uint32), cb, 4096)
    assert h[0] == 1000 and h[1:].sum() == 0 and imb == 4096.0
    # runs: code 3 x5 (one repeated key), code 7 x4 (two keys), code 9 x2
    code = np.array([3, 3, 3, 3, 3, 7, 7, 7, 7, 9, 9], np.uint32)
    keys = np.array([5, 5, 5, 5, 5, 8, 8, 8, 9, 10, 11], np.uint64)
    assert rmi.fallback_stats(keys, code, 2) == (2, 9, 5)
    assert rmi.fallback_stats(keys, code, 4) == (1, 5, 5)
    assert rmi.fallback_stats(keys, code, 5) == (0, 0, 0)
    # the runs are found by code, not by position
    p = np.random.default_rng(0).permutation(code.size)
    assert rmi.fallback_stats(keys[p], code[p], 2) == (2, 9, 5)
    f = np.array([-0.0, 0.0, -0.0], np.float32)     # distinct bit patterns: not constant
    assert rmi.fallback_stats(f, np.zeros(3, np.uint32), 2) == (1, 3, 0)
