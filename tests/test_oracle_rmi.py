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
