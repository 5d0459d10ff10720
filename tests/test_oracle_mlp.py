"""Pins of the MLP CDF oracle (oracle/mlp.py) against facts other than its
own formulas: finite differences and reverse-mode autodiff for the
gradient, hand-worked saturation cases for the forward pass, Adam's closed
forms, exact training points for keys with known features, and the table's
invariants.  Planted mistakes in the oracle are shown to be caught."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp, rmi

f32 = np.float32


def _point(seed=0, K=512):
    """A generic parameter point and training set (off the initial values,
    so no gradient block is accidentally zero)."""
    rng = np.random.default_rng(seed)
    u = np.sort(rng.random(K)).astype(f32)
    y = np.sort(rng.random(K)).astype(f32)
    p = mlp.init_params(u)
    p += rng.normal(0, 0.3, size=p.size)
    return p, u, y


def test_layout():
    assert mlp.P == 4353
    assert (mlp.OFF_A1, mlp.OFF_C1, mlp.OFF_A2, mlp.OFF_C2, mlp.OFF_A3, mlp.OFF_C3) == (0, 64, 128, 4224, 4288, 4352)


def test_gradient_matches_central_differences():
    p, u, y = _point()
    _, g = mlp.loss_grad(p, u, y)
    rng = np.random.default_rng(1)
    blocks = [(mlp.OFF_A1, mlp.OFF_C1), (mlp.OFF_C1, mlp.OFF_A2), (mlp.OFF_A2, mlp.OFF_C2),
              (mlp.OFF_C2, mlp.OFF_A3), (mlp.OFF_A3, mlp.OFF_C3), (mlp.OFF_C3, mlp.P)]
    idx = np.concatenate([rng.integers(a, b, size=min(8, b - a)) for a, b in blocks])
    for q in idx:
        h = 1e-6 * max(1.0, abs(p[q]))
        pp, pm = p.copy(), p.copy()
        pp[q] += h
        pm[q] -= h
        fd = (mlp.loss_grad(pp, u, y)[0] - mlp.loss_grad(pm, u, y)[0]) / (2 * h)
        assert abs(fd - g[q]) <= 1e-6 * max(abs(fd), abs(g[q])) + 1e-11, (q, fd, g[q])


def test_gradient_matches_reverse_mode_autodiff():
    """torch.autograd (float64) differentiates a torch transcription of the
    forward pass; the oracle's backward pass is written out by hand."""
    p, u, y = _point(seed=3)
    loss, g = mlp.loss_grad(p, u, y)
    t = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    H = mlp.H
    W1 = torch.nn.functional.softplus(t[mlp.OFF_A1:mlp.OFF_C1])
    W2 = torch.nn.functional.softplus(t[mlp.OFF_A2:mlp.OFF_C2]).reshape(H, H)
    w3 = torch.nn.functional.softplus(t[mlp.OFF_A3:mlp.OFF_C3])
    ut = torch.tensor(u, dtype=torch.float64)
    h1 = torch.tanh(ut[:, None] * W1[None, :] + t[mlp.OFF_C1:mlp.OFF_A2][None, :])
    h2 = torch.tanh(h1 @ W2.T + t[mlp.OFF_C2:mlp.OFF_A3][None, :])
    f = h2 @ w3 + t[mlp.OFF_C3]
    lt = ((f - torch.tensor(y, dtype=torch.float64)) ** 2).mean()
    lt.backward()
    assert lt.item() == pytest.approx(loss, rel=1e-12)
    np.testing.assert_allclose(g, t.grad.numpy(), rtol=1e-9, atol=1e-14)


def test_planted_mistake_in_the_backward_is_caught(monkeypatch):
    """A plausible slip (the softplus derivative taken at -a) must fail the
    finite-difference pin."""
    p, u, y = _point(seed=5)
    monkeypatch.setattr(mlp, "sigmoid", lambda x: 0.5 * (1.0 - np.tanh(0.5 * x)))
    _, g = mlp.loss_grad(p, u, y)
    q = mlp.OFF_A2 + 7
    h = 1e-6
    pp, pm = p.copy(), p.copy()
    pp[q] += h
    pm[q] -= h
    fd = (mlp.loss_grad(pp, u, y)[0] - mlp.loss_grad(pm, u, y)[0]) / (2 * h)
    assert abs(fd - g[q]) > 1e-3 * abs(fd)


def _silent(p):
    """Every weight raw -1e4 (softplus underflows to exactly 0)."""
    p[mlp.OFF_A1:mlp.OFF_C1] = -1e4
    p[mlp.OFF_A2:mlp.OFF_C2] = -1e4
    p[mlp.OFF_A3:mlp.OFF_C3] = -1e4
    return p


def test_forward_closed_forms():
    u = np.linspace(0, 1, 101)
    # no layer-2 weights: f = sum_i sp(a3_i) tanh(c2_i) + c3 whatever u is;
    # with a3 = 0 (sp = ln 2) and tanh(c2) = 1/2: f = 32 ln 2 + c3
    p = np.zeros(mlp.P)
    p[mlp.OFF_A1:mlp.OFF_C1] = 3.0
    p[mlp.OFF_A2:mlp.OFF_C2] = -1e4
    p[mlp.OFF_C2:mlp.OFF_A3] = math.atanh(0.5)
    p[mlp.OFF_A3:mlp.OFF_C3] = 0.0
    p[mlp.OFF_C3] = 0.25
    f, _, _ = mlp.forward(p, u)
    np.testing.assert_allclose(f, 32 * math.log(2) + 0.25, rtol=1e-13)
    # one path: a saturated step at u = 1/2 (A1 = 1e4, c1 = -5e3), one
    # layer-2 weight sp(0) = ln 2, one output weight ln 2, c2 = 0:
    # f = c3 +- ln 2 * tanh(ln 2) = c3 +- 0.6 ln 2 (tanh(ln 2) = 3/5)
    p = _silent(np.zeros(mlp.P))
    p[mlp.OFF_A1] = 1e4
    p[mlp.OFF_C1] = -5e3
    p[mlp.OFF_A2] = 0.0
    p[mlp.OFF_A3] = 0.0
    p[mlp.OFF_C3] = 0.5
    f, _, _ = mlp.forward(p, np.array([0.0, 0.25, 0.49, 0.51, 0.9, 1.0]))
    lo, hi = 0.5 - 0.6 * math.log(2), 0.5 + 0.6 * math.log(2)
    np.testing.assert_allclose(f, [lo, lo, lo, hi, hi, hi], rtol=1e-12)


def test_forward_is_monotone_for_any_parameters():
    rng = np.random.default_rng(7)
    u = np.linspace(0, 1, 2001)
    for _ in range(5):
        p = rng.normal(0, 3, size=mlp.P)
        f, _, _ = mlp.forward(p, u)
        assert np.all(np.diff(f) >= -1e-12)


def test_adam_closed_forms():
    """Step 1 moves every parameter by lr * g / (|g| + eps) (bias-corrected
    moments equal g and g^2); a constant gradient keeps that step size at
    every later step too."""
    rng = np.random.default_rng(9)
    g = rng.normal(0, 1, size=50)
    p0 = rng.normal(0, 1, size=50)
    p = p0.copy()
    m = np.zeros(50)
    v = np.zeros(50)
    for t in range(1, 6):
        mlp.adam_step(p, g, m, v, t)
        # |g| / (|g| + eps) differs from 1 by at most eps / |g| per step
        err = np.abs(p - (p0 - t * mlp.LR * np.sign(g)))
        assert np.all(err <= t * mlp.LR * mlp.EPS / np.abs(g) + 1e-12), t


def test_training_points_exact():
    """uint32 keys 2^e: x = 2^e exactly, its bits (127 + e) << 23 are a
    float32 integer, so the feature is linear in e and u = e / 31; with
    m = 2K the ranks are j_k = 2k + 1."""
    keys = (np.uint64(1) << np.arange(32, dtype=np.uint64)).astype(np.uint32)
    u, y = mlp.training_points(keys, 64)          # m = 32 <= K: every rank
    np.testing.assert_allclose(u, np.arange(32) / 31, rtol=1e-6)
    assert u[0] == 0 and u[-1] == 1
    np.testing.assert_array_equal(y, (np.arange(32, dtype=f32) / f32(32)))
    rng = np.random.default_rng(0)
    srt = np.sort(rng.integers(0, 1 << 32, size=8192, dtype=np.uint64).astype(np.uint32))
    u, y = mlp.training_points(srt, 4096)
    np.testing.assert_array_equal(y, (2 * np.arange(4096) + 1).astype(f32) / f32(8192))
    assert np.all(np.diff(u) >= 0)


def test_init_at_the_quantiles():
    u = (np.arange(4096) / f32(4096)).astype(f32)
    p = mlp.init_params(u)
    c = -p[mlp.OFF_C1:mlp.OFF_A2] / p[mlp.OFF_A1:mlp.OFF_C1]
    np.testing.assert_allclose(c, (2 * np.arange(64) + 1) / 128, atol=2e-4)
    # inner slopes 4 / (2 / 64) = 128; the ends see one gap
    np.testing.assert_allclose(p[mlp.OFF_A1 + 1:mlp.OFF_C1 - 1], 128, rtol=1e-3)
    # repeated keys (zero gaps) take the slope cap
    p = mlp.init_params(np.zeros(4096, f32))
    assert np.all(p[mlp.OFF_A1:mlp.OFF_C1] == 4096)


def test_training_fits_a_known_cdf_and_is_deterministic():
    u = np.linspace(0, 1, 1024).astype(f32)
    y = (u.astype(np.float64) ** 2).astype(f32)
    p, losses = mlp.train(u, y, 300)
    assert losses[-1] < losses[0] / 100
    f, _, _ = mlp.forward(p, u)
    assert np.sqrt(np.mean((f - y) ** 2)) < 0.01
    p2, _ = mlp.train(u, y, 300)
    np.testing.assert_array_equal(p, p2)


def test_table_invariants():
    rng = np.random.default_rng(2)
    k = np.floor(rng.lognormal(30, 3, size=100_000)).clip(0, 2.0 ** 63).astype(np.uint64)
    srt = np.sort(k[:20_000])
    u, y = mlp.training_points(srt, 4096)
    p, _ = mlp.train(u, y, 50)
    root = rmi.fit(srt, 1024)
    t = mlp.tabulate(p, root, 1024)
    assert t.lo[0] == 0 and np.all(np.diff(t.lo) >= 0) and t.hi[-1] == 1
    assert np.all(t.a >= 0)
    # at its knot every leaf's CDF is its lower clamp, which follows f
    f, _, _ = mlp.forward(p, np.arange(1, 1024) / 1024)
    run = np.maximum.accumulate(np.clip(f, 0, 1))
    np.testing.assert_allclose(t.lo[1:], run, atol=1e-6)
    # codes from the table never decrease along sorted keys
    c = rmi.codes(t, np.sort(k), 16)
    assert np.all(np.diff(c.astype(np.int64)) >= 0)
