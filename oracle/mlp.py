"""MLP CDF model oracle: TEST INFRASTRUCTURE ONLY (never imported by the
library; only tests, the smoke check and the benchmark's CPU leg use it).

The paper's library has no learned model (its sorter is a merge sort,
Sec. II-B).  The learned partition sort this package checks may use, in
place of the two-level linear model, a small network: 1 input, two hidden
layers of 64 units, 1 output.  This module is that network's definition,
written out plainly in float64:

  input    u in [0, 1]: the log-like key feature of the linear model's root
           (the bits of float32(image(key)) read as an unsigned integer and
           rounded to float32), shifted and scaled over the sample's range:
           u = (r - r_first) * s, s = float32(1 / (r_last - r_first)), in
           float32 (the GPU forms the same float32 values);
  layer 1  h1 = tanh(W1 * u + c1)                 (64 units)
  layer 2  h2 = tanh(W2 @ h1 + c2)                (64 x 64 weights)
  output   f  = w3 . h2 + c3
  weights  W1 = sp(A1), W2 = sp(A2), w3 = sp(a3), sp = softplus: every
           weight is positive and tanh increases, so f increases with u
           (a monotone CDF estimate by construction); biases are free.
  loss     L = mean over the training points k of (f(u_k) - y_k)^2, with
           the points at evenly spaced ranks j_k of the sorted sample of m
           keys and y_k = j_k / m (the empirical CDF).
  training Adam (Kingma & Ba, ICLR 2015) on the raw parameters
           (A1, c1, A2, c2, a3, c3), from a start placed at the quantiles
           of the training inputs (init_params).
  table    the trained f is evaluated at the left edges u_i = i / L of the
           root's L equal feature widths and turned into the linear model's
           leaf records: leaf i interpolates linearly in x = float32(key
           image) between its knot and the next, clamped to [lo_i,
           lo_{i+1}], lo_i = the running maximum of clamp(f(u_i), 0, 1),
           lo_0 = 0, lo_L = 1.  The per-key inference then costs what the
           linear model's does.

Parameter layout (flat, P = 4353 floats): A1[64] | c1[64] | A2[64 x 64]
(row i: layer-2 unit i, column j: layer-1 unit j) | c2[64] | a3[64] | c3.

Parity: the analytic gradient is pinned by central finite differences, the
forward pass by hand-worked special cases, Adam's first step by its closed
form (every parameter moves by lr * sign(gradient)), the table by
monotonicity and by agreement with f at the knots.
"""
from __future__ import annotations

import numpy as np

from . import rmi

H = 64
P = H + H + H * H + H + H + 1
OFF_A1, OFF_C1, OFF_A2 = 0, H, 2 * H
OFF_C2 = OFF_A2 + H * H
OFF_A3 = OFF_C2 + H
OFF_C3 = OFF_A3 + H

# Adam's constants (the published defaults, with the step size used here)
LR, BETA1, BETA2, EPS = 1e-2, 0.9, 0.999, 1e-8


def unpack(params: np.ndarray):
    p = np.asarray(params, np.float64)
    return (p[OFF_A1:OFF_C1], p[OFF_C1:OFF_A2], p[OFF_A2:OFF_C2].reshape(H, H), p[OFF_C2:OFF_A3],
            p[OFF_A3:OFF_C3], p[OFF_C3])


def softplus(x: np.ndarray) -> np.ndarray:
    return np.logaddexp(0.0, x)


def sigmoid(x: np.ndarray) -> np.ndarray:
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def init_params(u: np.ndarray) -> np.ndarray:
    """Fixed start from the training inputs u (nondecreasing, as the
    training points come in rank order), in float32 so both sides start
    from the same values: layer-1 unit i steps at the centre c_i =
    u[floor((2i + 1) K / 128)] (the 64 quantiles of the points) with slope
    s_i = clamp(4 / (c_{i+1} - c_{i-1}), 16, 4096) (one-sided at the ends),
    i.e. A1_i = s_i (softplus(s) = s to float32 precision for s >= 16) and
    c1_i = -(s_i * c_i); layer 2 passes every unit on (raw weights 2 on the
    diagonal, -7 elsewhere: 2.13 and 9.1e-4); the output adds them with raw
    weight -5 (0.0067) around c3 = 1/2.  So f starts as a smoothed staircase
    through the points' quantiles."""
    f32 = np.float32
    u = np.asarray(u, f32)
    K = u.size
    c = u[((2 * np.arange(H) + 1) * K) // (2 * H)].astype(f32)
    nxt = c[np.minimum(np.arange(H) + 1, H - 1)]
    prv = c[np.maximum(np.arange(H) - 1, 0)]
    gap = (nxt - prv).astype(f32)
    with np.errstate(divide="ignore"):
        s = np.where(gap > 0, (f32(4.0) / np.where(gap > 0, gap, f32(1))).astype(f32), f32(4096))
    s = np.minimum(np.maximum(s, f32(16)), f32(4096)).astype(f32)
    p = np.zeros(P, f32)
    p[OFF_A1:OFF_C1] = s
    p[OFF_C1:OFF_A2] = -(s * c).astype(f32)
    a2 = np.full((H, H), f32(-7.0), f32)
    np.fill_diagonal(a2, f32(2.0))
    p[OFF_A2:OFF_C2] = a2.ravel()
    p[OFF_A3:OFF_C3] = f32(-5.0)
    p[OFF_C3] = f32(0.5)
    return p.astype(np.float64)


def forward(params: np.ndarray, u: np.ndarray):
    """f(u) for a vector of inputs; also returns the hidden activations."""
    A1, c1, A2, c2, a3, c3 = unpack(params)
    W1, W2, w3 = softplus(A1), softplus(A2), softplus(a3)
    u = np.asarray(u, np.float64)
    h1 = np.tanh(np.outer(u, W1) + c1)          # [K, 64]
    h2 = np.tanh(h1 @ W2.T + c2)                # [K, 64]
    f = h2 @ w3 + c3                            # [K]
    return f, h1, h2


def loss_grad(params: np.ndarray, u: np.ndarray, y: np.ndarray):
    """(loss, gradient with respect to the raw parameters), by the chain
    rule written out layer by layer."""
    A1, c1, A2, c2, a3, c3 = unpack(params)
    W1, W2, w3 = softplus(A1), softplus(A2), softplus(a3)
    u = np.asarray(u, np.float64)
    y = np.asarray(y, np.float64)
    K = u.size
    f, h1, h2 = forward(params, u)
    r = f - y
    loss = float(np.mean(r * r))
    df = 2.0 * r / K                            # dL/df per point
    g = np.zeros(P, np.float64)
    dw3 = h2.T @ df
    g[OFF_C3] = df.sum()
    dz2 = np.outer(df, w3) * (1.0 - h2 * h2)    # [K, 64]
    dW2 = dz2.T @ h1                            # [64, 64]
    g[OFF_C2:OFF_A3] = dz2.sum(axis=0)
    dh1 = dz2 @ W2                              # [K, 64]
    dz1 = dh1 * (1.0 - h1 * h1)
    dW1 = dz1.T @ u
    g[OFF_C1:OFF_A2] = dz1.sum(axis=0)
    # through the softplus of every weight: d sp(a) / da = sigmoid(a)
    g[OFF_A1:OFF_C1] = dW1 * sigmoid(A1)
    g[OFF_A2:OFF_C2] = (dW2 * sigmoid(A2)).ravel()
    g[OFF_A3:OFF_C3] = dw3 * sigmoid(a3)
    return loss, g


def adam_step(params: np.ndarray, grad: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, lr: float = LR):
    """One Adam update (step t >= 1) of params, m, v in place."""
    m *= BETA1
    m += (1.0 - BETA1) * grad
    v *= BETA2
    v += (1.0 - BETA2) * grad * grad
    mhat = m / (1.0 - BETA1 ** t)
    vhat = v / (1.0 - BETA2 ** t)
    params -= lr * mhat / (np.sqrt(vhat) + EPS)


def training_points(sorted_keys: np.ndarray, K: int):
    """(u, y) at ranks j_k = floor((2k + 1) m / (2K)) of the sorted sample
    (every rank if m <= K), as float32: u from the root's feature, y = j/m."""
    m = sorted_keys.size
    K = min(K, m)
    k = np.arange(K, dtype=np.int64)
    j = ((2 * k + 1) * m) // (2 * K)
    f32 = np.float32
    _, r = rmi.features(sorted_keys)
    r0, r1 = f32(r[0]), f32(r[-1])
    width = f32(r1 - r0)
    s = f32(f32(1.0) / width) if width > 0 else f32(0)
    u = ((r[j] - r0).astype(f32) * s).astype(f32)
    y = (j.astype(f32) / f32(m)).astype(f32)
    return u, y


def train(u: np.ndarray, y: np.ndarray, iters: int, lr: float = LR, params: np.ndarray | None = None):
    """Adam from init_params(u) (or `params`) for `iters` steps; returns the
    parameters and the loss before every step."""
    p = init_params(u) if params is None else np.asarray(params, np.float64).copy()
    m = np.zeros(P)
    v = np.zeros(P)
    losses = []
    for t in range(1, iters + 1):
        loss, g = loss_grad(p, u, y)
        losses.append(loss)
        adam_step(p, g, m, v, t, lr)
    return p, np.array(losses)


def tabulate(params: np.ndarray, root: "rmi.Model", L: int) -> "rmi.Model":
    """Leaf records of the linear model's format from the network: root as
    given (rc, ra over the sample's feature range), knots u_i = i / L, F_i =
    f(u_i) clamped to [0, 1] with F_0 = 0 and F_L = 1, then made
    nondecreasing (running maximum); leaf i interpolates in x between its
    knot x_i and x_{i+1}, where x_i is the float32 whose bits are the knot's
    feature value rc + i * (1 / ra) (float32 operations, truncated to an
    integer)."""
    f32 = np.float32
    mdl = rmi.Model(L)
    mdl.rc, mdl.ra, mdl.rb = root.rc, root.ra, root.rb
    u = np.arange(L + 1, dtype=np.float64) / L
    F, _, _ = forward(params, u)
    F = np.clip(F, 0.0, 1.0)
    F[0], F[L] = 0.0, 1.0
    lo = np.maximum.accumulate(F).astype(f32)
    step = f32(f32(1.0) / f32(root.ra)) if root.ra > 0 else f32(0)
    r_knot = (f32(root.rc) + (np.arange(L + 1, dtype=f32) * step).astype(f32)).astype(f32)
    xk = r_knot.astype(np.float64).astype(np.uint64).astype(np.uint32).view(np.float32)
    dx = (xk[1:] - xk[:-1]).astype(f32)
    dlo = (lo[1:] - lo[:-1]).astype(f32)
    a = np.where(dx > 0, (dlo / np.where(dx > 0, dx, f32(1))).astype(f32), f32(0)).astype(f32)
    mdl.a = a[:L].copy()
    mdl.b = lo[:L].copy()
    mdl.x0 = xk[:L].copy()
    mdl.lo = lo[:L].copy()
    return mdl
