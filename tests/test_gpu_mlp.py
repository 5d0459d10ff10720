"""GPU parity of the MLP CDF model (the second learned model): forward and
backward against the float64 oracle, the start and Adam's first step, a
full training run against the oracle's, the table, and the learned sort
with the MLP table (bit-exact output, statistics equal to the oracle's
counts for that table)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2507_16710_amd as ak
import synth
from gpucheck import to_gpu, to_host
from oracle import mlp, rmi
from pools import bits

pytestmark = pytest.mark.gpu

F32_FRAC = float(np.float32(0.01))


def _keys(dist: str, n: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    if dist == "mixture":
        return synth.as_numpy(synth.workload5(n=n, seed=seed), "u64"), "u64"
    if dist == "lognormal":
        return np.floor(rng.lognormal(30, 3, size=n)).clip(0, 2.0 ** 63).astype(np.uint64), "u64"
    if dist == "uniform":
        return rng.integers(0, 1 << 64, size=n, dtype=np.uint64), "u64"
    if dist == "f32":
        return synth.as_numpy(synth.workload2(n=n, seed=seed), "f32"), "f32"
    if dist == "zipf":
        return rng.zipf(1.1, size=n).clip(1, 10_000_000).astype(np.int64), "i64"
    raise ValueError(dist)


def _sample(k: np.ndarray) -> np.ndarray:
    n = k.size
    return oracle.sort(k[rmi.sample_positions(0, n, rmi.sample_count(n, F32_FRAC))])


def _cuda(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("dist", ["mixture", "lognormal", "uniform", "f32"])
def test_loss_and_gradient_match_oracle(dist):
    """float32 sums on the GPU vs float64: the loss within 1e-4 relative,
    every gradient entry within 1e-3 of itself plus 2e-4 of its block's
    largest entry (sums of 4096 signed terms, tanh to a few ulps)."""
    k, dt = _keys(dist, 1 << 21, seed=2)
    u, y = mlp.training_points(_sample(k), 4096)
    rng = np.random.default_rng(5)
    for p in (mlp.init_params(u), mlp.init_params(u) + rng.normal(0, 0.2, size=mlp.P)):
        p32 = p.astype(np.float32)
        out = ak.mlp_loss_grad(_cuda(u), _cuda(y), _cuda(p32)).cpu().numpy().astype(np.float64)
        loss, g = mlp.loss_grad(p32.astype(np.float64), u, y)
        assert out[-1] == pytest.approx(loss, rel=1e-4)
        blocks = [(mlp.OFF_A1, mlp.OFF_C1), (mlp.OFF_C1, mlp.OFF_A2), (mlp.OFF_A2, mlp.OFF_C2),
                  (mlp.OFF_C2, mlp.OFF_A3), (mlp.OFF_A3, mlp.OFF_C3), (mlp.OFF_C3, mlp.P)]
        for a, b in blocks:
            err = np.abs(out[a:b] - g[a:b])
            tol = 1e-3 * np.abs(g[a:b]) + 2e-4 * np.abs(g[a:b]).max() + 1e-12
            assert np.all(err <= tol), (dist, a, float(err.max()), float(np.abs(g[a:b]).max()))


def test_start_and_first_adam_step():
    """The start is the oracle's, bit for bit (the same float32 operations);
    after one step every parameter whose gradient is not tiny moved by
    exactly lr against its sign (Adam's first step)."""
    k, dt = _keys("lognormal", 1 << 21, seed=3)
    srt = _sample(k)
    u, y = mlp.training_points(srt, 4096)
    p0_gpu, _ = ak.mlp_fit(to_gpu(srt, dt), iters=0, leaves=1024, dtype=dt)
    p0 = mlp.init_params(u)
    assert np.array_equal(p0_gpu.cpu().numpy(), p0.astype(np.float32))
    p1_gpu, _ = ak.mlp_fit(to_gpu(srt, dt), iters=1, leaves=1024, dtype=dt)
    _, g = mlp.loss_grad(p0, u, y)
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    d = p1_gpu.cpu().numpy().astype(np.float64) - p0
    np.testing.assert_allclose(d[big], -mlp.LR * np.sign(g[big]), atol=2e-6 * np.abs(p0[big]).max() + 1e-6)
    assert np.all(np.abs(d) <= mlp.LR * 1.0001 + 1e-6)


@pytest.mark.parametrize("dist", ["mixture", "lognormal"])
def test_training_run_and_table(dist):
    """300 Adam steps on the GPU (float32) and in the oracle (float64) from
    the same start reach losses within a factor of 2 of each other; the
    GPU's table is the oracle's table of the GPU's parameters (knot values
    within float32 evaluation error), with the root of the linear model."""
    k, dt = _keys(dist, 1 << 22, seed=4)
    srt = _sample(k)
    u, y = mlp.training_points(srt, 4096)
    params, model = ak.mlp_fit(to_gpu(srt, dt), iters=300, leaves=4096, dtype=dt)
    pg = params.cpu().numpy().astype(np.float64)
    loss_gpu = mlp.loss_grad(pg, u, y)[0]
    p_ref, losses = mlp.train(u, y, 300)
    loss_ref = mlp.loss_grad(p_ref, u, y)[0]
    assert losses[-1] < losses[0] / 10
    assert loss_ref / 2 <= loss_gpu <= loss_ref * 2, (loss_gpu, loss_ref)
    got = rmi.Model.from_array(model.cpu().numpy())
    root = rmi.Model(4096)
    rmi.fit_root(root, srt)
    assert (got.rc, got.ra, got.rb) == (root.rc, root.ra, root.rb)
    ref = mlp.tabulate(pg, root, 4096)
    assert got.lo[0] == 0 and np.all(np.diff(got.lo) >= 0) and np.all(got.a >= 0)
    np.testing.assert_allclose(got.lo, ref.lo, atol=2e-5)
    assert np.array_equal(got.x0, ref.x0)


def _mlp_stats(k: np.ndarray, dt: str, cap: int = 2048) -> dict:
    """Statistics the learned sort with the MLP model must report: the table
    ak_mlp_fit makes from the sort's own sample (the oracle cannot train a
    float32 network bit for bit), then the oracle's codes and counts."""
    n = k.size
    srt = _sample(k)
    _, model = ak.mlp_fit(to_gpu(srt, dt), iters=300, leaves=4096, dtype=dt)
    tab = rmi.Model.from_array(model.cpu().numpy())
    cb = rmi.code_bits(n)
    code = rmi.codes(tab, k, cb)
    h, imb = rmi.bucket_stats(code, cb, 4096)
    runs, fkeys, ckeys = rmi.fallback_stats(k, code, cap)
    return {"max_bucket": int(h.max()), "imbalance": float(imb), "fallback_runs": runs, "fallback_keys": fkeys,
            "constant_keys": ckeys, "code_bits": cb}


@pytest.mark.parametrize("dist,n", [("mixture", 4096 * 512), ("lognormal", 1_500_007), ("f32", 1 << 20),
                                    ("zipf", 1_000_003), ("uniform", 1 << 21)])
def test_learned_sort_with_mlp(dist, n):
    k, dt = _keys(dist, n, seed=6)
    ref = _mlp_stats(k, dt)
    t = to_gpu(k, dt)
    _, st = ak.sort_learned_(t, dtype=dt, cfg=ak.make_cfg(model="mlp"), stats=True)
    print(dist, "mlp", st)
    assert np.array_equal(bits(to_host(t, dt)), bits(oracle.sort(k)))
    for f in ("max_bucket", "fallback_runs", "fallback_keys", "constant_keys", "code_bits"):
        assert st[f] == ref[f], (f, st[f], ref[f])


def test_mlp_gain_over_untrained_and_beside_rmi():
    """On the skewed mixture the trained network leaves far fewer keys to
    the fallback than the method without a model; the two-level model's
    figures are printed beside it."""
    k, dt = _keys("mixture", 4096 * 1024, seed=1)
    ref = oracle.sort(k)
    out = {}
    for name, cfg in (("mlp", ak.make_cfg(model="mlp")), ("rmi", None), ("untrained", ak.make_cfg(untrained=True))):
        t = to_gpu(k, dt)
        _, out[name] = ak.sort_learned_(t, dtype=dt, cfg=cfg, stats=True)
        assert np.array_equal(to_host(t, dt), ref), name
    print(out)
    nonconst = {k_: v["fallback_keys"] - v["constant_keys"] for k_, v in out.items()}
    assert out["mlp"]["imbalance"] * 10 < out["untrained"]["imbalance"]
    assert nonconst["mlp"] * 10 < max(nonconst["untrained"], 1)
