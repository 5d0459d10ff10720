"""GPU parity of the learned-CDF partition sort and its building blocks.

Sorting results are bit-exact against the oracle sort; model codes and
routing (integers decided in float32) are bit-exact against the oracle's
float32 evaluation of the same parameters; fitted parameters, losses and
gradients (float32 sums on the GPU, float64 in the oracle) within stated
tolerances.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2507_16710_amd as ak
import synth
from gpucheck import fingerprint, is_sorted, rank_checks, to_gpu, to_host
from pools import DTYPES, bits, random_keys
from oracle import rmi

pytestmark = pytest.mark.gpu


def _keys(dist: str, n: int, seed: int = 0) -> tuple:
    rng = np.random.default_rng(seed)
    if dist == "mixture":
        return synth.as_numpy(synth.workload5(n=n, seed=seed), "u64"), "u64"
    if dist == "lognormal":
        return np.floor(rng.lognormal(30, 3, size=n)).clip(0, 2.0 ** 63).astype(np.uint64), "u64"
    if dist == "zipf":
        return rng.zipf(1.1, size=n).clip(1, 10_000_000).astype(np.int64), "i64"
    if dist == "uniform":
        return rng.integers(0, 1 << 64, size=n, dtype=np.uint64), "u64"
    if dist == "f32":
        return synth.as_numpy(synth.workload2(n=n, seed=seed), "f32"), "f32"
    raise ValueError(dist)


def _sorted_sample(k: np.ndarray, dt: str, m: int, seed: int = 7) -> np.ndarray:
    pos = rmi.sample_positions(seed, k.size, m)
    return oracle.sort(k[pos])


def test_sample_gather_exact():
    k, dt = _keys("uniform", 100_000)
    got = ak.learned_sample(to_gpu(k, dt), 5000, seed=123, dtype=dt)
    assert np.array_equal(to_host(got, dt), k[rmi.sample_positions(123, k.size, 5000)])


@pytest.mark.parametrize("dist", ["lognormal", "zipf", "f32", "uniform"])
def test_codes_bit_exact(dist):
    """Given the oracle's model, the GPU's leaf routing and codes match the
    oracle's float32 evaluation exactly."""
    k, dt = _keys(dist, 200_000)
    srt = _sorted_sample(k, dt, 20_000)
    mdl = rmi.fit(srt, 512)
    model = torch.from_numpy(mdl.as_array()).cuda()
    for cb in (12, 20, 24):
        got = ak.rmi_codes(to_gpu(k, dt), model, cb, dtype=dt)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy().view(np.uint32), rmi.codes(mdl, k, cb)), cb


@pytest.mark.parametrize("dist", ["lognormal", "mixture", "zipf", "f32"])
def test_fit_matches_least_squares(dist):
    n = 4096 * 64 if dist == "mixture" else 300_000
    k, dt = _keys(dist, n)
    srt = _sorted_sample(k, dt, 30_000)
    L = 256
    model = ak.rmi_fit(to_gpu(srt, dt), leaves=L, iters=3, dtype=dt)
    got = rmi.Model.from_array(model.cpu().numpy())
    ref = rmi.fit(srt, L)
    # root and leaf ranges: float32 formulas, exact
    assert (got.rc, got.ra, got.rb) == (ref.rc, ref.ra, ref.rb)
    assert np.array_equal(got.lo, ref.lo)
    assert got.as_array()[-1] == 1.0                       # sentinel lower clamp
    st, en, _ = rmi.leaf_ranges(ref, srt)
    nonempty = en > st
    assert np.array_equal(got.x0[nonempty], ref.x0[nonempty])
    assert np.all(got.a >= 0)
    # fitted CDF at the samples: float32 Newton vs float64 least squares
    Fg = rmi.cdf(got, srt).astype(np.float64)
    Fr = rmi.cdf(ref, srt).astype(np.float64)
    width = (got.hi - got.lo)[rmi.route(ref, rmi.features(srt)[1])]
    assert np.all(np.abs(Fg - Fr) <= 1e-3 * width + 2e-6), np.max(np.abs(Fg - Fr))
    # the GPU fit is a least-squares optimum: its loss is within 1% (plus a
    # float32 floor) of the float64 optimum, leaf by leaf
    lg = rmi.leaf_loss_grad(got, srt)[0]
    lr = rmi.leaf_loss_grad(ref, srt)[0]
    cnt = (en - st).astype(np.float64)
    assert np.all(lg <= lr * 1.01 + cnt * 1e-13 + 1e-12)


@pytest.mark.parametrize("dist", ["lognormal", "mixture"])
def test_forward_backward_match_oracle(dist):
    """Loss, gradient and curvature of every leaf for parameters moved off
    the optimum: GPU float32 sums vs oracle float64, relative 2e-3."""
    n = 4096 * 64 if dist == "mixture" else 300_000
    k, dt = _keys(dist, n)
    srt = _sorted_sample(k, dt, 30_000)
    mdl = rmi.fit(srt, 128)
    mdl.a = (mdl.a * np.float32(1.05)).astype(np.float32)
    mdl.b = (mdl.b + np.float32(2e-4)).astype(np.float32)
    out = ak.rmi_leaf_grad(to_gpu(srt, dt), torch.from_numpy(mdl.as_array()).cuda(), dtype=dt).cpu().numpy()
    assert out.shape == (128, 8)
    ref = rmi.leaf_grad_scaled(mdl, srt)
    assert np.array_equal(out[:, 6], ref[:, 6].astype(np.float32))       # scales: exact
    assert np.array_equal(out[:, 5], ref[:, 5].astype(np.float32))       # counts: exact
    for col in range(5):
        scale = np.abs(ref[:, col]).max() + 1e-30
        err = np.abs(out[:, col] - ref[:, col])
        assert np.all(err <= 2e-3 * np.abs(ref[:, col]) + 1e-5 * scale), (col, err.max())


@pytest.mark.parametrize("dist", ["mixture", "lognormal", "zipf", "uniform", "f32"])
def test_learned_sort_bit_exact(dist):
    n = 4096 * 300 if dist == "mixture" else 1_000_003
    k, dt = _keys(dist, n, seed=3)
    t = to_gpu(k, dt)
    _, st = ak.sort_learned_(t, dtype=dt, stats=True)
    assert np.array_equal(bits(to_host(t, dt)), bits(oracle.sort(k))), st


@pytest.mark.parametrize("dt", DTYPES)
def test_learned_sort_all_dtypes_and_edges(dt):
    rng = np.random.default_rng(11)
    for n in [1, 7, 4096, 4097, 50_000, 200_001]:
        for kind in ["mixed", "ties", "uniform"]:
            k = random_keys(dt, n, rng, kind)
            t = to_gpu(k, dt)
            ak.sort_learned_(t, dtype=dt)
            torch.cuda.synchronize()
            assert np.array_equal(bits(to_host(t, dt)), bits(oracle.sort(k))), (dt, n, kind)


def test_learned_chunks_with_repeated_spread_keys():
    """Chunks whose keys spread over all 64 bits and repeat: values drawn
    once to 99 times each.  A chunk whose groups of equal top bits stay
    short is finished by comparisons inside the groups; one holding a long
    run of equal keys takes the passes over every varying bit."""
    rng = np.random.default_rng(21)
    for dt, hi in (("u64", 1 << 64), ("i64", 1 << 63)):
        vals = rng.integers(0, hi, size=20_000, dtype=np.uint64)
        k = np.repeat(vals, rng.integers(1, 100, size=vals.size))
        rng.shuffle(k)
        k = k.view(np.int64) if dt == "i64" else k
        t = to_gpu(k, dt)
        ak.sort_learned_(t, dtype=dt)
        torch.cuda.synchronize()
        assert np.array_equal(bits(to_host(t, dt)), bits(oracle.sort(k))), dt


def test_learned_degenerate_and_configs():
    rng = np.random.default_rng(5)
    n = 300_000
    cases = {
        "constant": np.full(n, 42, dtype=np.uint64),
        "two_values": rng.choice(np.array([5, 1 << 60], dtype=np.uint64), size=n),
        "presorted": np.sort(rng.integers(0, 1 << 64, size=n, dtype=np.uint64)),
        "reversed": np.sort(rng.integers(0, 1 << 64, size=n, dtype=np.uint64))[::-1].copy(),
    }
    for name, k in cases.items():
        for cfg in [None, ak.make_cfg(untrained=True), ak.make_cfg(leaves=1), ak.make_cfg(leaves=65536),
                    ak.make_cfg(sample_frac=1.0, train_iters=1)]:
            t = to_gpu(k, "u64")
            ak.sort_learned_(t, dtype="u64", cfg=cfg)
            torch.cuda.synchronize()
            assert np.array_equal(to_host(t, "u64"), oracle.sort(k)), name
    nan = np.full(100_000, np.nan, dtype=np.float32)
    nan.view(np.uint32)[:] = rng.integers(0x7F800001, 0x7FFFFFFF, size=nan.size, dtype=np.uint32)
    t = to_gpu(nan, "f32")
    ak.sort_learned_(t, dtype="f32")
    assert np.array_equal(bits(to_host(t, "f32")), bits(nan))       # NaNs keep input order


def test_trained_model_gains_over_untrained():
    """On the skewed mixture the trained model leaves far fewer keys to the
    radix fallback and balances the 4096 buckets far better than the
    method without it (equal-width key ranges)."""
    k, dt = _keys("mixture", 4096 * 1024, seed=1)
    t = to_gpu(k, dt)
    _, st_tr = ak.sort_learned_(t, dtype=dt, stats=True)
    ref = oracle.sort(k)
    assert np.array_equal(to_host(t, dt), ref)
    t = to_gpu(k, dt)
    _, st_un = ak.sort_learned_(t, dtype=dt, cfg=ak.make_cfg(untrained=True), stats=True)
    assert np.array_equal(to_host(t, dt), ref)
    nonconst_tr = st_tr["fallback_keys"] - st_tr["constant_keys"]
    nonconst_un = st_un["fallback_keys"] - st_un["constant_keys"]
    print("trained", st_tr, "untrained", st_un)
    assert st_tr["imbalance"] * 10 < st_un["imbalance"]
    assert nonconst_tr * 10 < max(nonconst_un, 1)


def test_workload5_full_size():
    """2**31 uint64 mixture keys (17 GiB): learned sort == plain radix sort
    bit for bit; sorted, same multiset, sampled ranks."""
    keys = synth.workload5(device="cuda")
    fp = fingerprint(keys)
    plain = keys.clone()
    ak.sort_(plain, dtype="u64")
    lrn = keys.clone()
    _, st = ak.sort_learned_(lrn, dtype="u64", stats=True)
    torch.cuda.synchronize()
    print(st)
    assert torch.equal(plain, lrn)
    assert is_sorted(lrn, "u64") and fingerprint(lrn) == fp
    del plain
    rank_checks(keys, lrn, "u64", samples=8)


# the library's default sample fraction, 0.01 as a float32
F32_FRAC = float(np.float32(0.01))


def _oracle_stats(k: np.ndarray, dt: str, seed: int = 0, leaves: int = 4096, iters: int = 3,
                  cap: int = 2048) -> dict:
    """What ak_sort_learned must report, computed on the host: the sample the
    sort draws (positions from the oracle's SplitMix64), sorted by the
    oracle; the model fitted to it by ak_rmi_fit (the sort's own fit, whose
    parameters the oracle cannot reproduce bit for bit from float64); then
    the oracle's float32 codes of every key under that model, the top-bucket
    histogram and the runs of one code longer than one on-chip chunk."""
    n = k.size
    m = rmi.sample_count(n, F32_FRAC)
    srt = oracle.sort(k[rmi.sample_positions(seed, n, m)])
    model = ak.rmi_fit(to_gpu(srt, dt), leaves=leaves, iters=iters, dtype=dt)
    mdl = rmi.Model.from_array(model.cpu().numpy())
    cb = rmi.code_bits(n)
    code = rmi.codes(mdl, k, cb)
    h, imb = rmi.bucket_stats(code, cb, 4096)
    runs, fkeys, ckeys = rmi.fallback_stats(k, code, cap)
    return {"n": n, "sample_size": m, "leaves": leaves, "code_bits": cb, "max_bucket": int(h.max()),
            "imbalance": float(imb), "fallback_runs": runs, "fallback_keys": fkeys, "constant_keys": ckeys}


@pytest.mark.parametrize("dist,n", [("mixture", 4096 * 512), ("uniform", 1 << 21), ("lognormal", 1_500_007),
                                    ("zipf", 1_000_003), ("f32", 1 << 20)])
def test_learned_stats_match_oracle(dist, n):
    """The statistics the sort reports (largest of the 4096 buckets, its
    ratio to the ideal bucket, fallback runs and their keys, runs of one
    repeated key) equal the oracle's counts for the model the sort fits,
    exactly; and the sort still equals the oracle's."""
    k, dt = _keys(dist, n, seed=4)
    ref = _oracle_stats(k, dt)
    t = to_gpu(k, dt)
    _, st = ak.sort_learned_(t, dtype=dt, stats=True)
    print(dist, st, ref)
    for f in ("n", "sample_size", "leaves", "code_bits", "max_bucket", "fallback_runs", "fallback_keys",
              "constant_keys"):
        assert st[f] == ref[f], (f, st[f], ref[f])
    assert st["imbalance"] == pytest.approx(ref["imbalance"], rel=1e-12)
    # every key outside the fallback runs went through an on-chip chunk of at
    # most 2048 keys
    assert st["chunks"] >= -(-(n - st["fallback_keys"]) // 2048)
    assert np.array_equal(bits(to_host(t, dt)), bits(oracle.sort(k)))


def test_uniform_bucket_balance_statistical_pin():
    """Uniform uint64 keys: a bucket's share of the sample has relative
    standard error sqrt(B/m) (B = 4096 buckets, m samples), so the largest
    of 4096 buckets stays below 1 + 4.5 sqrt(B/m) of the ideal."""
    n = 1 << 22
    k, dt = _keys("uniform", n, seed=9)
    t = to_gpu(k, dt)
    _, st = ak.sort_learned_(t, dtype=dt, stats=True)
    m = st["sample_size"]
    assert m == rmi.sample_count(n, F32_FRAC)
    assert st["imbalance"] <= 1 + 4.5 * np.sqrt(4096 / m), st
    assert st["fallback_keys"] == 0
    assert np.array_equal(to_host(t, dt), oracle.sort(k))
