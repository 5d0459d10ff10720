"""GPU parity of ak_accumulate (Sec. II-B prefix sums with +) against the
oracle: integer keys bit-exact (wrap-around sums), float keys within the
first-order bound of the summation: d x u x (running sum of |x|), with u
the unit roundoff and d = 88 + 2 ceil(n / 2^22) the most roundings one term
passes through in the kernels' association (16 keys per thread, wave and
workgroup trees, one scan of the 4096-key chunk totals)."""
import zlib

import numpy as np
import pytest
import torch

import oracle
import paper_2507_16710_amd as ak
from gpucheck import NP, to_gpu, to_host
from pools import random_keys

pytestmark = pytest.mark.gpu

CHUNK = 4096
SIZES = [1, 5, CHUNK - 1, CHUNK, CHUNK + 1, 3 * CHUNK + 17, 1000003]


def _inputs(dt, n, rng):
    if dt.startswith("f"):
        x = rng.standard_normal(n) * np.exp(rng.uniform(-8, 8, n))
        return x.astype(NP[dt])
    return random_keys(dt, n, rng, "uniform")


def _check(dt, x, got, inclusive):
    ref = oracle.accumulate(x, inclusive)
    if not dt.startswith("f"):
        assert np.array_equal(got, ref), (dt, x.size, inclusive)
        return
    u = 2.0 ** -24 if dt == "f32" else 2.0 ** -53
    d = 88 + 2 * -(-x.size // (1 << 22))
    s = np.cumsum(np.abs(x.astype(np.float64)))
    if not inclusive:
        s = np.concatenate([[0.0], s[:-1]])
    err = np.abs(got.astype(np.float64) - ref)
    bound = 1.5 * d * u * s + 1e-300
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, (dt, x.size, inclusive, int(bad[0]), float(err[bad[0]]), float(bound[bad[0]]))


@pytest.mark.parametrize("dt", ["i32", "i64", "u32", "u64", "f32", "f64"])
def test_accumulate_matches_oracle(dt):
    rng = np.random.default_rng(zlib.crc32(f"gpuacc{dt}".encode()))
    for n in SIZES:
        x = _inputs(dt, n, rng)
        for inclusive in (True, False):
            print(f"accumulate dt={dt} n={n} inclusive={inclusive}", flush=True)
            t = to_gpu(x, dt)
            got = to_host(ak.accumulate(t, inclusive, dtype=dt), dt)
            _check(dt, x, got, inclusive)
            # in place gives the same result
            ak.accumulate_(t, inclusive, dtype=dt)
            assert np.array_equal(to_host(t, dt).view(np.uint8), got.view(np.uint8))


def test_accumulate_empty_and_closed_forms():
    t = torch.empty(0, dtype=torch.int64, device="cuda")
    assert ak.accumulate(t, dtype="i64").numel() == 0
    n = (1 << 22) + 7
    ones = torch.ones(n, dtype=torch.int64, device="cuda")
    assert torch.equal(ak.accumulate(ones, True, dtype="i64"), torch.arange(1, n + 1, device="cuda"))
    assert torch.equal(ak.accumulate(ones, False, dtype="i64"), torch.arange(n, device="cuda"))
    # int32 wrap-around
    w = to_gpu(np.array([2**31 - 1, 1, 5], dtype=np.int32), "i32")
    assert ak.accumulate(w, True, dtype="i32").cpu().tolist() == [2**31 - 1, -(2**31), -(2**31) + 5]


def test_accumulate_large_int64():
    """2^28 + 5 int64 keys (a full-size array of the 2^28 workloads):
    bit-exact against the oracle."""
    rng = np.random.default_rng(31)
    n = (1 << 28) + 5
    x = rng.integers(-(1 << 40), 1 << 40, size=n, dtype=np.int64)
    print(f"accumulate large n={n}", flush=True)
    got = to_host(ak.accumulate(to_gpu(x, "i64"), True, dtype="i64"), "i64")
    assert np.array_equal(got, oracle.accumulate(x, True))


def test_accumulate_repeats_bit_for_bit():
    """The association does not depend on which chunks finish first, so
    repeated calls agree bit for bit (float sums included)."""
    rng = np.random.default_rng(33)
    for dt in ("u64", "f32", "f64"):
        x = _inputs(dt, 300 * CHUNK + 11, rng)
        t = to_gpu(x, dt)
        first = to_host(ak.accumulate(t, True, dtype=dt), dt).view(np.uint8).copy()
        for _ in range(3):
            again = to_host(ak.accumulate(t, True, dtype=dt), dt).view(np.uint8)
            assert np.array_equal(again, first), dt
        _check(dt, x, first.view(NP[dt]), True)
