"""The seeded input generators: reproducible, and with the stated shapes."""
import numpy as np
import torch

import synth


def test_reproducible_and_seed_sensitive():
    a = synth.workload1(n=10000, seed=0)
    b = synth.workload1(n=10000, seed=0)
    c = synth.workload1(n=10000, seed=1)
    assert torch.equal(a, b) and not torch.equal(a, c)


def test_workload2_specials():
    n = 200_000
    v = synth.workload2(n=n)
    k = n // 1000
    assert int(torch.isnan(v).sum()) == k
    assert int((v == 0).sum()) == k
    assert int(torch.isinf(v).sum()) == k
    z = v[v == 0]
    assert 0 < int(torch.signbit(z).sum()) < k          # both zero signs drawn
    fin = v[torch.isfinite(v) & (v != 0)].double()
    assert abs(float(fin.std()) - 1e3) < 30 and abs(float(fin.mean())) < 30


def test_workload3_variants():
    z = synth.workload3("zipf", n=200_000)
    assert int(z.min()) >= 1 and int(z.max()) <= 1_000_000
    p1 = float((z == 1).double().mean())
    H = (np.arange(1, 1_000_001, dtype=np.float64) ** -1.2).sum()
    assert abs(p1 - 1 / H) < 0.005                       # P(rank 1) = 1/H
    ln = synth.workload3("lognormal", n=200_000)
    lg = torch.log(ln.double().clamp(min=1))
    assert abs(float(lg.mean()) - 20) < 0.05 and abs(float(lg.std()) - 2) < 0.05


def test_workload4_sizes_and_offsets():
    s = synth.workload4_sizes(nseg=100_000)
    assert int(s.min()) >= 16 and int(s.max()) <= 1 << 20
    assert abs(float(s.double().mean()) - 5000) < 250
    keys, off = synth.workload4(nseg=50, seed=3)
    assert off[0] == 0 and torch.all(off[1:] >= off[:-1]) and int(off[-1]) == keys.numel()


def test_workload5_blocks():
    n = 4096 * 64
    v = synth.as_numpy(synth.workload5(n=n), "u64").reshape(-1, 4096)
    sorted_blocks = np.all(np.diff(v.astype(np.float64), axis=1) >= 0, axis=1)
    zipf_blocks = np.all(v <= 10_000_000, axis=1)
    assert sorted_blocks.sum() >= 1 and zipf_blocks.sum() >= 1
    assert np.array_equal(synth.as_numpy(synth.workload5(n=n), "u64").reshape(-1, 4096), v)
