"""Autotuner of the segmented sort (run on the GPU; writes tune_gfx950.json).

For 32- and 64-bit keys it times the batched segmented sort on seeded
segment batches with lognormal lengths (the same family as the 100,000-segment
workload: sizes clipped to [16, 2**20], mean about 5,000, scaled down so a
sweep takes seconds) under every tuning the library accepts:

  ipt_a      keys per lane of the one-wave class      (2, 4)
  ipt_b      keys per lane of the one-workgroup class  (8, 16; 32 for 32-bit)
  grid_mult  persistent workgroups per CU             (2, 4, 8)
  b_max      on-chip limit of the one-workgroup class (full capacity, half)
  xl_min     shortest segment of the many-workgroup class (8192 ... 131072)

and writes the fastest per key width to ``tune_gfx950.json`` next to
``libak.so`` (read by the library at its first segmented call).  Every
configuration's output is checked against the first one's, so a tuning
can only be chosen if it sorts identically.

Usage:  python -m paper_2507_16710_amd.autotune [--nseg 20000] [--reps 3]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tune_gfx950.json")


def candidates(key_bits: int):
    b_opts = (8, 16, 32) if key_bits == 32 else (8, 16)
    for ipt_a, ipt_b, gm, xl in itertools.product((2, 4), b_opts, (2, 4, 8), (8192, 16384, 32768, 65536, 131072)):
        cap = 256 * ipt_b
        for b_max in (0, cap // 2):
            yield {"ipt_a": ipt_a, "ipt_b": ipt_b, "grid_mult": gm, "b_max": b_max, "xl_min": xl}


def run(nseg: int, reps: int, seed: int = 0) -> dict:
    import torch

    sys.path.insert(0, os.path.dirname(HERE))
    import paper_2507_16710_amd as ak
    import synth

    table = {"arch": "gfx950", "written": time.strftime("%Y-%m-%d %H:%M:%S"), "nseg": nseg}
    for key_bits, dt in ((32, "u32"), (64, "u64")):
        sizes = synth.workload4_sizes(nseg=nseg, seed=seed, device="cuda")
        off = torch.zeros(nseg + 1, dtype=torch.int64, device="cuda")
        off[1:] = torch.cumsum(sizes, 0)
        n = int(off[-1])
        g = torch.Generator(device="cuda").manual_seed(1234 + key_bits)
        if key_bits == 32:
            src = torch.randint(-(1 << 31), 1 << 31, (n,), generator=g, device="cuda", dtype=torch.int64).to(torch.int32)
        else:
            src = torch.randint(-(1 << 62), 1 << 62, (n,), generator=g, device="cuda", dtype=torch.int64)
        work = torch.empty_like(src)
        ref = None
        results = []
        for cfg in candidates(key_bits):
            ak.seg_set_tuning(key_bits, cfg["ipt_a"], cfg["ipt_b"], cfg["grid_mult"], cfg["b_max"], cfg["xl_min"])
            ts = []
            for r in range(reps + 1):
                work.copy_(src)
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                ak.segmented_sort_(work, off, dtype=dt, check=False)
                b.record()
                torch.cuda.synchronize()
                if r:
                    ts.append(a.elapsed_time(b))
            if ref is None:
                ref = work.clone()
            elif not torch.equal(ref, work):
                raise RuntimeError(f"tuning {cfg} sorted differently")
            ms = min(ts)
            results.append((ms, cfg))
            print(f"seg{key_bits} {cfg} {ms:.3f} ms", flush=True)
        best_ms, best = min(results, key=lambda x: x[0])
        table[f"seg{key_bits}"] = dict(best, ms=round(best_ms, 4), n=n)
        print(f"best seg{key_bits}: {best} {best_ms:.3f} ms", flush=True)
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nseg", type=int, default=20000)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=TABLE)
    a = ap.parse_args()
    table = run(a.nseg, a.reps)
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
    print("wrote", a.out)


if __name__ == "__main__":
    main()
