"""Benchmark of the sort hot path on one MI355X; prints ONE JSON line.

Default workload: 2**31 uint64 keys (17.2 GB) from the seeded mixture
(in blocks of 4096: 50% lognormal(30, 3), 30% Zipf(1.1) over 1e7 ranks, 20%
presorted runs of uniform keys).  One step = one learned-CDF partition sort
of those keys (sampling, sample sort, model fit, code-digit one-sweep passes,
on-chip chunk sorts, radix fallback), with the input already resident in HBM.
The plain radix sort of the same keys is timed the same way beside it; both
outputs are checked bit for bit against each other after the timed steps.

value = input bytes sorted per second (GB/s) of the learned sort.
roofline: the kernel with the largest share of the learned sort's time,
  algorithmic bytes per launch / its mean launch time (HIP events recorded
  by the library on the launch stream during the timed steps), against the
  nominal 8 TB/s and against this GPU's measured streaming-copy bandwidth.
cpu_baseline: the oracle's threaded merge sort on a bounded sample of the
  same keys, on this host's cores.
extras: the other workloads (1M int64 latency, 2**28 float32 sort and
  sortperm, 2**30 int64 in three distributions, binary search of 2**24
  int64 keys in 2**28 sorted ones, prefix sums of 2**28 int64 keys,
  100,000 segments).
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sorted GB/s on 1 MI355X, learned-CDF vs plain radix, bit-exact; % HBM peak"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2507_16710_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def timed_steps(torch, fn, src, work, steps, warmup):
    """Runs warmup + steps sorts of a fresh copy of src; returns per-step ms
    (HIP events on the current stream around the sort call only)."""
    for _ in range(warmup):
        work.copy_(src)
        fn(work)
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        work.copy_(src)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn(work)
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    return times


def cpu_baseline(torch, keys, dtype_np, seconds_hint=None):
    import numpy as np
    import oracle
    cores = len(os.sched_getaffinity(0))
    # a bounded sample: the first 2**30 keys take the threaded oracle about
    # 10-15 s on a 16-core share
    m = min(keys.numel(), 1 << 30)
    sample = keys[:m].cpu().numpy().view(dtype_np)
    t0 = time.perf_counter()
    oracle.sort_mt(sample, cores)
    dt = time.perf_counter() - t0
    return {"value": round(m * sample.itemsize / dt / 1e9, 4), "unit": "GB/s", "cores": cores,
            "kind": "oracle",
            "sample": f"first {m} keys of the same input, oracle threaded merge sort, {dt:.2f} s"}


def roofline(prof: dict, n: int, key_bytes: int, traffic):
    """Dominant kernel of a profile; algorithmic bytes per launch:
    one-sweep passes and chunk sorts read and write every key once
    (2*n*key_bytes); histograms read every key once."""
    per_launch = {"onesweep_pass": 2 * n * key_bytes, "onesweep_code_pass": 2 * n * key_bytes,
                  "chunk_sort": 2 * n * key_bytes, "digit_hist": n * key_bytes, "code_hist": n * key_bytes}
    cands = [(ms, name, cnt) for name, (cnt, ms) in prof.items() if name in per_launch]
    if not cands:
        return None
    ms, name, cnt = max(cands)
    avg_s = ms / cnt / 1e3
    achieved = per_launch[name] / avg_s / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "avg_launch_ms": round(ms / cnt, 4), "launches": cnt}


def load_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("source_hash") != source_hash():
        return None
    return d.get("kernels", {}).get(kernel)


def cpu_single(ak_unused, synth, np):
    """The oracle's plain (single-threaded) stable sort on workload 1 (the
    whole 1M int64 input, median of 3) and on a 2^24-key sample of workload
    2 (one run): the single-core baseline of the small configurations."""
    import oracle
    out = {}
    k = synth.workload1(device="cpu").numpy()
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.sort(k)
        ts.append(time.perf_counter() - t0)
    ts.sort()
    out["w1_i64_1M"] = {"ms": round(ts[1] * 1e3, 2), "GBps": round(k.size * 8 / ts[1] / 1e9, 4), "cores": 1}
    k = synth.workload2(device="cpu").numpy()[: 1 << 24]
    t0 = time.perf_counter()
    oracle.sort(k)
    dt = time.perf_counter() - t0
    out["w2_f32_2^24_sample"] = {"ms": round(dt * 1e3, 1), "GBps": round(k.size * 4 / dt / 1e9, 4), "cores": 1,
                                 "sample": "first 2^24 keys of workload 2"}
    return out


def route_bytes(ak, n: int, kb: int) -> int:
    """HBM bytes of the last plain sort by the route it took: one histogram
    read, a read and a write per digit pass, and a read and a write of the
    on-chip finish when the prefix route ran."""
    r = ak.sort_route()
    passes = r["passes"]
    return n * kb * (1 + 2 * passes + (2 if r["prefix_places"] else 0))


def extras(torch, ak, synth, reps=3):
    out = {}

    def t_of(fn, src):
        work = torch.empty_like(src)
        ts = timed_steps(torch, fn, src, work, reps, 1)
        return min(ts)

    k = synth.workload1(device="cuda")
    ms = t_of(lambda t: ak.sort_(t, dtype="i64"), k)
    msp = t_of(lambda t: ak.sortperm(t, dtype="i64"), k)
    out["w1_i64_1M"] = {"sort_us": round(ms * 1e3, 1), "sortperm_us": round(msp * 1e3, 1)}
    del k
    k = synth.workload2(device="cuda")
    ms = t_of(lambda t: ak.sort_(t, dtype="f32"), k)
    msp = t_of(lambda t: ak.sortperm(t, dtype="f32"), k)
    n = k.numel()
    out["w2_f32_2^28"] = {"sort_ms": round(ms, 3), "sort_GBps": round(n * 4 / ms / 1e6, 1),
                          "sortperm_ms": round(msp, 3), "sortperm_GBps": round(n * 4 / msp / 1e6, 1)}
    del k
    k = synth.workload2(device="cuda")
    msl = t_of(lambda t: ak.sortperm_lowmem(t, dtype="f32"), k)
    iota = torch.arange(k.numel(), dtype=torch.int32, device="cuda")
    idx = torch.empty_like(iota)

    def by_key(t):
        # the payload is reset inside the timed region (a 1 GB device copy)
        idx.copy_(iota)
        ak.sort_by_key_(t, idx, dtype="f32")
    msk = t_of(by_key, k)
    out["w2_f32_2^28"].update({"sortperm_lowmem_ms": round(msl, 3), "sort_by_key_u32_ms": round(msk, 3)})
    del k, idx, iota
    for v in ("uniform", "zipf", "lognormal"):
        k = synth.workload3(v, device="cuda")
        ms = t_of(lambda t: ak.sort_(t, dtype="i64"), k)
        n = k.numel()
        rb = route_bytes(ak, n, 8)
        out[f"w3_{v}_i64_2^30"] = {"sort_ms": round(ms, 3), "sort_GBps": round(n * 8 / ms / 1e6, 1),
                                   "route": ak.sort_route(),
                                   "hbm_frac_route": round(rb / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                                   "hbm_frac_lsd136": round(n * 136 / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        del k
        torch.cuda.empty_cache()
    # binary search (Sec. II-B): 2^24 int64 needles (half haystack members,
    # half random) in 2^28 sorted uniform int64 keys
    k = synth.workload3("uniform", n=1 << 28, device="cuda")
    ak.sort_(k, dtype="i64")
    g = torch.Generator(device="cuda").manual_seed(28)
    m = 1 << 24
    idx = torch.randint(0, k.numel(), (m // 2,), generator=g, device="cuda")
    q = torch.cat([k[idx], torch.randint(-(1 << 62), 1 << 62, (m - m // 2,), generator=g, device="cuda")])
    res = torch.empty(m, dtype=torch.int64, device="cuda")

    def t_search(fn):
        ts = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            if r:
                ts.append(a.elapsed_time(b))
        return min(ts)

    msf = t_search(lambda: ak.searchsortedfirst(k, q, dtype="i64", out=res))
    msl = t_search(lambda: ak.searchsortedlast(k, q, dtype="i64", out=res))
    out["search_i64_2^24_in_2^28"] = {"first_ms": round(msf, 3), "last_ms": round(msl, 3),
                                      "first_Gkeys_s": round(m / msf / 1e6, 2),
                                      "last_Gkeys_s": round(m / msl / 1e6, 2)}
    del q, res, idx
    # prefix sums (Sec. II-B accumulate): 2^28 int64 keys, inclusive
    acc = torch.empty_like(k)
    msa = t_search(lambda: ak.accumulate(k, True, dtype="i64", out=acc))
    out["accumulate_i64_2^28"] = {"ms": round(msa, 3), "GBps_alg": round(2 * k.numel() * 8 / msa / 1e6, 1)}
    del k, acc
    torch.cuda.empty_cache()
    keys, off = synth.workload4(device="cuda")
    work = torch.empty_like(keys)
    ts = []
    for r in range(reps + 1):
        work.copy_(keys)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        ak.segmented_sort_(work, off, dtype="u32", check=False)
        b.record()
        torch.cuda.synchronize()
        if r:
            ts.append(a.elapsed_time(b))
    ms = min(ts)
    out["w4_segmented_u32"] = {"n": int(keys.numel()), "nseg": int(off.numel() - 1), "ms": round(ms, 3),
                               "GBps": round(keys.numel() * 4 / ms / 1e6, 1)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 31, help="keys (multiple of 4096)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--only", default="", help="time one workload only (for profiler runs): learned, plain, "
                    "learned_mlp, w1, w2, w2_sortperm, w3_uniform, w3_zipf, w3_lognormal, w4")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported by this build "
              "(the multi-GPU sample sort is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2507_16710_amd as ak
    import synth

    ak.load_library()
    if args.only:
        only(args, torch, ak, synth)
        return
    n = args.n
    t0 = time.time()
    keys = synth.workload5(n=n, device="cuda")
    torch.cuda.synchronize()
    log(f"generated {n} keys in {time.time() - t0:.1f} s")
    work = torch.empty_like(keys)

    # streaming-copy bandwidth of this GPU (a device copy of the keys: one
    # read and one write of n*8 bytes), the practical ceiling beside the
    # nominal 8 TB/s
    copy_ms = []
    for r in range(4):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        work.copy_(keys)
        b.record()
        torch.cuda.synchronize()
        if r:
            copy_ms.append(a.elapsed_time(b))
    copy_gbps = 2 * n * 8 / (min(copy_ms) / 1e3) / 1e9

    # plain radix sort of the same keys (reference path)
    plain_ms = timed_steps(torch, lambda t: ak.sort_(t, dtype="u64"), keys, work, args.steps, args.warmup)
    plain_out = work.clone()
    log(f"plain radix: {min(plain_ms):.2f} ms")

    # learned sort: the timed steps, with the library's per-kernel timing on
    ak.profile_read()
    ak.profile_enable(True)
    torch.cuda.synchronize()
    learned_ms = timed_steps(torch, lambda t: ak.sort_learned_(t, dtype="u64"), keys, work, args.steps, args.warmup)
    ak.profile_enable(False)
    prof = ak.profile_read()
    log(f"learned: {min(learned_ms):.2f} ms; kernels {prof}")
    assert torch.equal(work, plain_out), "learned sort differs from the plain radix sort"
    del plain_out

    work.copy_(keys)
    _, stats = ak.sort_learned_(work, dtype="u64", stats=True)
    # the same pipeline with the method's model replaced: the 1-64-64-1
    # network (trained, tabulated), and no model (equal-width key ranges)
    others = {}
    for name, cfg in (("mlp", ak.make_cfg(model="mlp")), ("untrained", ak.make_cfg(untrained=True))):
        ms_o = timed_steps(torch, lambda t: ak.sort_learned_(t, dtype="u64", cfg=cfg), keys, work, 3, 1)
        work.copy_(keys)
        _, st_o = ak.sort_learned_(work, dtype="u64", cfg=cfg, stats=True)
        others[name] = {"ms_per_step": round(sum(ms_o) / len(ms_o), 3),
                        "value": round(n * 8 / (sum(ms_o) / len(ms_o) / 1e3) / 1e9, 2), "unit": "GB/s",
                        "imbalance": round(st_o["imbalance"], 3), "fallback_keys": st_o["fallback_keys"],
                        "constant_keys": st_o["constant_keys"]}
        log(f"learned ({name}): {min(ms_o):.2f} ms, imbalance {st_o['imbalance']:.2f}")

    ms_step = sum(learned_ms) / len(learned_ms)
    value = n * 8 / (ms_step / 1e3) / 1e9
    plain_step = sum(plain_ms) / len(plain_ms)
    learned_launches = {k: v for k, v in prof.items()}
    # profile counts span warmup + timed steps
    rl = roofline(learned_launches, n, 8, None)
    if rl is not None:
        rl["traffic"] = load_traffic(rl["kernel"])
        rl["copy_GBps"] = round(copy_gbps, 1)
        rl["frac_of_copy"] = round(rl["achieved"] / copy_gbps, 4)
    # learned-path algorithmic bytes: histogram read + 2 per code pass + chunk sort
    passes = (stats["code_bits"] + 7) // 8
    alg_bytes = n * 8 * (1 + 2 * passes + 2)
    # by the route the keys took: the chunk sorts read and write only the
    # keys outside fallback runs; the fallback reads its keys once (digit
    # counts) and moves its non-constant ones through at most 8 LSD passes;
    # the sample (gather, its own radix sort) and the model fit
    fb, const = stats["fallback_keys"], stats["constant_keys"]
    m = stats["sample_size"]
    route_bytes_learned = (n * 8 * (1 + 2 * passes) + (n - fb) * 16 + fb * 8 + (fb - const) * 8 * 16
                           + m * 8 * (2 + 1 + 2 * 8))
    plain_alg = n * 8 * (1 + 2 * 8)
    work.copy_(keys)
    ak.sort_(work, dtype="u64")
    plain_route = ak.sort_route()
    plain_route_bytes = route_bytes(ak, n, 8)
    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "learned-CDF partition sort of 2^31 uint64 mixture keys "
                               "(50% lognormal(30,3), 30% Zipf(1.1) over 1e7, 20% presorted runs of 4096), "
                               "4096 leaves, 1% sample", "n": n, "key_bytes": 8, "seed": 0},
        "plain_radix": {"value": round(n * 8 / (plain_step / 1e3) / 1e9, 2), "unit": "GB/s",
                        "ms_per_step": round(plain_step, 3),
                        "hbm_frac_alg": round(plain_alg / (plain_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                        "route": plain_route,
                        "hbm_frac_route": round(plain_route_bytes / (plain_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "learned_other_models": others,
        "learned_vs_plain": round(plain_step / ms_step, 3),
        "learned_hbm_frac_alg": round(alg_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "learned_route_bytes": int(route_bytes_learned),
        "learned_hbm_frac_route": round(route_bytes_learned / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "learned_stats": stats,
        "roofline": rl,
        "kernels_ms": {k: [c, round(ms, 3)] for k, (c, ms) in prof.items()},
        "bit_exact_vs_plain": True,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(torch, keys, np.uint64)
        line["cpu_single_thread"] = cpu_single(ak, synth, np)
    del keys, work
    torch.cuda.empty_cache()
    if not args.no_extras:
        line["extras"] = extras(torch, ak, synth)
    print(json.dumps(line), flush=True)


def only(args, torch, ak, synth):
    """One workload, `--steps` timed sorts after `--warmup` (profiler runs)."""
    name = args.only
    if name in ("learned", "plain", "learned_mlp"):
        src = synth.workload5(n=args.n, device="cuda")
        fn = {"learned": lambda t: ak.sort_learned_(t, dtype="u64"),
              "plain": lambda t: ak.sort_(t, dtype="u64"),
              "learned_mlp": lambda t: ak.sort_learned_(t, dtype="u64", cfg=ak.make_cfg(model="mlp"))}[name]
    elif name == "w1":
        src, fn = synth.workload1(device="cuda"), (lambda t: ak.sort_(t, dtype="i64"))
    elif name in ("w2", "w2_sortperm"):
        src = synth.workload2(device="cuda")
        fn = (lambda t: ak.sort_(t, dtype="f32")) if name == "w2" else (lambda t: ak.sortperm(t, dtype="f32"))
    elif name.startswith("w3_"):
        src, fn = synth.workload3(name[3:], device="cuda"), (lambda t: ak.sort_(t, dtype="i64"))
    elif name == "w4":
        src, off = synth.workload4(device="cuda")
        fn = lambda t: ak.segmented_sort_(t, off, dtype="u32", check=False)
    else:
        raise SystemExit(f"unknown workload {name}")
    work = torch.empty_like(src)
    ts = timed_steps(torch, fn, src, work, args.steps, args.warmup)
    print(json.dumps({"only": name, "n": int(src.numel()), "ms": [round(t, 3) for t in ts]}), flush=True)


if __name__ == "__main__":
    main()
