#!/usr/bin/env python3
"""Measures, on the GPU this runs on, which decision (COUNTING, RADIX,
QUICK) makes AUTO fastest on each of a grid of synthetic workloads, and
writes one CSV row per workload: its features (n, span, nbins, entropy) and
the three wall times of ahs_sort(AUTO) with the decision pinned to that
strategy (inputs resident on the device, the host round trips included).
AUTO computes the features first and the strategies reuse what they can
(radix the fused digit counts, counting the exact histogram; the sample
sort nothing), so a strategy's time here is its cost after the features,
not its forced time: forced radix and counting recompute the min/max and
their counts.  The decision is pinned by a constant model (no trees; the
initial scores favour one class) attached to the context.  These are the
labels the selector model of Sec. III-H is trained on (train_gbt.py).

Workloads: u32 keys uniform over k values (k from 16 to 2^32), 64..65,536
distinct values drawn with Zipf ranks, 4..64 equally likely values spread
over the whole range, sorted and reversed uniform keys; u64 keys uniform
over 2^64 / 2^48 / 2^32 / 2^16 values, Zipf over 4,096 values and 4..256
equally likely values spread over [0, 2^40), [0, 2^60) or the whole range
(both ends present, so the span is exact); u32 keys uniform inside 2 to 64
clusters of 2^16 to 2^23 consecutive values spread over the whole range
(mostly distinct keys whose binned entropy is as low as that of a few
repeated values); u32 Zipf(1.1) and Zipf(1.5) ranks over [0, 2^20) or
[0, 2^26) (the key is the rank: a narrow span with low entropy); f32 and f64 Normal(0, 1e3); n from 2^10 to 2^28.  Keys are
drawn on the device from a seeded torch generator (the labels are
measurements, not parity data).  --dists times only the named families and
--merge replaces their rows in an existing label file, keeping the others.
"""
import argparse
import csv
import os
import statistics
import sys
import tempfile
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import torch  # noqa: E402

import paper_2506_20677_amd as ahs  # noqa: E402


def workloads(max_log2n):
    out = []
    for lg in range(10, max_log2n + 1, 2):
        for k in (16, 256, 1024, 4096, 65536, 1 << 20, 1 << 24, 1 << 32):
            out.append(("u32", lg, "uniform", k))
        for m, s in ((64, 1.1), (256, 1.1), (4096, 1.1), (65536, 1.1), (256, 1.5)):
            out.append(("u32", lg, f"zipf{s}", m))
        for m in (4, 16, 64):
            out.append(("u32", lg, "fewvals32", m))
        # (clusters, log2 width): 2 x 2^23 and 16 x 2^20 fill 256 of the 65,536
        # bins (H = 8), 64 x 2^16 about 64 bins
        for c, w in ((2, 23), (16, 20), (64, 16)):
            out.append(("u32", lg, f"clustered{w}", c))
        for s in (1.1, 1.5):
            for k in (1 << 20, 1 << 26):
                out.append(("u32", lg, f"zipfrank{s}", k))
        out.append(("u32", lg, "sorted", 1 << 32))
        out.append(("u32", lg, "reverse", 1 << 32))
        # 64-bit and float keys at the same sizes (2^28 u64 keys = 2 GiB)
        for k in (1 << 16, 1 << 32, 1 << 48, 1 << 64):
            out.append(("u64", lg, "uniform", k))
        out.append(("u64", lg, "zipf1.0", 4096))
        for bits in (40, 60, 64):
            for m in (4, 16, 256):
                out.append(("u64", lg, f"fewvals{bits}", m))
        out.append(("f32", lg, "normal", 0))
        out.append(("f64", lg, "normal", 0))
    return out


def make_keys(dtype, lg, dist, param, g, dev):
    n = 1 << lg
    if dist in ("uniform", "sorted", "reverse"):
        if param >= 1 << 63:
            x = torch.randint(-(1 << 63), (1 << 63) - 1, (n,), generator=g, device=dev, dtype=torch.int64)
        else:
            x = torch.randint(0, param, (n,), generator=g, device=dev, dtype=torch.int64)
        if dist != "uniform":
            x = torch.sort(x, descending=(dist == "reverse")).values
    elif dist.startswith("fewvals"):
        # param equally likely values over [0, 2^bits), both ends among them
        bits = int(dist[7:])
        if bits >= 64:
            vals = torch.randint(-(1 << 63), (1 << 63) - 1, (param,), generator=g, device=dev, dtype=torch.int64)
            vals[0], vals[1] = 0, -1  # 0 and 2^64 - 1 as two's complement
        else:
            vals = torch.randint(0, 1 << bits, (param,), generator=g, device=dev, dtype=torch.int64)
            vals[0], vals[1] = 0, (1 << bits) - 1
        x = vals[torch.randint(0, param, (n,), generator=g, device=dev, dtype=torch.int64)]
    elif dist.startswith("clustered"):
        # param clusters of 2^w consecutive values, the first at 0 and the
        # last ending at 2^32 - 1, each key uniform inside a uniform cluster
        w = int(dist[9:])
        base = torch.randint(0, (1 << 32) - (1 << w) + 1, (param,), generator=g, device=dev, dtype=torch.int64)
        base[0], base[1] = 0, (1 << 32) - (1 << w)
        x = base[torch.randint(0, param, (n,), generator=g, device=dev, dtype=torch.int64)]
        x += torch.randint(0, 1 << w, (n,), generator=g, device=dev, dtype=torch.int64)
        x[0], x[-1] = 0, (1 << 32) - 1
    elif dist.startswith("zipfrank"):
        # the rank itself (0 = most frequent), so the span is at most param - 1
        s = float(dist[8:])
        w = torch.arange(1, param + 1, device=dev, dtype=torch.float64) ** (-s)
        cdf = torch.cumsum(w, 0)
        cdf /= cdf[-1].clone()
        u = torch.rand(n, generator=g, device=dev, dtype=torch.float64)
        x = torch.searchsorted(cdf, u).clamp_(max=param - 1)
    elif dist.startswith("zipf"):
        s = float(dist[4:])
        vals = torch.randint(0, 1 << 32 if dtype == "u32" else (1 << 62), (param,), generator=g, device=dev,
                             dtype=torch.int64)
        w = torch.arange(1, param + 1, device=dev, dtype=torch.float64) ** (-s)
        cdf = torch.cumsum(w, 0)
        cdf /= cdf[-1].clone()
        u = torch.rand(n, generator=g, device=dev, dtype=torch.float64)
        x = vals[torch.searchsorted(cdf, u).clamp_(max=param - 1)]
    else:  # normal
        fdt = torch.float32 if dtype == "f32" else torch.float64
        return (torch.randn(n, generator=g, device=dev, dtype=torch.float64) * 1e3).to(fdt)
    if dtype == "u32":
        # low 32 bits as two's complement int32, viewed unsigned
        x = x.bitwise_and(0xFFFFFFFF)
        x = torch.where(x >= (1 << 31), x - (1 << 32), x)
        return x.to(torch.int32).view(torch.uint32)
    return x.view(torch.uint64)


def time_sort(keys, out, strategy, ctx, cfg, reps):
    ts = []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, chosen, _ = ahs.ahs_sort(keys, strategy=strategy, cfg=cfg, out=out, ctx=ctx)
        torch.cuda.synchronize()
        if r:
            ts.append(time.perf_counter() - t)
    return statistics.median(ts), chosen


def constant_models(tmpdir):
    """One model file per strategy whose prediction is always that strategy."""
    out = {}
    for i, name in enumerate(("counting", "radix", "quick")):
        path = os.path.join(tmpdir, f"always_{name}.gbt")
        base = ["0.0"] * 3
        base[i] = "1.0"
        with open(path, "w") as fh:
            fh.write(f"ahs-gbt 1\nnum_class 3\nbase_score {' '.join(base)}\nnum_trees 0\n")
        out[name] = ahs.ahs_model_load(path)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "mi355x_labels.csv"))
    ap.add_argument("--max-log2n", type=int, default=28)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--dists", default="", help="comma-separated families to time (default: all)")
    ap.add_argument("--merge", action="store_true", help="replace only these families' rows in --out")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(2506)
    ctx = ahs.default_context(0)
    ctx.workspace(ahs.ahs_workspace_bytes(1 << args.max_log2n, ahs.U64, False, ahs.AUTO))
    cfg = ahs.ahs_config_init(ahs.PRESET_GPU)
    cfg_m = ahs.ahs_config_init(ahs.PRESET_GPU, use_model=1)
    with tempfile.TemporaryDirectory() as tmpdir:  # the files are parsed at load
        pinned = constant_models(tmpdir)
    rows = []
    wl = workloads(args.max_log2n)
    only = [d for d in args.dists.split(",") if d]
    if only:
        wl = [w for w in wl if w[2] in only]
    if not wl:
        raise SystemExit("no workload matches --dists")
    for i, (dtype, lg, dist, param) in enumerate(wl):
        keys = make_keys(dtype, lg, dist, param, g, dev)
        out = torch.empty_like(keys)
        f = ahs.ahs_features(keys, ctx=ctx)
        fsm = ahs.ahs_select(f, cfg)
        t = {}
        for name, s in (("counting", ahs.COUNTING), ("radix", ahs.RADIX), ("quick", ahs.QUICK)):
            if s == ahs.COUNTING and f.span >= 65536:
                t[name] = float("inf")
                continue
            ctx.set_model(pinned[name])
            t[name], chosen = time_sort(keys, out, ahs.AUTO, ctx, cfg_m, args.reps)
            if chosen != s:
                raise SystemExit(f"AUTO ran {ahs.STRATEGY_NAMES[chosen]} with the decision pinned to {name}")
        ctx.set_model(None)
        best = min(t, key=t.get)
        rows.append({"dtype": dtype, "n": f.n, "dist": dist, "param": param, "span": f.span, "nbins": f.nbins,
                     "entropy_bits": repr(f.entropy_bits), "t_counting": t["counting"], "t_radix": t["radix"],
                     "t_quick": t["quick"], "best": best, "fsm": ahs.STRATEGY_NAMES[fsm]})
        print(f"[labels] {i + 1}/{len(wl)} {dtype} 2^{lg} {dist} {param}: best {best} "
              f"({', '.join(f'{k} {v * 1e3:.3f}' for k, v in t.items())} ms), fsm {ahs.STRATEGY_NAMES[fsm]}",
              flush=True)
        del keys, out
    if args.merge and os.path.exists(args.out):
        fams = {r["dist"] for r in rows}
        with open(args.out, newline="") as fh:
            kept = [r for r in csv.DictReader(fh) if r["dist"] not in fams]
        rows = kept + rows
    with open(args.out, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    print(f"[labels] wrote {len(rows)} rows to {args.out}", flush=True)


if __name__ == "__main__":
    main()
