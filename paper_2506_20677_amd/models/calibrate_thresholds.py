#!/usr/bin/env python3
"""Threshold calibration of the FSM on the target GPU (Sec. III-C).

The paper picks the small-input threshold n_t and the counting threshold k_t
by minimising eq. (1), alpha * T(n_t, k_t) + (1 - alpha) * M(n_t, k_t) with
alpha = 0.7, T the normalised execution time over its datasets and M the
peak memory, over n_t in [10, 50] and k_t in [500, 5000].

``collect`` (needs the GPU) times, once per workload, every state the FSM
can reach on it: the n <= n_t state (AUTO with n_small raised above n, so
the small-input sort runs), COUNTING, RADIX and QUICK forced, and records
the features.  Workloads: n = 8 ... 64 keys (the n_t range and beyond) and
spans k = 256 ... 8,192 around the k_t range at 2^12 ... 2^24 keys, uniform
and Zipf(1.5).

The library never allocates (the caller passes one workspace sized for the
worst strategy), so peak memory is each state's algorithmic footprint: the
output (4n bytes) for all; plus the histogram (4 bytes per value of the
span) for counting; plus the ping-pong copy (4n) and 1 KiB of digit counts
per pass for radix; plus the bucket copy (4n) and 64 KiB of splitter and
bucket tables for the sample sort.

``analyze`` (CPU) evaluates eq. (1) on the full grid without running any
sort: for each (n_t, k_t) the library's own decision function (ahs_select,
a host call) picks the state per workload; T is the mean of the chosen
state's time over the workload's best time, M the mean peak memory of the
chosen state in MB; each is divided by its largest value over the grid
(the paper leaves the normalisation open) before weighting.  A grid search
replaces the paper's Bayesian refinement: two integer parameters on a
21 x 19 grid are evaluated exhaustively in milliseconds.

The GPU form of eq. (2) is reported beside the result: the paper bounds the
counting range by cache size over 4 bytes per counter per thread; here the
counting histogram lives in LDS, so k_max = LDS bytes per CU / (4 bytes x
resident histogram workgroups per CU).
"""
import argparse
import csv
import json
import math
import os
import statistics
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

ALPHA = 0.7
N_GRID = list(range(10, 51, 2))
K_GRID = list(range(500, 5001, 250))
STATES = ("insertion", "counting", "radix", "quick")
TIMES_CSV = os.path.join(HERE, "mi355x_threshold_times.csv")
RESULT_JSON = os.path.join(HERE, "mi355x_thresholds.json")


# ------------------------------------------------------------------ collect
def workloads():
    out = []
    for n in (8, 10, 12, 14, 16, 18, 20, 22, 24, 28, 32, 40, 48, 56, 64):
        for dist in ("uniform32", "uniform100", "sorted32"):
            out.append((n, dist, 0))
    for lg in (12, 16, 20, 24):
        for k in (256, 500, 1000, 1500, 2000, 2500, 3000, 3500, 4000, 4096, 4500, 5000, 6000, 8192):
            for dist in ("uniformk", "zipfk"):
                out.append((1 << lg, dist, k))
    return out


def make_keys(n, dist, k, g, torch, dev):
    if dist == "uniform32":
        x = torch.randint(-(1 << 31), 1 << 31, (n,), generator=g, device=dev, dtype=torch.int64)  # all 32 bits
    elif dist == "uniform100":
        x = torch.randint(0, 100, (n,), generator=g, device=dev, dtype=torch.int64)
    elif dist == "sorted32":
        x = torch.sort(torch.randint(0, 1 << 31, (n,), generator=g, device=dev, dtype=torch.int64)).values
    elif dist == "uniformk":
        x = torch.randint(0, k, (n,), generator=g, device=dev, dtype=torch.int64)
    else:  # Zipf(1.5) ranks 0 .. k-1
        w = torch.arange(1, k + 1, device=dev, dtype=torch.float64) ** -1.5
        cdf = torch.cumsum(w, 0)
        cdf /= cdf[-1].clone()
        u = torch.rand(n, generator=g, device=dev, dtype=torch.float64)
        x = torch.searchsorted(cdf, u).clamp_(max=k - 1)
    return x.to(torch.int32).view(torch.uint32)


def collect(out_path, reps):
    import torch
    import paper_2506_20677_amd as ahs

    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(25063)
    ctx = ahs.default_context(0)
    ctx.workspace(ahs.ahs_workspace_bytes(1 << 24, ahs.U32, False, ahs.AUTO))
    base = ahs.ahs_config_init(ahs.PRESET_GPU)
    small = ahs.ahs_config_init(ahs.PRESET_GPU, n_small=1024)  # every n here takes the small-input state

    def timed(keys, out, strategy, cfg):
        ts = []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, _, ch, _ = ahs.ahs_sort(keys, strategy=strategy, cfg=cfg, out=out, ctx=ctx)
            torch.cuda.synchronize()
            if r:
                ts.append(time.perf_counter() - t)
        return statistics.median(ts), ch

    rows = []
    wl = workloads()
    for i, (n, dist, k) in enumerate(wl):
        keys = make_keys(n, dist, k, g, torch, dev)
        out = torch.empty_like(keys)
        f = ahs.ahs_features(keys, ctx=ctx)
        row = {"n": n, "dist": dist, "param": k, "span": f.span, "nbins": f.nbins,
               "entropy_bits": repr(f.entropy_bits)}
        for name, s in (("counting", ahs.COUNTING), ("radix", ahs.RADIX), ("quick", ahs.QUICK)):
            if s == ahs.COUNTING and f.span >= base.k_count_cap:
                row["t_" + name] = float("inf")
            else:
                row["t_" + name], _ = timed(keys, out, s, base)
        if n <= 64:
            t, ch = timed(keys, out, ahs.AUTO, small)
            assert ch == ahs.INSERTION, ch
            row["t_insertion"] = t
        else:
            row["t_insertion"] = float("inf")
        rows.append(row)
        print(f"[calib] {i + 1}/{len(wl)} n={n} {dist} {k}: " +
              ", ".join(f"{s} {row['t_' + s] * 1e3:.4f}" for s in STATES) + " ms", flush=True)
        del keys, out
    props = torch.cuda.get_device_properties(0)
    hw = {"lds_bytes_per_cu": int(getattr(props, "shared_memory_per_multiprocessor", 160 * 1024)),
          "cus": props.multi_processor_count, "name": props.name}
    with open(out_path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    with open(out_path + ".hw.json", "w") as fh:
        json.dump(hw, fh)
    print(f"[calib] wrote {len(rows)} rows to {out_path}", flush=True)


# ------------------------------------------------------------------ analyze
def footprint(state, n, span):
    """Algorithmic peak device memory of a state in bytes (u32 keys)."""
    out = 4 * n
    if state == "counting":
        return out + 4 * (span + 1)
    if state == "radix":
        passes = max(1, (span.bit_length() + 7) // 8)
        return out + 4 * n + 1024 * passes
    if state == "quick":
        return out + 4 * n + 65536
    return out


def load(path):
    rows = []
    for r in csv.DictReader(open(path)):
        n, span = int(r["n"]), int(r["span"])
        rows.append({"n": n, "span": span, "nbins": int(r["nbins"]), "entropy_bits": float(r["entropy_bits"]),
                     "t": {s: float(r["t_" + s]) for s in STATES},
                     "mem": {s: footprint(s, n, span) for s in STATES}})
    return rows


def objective_grid(rows, decide, n_grid=N_GRID, k_grid=K_GRID, alpha=ALPHA):
    """Eq. (1) over the grid.  decide(row, n_t, k_t) -> state name.  Returns
    {(n_t, k_t): (J, T, M)} with T the mean time over the best, M the mean
    peak memory in MB, both before normalisation, and J the weighted sum of
    T and M each divided by its largest value over the grid."""
    raw = {}
    for nt in n_grid:
        for kt in k_grid:
            ts, ms = [], []
            for r in rows:
                s = decide(r, nt, kt)
                best = min(v for v in r["t"].values() if math.isfinite(v))
                ts.append(r["t"][s] / best)
                ms.append(r["mem"][s] / 1e6)
            raw[(nt, kt)] = (sum(ts) / len(ts), sum(ms) / len(ms))
    tmax = max(v[0] for v in raw.values())
    mmax = max(v[1] for v in raw.values()) or 1.0
    return {key: (alpha * t / tmax + (1 - alpha) * m / mmax, t, m) for key, (t, m) in raw.items()}


def best_point(grid):
    """Smallest J; ties go to the smaller n_t, then the smaller k_t."""
    return min(grid, key=lambda key: (round(grid[key][0], 12), key[0], key[1]))


def library_decider():
    import paper_2506_20677_amd as ahs

    names = {ahs.INSERTION: "insertion", ahs.COUNTING: "counting", ahs.RADIX: "radix", ahs.QUICK: "quick"}

    def decide(r, nt, kt):
        cfg = ahs.ahs_config_init(ahs.PRESET_GPU, n_small=nt, k_count=kt)
        f = ahs.FeatureVector(n=r["n"], span=r["span"], nbins=r["nbins"], entropy_bits=r["entropy_bits"])
        return names[ahs.ahs_select(f, cfg)]
    return decide


def analyze(times_path, out_path, hw_path=None):
    rows = load(times_path)
    grid = objective_grid(rows, library_decider())
    nt, kt = best_point(grid)
    J, T, M = grid[(nt, kt)]

    def time_at(n_t, k_t):
        return round(objective_grid(rows, library_decider(), [n_t], [k_t])[(n_t, k_t)][1], 4)
    hw = json.load(open(hw_path)) if hw_path and os.path.exists(hw_path) else {"lds_bytes_per_cu": 160 * 1024}
    res = {"alpha": ALPHA, "n_grid": [N_GRID[0], N_GRID[-1], N_GRID[1] - N_GRID[0]],
           "k_grid": [K_GRID[0], K_GRID[-1], K_GRID[1] - K_GRID[0]], "workloads": len(rows),
           "best": {"n_small": nt, "k_count": kt, "J": round(J, 6), "time_over_best": round(T, 4),
                    "peak_MB": round(M, 3)},
           "gpu_preset": {"n_small": 20, "k_count": 4096, "time_over_best": time_at(20, 4096)},
           "paper_table2": {"n_small": 20, "k_count": 1024, "time_over_best": time_at(20, 1024)},
           "k_max_eq2_gpu": hw["lds_bytes_per_cu"] // (4 * 2),
           "k_max_eq2_note": "LDS bytes per CU / (4 bytes per counter x 2 resident histogram workgroups per CU)"}
    with open(out_path, "w") as fh:
        json.dump(res, fh, indent=1)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=("collect", "analyze"))
    ap.add_argument("--times", default=TIMES_CSV)
    ap.add_argument("--out", default=RESULT_JSON)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    if args.mode == "collect":
        collect(args.times, args.reps)
    else:
        print(json.dumps(analyze(args.times, args.out, args.times + ".hw.json"), indent=1))


if __name__ == "__main__":
    main()
