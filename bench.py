#!/usr/bin/env python3
"""Benchmark of the Adaptive Hybrid Sort hot path on one MI355X.

Workload (default): the strategy sweep at scale -- six arrays of 2^28
uint32 keys: (a) uniform on [0, 4095] (counting), (b) 256 distinct random
32-bit values with Zipf(1.1) ranks (radix), (c) uniform 32-bit keys,
unsorted, sorted, reversed and sorted with n/200 random transpositions
(general path).  One step sorts all six with AHS AUTO (features, decision,
the chosen sort); inputs are resident in HBM before the timed region.

The last stdout line is one compact JSON object (under 4 KB): whole-job
Gkeys/s, the dominant kernel's roofline (algorithmic bytes per launch over
its average launch time, both measured with HIP events on the launch
stream), the CPU oracle on a bounded sample (one pinned core, median of
runs) and a few summary figures per section.  Every section in full goes to
--detail-out (and to stderr).

Sections reported beside the headline (not in `value`):
* per_case: each sweep array under AUTO and each forced strategy, %HBM of
  each path.
* pr1: 10^6 uint32 keys on [0, 1023]: AUTO, forced RADIX and QUICK, keys
  only and with payload, checked bitwise against the oracle, whose own time
  is reported.
* wide: 2^27 u64 uniform, u64 Zipf(1.0) over 4,096 values, f32 and f64
  Normal(0, 1e3) with duplicates and signed zeros; AUTO against forced
  RADIX and QUICK, keys only and with payload = index.
* paper_sweep: the paper's dataset families (uniform, rounded Gaussian as
  signed keys, Zipf(1.5), edge patterns, full-range signed keys, stand-ins
  with the (n, k, H) of its real datasets); AUTO against each forced strategy.
* batched: 65,536 uint32 segments, sizes log-uniform on [16, 2^20] (about
  6.2e9 keys), distributions mixed per segment; the autotuned, graph-captured
  batched sort against a host loop of per-array AHS AUTO calls.
* serving: Poisson arrivals at 2,000 requests/s for 60 s, sizes log-uniform
  on [2^10, 2^24], key types u32/u64/f32, half with payload, 48 GB admission
  budget; the serving loop against one-at-a-time AHS AUTO on one stream, in
  real time (latency p50/p99) and as a burst of the trace's first seconds
  (throughput).
"""
import argparse
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Gkeys/s & %HBM peak per strategy, 2^28 uint32; batched p99 latency vs plain"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


# The sources each timed kernel family is compiled from: a committed
# counter summary describes a kernel only while these are unchanged.
KERNEL_SOURCES = {
    "onesweep_pass": ["radix.hip", "onesweep.hpp", "common.hpp", "kernels.hpp"],
    "minmax": ["features.hip", "histcommon.hpp", "common.hpp", "kernels.hpp"],
    "feature_hist": ["features.hip", "histcommon.hpp", "common.hpp", "kernels.hpp"],
    "counting_expand": ["counting.hip", "common.hpp", "kernels.hpp"],
    "ss_block_sort": ["samplesort.hip", "blocksort.hpp", "onesweep.hpp", "samplesort.hpp", "common.hpp", "kernels.hpp"],
    "ss_scatter": ["samplesort.hip", "onesweep.hpp", "samplesort.hpp", "common.hpp", "kernels.hpp"],
    "ss_count": ["samplesort.hip", "samplesort.hpp", "common.hpp", "kernels.hpp"],
}


def source_sha(kernel=None):
    """Hash of the kernel family's sources (all library sources when the
    family is unknown)."""
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_2506_20677_amd", "csrc")
    files = [os.path.join(csrc, f) for f in KERNEL_SOURCES[kernel]] if kernel in KERNEL_SOURCES else \
        sorted(glob.glob(os.path.join(csrc, "*")))
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, tag):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload, or None when the kernel's sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except OSError:
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k or k.get("source_sha") != source_sha(kernel) or k["fetch_bytes_per_launch"] is None:
        return None
    return k["fetch_bytes_per_launch"] + (k["write_bytes_per_launch"] or 0)


def percentile(xs, q):
    """Nearest-rank percentile."""
    import math
    v = sorted(xs)
    if not v:
        return None
    return v[max(1, min(len(v), math.ceil(q / 100.0 * len(v)))) - 1]


def batched_section(args, ahs, gen, torch, np):
    """65,536 segments in one batched call (autotuned, graph-captured) against
    a host loop of per-array AUTO sorts of the same segments."""
    dev = torch.device("cuda:0")
    t = time.time()
    keys_h, offs_h, kinds = gen.segments(nseg=args.seg_count, seed=8)
    n = keys_h.size
    log(f"[bench] batched workload: {args.seg_count} segments, {n} keys, generated in {time.time() - t:.1f}s")
    keys = torch.from_numpy(keys_h).to(dev)
    offs = torch.from_numpy(offs_h.view(np.int64)).to(dev)
    sizes = np.diff(offs_h.astype(np.int64))
    del keys_h
    torch.cuda.synchronize()
    ctx = ahs.default_context(0)
    caps, tune_ms = ahs.ahs_segmented_autotune(ahs.U32, False, ctx)
    radix_tile = ahs.ahs_segmented_get_radix_tile(ahs.U32, False, ctx)
    log(f"[bench] autotuned size-class variants {caps}, radix tile {radix_tile} keys")
    # blocking call (one host read per sample-sort level)
    out_b, _, chosen_b, _ = ahs.ahs_sort_segmented(keys, offs, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.seg_reps):
        ahs.ahs_sort_segmented(keys, offs, out=out_b, ctx=ctx)
    torch.cuda.synchronize()
    blocking_s = (time.perf_counter() - t0) / args.seg_reps
    # graph-captured enqueue-only call
    g = ahs.SegmentedGraph(keys, offs, ctx=ctx, max_seg_hint=int(sizes.max()))
    g.launch()
    torch.cuda.synchronize()
    status = int(g.status.item())
    t0 = time.perf_counter()
    for _ in range(args.seg_reps):
        g.launch()
    torch.cuda.synchronize()
    graph_s = (time.perf_counter() - t0) / args.seg_reps
    same_graph = bool(torch.equal(g.out.view(torch.int32), out_b.view(torch.int32)))
    same_chosen = bool(torch.equal(g.chosen, chosen_b))
    del g
    torch.cuda.empty_cache()
    if not args.seg_loop:
        res = {"workload": f"{args.seg_count} uint32 segments, sizes log-uniform on [16, 2^20] (seed 8), {n} keys",
               "keys": n, "autotuned_caps": caps, "autotuned_radix_tile": radix_tile,
               "graph_ms": round(graph_s * 1e3, 3),
               "graph_gkeys_s": round(n / graph_s / 1e9, 3), "blocking_ms": round(blocking_s * 1e3, 3),
               "blocking_gkeys_s": round(n / blocking_s / 1e9, 3), "graph_status": status,
               "identical_outputs": same_graph, "decisions_equal_graph_blocking": same_chosen}
        log(f"[bench] batched {json.dumps(res)}")
        del keys, offs, out_b
        torch.cuda.empty_cache()
        return res
    # host loop of plain per-array calls
    out_l = torch.empty_like(keys)
    ws = ctx.workspace(ahs.ahs_workspace_bytes(int(sizes.max()), ahs.U32, False, ahs.AUTO))
    bounds = offs_h.astype(np.int64).tolist()
    loop_chosen = np.empty(args.seg_count, np.uint8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.seg_count):
        a, b = bounds[i], bounds[i + 1]
        _, _, ch, _ = ahs.ahs_sort(keys[a:b], out=out_l[a:b], ctx=ctx)
        loop_chosen[i] = ch
    torch.cuda.synchronize()
    loop_s = time.perf_counter() - t0
    same_loop = bool(torch.equal(out_l.view(torch.int32), out_b.view(torch.int32)))
    agree = float(np.mean(loop_chosen == chosen_b.cpu().numpy()))
    del out_l, ws
    kinds_count = {k: int(np.sum(kinds == i)) for i, k in enumerate(gen.SEG_KINDS)}
    res = {
        "workload": f"{args.seg_count} uint32 segments, sizes log-uniform on [16, 2^20] (seed 8), "
                    f"{n} keys; per-segment kinds {kinds_count}",
        "keys": n, "autotuned_caps": caps, "autotuned_radix_tile": radix_tile,
        "autotune_kernel_ms": [round(x, 4) for x in tune_ms],
        "graph_ms": round(graph_s * 1e3, 3), "graph_gkeys_s": round(n / graph_s / 1e9, 3),
        "blocking_ms": round(blocking_s * 1e3, 3), "blocking_gkeys_s": round(n / blocking_s / 1e9, 3),
        "loop_ms": round(loop_s * 1e3, 3), "loop_gkeys_s": round(n / loop_s / 1e9, 3),
        "speedup_graph_vs_loop": round(loop_s / graph_s, 2), "graph_status": status,
        "identical_outputs": same_graph and same_loop, "decisions_equal_graph_blocking": same_chosen,
        "decisions_agree_with_loop": round(agree, 6),
    }
    log(f"[bench] batched {json.dumps(res)}")
    del keys, offs, out_b
    torch.cuda.empty_cache()
    return res


def serving_section(args, ahs, gen, torch, np):
    """The request trace through the serving loop and through one-at-a-time
    plain AUTO sorts, in real time and as a burst."""
    dev = torch.device("cuda:0")
    tr = gen.request_trace(duration_s=args.serve_seconds)
    m = len(tr["arrival_s"])
    pool_n = 1 << 26
    pools = {}
    for k in gen.POOL_KINDS:
        pools[k] = torch.from_numpy(gen.request_pool(k, n=pool_n)).to(dev)
    pay_pool = torch.arange(pool_n, dtype=torch.int32, device=dev).view(torch.uint32)
    torch.cuda.synchronize()
    reqs = []
    for i in range(m):
        n = int(tr["size"][i])
        kind = gen.request_pool_kind(int(tr["dtype"][i]), int(tr["dist"][i]))
        off = int(tr["offset"][i]) % (pool_n - n + 1)
        reqs.append((float(tr["arrival_s"][i]) * 1e3, kind, off, n, bool(tr["payload"][i])))
    total_keys = sum(r[3] for r in reqs)
    log(f"[bench] serving trace: {m} requests over {args.serve_seconds}s, {total_keys} keys")

    def view(r):
        _, kind, off, n, pay = r
        return pools[kind][off:off + n], (pay_pool[off:off + n] if pay else None)

    burst_reqs = [r for r in reqs if r[0] < args.burst_seconds * 1e3]

    def served(burst):
        rs = burst_reqs if burst else reqs
        m = len(rs)
        srv = ahs.Server(hbm_budget_bytes=int(args.serve_budget_gb * 1e9), slots=args.serve_slots, autotune=True)
        start = srv.now_ms() + 20.0
        i, outstanding, done = 0, 0, 0
        held = []  # every 997th result, checked after the replay (its temporaries
        #            would allocate device memory, which synchronises the device)
        while i < m or outstanding:
            now = srv.now_ms()
            while i < m and (burst or start + rs[i][0] <= now):
                k, v = view(rs[i])
                srv.submit(k, v, arrival_ms=start if burst else start + rs[i][0])
                i += 1
                outstanding += 1
            for r in srv.poll(wait_ms=0.0 if i < m else 50.0):
                if r["status"] != ahs.OK:
                    raise RuntimeError(f"request {r['id']} failed with status {r['status']}")
                if done % 997 == 0 and r["n"] > 1:
                    held.append(r)
                else:
                    srv.release(r["id"])
                outstanding -= 1
                done += 1
        st = srv.stats()
        for r in held:  # spot check on the device
            x = r["keys"]
            if x.dtype == torch.uint32:
                x = x.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
            elif x.dtype == torch.uint64:
                x = x.view(torch.int64) ^ (-(2 ** 63))  # unsigned order as signed
            assert bool((x[1:] >= x[:-1]).all().item()), "unsorted result"
            srv.release(r["id"])
        checked = len(held)
        srv.close()
        return {"requests": m, "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
                "max_ms": round(st["max_ms"], 3), "gkeys_s": round(st["gkeys_per_s"], 3), "batches": st["batches"],
                "mean_batch_requests": round(st["mean_batch_requests"], 2),
                "arena_peak_GB": round(st["arena_peak_bytes"] / 1e9, 3), "spot_checked": checked}

    def plain(burst):
        rs = burst_reqs if burst else reqs
        ctx = ahs.default_context(0)
        ctx.workspace(ahs.ahs_workspace_bytes(1 << 24, ahs.U64, True, ahs.AUTO))
        out_k = torch.empty(1 << 24, dtype=torch.int64, device=dev)
        out_v = torch.empty(1 << 24, dtype=torch.int32, device=dev).view(torch.uint32)
        torch.cuda.synchronize()
        t0 = time.perf_counter() * 1e3 + 20.0
        lat, last = [], 0.0
        for r in rs:
            a = t0 if burst else t0 + r[0]
            while time.perf_counter() * 1e3 < a:
                pass
            k, v = view(r)
            o = out_k.view(k.dtype)[:k.numel()] if k.element_size() == 8 else \
                out_k.view(torch.int32)[:k.numel()].view(k.dtype)
            ahs.ahs_sort(k, v, out=o, out_values=out_v[:k.numel()] if v is not None else None, ctx=ctx)
            torch.cuda.synchronize()
            last = time.perf_counter() * 1e3
            lat.append(last - a)
        del out_k, out_v
        keys_done = sum(r[3] for r in rs)
        return {"requests": len(rs), "p50_ms": round(percentile(lat, 50), 3), "p99_ms": round(percentile(lat, 99), 3),
                "max_ms": round(max(lat), 3), "gkeys_s": round(keys_done / ((last - t0) * 1e-3) / 1e9, 3)}

    res = {"workload": f"Poisson arrivals 2000/s for {args.serve_seconds}s ({m} requests, {total_keys} keys), "
                       "sizes log-uniform on [2^10, 2^24], u32/u64/f32 (uniform or Zipf(1.0) over 4,096 values; "
                       f"f32 Normal), half with payload; budget {args.serve_budget_gb} GB, {args.serve_slots} slots",
           "offered_gkeys_s": round(total_keys / args.serve_seconds / 1e9, 3),
           "burst": f"the first {args.burst_seconds}s of the trace ({len(burst_reqs)} requests) submitted at once"}
    modes = args.serve_modes.split(",")
    for mode, burst in (("realtime", False), ("burst", True)):
        for kind, fn in (("served", served), ("plain", plain)):
            if kind not in modes:
                continue
            t = time.time()
            res[f"{kind}_{mode}"] = fn(burst)
            log(f"[bench] {kind} {mode} in {time.time() - t:.1f}s: {res[f'{kind}_{mode}']}")
    if "served" in modes and "plain" in modes:
        res["p99_served_over_plain_realtime"] = round(
            res["served_realtime"]["p99_ms"] / res["plain_realtime"]["p99_ms"], 3)
        res["throughput_served_over_plain_burst"] = round(
            res["served_burst"]["gkeys_s"] / res["plain_burst"]["gkeys_s"], 3)
    del pools, pay_pool
    torch.cuda.empty_cache()
    return res


def paper_sweep_section(args, ahs, gen, torch, np):
    """The paper's dataset families (Sec. III-B) at their default sizes: AUTO
    (FSM + selector, and FSM only) against each forced strategy, with every
    strategy's output checked bitwise against the others and for order."""
    dev = torch.device("cuda:0")
    ctx = ahs.default_context(0)
    ctx.set_model(ahs.default_model())
    cfg_auto = ahs.ahs_config_init(ahs.PRESET_GPU, use_model=1)
    cfg_fsm = ahs.ahs_config_init(ahs.PRESET_GPU)
    cfg_cal = ahs.ahs_config_init(ahs.PRESET_MI355X_CALIBRATED)  # thresholds recalibrated by eq. (1)
    rows = []
    for case in gen.PAPER_CASES:
        t = time.time()
        keys = torch.from_numpy(gen.paper_sweep(case)).to(dev)
        n = keys.numel()
        out = torch.empty_like(keys)
        torch.cuda.synchronize()
        row = {"case": case, "dtype": str(keys.dtype).replace("torch.", ""), "n": n}
        ref = None
        for sname, strat, cfg in (("auto", ahs.AUTO, cfg_auto), ("auto_fsm", ahs.AUTO, cfg_fsm),
                                  ("auto_fsm_calibrated", ahs.AUTO, cfg_cal),
                                  ("counting", ahs.COUNTING, cfg_fsm), ("radix", ahs.RADIX, cfg_fsm),
                                  ("quick", ahs.QUICK, cfg_fsm)):
            times = []
            try:
                for r in range(args.reps + 1):  # the first run is not timed
                    torch.cuda.synchronize()
                    a = time.perf_counter()
                    _, _, ch, f = ahs.ahs_sort(keys, strategy=strat, cfg=cfg, out=out, ctx=ctx, want_features=r == 0)
                    torch.cuda.synchronize()
                    if r == 0:
                        feats = f
                    else:
                        times.append(time.perf_counter() - a)
            except ahs.AhsError as e:
                row[sname] = {"status": e.status}
                continue
            if ref is None:
                ref = out.clone()
                if keys.dtype in (torch.int32, torch.int64):
                    x = out
                elif keys.dtype == torch.uint32:
                    x = out.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
                else:
                    x = out.view(torch.int64) ^ (-(2 ** 63))  # unsigned order as signed
                row["sorted_ok"] = bool((x[1:] >= x[:-1]).all().item())
                row.update({"span": feats.span, "nbins": feats.nbins, "entropy_bits": round(feats.entropy_bits, 4)})
                del x
                agree = True
            else:
                agree = bool(torch.equal(ref.view(torch.uint8), out.view(torch.uint8)))
            med = statistics.median(times)
            row[sname] = {"ms": round(med * 1e3, 4), "Gkeys_s": round(n / med / 1e9, 2),
                          "chosen": ahs.STRATEGY_NAMES[ch], "agrees": agree}
        forced = {k: row[k]["ms"] for k in ("counting", "radix", "quick") if "ms" in row[k]}
        best = min(forced, key=forced.get)
        row["best_forced"] = best
        row["auto_over_best"] = round(row["auto"]["ms"] / forced[best], 4)
        row["auto_fsm_over_best"] = round(row["auto_fsm"]["ms"] / forced[best], 4)
        row["auto_fsm_calibrated_over_best"] = round(row["auto_fsm_calibrated"]["ms"] / forced[best], 4)
        rows.append(row)
        log(f"[bench] paper case {case} in {time.time() - t:.1f}s: auto {row['auto']['chosen']} "
            f"{row['auto']['ms']} ms, best {best} {forced[best]} ms, fsm {row['auto_fsm']['chosen']}")
        del keys, out, ref
        torch.cuda.empty_cache()
    ratios = [r["auto_over_best"] for r in rows]
    fsm = [r["auto_fsm_over_best"] for r in rows]
    cal = [r["auto_fsm_calibrated_over_best"] for r in rows]
    return {"workload": "the paper's dataset families: uniform k in {1e2, 1e4, 1e6}, Normal(0, k/4) rounded "
                        "(int32) for k in 1e2..1e6, Zipf(1.5) ranks over k in {1e2, 1e4, 1e6}, constant, ascending, "
                        "descending, sawtooth, alternating, full-range int32/int64, and synthetic (n, k, H) "
                        "stand-ins for the taxi, sensor and k-mer datasets; 2^24 keys unless the paper gives n",
            "auto_over_best_geomean": round(float(np.exp(np.mean(np.log(ratios)))), 4),
            "auto_over_best_max": max(ratios),
            "auto_fsm_over_best_geomean": round(float(np.exp(np.mean(np.log(fsm)))), 4),
            "auto_fsm_over_best_max": max(fsm),
            "auto_fsm_calibrated_over_best_geomean": round(float(np.exp(np.mean(np.log(cal)))), 4),
            "auto_fsm_calibrated_over_best_max": max(cal),
            "all_sorted_and_agreeing": all(r["sorted_ok"] and all(r[k].get("agrees", True) for k in
                                                                  ("auto", "auto_fsm", "auto_fsm_calibrated",
                                                                   "counting", "radix", "quick"))
                                           for r in rows),
            "cases": rows}


def _timed_sort(ahs, torch, keys, values, strat, cfg, out, out_v, ctx, reps):
    """Median wall time of `reps` AHS calls (the first, untimed, warms up),
    with the algorithmic bytes of one call's kernels and the chosen strategy."""
    times, path_bytes, ch = [], None, None
    for r in range(reps + 1):
        ahs.ahs_profile_enable(ctx, True)
        ahs.ahs_profile_reset(ctx)
        torch.cuda.synchronize()
        a = time.perf_counter()
        _, _, ch, _ = ahs.ahs_sort(keys, values, strategy=strat, cfg=cfg, out=out, out_values=out_v, ctx=ctx)
        torch.cuda.synchronize()
        if r:
            times.append(time.perf_counter() - a)
        path_bytes = sum(v[2] for v in ahs.ahs_profile_dump(ctx).values())
        ahs.ahs_profile_enable(ctx, False)
    return statistics.median(times), path_bytes, ch


def _ordered(torch, x):
    """Keys as int64 whose signed order is the sort order of the dtype (for
    the on-device order check of a result)."""
    if x.dtype == torch.uint32:
        return x.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    if x.dtype == torch.float32:
        b = x.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        return torch.where(b >= 2 ** 31, (2 ** 32 - 1) - b, b + 2 ** 31)
    if x.dtype == torch.float64:
        b = x.view(torch.int64)
        return torch.where(b < 0, ~b, b ^ (-(2 ** 63))) ^ (-(2 ** 63))
    if x.dtype == torch.uint64:
        return x.view(torch.int64) ^ (-(2 ** 63))
    return x.to(torch.int64)


def strategy_table(reps, ahs, torch, keys, with_payload, strategies, ctx):
    """AUTO and forced strategies on one device array: median ms, Gkeys/s,
    path %HBM, and whether every strategy produced the same bytes."""
    n = keys.numel()
    vals = torch.arange(n, dtype=torch.int32, device=keys.device).view(torch.uint32) if with_payload else None
    out = torch.empty_like(keys)
    out_v = torch.empty_like(vals) if with_payload else None
    row, ref, ref_v = {}, None, None
    for sname, strat, cfg in strategies:
        try:
            med, pb, ch = _timed_sort(ahs, torch, keys, vals, strat, cfg, out, out_v, ctx, reps)
        except ahs.AhsError as e:
            ahs.ahs_profile_enable(ctx, False)
            row[sname] = {"status": e.status}
            continue
        if ref is None:
            ref, ref_v = out.clone(), (out_v.clone() if with_payload else None)
            x = _ordered(torch, out)
            row["sorted_ok"] = bool((x[1:] >= x[:-1]).all().item())
            del x
            agree = True
        else:
            agree = bool(torch.equal(ref.view(torch.uint8), out.view(torch.uint8)))
            if with_payload:
                agree = agree and bool(torch.equal(ref_v.view(torch.int32), out_v.view(torch.int32)))
        row[sname] = {"ms": round(med * 1e3, 4), "Gkeys_s": round(n / med / 1e9, 2),
                      "chosen": ahs.STRATEGY_NAMES[ch], "path_GB": round(pb / 1e9, 3),
                      "hbm_frac_path": round(pb / med / 1e9 / HBM_PEAK_GBS, 4), "agrees": agree}
    forced = {k: row[k]["ms"] for k in ("counting", "radix", "quick") if "ms" in row.get(k, {})}
    if forced:
        best = min(forced, key=forced.get)
        row["best_forced"] = best
        for a in ("auto", "auto_fsm"):
            if "ms" in row.get(a, {}):
                row[f"{a}_over_best"] = round(row[a]["ms"] / forced[best], 4)
    del vals, out, out_v, ref, ref_v
    return row


def _pin_one_core():
    """Pins this process to one core for the single-threaded oracle; returns
    the previous affinity (to restore) and the core."""
    old = os.sched_getaffinity(0)
    core = max(old)
    os.sched_setaffinity(0, {core})
    return old, core


def pr1_section(args, ahs, gen, torch, np):
    """PR1: 10^6 uint32 keys uniform on [0, 1023] (seed 0): AUTO, forced
    RADIX and forced QUICK, keys only and with payload = index, each checked
    bitwise against the CPU oracle; the oracle timed on one pinned core."""
    import oracle
    dev = torch.device("cuda:0")
    ctx = ahs.default_context(0)
    ctx.set_model(ahs.default_model())
    keys_h = gen.pr1()
    keys = torch.from_numpy(keys_h).to(dev)
    n = keys.numel()
    cfg = ahs.ahs_config_init(ahs.PRESET_GPU)
    cfg_m = ahs.ahs_config_init(ahs.PRESET_GPU, use_model=1)
    strategies = (("auto", ahs.AUTO, cfg_m), ("auto_fsm", ahs.AUTO, cfg), ("counting", ahs.COUNTING, cfg),
                  ("radix", ahs.RADIX, cfg), ("quick", ahs.QUICK, cfg))
    res = {"workload": "PR1: 1,000,000 uint32 keys uniform on [0, 1023] (seed 0)", "n": n}
    vals_h = np.arange(n, dtype=np.uint32)
    exact = True
    for pay in (False, True):
        tab = strategy_table(max(args.reps, 10), ahs, torch, keys, pay, strategies, ctx)
        # bitwise against the oracle for AUTO, RADIX and QUICK
        for sname, strat in (("auto_fsm", ahs.AUTO), ("radix", ahs.RADIX), ("quick", ahs.QUICK)):
            v = torch.from_numpy(vals_h).to(dev) if pay else None
            ko, vo, ch, _ = ahs.ahs_sort(keys, v, strategy=strat, cfg=cfg, ctx=ctx)
            st, rk, rv, rch, _ = oracle.sort(keys_h, vals_h if pay else None, strat)
            ok = st == 0 and np.array_equal(ko.cpu().numpy(), rk) and ch == rch
            if pay:
                ok = ok and np.array_equal(vo.cpu().numpy(), rv)
            tab[sname]["oracle_exact"] = bool(ok)
            exact = exact and ok
        res["with_payload" if pay else "keys_only"] = tab
    old, core = _pin_one_core()
    try:
        for sname, strat in (("auto", oracle.AUTO), ("radix", oracle.RADIX), ("quick", oracle.QUICK)):
            ts = []
            for _ in range(10):
                a = time.perf_counter()
                st, _, _, _, _ = oracle.sort(keys_h, None, strat)
                ts.append(time.perf_counter() - a)
            res.setdefault("oracle_ms", {})[sname] = round(statistics.median(ts) * 1e3, 3)
    finally:
        os.sched_setaffinity(0, old)
    res["oracle_core"] = core
    res["all_oracle_exact"] = exact
    log(f"[bench] pr1 {json.dumps(res)}")
    del keys
    torch.cuda.empty_cache()
    return res


def wide_section(args, ahs, gen, torch, np):
    """Wide and floating keys at 2^27: u64 uniform, u64 Zipf(1.0) over 4,096
    values, f32 and f64 Normal(0, 1e3) with duplicates and signed zeros; AUTO
    against forced RADIX and QUICK, keys only and with payload = index."""
    dev = torch.device("cuda:0")
    ctx = ahs.default_context(0)
    ctx.set_model(ahs.default_model())
    cfg = ahs.ahs_config_init(ahs.PRESET_GPU)
    cfg_m = ahs.ahs_config_init(ahs.PRESET_GPU, use_model=1)
    strategies = (("auto", ahs.AUTO, cfg_m), ("auto_fsm", ahs.AUTO, cfg), ("radix", ahs.RADIX, cfg),
                  ("quick", ahs.QUICK, cfg))
    n = 1 << args.wide_log2n
    rows = []
    for case in gen.WIDE_CASES:
        t = time.time()
        keys = torch.from_numpy(gen.wide_keys(case, n=n)).to(dev)
        for pay in (False, True):
            row = {"case": case, "payload": pay, "n": n}
            row.update(strategy_table(args.reps, ahs, torch, keys, pay, strategies, ctx))
            rows.append(row)
            log(f"[bench] wide {case} payload={pay} in {time.time() - t:.1f}s: " + json.dumps(row))
        del keys
        torch.cuda.empty_cache()
    ratios = [r["auto_over_best"] for r in rows if "auto_over_best" in r]
    return {"workload": f"wide keys, 2^{args.wide_log2n} per array: " + ", ".join(gen.WIDE_CASES) +
                        "; keys only and with payload = index",
            "auto_over_best_max": max(ratios), "all_sorted_and_agreeing":
                all(r["sorted_ok"] and all(r[k].get("agrees", True) for k in ("auto", "auto_fsm", "radix", "quick"))
                    for r in rows),
            "cases": rows}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=28, help="keys per array (2^log2n)")
    ap.add_argument("--reps", type=int, default=5, help="runs per (array, strategy) for medians")
    ap.add_argument("--cases", action=argparse.BooleanOptionalAction, default=True,
                    help="per-array AUTO vs forced strategies")
    ap.add_argument("--cpu-baseline", action=argparse.BooleanOptionalAction, default=True)
    ap.add_argument("--cpu-sample-log2", type=int, default=26,
                    help="keys of each array the oracle sorts for the CPU baseline")
    ap.add_argument("--cpu-runs", type=int, default=3, help="oracle runs for the CPU baseline median")
    ap.add_argument("--pr1", action=argparse.BooleanOptionalAction, default=True,
                    help="PR1: 10^6 keys on [0, 1023], AUTO vs forced RADIX/QUICK, against the oracle")
    ap.add_argument("--wide", action=argparse.BooleanOptionalAction, default=True,
                    help="wide and floating keys: AUTO vs forced strategies, keys only and with payload")
    ap.add_argument("--wide-log2n", type=int, default=27)
    ap.add_argument("--detail-out", default=os.path.join("gpurun_out", "bench_detail.json"),
                    help="file that receives every section in full (the stdout line carries summaries)")
    ap.add_argument("--only", default=None, help="comma list of sweep cases to run")
    ap.add_argument("--force", default="auto", choices=("auto", "counting", "radix", "quick"),
                    help="strategy of the timed steps (auto: the method; a forced one for kernel profiles)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain elementwise copy of 2^log2n 32-bit words first (counter calibration)")
    ap.add_argument("--headline", action=argparse.BooleanOptionalAction, default=True,
                    help="the strategy sweep (the reported value); --no-headline runs only the other sections")
    ap.add_argument("--paper-sweep", action=argparse.BooleanOptionalAction, default=True,
                    help="the paper's dataset families, AUTO vs each forced strategy")
    ap.add_argument("--batched", action=argparse.BooleanOptionalAction, default=True)
    ap.add_argument("--seg-count", type=int, default=65536, help="segments in the batched workload")
    ap.add_argument("--seg-reps", type=int, default=3, help="timed graph replays of the batched sort")
    ap.add_argument("--seg-loop", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the host loop of per-array calls over the same segments")
    ap.add_argument("--serve", action=argparse.BooleanOptionalAction, default=True)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="seconds of the Poisson request trace replayed in real time")
    ap.add_argument("--burst-seconds", type=float, default=10.0,
                    help="seconds of the same trace submitted at once (throughput runs)")
    ap.add_argument("--serve-budget-gb", type=float, default=48.0)
    ap.add_argument("--serve-slots", type=int, default=4, help="stream slots of the server")
    ap.add_argument("--serve-modes", default="served,plain", help="which serving runs: served, plain or both")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(how the sort would shard is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2506_20677_amd as ahs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if not args.headline:
        side = {"paper_sweep": paper_sweep_section(args, ahs, gen, torch, np) if args.paper_sweep else None,
                "batched": batched_section(args, ahs, gen, torch, np) if args.batched else None,
                "serving": serving_section(args, ahs, gen, torch, np) if args.serve else None}
        print(json.dumps({"metric": METRIC, "value": None, "note": "sections only (--no-headline)", **side}),
              flush=True)
        return
    n = 1 << args.log2n
    cases = list(gen.SWEEP_CASES) if not args.only else args.only.split(",")

    # ------------------------------------------------------------ inputs
    host = {}
    dkeys = {}
    for c in cases:
        t = time.time()
        host[c] = gen.strategy_sweep(c, n=n)
        dkeys[c] = torch.from_numpy(host[c]).to(dev)
        log(f"[bench] generated {c} n=2^{args.log2n} in {time.time() - t:.1f}s")
    out = torch.empty(n, dtype=torch.uint32, device=dev)
    ctx = ahs.default_context(0)
    ws_bytes = ahs.ahs_workspace_bytes(n, ahs.U32, False, ahs.AUTO)
    ctx.workspace(ws_bytes)
    # AUTO = the FSM plus the gradient-boosted selector trained on MI355X
    # measurements (the paper's two decision mechanisms)
    model = ahs.default_model()
    ctx.set_model(model)
    cfg_auto = ahs.ahs_config_init(ahs.PRESET_GPU, use_model=1)
    cfg_fsm = ahs.ahs_config_init(ahs.PRESET_GPU)
    torch.cuda.synchronize()

    strat = ahs.STRATEGY_CODES[args.force]

    def step():
        chosen = {}
        for c in cases:
            _, _, ch, _ = ahs.ahs_sort(dkeys[c], strategy=strat, cfg=cfg_auto if strat == ahs.AUTO else cfg_fsm,
                                       out=out, ctx=ctx)
            chosen[c] = ahs.STRATEGY_NAMES[ch]
        return chosen

    if args.calib_copy:
        # plain copy kernel of known size: reads and writes 4 bytes per element
        a32 = dkeys[cases[0]].view(torch.int32)
        torch.neg(a32, out=out.view(torch.int32))
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {4 * n} bytes read + {4 * n} bytes written")
    for _ in range(args.warmup):
        chosen = step()
    torch.cuda.synchronize()
    log(f"[bench] warmup done, AUTO choices {chosen}")

    # ------------------------------------------------------------ timed steps
    ahs.ahs_profile_enable(ctx, True)
    ahs.ahs_profile_reset(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        chosen = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ahs.ahs_profile_dump(ctx)
    ahs.ahs_profile_enable(ctx, False)
    elapsed = t1 - t0
    keys_total = n * len(cases) * args.steps
    value = keys_total / elapsed / 1e9
    ms_per_step = elapsed / args.steps * 1e3
    log(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.2f} Gkeys/s")

    dom = max(prof.items(), key=lambda kv: kv[1][1])
    dname, (dl, dms, dbytes) = dom
    achieved = dbytes / (dms / 1e3) / 1e9 if dms > 0 else 0.0
    tag = f"strategy_sweep_2p{args.log2n}_u32" if not args.only and args.force == "auto" else None
    traffic = measured_traffic(dname, tag) if tag else None
    roofline = {
        "bound": "hbm", "kernel": dname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
        "traffic_over_algorithmic": round(traffic / (dbytes / dl), 3) if traffic and dl else None,
        "launches": dl, "avg_launch_ms": round(dms / dl, 5) if dl else None,
        "algo_bytes_per_launch": round(dbytes / dl) if dl else None,
    }
    step_kernels = {k: {"launches": v[0], "ms_total": round(v[1], 4), "algo_GB": round(v[2] / 1e9, 4),
                        "GBps": round(v[2] / (v[1] / 1e3) / 1e9, 1) if v[1] > 0 else None}
                    for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])}

    # ------------------------------------------------------------ practical ceilings
    # a plain device copy (read + write) and a plain read-only reduction of
    # one array, timed with events: what streaming kernels reach on this GPU
    def event_ms(fn, reps=5):
        ts = []
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return statistics.median(ts[1:])
    src32 = dkeys[cases[0]].view(torch.int32)
    copy_ms = event_ms(lambda: out.view(torch.int32).copy_(src32))
    read_ms = event_ms(lambda: torch.amax(src32))
    ceilings = {"copy_GBps": round(2 * 4 * n / copy_ms / 1e6, 1), "read_GBps": round(4 * n / read_ms / 1e6, 1),
                "how": f"torch copy (read + write) and torch.amax (read) of 2^{args.log2n} int32, event-timed medians"}
    ceilings["copy_frac"] = round(ceilings["copy_GBps"] / HBM_PEAK_GBS, 4)
    ceilings["read_frac"] = round(ceilings["read_GBps"] / HBM_PEAK_GBS, 4)
    log(f"[bench] ceilings {ceilings}")

    # ------------------------------------------------------------ per array and strategy
    per_case = []
    if args.cases:
        for c in cases:
            row = {"case": c, "auto_choice": chosen[c]}
            ref = None
            for sname, s, cfg in (("auto", ahs.AUTO, cfg_auto), ("auto_fsm", ahs.AUTO, cfg_fsm),
                                  ("counting", ahs.COUNTING, cfg_fsm), ("radix", ahs.RADIX, cfg_fsm),
                                  ("quick", ahs.QUICK, cfg_fsm)):
                times = []
                path_bytes = None
                try:
                    for r in range(args.reps):
                        ahs.ahs_profile_enable(ctx, True)
                        ahs.ahs_profile_reset(ctx)
                        torch.cuda.synchronize()
                        a = time.perf_counter()
                        _, _, ch, _ = ahs.ahs_sort(dkeys[c], strategy=s, cfg=cfg, out=out, ctx=ctx)
                        torch.cuda.synchronize()
                        times.append(time.perf_counter() - a)
                        p = ahs.ahs_profile_dump(ctx)
                        path_bytes = sum(v[2] for v in p.values())
                    ahs.ahs_profile_enable(ctx, False)
                except ahs.AhsError as e:
                    ahs.ahs_profile_enable(ctx, False)
                    row[sname] = {"status": e.status}
                    continue
                # every strategy must produce the same bits (stable sort is unique)
                o = out.view(torch.int32)
                if ref is None:
                    ref = o.clone()
                    u = o.to(torch.int64) & 0xFFFFFFFF
                    row["sorted_ok"] = bool((u[1:] >= u[:-1]).all().item())
                    del u
                    agree = True
                else:
                    agree = bool(torch.equal(ref, o))
                med = statistics.median(times)
                row[sname] = {"ms": round(med * 1e3, 4), "Gkeys_s": round(n / med / 1e9, 2),
                              "chosen": ahs.STRATEGY_NAMES[ch],
                              "path_GB": round(path_bytes / 1e9, 3),
                              "hbm_frac_path": round(path_bytes / med / 1e9 / HBM_PEAK_GBS, 4),
                              "agrees": agree, "kernels": {k: [v[0], round(v[1], 4)] for k, v in p.items()}}
            forced = {k: row[k]["ms"] for k in ("counting", "radix", "quick") if "ms" in row.get(k, {})}
            best = min(forced.values(), default=None)
            if forced:
                row["best_forced"] = min(forced, key=forced.get)
            if best and "ms" in row.get("auto", {}):
                row["auto_over_best"] = round(row["auto"]["ms"] / best, 4)
            if best and "ms" in row.get("auto_fsm", {}):
                row["auto_fsm_over_best"] = round(row["auto_fsm"]["ms"] / best, 4)
            per_case.append(row)
            log(f"[bench] case {c}: " + json.dumps(row))
            del ref

    # ------------------------------------------------------------ CPU oracle baseline
    cpu = None
    if args.cpu_baseline:
        import oracle

        m = min(n, 1 << args.cpu_sample_log2)
        omodel = oracle.Model(ahs.SELECTOR_MODEL)
        ocfg = oracle.config(0, use_model=1)
        samples = [np.ascontiguousarray(host[c][:m]) for c in cases]
        old_aff, core = _pin_one_core()
        runs = []
        try:
            for _ in range(args.cpu_runs):
                a = time.perf_counter()
                for c, sample in zip(cases, samples):
                    st, _, _, _, _ = oracle.sort(sample, None, oracle.AUTO, ocfg, omodel)
                    if st != 0:
                        log(f"[bench] oracle status {st} on {c}")
                runs.append(time.perf_counter() - a)
        finally:
            os.sched_setaffinity(0, old_aff)
        med = statistics.median(runs)
        tot_k = m * len(cases)
        cpu = {"value": round(tot_k / med / 1e9, 6), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
               "sample": f"first 2^{int(np.log2(m))} keys of each of the {len(cases)} arrays, AHS AUTO "
                         f"(FSM + the same selector model), single-threaded C oracle pinned to core {core}, "
                         f"median of {len(runs)} runs of {med:.1f} s",
               **host_info()}
        log(f"[bench] cpu baseline {cpu}")

    # ------------------------------------------------------------ other configurations
    del dkeys, out, host
    torch.cuda.empty_cache()
    pr1 = pr1_section(args, ahs, gen, torch, np) if args.pr1 else None
    wide = wide_section(args, ahs, gen, torch, np) if args.wide else None
    paper = paper_sweep_section(args, ahs, gen, torch, np) if args.paper_sweep else None
    batched = batched_section(args, ahs, gen, torch, np) if args.batched else None
    serving = serving_section(args, ahs, gen, torch, np) if args.serve else None

    res = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gkeys/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"strategy sweep: {len(cases)} arrays x 2^{args.log2n} uint32 ({', '.join(cases)}), "
                               + ("AHS AUTO per array (FSM + selector trained on MI355X measurements)"
                                  if args.force == "auto" else f"strategy forced to {args.force.upper()}"),
                   "n_per_array": n, "auto_choices": chosen},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    detail = dict(res, ceilings=ceilings, step_kernels=step_kernels, per_case=per_case, pr1=pr1, wide=wide,
                  paper_sweep=paper, batched=batched, serving=serving)
    try:
        os.makedirs(os.path.dirname(args.detail_out) or ".", exist_ok=True)
        with open(args.detail_out, "w") as f:
            json.dump(detail, f, indent=1)
    except OSError as e:
        log(f"[bench] cannot write {args.detail_out}: {e}")
    log("[bench] detail " + json.dumps(detail))
    res["summary"] = summarise(per_case, pr1, wide, paper, batched, serving, ceilings)
    line = json.dumps(res, separators=(",", ":"))
    if len(line) > 3900:  # the stdout line stays short: drop summary parts, largest first
        for k in sorted(res["summary"], key=lambda k: -len(json.dumps(res["summary"][k]))):
            del res["summary"][k]
            line = json.dumps(res, separators=(",", ":"))
            if len(line) <= 3900:
                break
    print(line, flush=True)


def summarise(per_case, pr1, wide, paper, batched, serving, ceilings):
    """A few figures per section for the stdout line (the detail file has all)."""
    out = {"ceilings": {k: ceilings[k] for k in ("copy_GBps", "read_GBps")}}
    if per_case:
        out["sweep"] = {r["case"]: [r.get("auto", {}).get("ms"), r.get("best_forced"), r.get("auto_over_best"),
                                    max((r[k].get("hbm_frac_path", 0) for k in ("counting", "radix", "quick")
                                         if k in r and "ms" in r[k]), default=None)]
                        for r in per_case}
        out["sweep_cols"] = "auto_ms, best forced, auto/best, best path hbm frac"
    if pr1:
        out["pr1"] = {"ms": {k: pr1["keys_only"][k].get("ms") for k in ("auto", "radix", "quick")},
                      "oracle_ms": pr1["oracle_ms"], "oracle_exact": pr1["all_oracle_exact"]}
    if wide:
        out["wide"] = {f"{r['case']}{'+p' if r['payload'] else ''}": [r.get("auto", {}).get("ms"),
                                                                      r.get("best_forced"), r.get("auto_over_best")]
                       for r in wide["cases"]}
        out["wide_ok"] = wide["all_sorted_and_agreeing"]
    if paper:
        out["paper_sweep"] = {k: paper[k] for k in ("auto_over_best_geomean", "auto_over_best_max",
                                                    "all_sorted_and_agreeing")}
    if batched:
        out["batched"] = {k: batched.get(k) for k in ("graph_ms", "blocking_ms", "loop_ms", "speedup_graph_vs_loop",
                                                      "identical_outputs", "graph_status")}
    if serving:
        out["serving"] = {k: serving.get(k) for k in ("p99_served_over_plain_realtime",
                                                      "throughput_served_over_plain_burst")}
        for k in ("served_realtime", "plain_realtime", "served_burst", "plain_burst"):
            if k in serving:
                out["serving"][k] = [serving[k]["p50_ms"], serving[k]["p99_ms"], serving[k]["gkeys_s"]] + \
                    ([serving[k]["mean_batch_requests"]] if "mean_batch_requests" in serving[k] else [])
        out["serving_cols"] = "p50_ms, p99_ms, Gkeys/s, mean requests per batch"
    return out


if __name__ == "__main__":
    main()
