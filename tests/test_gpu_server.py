"""GPU tests of the serving loop: every request's result equals the oracle's
sort of that request (keys and payload bit-exact, decision as the FSM's up
to the entropy-threshold tie), the same alone and in a mix, under
continuous batching with several slots and under a tight HBM budget."""
import math
import sys

import numpy as np
import pytest

import gen
import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_20677_amd as ahs  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def bits(a):
    return a.view(np.uint32 if a.itemsize == 4 else np.uint64)


def host_bits(t):
    """Host copy of a result tensor as raw bits."""
    if t.dtype in (torch.uint32, torch.uint64):
        t = t.view(torch.int32 if t.dtype == torch.uint32 else torch.int64)
    a = t.cpu().numpy()
    return a.view(np.uint32 if a.itemsize == 4 else np.uint64)


def make_requests(count, seed, lo_exp=4, span_exp=12):
    """Mixed key types, sizes, distributions and payloads (the serving mix)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        n = int(2 ** (lo_exp + span_exp * rng.random()))
        kind = i % 3
        if kind == 0:
            keys = gen.u32(seed, 100 + i, n) if rng.random() < 0.5 else gen.zipf_keys(seed + i, n, 64, 1.1, 32)
            keys = keys.astype(np.uint32)
        elif kind == 1:
            keys = gen.u64(seed, 100 + i, n) if rng.random() < 0.5 else gen.zipf_keys(seed + i, n, 4096, 1.0, 64)
        else:
            keys = gen.wide_keys("f32normal", n=n, seed=seed + i)
        vals = np.arange(n, dtype=np.uint32) if rng.random() < 0.5 else None
        reqs.append((keys, vals))
    reqs[3] = (np.zeros(0, np.uint32), None)          # an empty request
    reqs[4] = (np.full(1000, 7, np.uint64), None)      # all equal
    return reqs


def check_result(res, keys, vals):
    assert res["status"] == ahs.OK, res
    st, rk, rv, rchosen, rf = O.sort(keys, vals, O.AUTO, O.config(0))
    assert st == O.OK
    if keys.size:
        assert np.array_equal(host_bits(res["keys"]), bits(rk))
    if vals is not None and keys.size:
        assert np.array_equal(host_bits(res["values"]), rv)
    if res["chosen"] != rchosen:
        thr = 0.7 * math.log2(rf.nbins) if rf.nbins > 1 else 0.0
        assert abs(rf.entropy_bits - thr) <= 1e-6 * thr, (res["chosen"], rchosen)


def drain(server, want, wait_ms=200.0, limit_s=60.0):
    import time
    out = {}
    t = time.time()
    while len(out) < want:
        for r in server.poll(wait_ms=wait_ms):
            out[r["id"]] = r
        assert time.time() - t < limit_s, "server did not finish"
    return out


def run_mix(server, reqs):
    dev = [(to_dev(k), to_dev(v) if v is not None else None) for k, v in reqs]
    torch.cuda.synchronize()
    ids = [server.submit(k, v) for k, v in dev]
    done = drain(server, len(ids))
    results = []
    for i, rid in enumerate(ids):
        r = done[rid]
        results.append((host_bits(r["keys"]) if r["keys"] is not None and r["n"] else np.zeros(0),
                        host_bits(r["values"]) if r["values"] is not None and r["n"] else None, r["chosen"]))
        check_result(r, *reqs[i])
        server.release(rid)
    return results


def test_server_mix_matches_oracle_and_batches():
    reqs = make_requests(60, seed=61)
    # lazy dispatch: all 60 requests are pending when the first poll forms batches
    s = ahs.Server(hbm_budget_bytes=2 << 30, slots=3, lazy_dispatch=True)
    say("server mix of 60 requests")
    run_mix(s, reqs)
    st = s.stats()
    say(st)
    assert st["completed"] == 60 and st["failed"] == 0 and st["pending"] == 0
    assert st["batches"] < 60 and st["mean_batch_requests"] > 1.0  # requests were grouped
    assert st["arena_used_bytes"] == 0 and st["arena_peak_bytes"] <= 2 << 30
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    s.close()


def test_server_result_same_alone_and_in_mix():
    reqs = make_requests(30, seed=62)
    s = ahs.Server(hbm_budget_bytes=1 << 30, slots=4)
    mixed = run_mix(s, reqs)
    alone = []
    for k, v in reqs:
        alone.extend(run_mix(s, [(k, v)]))
    for (ka, va, ca), (kb, vb, cb) in zip(mixed, alone):
        assert np.array_equal(ka, kb)
        assert (va is None and vb is None) or np.array_equal(va, vb)
        assert ca == cb
    s.close()


def test_server_tight_budget_admits_as_memory_frees():
    """The arena holds about one large request at a time: everything still
    completes, in order of admission, and never above the budget; a request
    larger than the whole budget fails with AHS_E_OOM."""
    budget = 48 << 20
    s = ahs.Server(hbm_budget_bytes=budget, slots=4, max_batch_keys=1 << 20)
    reqs = [(gen.u32(63, i, 1 << 20), None) for i in range(6)] + [(gen.u32(64, 0, 5000), None)]
    dev = [to_dev(k) for k, _ in reqs]
    torch.cuda.synchronize()
    ids = [s.submit(k) for k in dev]
    huge = torch.zeros(8 << 20, dtype=torch.int64, device=DEV).view(torch.uint64)  # 64 MiB of keys > budget
    hid = s.submit(huge)
    done = {}
    import time
    t = time.time()
    while len(done) < len(ids) + 1:
        for r in s.poll(wait_ms=100.0):
            done[r["id"]] = r
            if r["status"] == ahs.OK:
                i = ids.index(r["id"])
                check_result(r, *reqs[i])
            s.release(r["id"])  # frees memory for the next admission
        assert time.time() - t < 60
    assert done[hid]["status"] == ahs.E_OOM
    st = s.stats()
    assert st["completed"] == len(ids) and st["failed"] == 1
    assert st["arena_peak_bytes"] <= budget
    s.close()


def test_server_requests_arrive_while_others_run():
    """Continuous batching: new requests are submitted between polls while
    earlier batches are still on the device."""
    reqs = make_requests(40, seed=65, lo_exp=10, span_exp=8)
    s = ahs.Server(hbm_budget_bytes=2 << 30, slots=2)
    dev = [(to_dev(k), to_dev(v) if v is not None else None) for k, v in reqs]
    torch.cuda.synchronize()
    ids, done = [], {}
    for i, (k, v) in enumerate(dev):
        ids.append(s.submit(k, v))
        if i % 5 == 4:
            for r in s.poll():
                done[r["id"]] = r
    done.update(drain(s, len(ids) - len(done)) if len(done) < len(ids) else {})
    for i, rid in enumerate(ids):
        check_result(done[rid], *reqs[i])
        s.release(rid)
    assert s.stats()["completed"] == len(ids)
    s.close()


def test_server_signed_requests():
    """Signed 32- and 64-bit requests beside unsigned ones: each key type
    forms its own batches; results equal the oracle's."""
    rng = np.random.default_rng(63)
    reqs = []
    for i in range(24):
        n = int(2 ** (4 + 11 * rng.random()))
        dt = (np.int32, np.int64, np.uint32)[i % 3]
        info = np.iinfo(dt)
        if i % 2:  # narrow span (around zero for the signed types)
            lo = 0 if dt == np.uint32 else -1000
            keys = rng.integers(lo, lo + 2000, n).astype(dt)
        else:  # the whole range of the type
            keys = rng.integers(int(info.min), int(info.max), n, dtype=np.int64, endpoint=True).astype(dt) \
                if dt != np.uint32 else gen.u32(63, i, n)
        vals = np.arange(n, dtype=np.uint32) if i % 4 < 2 else None
        reqs.append((keys, vals))
    s = ahs.Server(hbm_budget_bytes=1 << 30, slots=2, lazy_dispatch=True)
    say("server signed mix of 24 requests")
    run_mix(s, reqs)
    assert s.stats()["failed"] == 0
    s.close()


def test_server_lone_large_request_with_nan_matches_batched_sort():
    """A lone large request holding NaN keys (sorted straight from the
    caller's buffers by the enqueue-only batched sort) is reported like a
    batched segment (status OK, decision code SEG_NAN, keys in bit-map
    order), identical to ahs_sort_segmented of it alone."""
    r = np.random.default_rng(66)
    keys = r.normal(0, 1e3, 20_000).astype(np.float32)
    keys[::997] = np.nan
    keys[5] = -np.nan
    vals = np.arange(keys.size, dtype=np.uint32)
    k, v = to_dev(keys), to_dev(vals)
    torch.cuda.synchronize()
    s = ahs.Server(hbm_budget_bytes=1 << 30, slots=2)
    rid = s.submit(k, v)
    res = drain(s, 1)[rid]
    assert res["status"] == ahs.OK and res["chosen"] == ahs.SEG_NAN
    offs = torch.tensor([0, keys.size], dtype=torch.int64, device=DEV)
    ko, vo, ch, _ = ahs.ahs_sort_segmented(k, offs, v)
    torch.cuda.synchronize()
    assert np.array_equal(host_bits(res["keys"]), host_bits(ko))
    assert np.array_equal(host_bits(res["values"]), host_bits(vo))
    assert int(ch[0].item()) == ahs.SEG_NAN
    s.release(rid)
    s.close()


def test_server_latency_is_bounded_by_wall_time():
    """The reported latency (completion on the GPU clock - arrival on the
    server clock) never exceeds the wall time from submit to the end of the
    drain: the two clocks share their origin even when the server autotunes
    at creation (regression: the host origin was taken after autotuning)."""
    import time
    s = ahs.Server(hbm_budget_bytes=1 << 30, slots=2, autotune=True)
    k = to_dev(gen.u32(67, 0, 50_000))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rid = s.submit(k)
    res = drain(s, 1)[rid]
    wall_ms = (time.perf_counter() - t0) * 1e3
    assert res["status"] == ahs.OK
    st = s.stats()
    say(st["max_ms"], wall_ms)
    assert 0 < st["max_ms"] <= wall_ms + 2.0
    s.release(rid)
    s.close()
