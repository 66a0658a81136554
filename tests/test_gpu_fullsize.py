"""Parity at the benchmark's full sizes, in the configuration bench.py times.

The oracle cannot sort 2^28 keys in seconds, so at these sizes the checks
are: the features and the AUTO decision against the oracle's (exact, which
the C oracle computes at any size in a few seconds); and, for the sorted
output, properties that define the stable sort at any size: ascending order,
the same multiset as the input (compared with torch.sort of the input), and
for payload runs the gather identity keys_out[i] == keys_in[vals_out[i]]
with vals_out ascending inside every run of equal keys.  The batched
workload at its full 65,536 segments is additionally compared with the
oracle segment by segment on a sample of segments.
"""
import functools
import sys
import time

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
H_RTOL = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def as_ordered_int64(t):
    """Device keys as int64 values whose signed order is the keys' sort order."""
    if t.dtype == torch.int32:
        return t.to(torch.int64)
    if t.dtype == torch.int64:
        return t
    if t.dtype == torch.uint32:
        return t.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    if t.dtype == torch.uint64:
        return t.view(torch.int64) ^ (-(2 ** 63))
    if t.dtype == torch.float32:  # the library's bit map, written out for the check
        b = t.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        return torch.where(b >= 2 ** 31, (~b) & 0xFFFFFFFF, b | 2 ** 31)
    b = t.view(torch.int64)
    return torch.where(b < 0, ~b, b ^ (-(2 ** 63))) ^ (-(2 ** 63))


def check_sorted_permutation(kin, kout, vout=None, chunk=1 << 27):
    n = kin.numel()
    a = as_ordered_int64(kout)
    assert bool((a[1:] >= a[:-1]).all().item()), "output not ascending"
    ref = torch.sort(as_ordered_int64(kin)).values
    assert torch.equal(ref, a), "output is not a permutation of the input"
    del ref
    if vout is not None:
        v = vout.view(torch.int32).to(torch.int64)
        ain = as_ordered_int64(kin)
        for s0 in range(0, n, chunk):
            s1 = min(n, s0 + chunk)
            assert torch.equal(ain[v[s0:s1]], a[s0:s1]), "payload does not point at its key"
        same = a[1:] == a[:-1]
        assert bool((v[1:][same] > v[:-1][same]).all().item()), "equal keys not in input order"


def check_features_vs_oracle(f, keys_host):
    st, rf, _ = O.features(keys_host)
    assert st == O.OK
    assert (f.n, f.min_key, f.max_key, f.span, f.shift, f.nbins, f.exact) == \
        (rf.n, rf.min_key, rf.max_key, rf.span, rf.shift, rf.nbins, rf.exact)
    assert abs(f.entropy_bits - rf.entropy_bits) <= H_RTOL * max(rf.entropy_bits, 1e-300)
    return rf


@pytest.fixture(scope="module")
def selector():
    ctx = ahs.default_context(0)
    ctx.set_model(ahs.default_model())
    yield ctx, ahs.ahs_config_init(0, use_model=1)
    ctx.set_model(None)


@pytest.mark.parametrize("case", gen.SWEEP_CASES)
def test_strategy_sweep_full_size(case, selector):
    ctx, cfg = selector
    n = 1 << 28
    t = time.time()
    keys = gen.strategy_sweep(case, n=n)
    say(f"full-size sweep {case}: 2^28 keys generated in {time.time() - t:.1f}s")
    k = torch.from_numpy(keys).to(DEV)
    out, _, chosen, f = ahs.ahs_sort(k, strategy=ahs.AUTO, cfg=cfg, ctx=ctx, want_features=True)
    torch.cuda.synchronize()
    rf = check_features_vs_oracle(f, keys)
    st, rchosen = O.select(rf, O.config(0, use_model=1), O.Model(ahs.SELECTOR_MODEL))
    assert st == O.OK and chosen == rchosen, (chosen, rchosen)
    check_sorted_permutation(k, out)
    say(f"full-size sweep {case}: {ahs.STRATEGY_NAMES[chosen]} ok")


@pytest.mark.parametrize("case", gen.WIDE_CASES)
def test_wide_keys_full_size_with_payload(case, selector):
    ctx, cfg = selector
    n = 1 << 27
    keys = gen.wide_keys(case, n=n)
    say(f"full-size wide {case}: 2^27 keys")
    k = torch.from_numpy(keys).to(DEV)
    v = torch.arange(n, dtype=torch.int32, device=DEV).view(torch.uint32)
    out, vout, chosen, f = ahs.ahs_sort(k, v, strategy=ahs.AUTO, cfg=cfg, ctx=ctx, want_features=True)
    torch.cuda.synchronize()
    rf = check_features_vs_oracle(f, keys)
    st, rchosen = O.select(rf, O.config(0, use_model=1), O.Model(ahs.SELECTOR_MODEL))
    assert st == O.OK and chosen == rchosen, (chosen, rchosen)
    check_sorted_permutation(k, out, vout)
    say(f"full-size wide {case}: {ahs.STRATEGY_NAMES[chosen]} ok")


@pytest.mark.parametrize("case", ["i32_uniform", "i64_uniform", "gauss_k1e6", "taxi_like", "kmer_like"])
def test_paper_families_full_size_with_payload(case, selector):
    """The paper's families at the sizes the benchmark's paper sweep runs
    (2^24 keys, 10^7 for the taxi stand-in, 10^8 u64 for the k-mer one),
    signed keys included, through AUTO with the selector and a payload."""
    ctx, cfg = selector
    keys = gen.paper_sweep(case)
    n = keys.size
    say(f"full-size paper family {case}: {n} keys {keys.dtype}")
    k = torch.from_numpy(keys).to(DEV)
    v = torch.arange(n, dtype=torch.int32, device=DEV).view(torch.uint32)
    out, vout, chosen, f = ahs.ahs_sort(k, v, strategy=ahs.AUTO, cfg=cfg, ctx=ctx, want_features=True)
    torch.cuda.synchronize()
    rf = check_features_vs_oracle(f, keys)
    st, rchosen = O.select(rf, O.config(0, use_model=1), O.Model(ahs.SELECTOR_MODEL))
    assert st == O.OK and chosen == rchosen, (chosen, rchosen)
    check_sorted_permutation(k, out, vout)
    say(f"full-size paper family {case}: {ahs.STRATEGY_NAMES[chosen]} ok")


def test_batched_full_size_graph():
    """The 65,536-segment workload (about 6.2e9 keys) through the autotuned,
    graph-captured batched sort, as bench.py times it."""
    t = time.time()
    keys, offs, kinds = gen.segments(nseg=65536, seed=8)
    say(f"full-size batch: {keys.size} keys generated in {time.time() - t:.1f}s")
    k = torch.from_numpy(keys).to(DEV)
    o = torch.from_numpy(offs.view(np.int64)).to(DEV)
    sizes = np.diff(offs.astype(np.int64))
    ahs.ahs_segmented_autotune(ahs.U32, False)
    g = ahs.SegmentedGraph(k, o, max_seg_hint=int(sizes.max()), want_features=True)
    g.launch()
    torch.cuda.synchronize()
    assert int(g.status.item()) == 0
    say("full-size batch: sorted; checking every segment's order")
    # every segment ascending: the only descents allowed are at segment starts
    a = g.out.view(torch.int32)
    starts = torch.zeros(k.numel(), dtype=torch.bool, device=DEV)
    first = o[:-1]
    starts[first[first < k.numel()]] = True
    chunk = 1 << 28
    for s0 in range(0, k.numel() - 1, chunk):
        s1 = min(k.numel() - 1, s0 + chunk)
        x = a[s0:s1 + 1].to(torch.int64) & 0xFFFFFFFF
        desc = x[1:] < x[:-1]
        assert not bool((desc & ~starts[s0 + 1:s1 + 1]).any().item()), f"descent inside a segment near {s0}"
    del starts
    # sampled segments against the oracle, including the largest and smallest
    rng = np.random.default_rng(7)
    pick = set(rng.choice(len(sizes), 48, replace=False).tolist())
    pick |= {int(np.argmax(sizes)), int(np.argmin(sizes))}
    feats = ahs.feature_records(g.feats)
    chosen = g.chosen.cpu().numpy()
    gk = None
    for s in sorted(pick):
        lo, hi = int(offs[s]), int(offs[s + 1])
        st, rk, _, rch, rf = O.sort(keys[lo:hi], None, O.AUTO, O.config(0))
        assert st == O.OK
        gk = a[lo:hi].cpu().numpy().view(np.uint32)
        assert np.array_equal(gk, rk), f"segment {s} (size {hi - lo}) differs"
        assert chosen[s] == rch or abs(rf.entropy_bits - 0.7 * np.log2(max(rf.nbins, 2))) <= 1e-6 * rf.entropy_bits
        f = feats[s]
        assert (f.n, f.min_key, f.max_key, f.span, f.nbins) == (rf.n, rf.min_key, rf.max_key, rf.span, rf.nbins)
    say(f"full-size batch: {len(pick)} sampled segments match the oracle")
    # the blocking form on the same batch: its host-driven levels finish more
    # buckets in one level than one workgroup per bucket can address in a
    # single dispatch (regression: the launch wrapped and left buckets unsorted)
    ob, _, cb, fb = ahs.ahs_sort_segmented(k, o, want_features=True)
    torch.cuda.synchronize()
    assert torch.equal(ob.view(torch.int32), a), "blocking and graph outputs differ"
    assert torch.equal(cb, g.chosen), "blocking and graph decisions differ"
    say("full-size batch: blocking form identical to the graph")


@pytest.mark.parametrize("case", ["uniform32", "sorted32", "reverse32", "swapped32"])
def test_general_path_full_size_forced_quick(case):
    """The general-path arrays at 2^28 under forced QUICK with payload =
    index: on uniform keys the sample sort takes three levels, the last one
    reading the output buffer; the keys-only run must give the same keys."""
    n = 1 << 28
    keys = gen.strategy_sweep(case, n=n)
    say(f"full-size forced quick {case}: 2^28 keys")
    k = torch.from_numpy(keys).to(DEV)
    del keys
    v = torch.arange(n, dtype=torch.int32, device=DEV).view(torch.uint32)
    out, vout, chosen, _ = ahs.ahs_sort(k, v, strategy=ahs.QUICK)
    torch.cuda.synchronize()
    assert chosen == ahs.QUICK
    check_sorted_permutation(k, out, vout)
    out2, _, _, _ = ahs.ahs_sort(k, strategy=ahs.QUICK)
    torch.cuda.synchronize()
    assert torch.equal(out.view(torch.int32), out2.view(torch.int32)), "keys-only run differs"
    say(f"full-size forced quick {case}: ok")


@functools.lru_cache(maxsize=1)
def _wide_host(case):
    return gen.wide_keys(case, n=1 << 27)


@pytest.mark.parametrize("strategy,payload", [("auto", False), ("radix", False), ("radix", True),
                                              ("quick", False), ("quick", True)])
@pytest.mark.parametrize("case", gen.WIDE_CASES)
def test_wide_keys_full_size_strategies(case, strategy, payload, selector):
    """Wide and floating keys at 2^27 under AUTO (keys only; the payload run
    is above) and forced RADIX and QUICK, keys only and with payload."""
    ctx, cfg = selector
    keys = _wide_host(case)
    n = keys.size
    say(f"full-size wide {case}: {strategy} payload={payload}")
    k = torch.from_numpy(keys).to(DEV)
    v = torch.arange(n, dtype=torch.int32, device=DEV).view(torch.uint32) if payload else None
    out, vout, chosen, f = ahs.ahs_sort(k, v, strategy=strategy, cfg=cfg, ctx=ctx, want_features=strategy == "auto")
    torch.cuda.synchronize()
    if strategy == "auto":
        rf = check_features_vs_oracle(f, keys)
        st, rchosen = O.select(rf, O.config(0, use_model=1), O.Model(ahs.SELECTOR_MODEL))
        assert st == O.OK and chosen == rchosen, (chosen, rchosen)
    else:
        assert chosen == ahs.STRATEGY_CODES[strategy]
    check_sorted_permutation(k, out, vout)
    say(f"full-size wide {case} {strategy}: ok")


@pytest.mark.parametrize("strategy", ["radix", "quick"])
def test_single_array_2p30_u32(strategy):
    """One array of 2^30 uniform 32-bit keys with payload = index: the
    look-back status words of the radix passes and of the sample-sort
    scatter switch to 64 bits at this size."""
    n = 1 << 30
    keys = gen.u32(12, 0, n)
    say(f"single array 2^30 u32: {strategy}")
    k = torch.from_numpy(keys).to(DEV)
    del keys
    v = torch.arange(n, dtype=torch.int32, device=DEV).view(torch.uint32)
    out, vout, chosen, _ = ahs.ahs_sort(k, v, strategy=strategy)
    torch.cuda.synchronize()
    assert chosen == ahs.STRATEGY_CODES[strategy]
    check_sorted_permutation(k, out, vout)
    say(f"single array 2^30 u32 {strategy}: ok")
