"""GPU parity of the batched segmented sort against the CPU oracle.

Each segment is checked as an independent array: its keys and payload
bit-exact against the oracle's sort of that segment alone, its decision
equal to the oracle's (up to the documented entropy-threshold tie), and its
feature vector to the same bar as the single-array path.  A segment holding
NaN keys has no oracle decision; its expected output is the stable order of
the oracle's bit map and its decision code is 0xFD.
"""
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
H_RTOL = 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def bits(a):
    return a.view(np.uint32 if a.itemsize == 4 else np.uint64)


def offsets_of(sizes):
    offs = np.zeros(len(sizes) + 1, np.uint64)
    np.cumsum(np.asarray(sizes, np.uint64), out=offs[1:])
    return offs


def check_features(f, rf):
    assert (f.n, f.min_key, f.max_key, f.span, f.nan_count) == (rf.n, rf.min_key, rf.max_key, rf.span, rf.nan_count)
    assert (f.shift, f.nbins, f.exact) == (rf.shift, rf.nbins, rf.exact)
    if rf.entropy_bits == 0.0:
        assert f.entropy_bits == 0.0
    else:
        assert abs(f.entropy_bits - rf.entropy_bits) <= H_RTOL * rf.entropy_bits, (f.entropy_bits, rf.entropy_bits)
        assert abs(f.entropy_ratio - rf.entropy_ratio) <= 2 * H_RTOL * rf.entropy_ratio


def near_threshold(rf):
    if rf.nbins <= 1:
        return False
    thr = 0.7 * math.log2(rf.nbins)
    return abs(rf.entropy_bits - thr) <= H_RTOL * thr


def run_segments(keys, offs, vals=None, strategy=ahs.AUTO, preset=0, in_place=False, mode="blocking", hint=0):
    """Sorts all segments in one call (blocking, enqueue-only or a captured
    graph) and checks every segment against the oracle.  Returns the host
    array of decisions."""
    nseg = len(offs) - 1
    say(f"segmented mode={mode} nseg={nseg} n={keys.size} dtype={keys.dtype} payload={vals is not None} "
        f"strategy={strategy} inplace={in_place} max_seg={int(np.max(np.diff(offs.astype(np.int64)), initial=0))}")
    k = to_dev(keys)
    v = to_dev(vals) if vals is not None else None
    o = to_dev(offs)
    cfg = ahs.ahs_config_init(preset)
    outs = dict(out=k, out_values=v) if in_place else {}
    if mode == "blocking":
        ko, vo, chosen, feats = ahs.ahs_sort_segmented(k, o, v, strategy, cfg, want_features=True, **outs)
    elif mode == "async":
        ko, vo, chosen, feats, status = ahs.ahs_sort_segmented_async(k, o, v, strategy, cfg, max_seg_hint=hint,
                                                                     want_features=True, **outs)
        assert int(status.item()) == 0
    else:
        g = ahs.SegmentedGraph(k, o, v, strategy, cfg, max_seg_hint=hint, want_features=True, **outs)
        g.launch()
        torch.cuda.synchronize()
        assert int(g.status.item()) == 0
        ko, vo, chosen, feats = g.out, g.out_values, g.chosen, g.feats
    torch.cuda.synchronize()
    ko = ko.cpu().numpy()
    vo = vo.cpu().numpy() if vals is not None else None
    chosen = chosen.cpu().numpy()
    fs = ahs.feature_records(feats)
    ocfg = O.config(preset)
    for s in range(nseg):
        a, b = int(offs[s]), int(offs[s + 1])
        seg = keys[a:b]
        sv = vals[a:b] if vals is not None else None
        st, rk, rv, rchosen, rf = O.sort(seg, sv, O.AUTO, ocfg)
        if st == O.E_NAN:
            _, mapped, nans = O.map_keys(seg)
            order = np.argsort(mapped, kind="stable")
            rk = seg[order]
            rv = sv[order] if sv is not None else None
            assert chosen[s] == ahs.SEG_NAN, (s, chosen[s])
            assert fs[s].n == b - a and fs[s].nan_count == nans
        else:
            assert st == O.OK, (s, st)
            check_features(fs[s], rf)
            if strategy != ahs.AUTO:
                assert chosen[s] == strategy, (s, chosen[s])
            elif chosen[s] != rchosen:
                assert near_threshold(rf), (s, chosen[s], rchosen)
        assert np.array_equal(bits(ko[a:b]), bits(rk)), f"segment {s} keys differ (size {b - a})"
        if vals is not None:
            assert np.array_equal(vo[a:b], rv), f"segment {s} payload differs"
    return chosen


def mixed_sizes(nseg, seed, cap):
    sizes = gen.segment_sizes(nseg, seed=seed, lo_exp=0, span_exp=math.log2(cap), cap=cap, lo=0)
    # boundaries of the method (n_small) and of the LDS path, and empty segments
    special = [0, 0, 1, 20, 21, 8191, 8192, 8193, 0]
    sizes[: len(special)] = special
    return sizes


def test_segmented_u32_mixed_auto():
    keys, offs, _ = gen.segments(nseg=400, seed=21, sizes=mixed_sizes(400, 21, 1 << 15))
    chosen = run_segments(keys, offs)
    # every decision occurs in this mix
    assert {ahs.INSERTION, ahs.COUNTING, ahs.QUICK} <= set(chosen.tolist())


def test_segmented_u32_payload():
    keys, offs, _ = gen.segments(nseg=150, seed=22, sizes=mixed_sizes(150, 22, 1 << 14))
    run_segments(keys, offs, np.arange(keys.size, dtype=np.uint32))


def test_segmented_large_multilevel():
    """Several segments above the LDS size, one needing more than one level,
    sorted by the same sample-sort levels together with small ones."""
    sizes = [(1 << 21) + 3, 9000, 0, 7, 300_000, 8193, 65_536, 5000]
    keys, offs, _ = gen.segments(nseg=len(sizes), seed=23, sizes=np.array(sizes))
    run_segments(keys, offs, np.arange(keys.size, dtype=np.uint32))
    run_segments(keys, offs)


def test_segmented_radix_decision():
    """Large low-entropy segments (few distinct 32-bit values) decide RADIX."""
    sizes = [200_000, 50_000, 20_000]
    parts = [gen.zipf_keys(31 + i, s, 64, 1.1, 32) for i, s in enumerate(sizes)]
    keys = np.concatenate(parts).astype(np.uint32)
    chosen = run_segments(keys, offsets_of(sizes))
    assert (chosen == ahs.RADIX).all(), chosen


def _dispatch_parts():
    """Large segments of every route: counting ranges (one and two digit
    passes, a constant segment whose one pass is a copy), low-entropy wide
    ranges (radix; one of them above 2^20 keys, so its entropy comes from two
    histogram units, with 16-bit bin wraps from eight values over two million
    keys), high-entropy wide ranges (sample sort; one over two units), and a
    span below k_radix (sample sort, no histogram)."""
    return [
        gen.u32(61, 0, 300_000, mask=255),
        gen.u32(61, 1, 20_000, mask=4095),
        np.full(50_000, 7, np.uint32),
        gen.zipf_keys(62, 200_000, 64, 1.1, 32),
        gen.zipf_keys(63, (1 << 21) + 5, 8, 1.1, 32),
        gen.u32(64, 0, (1 << 20) + 1),
        gen.u32(65, 0, 30_000, mask=(1 << 20) - 1),
        gen.u32(66, 0, 9000, mask=(1 << 19) - 1),
        gen.u32(67, 0, 5000),
    ]


@pytest.mark.parametrize("mode,in_place", [("blocking", False), ("async", True), ("graph", False)])
def test_segmented_large_dispatch(mode, in_place):
    parts = _dispatch_parts()
    sizes = [p.size for p in parts]
    keys = np.concatenate(parts)
    chosen = run_segments(keys, offsets_of(sizes), np.arange(keys.size, dtype=np.uint32), mode=mode,
                          in_place=in_place, hint=max(sizes))
    assert list(chosen[:5]) == [ahs.COUNTING, ahs.COUNTING, ahs.COUNTING, ahs.RADIX, ahs.RADIX]
    assert list(chosen[5:8]) == [ahs.QUICK, ahs.QUICK, ahs.QUICK]


@pytest.mark.parametrize("strategy", [ahs.COUNTING, ahs.RADIX, ahs.QUICK])
def test_segmented_forced(strategy):
    keys, offs, _ = gen.segments(nseg=60, seed=24, sizes=mixed_sizes(60, 24, 1 << 15))
    run_segments(keys, offs, np.arange(keys.size, dtype=np.uint32), strategy=strategy)


def test_segmented_u64_payload():
    sizes = mixed_sizes(80, 25, 1 << 15)
    sizes[-1] = 40_000
    n = int(np.sum(sizes))
    keys = gen.wide_keys("u64zipf4096", n=n)
    keys[: n // 2] = gen.wide_keys("u64uniform", n=n // 2)
    run_segments(keys, offsets_of(sizes), np.arange(n, dtype=np.uint32))


@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_segmented_signed_payload(dt):
    """Signed keys in every segment class: narrow spans around zero
    (counting), full-range uniform (quicksort), few values over the full
    range (radix), with both ends of the type planted."""
    sizes = mixed_sizes(90, 29, 1 << 15)
    sizes[-3:] = [40_000, 30_000, 20_000]
    n = int(np.sum(sizes))
    info = np.iinfo(dt)
    r = np.random.default_rng(29)
    keys = r.integers(int(info.min), int(info.max), n, dtype=np.int64, endpoint=True).astype(dt)
    offs = offsets_of(sizes)
    for s in range(0, len(sizes), 3):
        a, b = int(offs[s]), int(offs[s + 1])
        keys[a:b] = r.integers(-1500, 1500, b - a).astype(dt)
    a = int(offs[-2])
    bits_ = 32 if dt == np.int32 else 64
    z = gen.zipf_keys(30, n - a, 64, 1.1, bits_).astype(np.uint32 if dt == np.int32 else np.uint64).view(dt)
    keys[a:] = z
    keys[::97] = info.min
    keys[::89] = info.max
    chosen = run_segments(keys, offs, np.arange(n, dtype=np.uint32))
    assert {ahs.INSERTION, ahs.COUNTING, ahs.QUICK} <= set(chosen.tolist())
    run_segments(keys, offs)


@pytest.mark.parametrize("case", ["f32normal", "f64normal"])
def test_segmented_float_with_nan(case):
    sizes = mixed_sizes(60, 26, 1 << 14)
    sizes[-2:] = [30_000, 12_000]
    sizes[10] = 500
    n = int(np.sum(sizes))
    keys = gen.wide_keys(case, n=n)
    offs = offsets_of(sizes)
    # a small and a large segment with NaNs of both signs
    for s in (10, len(sizes) - 1):
        a, b = int(offs[s]), int(offs[s + 1])
        keys[a + 3] = np.nan
        keys[b - 2] = -np.nan
        keys[a + 5] = np.inf
    chosen = run_segments(keys, offs, np.arange(n, dtype=np.uint32))
    assert chosen[10] == ahs.SEG_NAN and chosen[-1] == ahs.SEG_NAN
    assert (chosen[:10] != ahs.SEG_NAN).all()


@pytest.mark.parametrize("mode,in_place", [("blocking", False), ("blocking", True), ("async", False),
                                           ("async", True), ("graph", False)])
@pytest.mark.parametrize("dt", [np.uint32, np.int32])
def test_segmented_quick_large_equal_key_buckets(dt, mode, in_place):
    """Segments the FSM sends to the sample sort (100 distinct values over a
    span below the radix threshold) holding up to 2^20 keys, so their
    buckets of equal keys exceed 4,096 keys and are scattered straight to
    the output; signed keys, payload, every dispatch mode, and in place."""
    r = np.random.default_rng(61)
    sizes = [1 << 20, 300_001, 150_000, 9000, 4097, 100, 1, 65_537]
    offs = offsets_of(sizes)
    n = int(offs[-1])
    lo = -250_000 if dt == np.int32 else 0
    vals = r.integers(lo, lo + 500_000, 100).astype(dt)
    keys = vals[r.integers(0, vals.size, n)]
    chosen = run_segments(keys, offs, np.arange(n, dtype=np.uint32), mode=mode, in_place=in_place,
                          hint=1 << 20)
    assert chosen[0] == ahs.QUICK


def test_segmented_in_place():
    keys, offs, _ = gen.segments(nseg=50, seed=27, sizes=mixed_sizes(50, 27, 1 << 15))
    run_segments(keys, offs, np.arange(keys.size, dtype=np.uint32), in_place=True)


def test_segmented_paper_preset():
    keys, offs, _ = gen.segments(nseg=80, seed=28, sizes=mixed_sizes(80, 28, 1 << 14))
    run_segments(keys, offs, preset=ahs.PRESET_PAPER_TABLE2)


def test_segmented_repeat_and_shrink():
    """Two calls on one context and workspace, the second smaller: the
    workspace's counters and tables carry nothing from the first."""
    k1, o1, _ = gen.segments(nseg=40, seed=29, sizes=mixed_sizes(40, 29, 1 << 16))
    run_segments(k1, o1)
    k2, o2, _ = gen.segments(nseg=7, seed=30, sizes=np.array([9000, 3, 0, 12_000, 100, 8192, 8193]))
    run_segments(k2, o2)


def test_segmented_matches_single_array_calls():
    keys, offs, _ = gen.segments(nseg=12, seed=31, sizes=np.array([5, 20, 21, 3000, 8192, 8193, 20_000, 70_000,
                                                                   1, 0, 4096, 100_000]))
    k = to_dev(keys)
    ko, _, chosen, _ = ahs.ahs_sort_segmented(k, to_dev(offs))
    chosen = chosen.cpu().tolist()
    for s in range(len(offs) - 1):
        a, b = int(offs[s]), int(offs[s + 1])
        so, _, ch, _ = ahs.ahs_sort(k[a:b].contiguous())
        assert torch.equal(so, ko[a:b])
        assert ch == chosen[s], (s, ch, chosen[s])


def test_segmented_errors():
    k = to_dev(np.arange(100, dtype=np.uint32))
    bad = [np.array([0, 60, 50, 100], np.uint64),   # decreasing
           np.array([0, 50, 99], np.uint64),        # does not end at n
           np.array([0, 50, 101], np.uint64)]       # past the end
    for offs in bad:
        with pytest.raises(ahs.AhsError) as e:
            ahs.ahs_sort_segmented(k, to_dev(offs))
        assert e.value.status == ahs.E_INVALID_ARG
    cfg = ahs.ahs_config_init()
    cfg.use_model = 1
    with pytest.raises(ahs.AhsError) as e:
        ahs.ahs_sort_segmented(k, to_dev(np.array([0, 100], np.uint64)), cfg=cfg)
    assert e.value.status == ahs.E_UNSUPPORTED
    # zero segments is a no-op
    out, _, chosen, _ = ahs.ahs_sort_segmented(k[:0], to_dev(np.array([0], np.uint64)))
    assert out.numel() == 0 and chosen.numel() == 0


# ------------------------------------------------------------------ enqueue-only form, graphs, autotuner
@pytest.mark.parametrize("hint", [0, 1 << 15])
def test_segmented_async_mixed(hint):
    keys, offs, _ = gen.segments(nseg=300, seed=41, sizes=mixed_sizes(300, 41, 1 << 15))
    run_segments(keys, offs, np.arange(keys.size, dtype=np.uint32), mode="async", hint=hint)


def test_segmented_async_multilevel_and_wide():
    sizes = [(1 << 21) + 3, 9000, 0, 7, 300_000, 8193, 65_536, 5000]
    keys, offs, _ = gen.segments(nseg=len(sizes), seed=42, sizes=np.array(sizes))
    run_segments(keys, offs, mode="async")
    n = int(offs[-1])
    wide = gen.wide_keys("u64zipf4096", n=n)
    run_segments(wide, offs, np.arange(n, dtype=np.uint32), mode="async", hint=(1 << 21) + 3)
    f = gen.wide_keys("f32normal", n=n)
    f[5] = np.nan
    run_segments(f, offs, np.arange(n, dtype=np.uint32), mode="async", in_place=True)


def test_segmented_async_invalid_offsets_write_nothing():
    k = to_dev(np.arange(100, dtype=np.uint32)[::-1].copy())
    out = torch.full((100,), 7, dtype=torch.int32, device=DEV).view(torch.uint32)
    o = to_dev(np.array([0, 60, 50, 100], np.uint64))
    _, _, _, _, status = ahs.ahs_sort_segmented_async(k, o, out=out)
    assert int(status.item()) & ahs.SEG_ERR_OFFSETS
    assert (out.view(torch.int32) == 7).all()


def test_segmented_async_hint_too_small_is_reported():
    """A segment above the size hint with no level launched for it is
    reported in the status word (its output is not sorted)."""
    sizes = [100, 20_000, 50]
    keys, offs, _ = gen.segments(nseg=3, seed=43, sizes=np.array(sizes))
    k = to_dev(keys)
    ko, _, _, _, status = ahs.ahs_sort_segmented_async(k, to_dev(offs), max_seg_hint=100)
    assert int(status.item()) == ahs.SEG_ERR_LEVELS | ahs.SEG_ERR_HINT
    # the small segments are still sorted
    ko = ko.cpu().numpy()
    assert np.array_equal(ko[:100], np.sort(keys[:100]))


def test_segmented_graph_replays():
    """One capture, several replays with the program's own eager work and
    synchronisations in between; every replay is checked against the eager
    (blocking) result for the inputs it saw."""
    sizes = mixed_sizes(120, 44, 1 << 15)
    sizes[-1] = 70_000
    offs = offsets_of(sizes)
    n = int(offs[-1])
    k = torch.empty(n, dtype=torch.uint32, device=DEV)
    o = to_dev(offs)
    g = ahs.SegmentedGraph(k, o, max_seg_hint=70_000, want_features=True)
    for rep in range(3):
        keys, _, _ = gen.segments(nseg=len(sizes), seed=50 + rep, sizes=sizes)
        k.copy_(to_dev(keys))
        torch.cuda.synchronize()
        say(f"graph replay {rep}")
        g.launch()
        torch.cuda.synchronize()
        assert int(g.status.item()) == 0
        eo, _, ech, ef = ahs.ahs_sort_segmented(k, o, want_features=True)
        torch.cuda.synchronize()
        assert torch.equal(g.out, eo), rep
        assert torch.equal(g.chosen, ech), rep
        assert torch.equal(g.feats, ef), rep
        # and against the oracle on a few segments
        gk = g.out.cpu().numpy()
        for s in (0, 9, len(sizes) - 1):
            a, b = int(offs[s]), int(offs[s + 1])
            assert np.array_equal(gk[a:b], np.sort(keys[a:b]))
        g.out.view(torch.int32).fill_(0)  # eager work between replays


def test_segmented_graph_matches_oracle():
    keys, offs, _ = gen.segments(nseg=200, seed=45, sizes=mixed_sizes(200, 45, 1 << 15))
    run_segments(keys, offs, np.arange(keys.size, dtype=np.uint32), mode="graph")


@pytest.mark.parametrize("dt", [ahs.U32, ahs.F64])
@pytest.mark.parametrize("pay", [False, True])
def test_autotune_choices_valid(dt, pay):
    caps, ms = ahs.ahs_segmented_autotune(dt, pay)
    say(f"autotune dtype={dt} payload={pay}: {caps} {ms}")
    for c, cap in enumerate(caps):
        assert cap in (1024, 2048, 4096, 8192) and cap >= (1024 << c)
        assert ms[c] > 0
    assert ahs.ahs_segmented_get_variants(dt, pay) == caps


RADIX_TILES = {(ahs.U32, False): (8192, 12288), (ahs.U32, True): (6144, 9216), (ahs.U64, False): (6144, 9216),
               (ahs.U64, True): (4096, 6144)}


@pytest.mark.parametrize("dt,pay", list(RADIX_TILES))
def test_radix_tile_choices_give_identical_results(dt, pay):
    """Both tile shapes of the segmented radix passes give the same keys,
    payloads and decisions (oracle-checked), and the autotuner keeps one of
    them."""
    sizes = [9000, 70_000, 300_000, 20, 12_345, 150_001]
    n = sum(sizes)
    if dt == ahs.U32:
        keys = np.concatenate([gen.zipf_keys(70 + i, s, 64, 1.1, 32) for i, s in enumerate(sizes)])
    else:
        keys = np.concatenate([gen.zipf_keys(70 + i, s, 4096, 1.0, 64) for i, s in enumerate(sizes)])
    vals = np.arange(n, dtype=np.uint32) if pay else None
    saved = ahs.ahs_segmented_get_radix_tile(dt, pay)
    outs = []
    try:
        for tile in RADIX_TILES[(dt, pay)]:
            ahs.ahs_segmented_set_radix_tile(dt, tile, pay)
            assert ahs.ahs_segmented_get_radix_tile(dt, pay) == tile
            chosen = run_segments(keys, offsets_of(sizes), vals, mode="async", hint=max(sizes))
            assert chosen[1] == ahs.RADIX and chosen[2] == ahs.RADIX
            outs.append(chosen)
    finally:
        ahs.ahs_segmented_set_radix_tile(dt, saved, pay)
    assert np.array_equal(outs[0], outs[1])
    ahs.ahs_segmented_autotune(dt, pay)
    assert ahs.ahs_segmented_get_radix_tile(dt, pay) in RADIX_TILES[(dt, pay)]
    with pytest.raises(ahs.AhsError):
        ahs.ahs_segmented_set_radix_tile(dt, 1000, pay)


def test_every_variant_gives_identical_results():
    keys, offs, _ = gen.segments(nseg=200, seed=46, sizes=mixed_sizes(200, 46, 1 << 13))
    vals = np.arange(keys.size, dtype=np.uint32)
    k, o, v = to_dev(keys), to_dev(offs), to_dev(vals)
    saved = ahs.ahs_segmented_get_variants(ahs.U32, True)
    results = []
    try:
        for caps in ([1024, 2048, 4096, 8192], [8192] * 4, [2048, 2048, 8192, 8192], [4096, 4096, 4096, 8192]):
            ahs.ahs_segmented_set_variants(ahs.U32, caps, True)
            ko, vo, ch, f = ahs.ahs_sort_segmented(k, o, v, want_features=True)
            torch.cuda.synchronize()
            results.append((ko.clone(), vo.clone(), ch.clone(), f.clone()))
    finally:
        ahs.ahs_segmented_set_variants(ahs.U32, saved, True)
    ref = ahs.feature_records(results[0][3])
    for r in results[1:]:
        for x, y in zip(results[0][:3], r[:3]):
            assert torch.equal(x, y)
        # features: integer fields equal; entropy sums differ only in the
        # order the workgroup adds its terms
        for fa, fb in zip(ref, ahs.feature_records(r[3])):
            assert (fa.n, fa.min_key, fa.max_key, fa.span, fa.nan_count, fa.shift, fa.nbins, fa.exact) == \
                (fb.n, fb.min_key, fb.max_key, fb.span, fb.nan_count, fb.shift, fb.nbins, fb.exact)
            assert abs(fa.entropy_bits - fb.entropy_bits) <= 1e-12 * max(1.0, fa.entropy_bits)
    with pytest.raises(ahs.AhsError):
        ahs.ahs_segmented_set_variants(ahs.U32, [1024, 1024, 4096, 8192], True)
