"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Bar: keys, payloads, min/max/span/shift/nbins, histograms and the chosen
strategy bit-exact; entropy within 1e-6 relative (0 exactly when the
oracle's is 0); strategy disagreement accepted only when the oracle's
entropy lies within 1e-6 relative of the radix threshold 0.7*log2(nbins).
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


def check_features(f, rf, hist=None, rhist=None):
    assert (f.n, f.min_key, f.max_key, f.span, f.nan_count) == (rf.n, rf.min_key, rf.max_key, rf.span, rf.nan_count)
    assert (f.shift, f.nbins, f.exact) == (rf.shift, rf.nbins, rf.exact)
    if rf.entropy_bits == 0.0:
        assert f.entropy_bits == 0.0
    else:
        assert abs(f.entropy_bits - rf.entropy_bits) <= H_RTOL * rf.entropy_bits, (f.entropy_bits, rf.entropy_bits)
    if hist is not None:
        assert np.array_equal(hist[: rf.nbins], rhist)


def near_threshold(rf, cfg=None):
    if rf.nbins <= 1:
        return False
    thr = 0.7 * math.log2(rf.nbins)
    return abs(rf.entropy_bits - thr) <= H_RTOL * thr


def run_pair(keys, vals=None, strategy=ahs.AUTO, cfg_preset=0, in_place=False):
    """Sorts on the GPU and with the oracle; asserts the bar."""
    say(f"case n={keys.size} dtype={keys.dtype} payload={vals is not None} strategy={strategy} inplace={in_place}")
    k = to_dev(keys)
    v = to_dev(vals) if vals is not None else None
    cfg = ahs.ahs_config_init(cfg_preset)
    if in_place:
        ko, vo, chosen, f = ahs.ahs_sort(k, v, strategy, cfg, out=k, out_values=v, want_features=True)
    else:
        ko, vo, chosen, f = ahs.ahs_sort(k, v, strategy, cfg, want_features=True)
    torch.cuda.synchronize()
    st, rk, rv, rchosen, rf = O.sort(keys, vals, strategy, O.config(cfg_preset))
    if st == O.E_DEPTH:
        # the oracle's median-of-three quicksort (forced, or chosen by AUTO)
        # refuses adversarial inputs (sawtooth); its four sorts are pinned to
        # agree, so radix gives the same unique stable result
        assert strategy in (ahs.QUICK, ahs.AUTO)
        rchosen = O.QUICK if strategy == ahs.QUICK else O.select(rf, O.config(cfg_preset))[1]
        assert rchosen == O.QUICK
        st, rk, rv, _, rf = O.sort(keys, vals, O.RADIX, O.config(cfg_preset))
    assert st == O.OK, st
    assert np.array_equal(bits(ko.cpu().numpy()), bits(rk)), "keys differ"
    if vals is not None:
        assert np.array_equal(vo.cpu().numpy(), rv), "payload differs"
    check_features(f, rf)
    if chosen != rchosen:
        assert near_threshold(rf), (chosen, rchosen, rf.as_dict())
    return chosen


# ------------------------------------------------------------------ features
def _packed_pair(runs):
    """Keys of the two bins sharing packed LDS word 0 (shift 16), each more
    than 65,535 times per workgroup, so both 16-bit halves wrap, also while
    the other half is full: in random order (dominant-bin adds of a wave)
    or in runs of random length (dominant-bin adds plus runs merged inside
    a lane), with sparse keys of other bins."""
    r = np.random.default_rng(23 + runs)
    n = 1 << 21
    if runs:
        lens = r.integers(1, 700, n // 100)
        keys = np.repeat(np.where(np.arange(lens.size) % 2 == 0, 3, 65539), lens)[:n]
        keys = np.concatenate([keys, np.full(n - keys.size, 3)])
    else:
        keys = np.where(r.random(n) < 0.5, 3, 65539)
    keys = keys.astype(np.uint32)
    other = r.integers(0, n, n // 500)
    keys[other] = r.integers(0, 2**32, other.size, dtype=np.uint64).astype(np.uint32)
    keys[0], keys[-1] = 0, 2**32 - 1
    return keys


FEATURE_CASES = [
    ("pr1", lambda: gen.pr1()),
    ("u32 uniform4096 1M", lambda: gen.strategy_sweep("uniform4096", n=1 << 20)),
    ("u32 zipf256 1M", lambda: gen.strategy_sweep("zipf256", n=1 << 20)),
    ("u32 uniform32 1M", lambda: gen.strategy_sweep("uniform32", n=1 << 20)),
    ("u64 uniform 300k", lambda: gen.wide_keys("u64uniform", n=300_001)),
    ("u64 zipf 300k", lambda: gen.wide_keys("u64zipf4096", n=300_001)),
    ("f32 normal 300k", lambda: gen.wide_keys("f32normal", n=300_001)),
    ("f64 normal 300k", lambda: gen.wide_keys("f64normal", n=300_001)),
    ("u32 constant", lambda: np.full(777, 9, np.uint32)),
    ("u32 span 8191", lambda: (np.arange(100_000) % 8192).astype(np.uint32)),
    ("u32 span 8192", lambda: (np.arange(100_000) % 8193).astype(np.uint32)),
    ("u32 span 65535", lambda: (np.arange(200_003) * 7 % 65536).astype(np.uint32)),
    ("u32 span 65536", lambda: (np.arange(200_003) * 7 % 65537).astype(np.uint32)),
    ("u32 one hot bin overflow", lambda: np.concatenate([np.zeros(300_000, np.uint32), np.full(300_000, 1, np.uint32),
                                                         np.array([2**32 - 1], np.uint32)])),
    ("u32 packed pair random", lambda: _packed_pair(False)),
    ("u32 packed pair runs", lambda: _packed_pair(True)),
    ("u32 swapped 4M", lambda: gen.strategy_sweep("swapped32", n=1 << 22)),
    ("u32 sorted 4M", lambda: gen.strategy_sweep("sorted32", n=1 << 22)),
    ("u64 two", lambda: np.array([0, 2**64 - 1], np.uint64)),
    ("f32 signed zeros", lambda: np.array([0.0, -0.0] * 50, np.float32)),
    ("u32 n=1", lambda: np.array([12345], np.uint32)),
]


@pytest.mark.parametrize("name,make", FEATURE_CASES, ids=[c[0] for c in FEATURE_CASES])
def test_features_parity(name, make):
    keys = make()
    say(f"features {name} n={keys.size}")
    hist = torch.zeros(65536, dtype=torch.int32, device=DEV)
    f = ahs.ahs_features(to_dev(keys), hist)
    torch.cuda.synchronize()
    st, rf, rhist = O.features(keys)
    assert st == O.OK
    check_features(f, rf, hist.cpu().numpy().view(np.uint32), rhist)


def test_features_bin_overflow_exact():
    """More than 65,535 keys of one bin inside one block: the packed 16-bit
    counters wrap and the corrections must restore the exact count."""
    n = 1 << 21
    keys = np.zeros(n, np.uint32)
    keys[::3] = 1
    keys[-1] = 2**32 - 1  # forces the 65,536-bin histogram (shift 16: keys 0, 1 share bin 0)
    keys[5] = 70000
    hist = torch.zeros(65536, dtype=torch.int32, device=DEV)
    f = ahs.ahs_features(to_dev(keys), hist)
    st, rf, rhist = O.features(keys)
    check_features(f, rf, hist.cpu().numpy().view(np.uint32), rhist)


def test_features_nan():
    keys = np.array([1.0, np.nan, 2.0], np.float32)
    with pytest.raises(ahs.AhsError) as e:
        ahs.ahs_features(to_dev(keys))
    assert e.value.status == ahs.E_NAN and e.value.features.nan_count == 1


def test_features_empty():
    f = ahs.ahs_features(torch.empty(0, dtype=torch.uint32, device=DEV))
    assert f.n == 0 and f.nbins == 0


# ------------------------------------------------------------------ sorts
def test_pr1_auto_radix_parity():
    """PR1 shape: 1,000,000 u32 uniform on [0, 1023]; AUTO picks counting."""
    keys = gen.pr1()
    assert run_pair(keys) == ahs.COUNTING
    vals = np.arange(keys.size, dtype=np.uint32)
    assert run_pair(keys, vals) == ahs.COUNTING
    assert run_pair(keys, vals, ahs.RADIX) == ahs.RADIX
    assert run_pair(keys, None, ahs.RADIX) == ahs.RADIX


@pytest.mark.parametrize("payload", [False, True])
def test_pr1_forced_quick_parity(payload):
    """PR1 with the strategy forced to QUICK: the sample sort on 1,024
    distinct values (every bucket an equality bucket after one level),
    keys and payload bit-exact to the oracle's quicksort."""
    keys = gen.pr1()
    vals = np.arange(keys.size, dtype=np.uint32) if payload else None
    assert run_pair(keys, vals, ahs.QUICK) == ahs.QUICK


SIZES = [1, 2, 19, 20, 21, 100, 4095, 4096, 4097, 8191, 8192, 8193, 3 * 8192 + 17, 65537, 300_001]


@pytest.mark.parametrize("n", SIZES)
def test_radix_sizes_u32(n):
    r = np.random.default_rng(n)
    keys = r.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    run_pair(keys, np.arange(n, dtype=np.uint32), ahs.RADIX)
    run_pair(keys, None, ahs.RADIX)


@pytest.mark.parametrize("n", [1, 21, 4095, 4097, 100_003])
@pytest.mark.parametrize("kind", ["u64", "f32", "f64"])
def test_radix_wide(n, kind):
    r = np.random.default_rng(n + 7)
    if kind == "u64":
        keys = r.integers(0, 2**64, n, dtype=np.uint64)
    elif kind == "f32":
        keys = r.normal(0, 1e3, n).astype(np.float32)
        keys[::97] = -0.0
        keys[::89] = 0.0
        keys[::1001] = np.inf
    else:
        keys = r.normal(0, 1.0, n)
        keys[::53] = -np.inf
        keys[::59] = -0.0
    vals = np.arange(n, dtype=np.uint32)
    run_pair(keys, vals, ahs.RADIX)
    run_pair(keys, None, ahs.RADIX)


@pytest.mark.parametrize("n", [21, 1000, 8193, 100_000, 1_000_003])
@pytest.mark.parametrize("k", [1, 2, 255, 256, 1000, 4096])
def test_counting(n, k):
    r = np.random.default_rng(n * 31 + k)
    keys = (r.integers(0, k, n) + 1_000_000).astype(np.uint32)
    run_pair(keys, None, ahs.COUNTING)
    run_pair(keys, np.arange(n, dtype=np.uint32), ahs.COUNTING)


@pytest.mark.parametrize("dt", [np.uint64, np.float32, np.float64])
def test_counting_wide(dt):
    r = np.random.default_rng(5)
    if dt == np.uint64:
        keys = r.integers(0, 3000, 50_001).astype(np.uint64) + np.uint64(2**63)
    elif dt == np.float32:
        keys = (r.integers(0, 3000, 50_001).astype(np.uint32) + np.uint32(0x3F800000)).view(np.float32)
    else:
        keys = (r.integers(0, 3000, 50_001).astype(np.uint64) + np.uint64(0xC000000000000000)).view(np.float64)
    run_pair(keys, None, ahs.COUNTING)
    run_pair(keys, np.arange(keys.size, dtype=np.uint32), ahs.COUNTING)


def test_auto_choices_match_oracle():
    cases = {
        "uniform4096": ahs.COUNTING,
        "zipf256": ahs.RADIX,
    }
    for case, want in cases.items():
        keys = gen.strategy_sweep(case, n=1 << 20)
        assert run_pair(keys) == want
        assert run_pair(keys, np.arange(keys.size, dtype=np.uint32)) == want
    for case, want in (("u64zipf4096", ahs.RADIX), ("f32normal", ahs.RADIX), ("f64normal", ahs.RADIX)):
        keys = gen.wide_keys(case, n=1 << 19)
        assert run_pair(keys, np.arange(keys.size, dtype=np.uint32)) == want


def test_radix_on_sorted_low_entropy():
    """Sorted keys of low entropy over a span above 2^20: AUTO plans radix
    digits during the feature pass (fused digit counts of sorted, wave-
    uniform digits) and picks radix; also nearly sorted."""
    r = np.random.default_rng(29)
    keys = (np.sort(r.zipf(1.3, 1 << 21) % 97).astype(np.uint64) * 40_009).astype(np.uint32)
    assert run_pair(keys) == ahs.RADIX
    assert run_pair(keys, np.arange(keys.size, dtype=np.uint32)) == ahs.RADIX
    sw = keys.copy()
    i = r.integers(0, keys.size, 5000)
    j = r.integers(0, keys.size, 5000)
    sw[i], sw[j] = keys[j], keys[i]
    assert run_pair(sw) == ahs.RADIX


def test_insertion_state():
    for n in (1, 2, 5, 20):
        r = np.random.default_rng(n)
        keys = r.integers(0, 5, n).astype(np.uint32)
        assert run_pair(keys, np.arange(n, dtype=np.uint32)) == ahs.INSERTION
    keys = np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.0], np.float32)
    assert run_pair(keys, np.arange(6, dtype=np.uint32)) == ahs.INSERTION


@pytest.mark.parametrize("strategy", [ahs.AUTO, ahs.RADIX, ahs.COUNTING])
def test_in_place(strategy):
    r = np.random.default_rng(11)
    keys = r.integers(0, 3000, 70_001).astype(np.uint32)
    run_pair(keys, np.arange(keys.size, dtype=np.uint32), strategy, in_place=True)
    run_pair(keys, None, strategy, in_place=True)
    if strategy == ahs.RADIX:
        keys = r.integers(0, 2**32, 70_001, dtype=np.uint64).astype(np.uint32)
        run_pair(keys, np.arange(keys.size, dtype=np.uint32), strategy, in_place=True)


def test_edge_patterns():
    n = 50_000
    asc = (np.arange(n, dtype=np.uint64) * 86_028_121 % 2**32).astype(np.uint32)
    asc.sort()
    pats = {
        "constant": np.full(n, 5, np.uint32),
        "ascending": asc,
        "descending": asc[::-1].copy(),
        "sawtooth": np.tile(np.concatenate([np.arange(500), np.arange(500)[::-1]]), n // 1000).astype(np.uint32) * 9973,
        "alternating": np.tile(np.array([1, 2**31], np.uint32), n // 2),
    }
    for name, keys in pats.items():
        say("pattern", name)
        run_pair(keys, np.arange(n, dtype=np.uint32), ahs.RADIX)
        run_pair(keys, np.arange(n, dtype=np.uint32), ahs.AUTO) if name in ("constant",) else None


def test_errors():
    k = to_dev(np.array([1.0, np.nan], np.float32))
    with pytest.raises(ahs.AhsError) as e:
        ahs.ahs_sort(k)
    assert e.value.status == ahs.E_NAN
    k = to_dev(np.array([0, 100_000], np.uint32))
    with pytest.raises(ahs.AhsError) as e:
        ahs.ahs_sort(k, strategy=ahs.COUNTING)
    assert e.value.status == ahs.E_UNSUPPORTED
    with pytest.raises(ahs.AhsError) as e:
        ahs.ahs_sort(k, strategy=ahs.INSERTION)
    assert e.value.status == ahs.E_INVALID_ARG
    ko, _, chosen, _ = ahs.ahs_sort(torch.empty(0, dtype=torch.uint32, device=DEV))
    assert ko.numel() == 0 and chosen == ahs.INSERTION


def test_repeatability():
    """Same input, many runs: identical bits (deterministic look-back)."""
    keys = gen.strategy_sweep("zipf256", n=1 << 20)
    vals = np.arange(keys.size, dtype=np.uint32)
    k, v = to_dev(keys), to_dev(vals)
    ref = None
    for i in range(20):
        ko, vo, _, _ = ahs.ahs_sort(k, v, ahs.RADIX)
        cur = (ko.cpu().numpy().copy(), vo.cpu().numpy().copy())
        if ref is None:
            ref = cur
        assert np.array_equal(cur[0], ref[0]) and np.array_equal(cur[1], ref[1])


# ------------------------------------------------------------------ general path (sample sort)
QUICK_SIZES = [1, 2, 21, 8191, 8192, 8193, 12_289, 100_003, 1_000_001]


@pytest.mark.parametrize("n", QUICK_SIZES)
def test_quick_sizes_u32(n):
    r = np.random.default_rng(n + 100)
    keys = r.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    run_pair(keys, np.arange(n, dtype=np.uint32), ahs.QUICK)
    run_pair(keys, None, ahs.QUICK)


@pytest.mark.parametrize("kind", ["u64", "f32", "f64", "u64zipf", "few"])
@pytest.mark.parametrize("n", [8193, 300_007])
def test_quick_wide_and_duplicates(kind, n):
    r = np.random.default_rng(n + len(kind))
    if kind == "u64":
        keys = r.integers(0, 2**64, n, dtype=np.uint64)
    elif kind == "f32":
        keys = r.normal(0, 1e3, n).astype(np.float32)
        keys[::97] = -0.0
        keys[::89] = 0.0
    elif kind == "f64":
        keys = r.normal(0, 1.0, n)
        keys[::53] = -np.inf
        keys[::59] = -0.0
    elif kind == "u64zipf":
        keys = gen.wide_keys("u64zipf4096", n=n)
    else:
        keys = r.choice(np.array([7, 7, 7, 9, 2**31, 5], np.uint32), n)
    run_pair(keys, np.arange(n, dtype=np.uint32), ahs.QUICK)
    run_pair(keys, None, ahs.QUICK)


@pytest.mark.parametrize("kind", ["u32", "u64", "f32"])
@pytest.mark.parametrize("n", [30_011, 120_007, 260_003])
def test_quick_buckets_with_repeated_keys(kind, n):
    """Each value 2-4 times, so equal keys fall inside block-sort buckets of
    about n/256 keys (one-pass rank sort up to 512 keys, LSD passes above)
    rather than into equality buckets: the payload pins their input order."""
    r = np.random.default_rng(n + 3 * len(kind))
    if kind == "u32":
        vals_ = r.integers(0, 2**32, n // 3, dtype=np.uint64).astype(np.uint32)
    elif kind == "u64":
        vals_ = r.integers(0, 2**64, n // 3, dtype=np.uint64)
    else:
        vals_ = r.normal(0, 1e3, n // 3).astype(np.float32)
        vals_[::7] = -0.0
        vals_[::11] = 0.0
    keys = vals_[r.integers(0, vals_.size, n)]
    run_pair(keys, np.arange(n, dtype=np.uint32), ahs.QUICK)
    run_pair(keys, None, ahs.QUICK)


def test_quick_patterns():
    n = 400_000
    base = gen.strategy_sweep("uniform32", n=n)
    srt = np.sort(base)
    pats = {
        "sorted": srt,
        "reverse": srt[::-1].copy(),
        "swapped": gen.apply_swaps(srt.copy(), 3, 5, n // 200),
        "constant": np.full(n, 77, np.uint32),
        "two-values": np.where(np.arange(n) % 3 == 0, 5, 2**32 - 1).astype(np.uint32),
        "sawtooth": np.tile(np.concatenate([np.arange(1000), np.arange(1000)[::-1]]), n // 2000).astype(np.uint32),
    }
    for name, keys in pats.items():
        say("pattern", name)
        run_pair(keys, np.arange(n, dtype=np.uint32), ahs.QUICK)


def test_quick_in_place():
    r = np.random.default_rng(4)
    for n in (5000, 250_001):
        keys = r.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
        run_pair(keys, np.arange(n, dtype=np.uint32), ahs.QUICK, in_place=True)
        keys = r.normal(0, 1, n).astype(np.float32)
        run_pair(keys, np.arange(n, dtype=np.uint32), ahs.QUICK, in_place=True)


@pytest.mark.parametrize("dtype", [np.uint32, np.int32, np.float32, np.uint64, np.int64, np.float64])
def test_quick_large_equal_key_buckets(dtype):
    """Forced QUICK where buckets of equal keys hold more than 4,096 keys and
    are scattered straight to the output: at level 0 (five distinct values,
    signed zeros and negative keys included, so signed and float keys are
    unmapped on the way) and at level 1 (24 values of 6,000 copies each
    among keys that need a second level); ragged size, with a payload, out
    of place and in place (level 0 then reads the output and the scatter
    keeps those buckets in the scratch buffer)."""
    r = np.random.default_rng(41)
    n = (1 << 22) + 777
    dt = np.dtype(dtype)
    if dt.kind == "f":
        vals = np.array([-3.5, -0.0, 0.0, 1.25, 7e3], dtype=dt)
        wide = (r.standard_normal(n) * 1e3).astype(dt)
    elif dt.kind == "i":
        info = np.iinfo(dt)
        vals = np.array([info.min, -1, 0, 3, info.max], dtype=dt)
        wide = r.integers(info.min, info.max, n, dtype=dt, endpoint=True)
    else:
        info = np.iinfo(dt)
        vals = np.array([0, 7, 1 << 20, info.max - 1, info.max], dtype=dt)
        wide = r.integers(0, info.max, n, dtype=dt, endpoint=True)
    few = vals[r.integers(0, vals.size, n)]
    mixed = wide.copy()
    heavy = wide[r.integers(0, n, 24)]
    mixed[r.permutation(n)[: 24 * 6000]] = np.repeat(heavy, 6000)
    pay = np.arange(n, dtype=np.uint32)
    for keys in (few, mixed):
        run_pair(keys, None, ahs.QUICK)
        run_pair(keys, pay, ahs.QUICK)
        run_pair(keys.copy(), pay.copy(), ahs.QUICK, in_place=True)


def test_auto_general_path():
    for case in ("uniform32", "sorted32", "reverse32", "swapped32"):
        keys = gen.strategy_sweep(case, n=1 << 20)
        assert run_pair(keys) == ahs.QUICK
    keys = gen.wide_keys("u64uniform", n=1 << 19)
    assert run_pair(keys, np.arange(keys.size, dtype=np.uint32)) == ahs.QUICK


SELECTOR_CASES = [("sweep", c, 1 << 20) for c in gen.SWEEP_CASES] + \
    [("wide", c, 1 << 19) for c in gen.WIDE_CASES] + [("pr1", "pr1", 1_000_000), ("sweep", "uniform32", 3000)]


@pytest.mark.parametrize("family,case,n", SELECTOR_CASES, ids=[f"{c[1]}-{c[2]}" for c in SELECTOR_CASES])
def test_auto_with_selector_model(family, case, n):
    """AUTO with the shipped selector model: the library's decision equals the
    oracle's (same model file, same features up to the entropy tolerance) and
    the output is the oracle's."""
    keys = gen.pr1() if family == "pr1" else (gen.strategy_sweep(case, n=n) if family == "sweep"
                                              else gen.wide_keys(case, n=n))
    vals = np.arange(keys.size, dtype=np.uint32)
    ctx = ahs.default_context(0)
    ctx.set_model(ahs.default_model())
    try:
        cfg = ahs.ahs_config_init(0, use_model=1)
        say(f"selector {case} n={keys.size}")
        ko, vo, chosen, f = ahs.ahs_sort(to_dev(keys), to_dev(vals), ahs.AUTO, cfg, want_features=True, ctx=ctx)
        torch.cuda.synchronize()
    finally:
        ctx.set_model(None)
    om = O.Model(ahs.SELECTOR_MODEL)
    st, rk, rv, rchosen, rf = O.sort(keys, vals, O.AUTO, O.config(0, use_model=1), om)
    assert st == O.OK
    assert np.array_equal(bits(ko.cpu().numpy()), bits(rk))
    assert np.array_equal(vo.cpu().numpy(), rv)
    check_features(f, rf)
    assert chosen == rchosen, (chosen, rchosen, rf.as_dict())


@pytest.mark.parametrize("kind,log2n", [("u32", 25), ("u64", 24), ("f32", 24)])
def test_quick_multilevel(kind, log2n):
    """Large enough that level 0 leaves buckets above the block-sort
    capacity, so later levels run with many segments at once."""
    n = 1 << log2n
    if kind == "u32":
        keys = gen.strategy_sweep("uniform32", n=n)
    elif kind == "u64":
        keys = gen.wide_keys("u64uniform", n=n)
    else:
        keys = gen.wide_keys("f32normal", n=n)
    vals = np.arange(n, dtype=np.uint32)
    say(f"multilevel quick {kind} n=2^{log2n}")
    ko, vo, chosen, _ = ahs.ahs_sort(to_dev(keys), to_dev(vals), ahs.QUICK)
    torch.cuda.synchronize()
    st, rk, rv, _, _ = O.sort(keys, vals, O.RADIX)  # same unique stable result, faster oracle
    assert st == O.OK
    assert np.array_equal(bits(ko.cpu().numpy()), bits(rk))
    assert np.array_equal(vo.cpu().numpy(), rv)


@pytest.mark.parametrize("case", ["zipf256", "uniform32", "uniform4096"])
def test_radix_counting_large(case):
    n = 1 << 25
    keys = gen.strategy_sweep(case, n=n)
    say(f"large {case}")
    ko, _, _, _ = ahs.ahs_sort(to_dev(keys), None, ahs.RADIX)
    st, rk, _, _, _ = O.sort(keys, None, O.RADIX)
    assert np.array_equal(ko.cpu().numpy(), rk)
    ko, _, chosen, _ = ahs.ahs_sort(to_dev(keys), None, ahs.AUTO)
    assert np.array_equal(ko.cpu().numpy(), rk)


# ------------------------------------------------------------------ signed keys
def _signed(kind, n, seed):
    """Signed keys of one family, with both ends of the type, -1 and 0 planted."""
    r = np.random.default_rng(seed)
    dt = np.int32 if kind.startswith("i32") else np.int64
    info = np.iinfo(dt)
    if kind.endswith("uniform"):
        keys = r.integers(int(info.min), int(info.max), n, dtype=np.int64, endpoint=True).astype(dt)
    elif kind.endswith("zipf"):
        # few distinct values spread over the whole signed range
        keys = gen.zipf_keys(seed, n, 256, 1.1, 32 if dt == np.int32 else 64)
        keys = keys.astype(np.uint32 if dt == np.int32 else np.uint64).view(dt)
        return keys
    else:  # narrow span straddling zero
        keys = r.integers(-1800, 1800, n).astype(dt)
        return keys
    if n > 4:
        keys[::101] = info.min
        keys[::103] = info.max
        keys[::107] = -1
        keys[::109] = 0
    return keys


@pytest.mark.parametrize("kind", ["i32uniform", "i32zipf", "i32narrow", "i64uniform", "i64zipf", "i64narrow"])
def test_signed_features_parity(kind):
    keys = _signed(kind, 300_007, 41)
    say(f"signed features {kind} n={keys.size}")
    hist = torch.zeros(65536, dtype=torch.int32, device=DEV)
    f = ahs.ahs_features(to_dev(keys), hist)
    torch.cuda.synchronize()
    st, rf, rhist = O.features(keys)
    assert st == O.OK
    check_features(f, rf, hist.cpu().numpy().view(np.uint32), rhist)


@pytest.mark.parametrize("n", [1, 21, 4097, 100_003, 1_000_003])
@pytest.mark.parametrize("kind", ["i32uniform", "i64uniform", "i32zipf"])
def test_signed_radix(n, kind):
    keys = _signed(kind, n, n + 3)
    run_pair(keys, np.arange(n, dtype=np.uint32), ahs.RADIX)
    run_pair(keys, None, ahs.RADIX)


@pytest.mark.parametrize("kind", ["i32narrow", "i64narrow"])
@pytest.mark.parametrize("n", [21, 8193, 1_000_003])
def test_signed_counting(kind, n):
    keys = _signed(kind, n, n + 5)
    run_pair(keys, None, ahs.COUNTING)
    run_pair(keys, np.arange(n, dtype=np.uint32), ahs.COUNTING)
    if kind == "i64narrow":
        # a narrow span at the bottom of the type
        run_pair(np.iinfo(np.int64).min + keys.astype(np.int64) + 1800, None, ahs.COUNTING)


@pytest.mark.parametrize("kind", ["i32uniform", "i64uniform", "i64zipf"])
@pytest.mark.parametrize("n", [8193, 300_007])
def test_signed_quick(kind, n):
    keys = _signed(kind, n, n + 9)
    run_pair(keys, np.arange(n, dtype=np.uint32), ahs.QUICK)
    run_pair(keys, None, ahs.QUICK)


def test_signed_auto_choices_and_in_place():
    """AUTO on signed keys takes the oracle's decision for each family:
    narrow span -> counting, few values over the full range -> radix,
    uniform over the full range -> quicksort; in place as well."""
    want = {"i32narrow": ahs.COUNTING, "i32zipf": ahs.RADIX, "i32uniform": ahs.QUICK,
            "i64narrow": ahs.COUNTING, "i64zipf": ahs.RADIX, "i64uniform": ahs.QUICK}
    for kind, s in want.items():
        keys = _signed(kind, 1 << 20, 43)
        assert run_pair(keys, np.arange(keys.size, dtype=np.uint32)) == s, kind
        assert run_pair(keys, None, in_place=True) == s, kind
    for n in (1, 7, 20):
        keys = np.array([-3, 2**31 - 1, -2**31, 0, -1, 5, -3] * 3, np.int32)[:n]
        assert run_pair(keys, np.arange(n, dtype=np.uint32)) == ahs.INSERTION


def test_small_input_state_without_features():
    """n <= n_small with integer keys and no feature request: the decision
    needs only n, so the sort runs without the feature pass; the result and
    the reported state equal the oracle's, in place too, and for a raised
    n_small up to the small sort's limit."""
    cfg0 = O.config(0)
    for dt in (np.uint32, np.int32, np.uint64, np.int64):
        for n in (1, 2, 7, 20):
            r = np.random.default_rng(n)
            info = np.iinfo(dt)
            keys = r.integers(int(info.min), int(info.max), n, dtype=np.int64 if dt != np.uint64 else np.uint64,
                              endpoint=True).astype(dt)
            keys[: n // 2] = keys[n - 1]  # duplicates
            vals = np.arange(n, dtype=np.uint32)
            st, rk, rv, rch, _ = O.sort(keys, vals, O.AUTO, cfg0)
            assert st == O.OK and rch == O.INSERTION
            k = to_dev(keys)
            ko, vo, ch, f = ahs.ahs_sort(k, to_dev(vals))
            assert f is None and ch == ahs.INSERTION
            assert np.array_equal(bits(ko.cpu().numpy()), bits(rk)) and np.array_equal(vo.cpu().numpy(), rv)
            ko, _, ch, _ = ahs.ahs_sort(k, out=k)
            torch.cuda.synchronize()
            assert ch == ahs.INSERTION and np.array_equal(bits(k.cpu().numpy()), bits(rk))
    keys = np.random.default_rng(3).integers(0, 50, 1000).astype(np.uint32)
    cfg = ahs.ahs_config_init(0, n_small=1000)
    ko, _, ch, _ = ahs.ahs_sort(to_dev(keys), cfg=cfg)
    st, rk, _, rch, _ = O.sort(keys, None, O.AUTO, O.config(0, n_small=1000))
    assert ch == ahs.INSERTION == rch and np.array_equal(ko.cpu().numpy(), rk)


def test_calibrated_preset_decisions():
    """The thresholds recalibrated by eq. (1) (n_small 48, K_c 5000): 48 keys
    take the small-input state, a span of 4,999 the counting sort, a span of
    5,000 the general path, matching the oracle under the same preset."""
    r = np.random.default_rng(47)
    keys = r.integers(0, 2**32, 48, dtype=np.uint64).astype(np.uint32)
    assert run_pair(keys, np.arange(48, dtype=np.uint32), cfg_preset=ahs.PRESET_MI355X_CALIBRATED) == ahs.INSERTION
    keys = (r.integers(0, 5000, 100_000) + 7).astype(np.uint32)
    keys[0], keys[1] = 7, 7 + 4999
    assert run_pair(keys, None, cfg_preset=ahs.PRESET_MI355X_CALIBRATED) == ahs.COUNTING
    keys[1] = 7 + 5000
    assert run_pair(keys, None, cfg_preset=ahs.PRESET_MI355X_CALIBRATED) == ahs.QUICK


@pytest.mark.parametrize("span_bits,nvals,dt", [(13, 30, np.uint32), (21, 200, np.uint32), (32, 300, np.uint32),
                                                (27, 100, np.uint64), (61, 13, np.uint64)])
def test_auto_radix_digits_from_histogram(span_bits, nvals, dt):
    """AUTO to radix on few values over spans of 2^13 (exact histogram, shift
    0: every digit summed from the bins), 2^21 (shift 5: digit 0 counted per
    key, digits 1 and 2 from runs of 8 and 2,048 bins), 2^32, 2^27 and 2^61
    (u64, shift 45: digits 6 and 7 from the bins): keys, payload and the
    decision equal the oracle's."""
    r = np.random.default_rng(span_bits)
    hi = (1 << span_bits) - 1
    vals = r.integers(0, hi, nvals, dtype=np.uint64, endpoint=True)
    vals[0], vals[1] = 0, hi
    keys = (vals[r.integers(0, nvals, 300_007)] + np.uint64(12345)).astype(dt)  # wraps for 2^32: still radix
    preset = 0
    if span_bits == 13:
        # lower the radix threshold so a span below 2^16 reaches the radix test
        cfg = ahs.ahs_config_init(0, k_count=100, k_radix=1000)
        ocfg = O.config(0, k_count=100, k_radix=1000)
        k = to_dev(keys)
        ko, vo, ch, f = ahs.ahs_sort(k, to_dev(np.arange(keys.size, dtype=np.uint32)), ahs.AUTO, cfg,
                                     want_features=True)
        st, rk, rv, rch, rf = O.sort(keys, np.arange(keys.size, dtype=np.uint32), O.AUTO, ocfg)
        assert st == O.OK and rch == O.RADIX and ch == ahs.RADIX and f.shift == 0
        assert np.array_equal(bits(ko.cpu().numpy()), bits(rk)) and np.array_equal(vo.cpu().numpy(), rv)
        return
    assert run_pair(keys, np.arange(keys.size, dtype=np.uint32), cfg_preset=preset) == ahs.RADIX
    assert run_pair(keys, None, cfg_preset=preset) == ahs.RADIX
