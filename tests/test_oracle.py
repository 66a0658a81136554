"""Pins the CPU oracle to the paper and to mathematics it does not share.

Each test checks the oracle against something other than itself: hand-worked
fixtures (tests/golden), closed forms of the entropy, brute force over all
permutations of tiny inputs against Python's stable ``sorted``, independent
library routines (numpy sorting and searching, scipy's entropy), and
invariants (sortedness, multiset, stability, idempotence, agreement of the
four sorts).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NP = {"u32": np.uint32, "u64": np.uint64, "f32": np.float32, "f64": np.float64}
STRAT = {"insertion": O.INSERTION, "counting": O.COUNTING, "radix": O.RADIX, "quick": O.QUICK}
SORTS = (O.INSERTION, O.COUNTING, O.RADIX, O.QUICK)


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def keys_of(case):
    dt = NP[case["dtype"]]
    if "keys_hex" in case:
        ut = np.uint32 if dt in (np.uint32, np.float32) else np.uint64
        return np.array([int(h, 16) for h in case["keys_hex"]], dtype=ut).view(dt)
    return np.array(case["keys"], dtype=dt)


def bits(a):
    return a.view(np.uint32 if a.itemsize == 4 else np.uint64)


def stable_reference(keys):
    """Stable order by the float or integer value, -0.0 before +0.0."""
    if keys.dtype.kind == "f":
        idx = range(keys.size)
        return sorted(idx, key=lambda i: (float(keys[i]), 0 if math.copysign(1.0, keys[i]) < 0 else 1))
    return sorted(range(keys.size), key=lambda i: int(keys[i]))


# ------------------------------------------------------------------ features
@pytest.mark.parametrize("case", load("features_cases.json")["cases"])
def test_features_golden(case):
    st, f, hist = O.features(keys_of(case))
    assert st == O.OK
    assert (f.n, f.min_key, f.max_key, f.span) == (len(keys_of(case)), case["min"], case["max"], case["span"])
    assert (f.shift, f.nbins, f.exact) == (case["shift"], case["nbins"], case["exact"])
    assert f.entropy_bits == pytest.approx(case["H"], rel=1e-12, abs=1e-15)
    if "ratio" in case:
        assert f.entropy_ratio == pytest.approx(case["ratio"], rel=1e-12, abs=1e-15)
    else:
        assert f.entropy_ratio == pytest.approx(case["H"] / math.log2(case["ratio_log2_bins"]), rel=1e-12)
    assert int(hist.sum()) == f.n
    for b, c in case.get("hist_nonzero", {}).items():
        assert hist[int(b)] == c
    assert np.count_nonzero(hist) == len(set(bits(keys_of(case)).tolist())) or f.shift > 0


def test_features_empty():
    st, f, hist = O.features(np.array([], np.uint32))
    assert st == O.OK and f.n == 0 and f.nbins == 0 and f.entropy_bits == 0.0 and hist.size == 0


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_features_nan_rejected(dt):
    a = np.array([1.0, np.nan, -2.0, np.nan], dtype=dt)
    st, f, _ = O.features(a)
    assert st == O.E_NAN and f.nan_count == 2 and f.n == 4


def test_entropy_constant_is_exactly_zero():
    for n in (1, 2, 21, 1000, 12345):
        st, f, _ = O.features(np.full(n, 77, np.uint32))
        assert st == O.OK and f.entropy_bits == 0.0 and f.entropy_ratio == 0.0 and f.nbins == 1


@pytest.mark.parametrize("m", [2, 3, 7, 64, 1000, 4096])
def test_entropy_equal_frequencies_is_log2_m(m):
    # m equally frequent values: H = log2 m exactly in real arithmetic
    keys = np.tile(np.arange(m, dtype=np.uint32) * 3 + 11, 5)
    np.random.default_rng(m).shuffle(keys)
    st, f, _ = O.features(keys)
    assert f.entropy_bits == pytest.approx(math.log2(m), rel=1e-12)


@pytest.mark.parametrize("a,b", [(1, 1), (1, 3), (5, 995), (333, 667)])
def test_entropy_two_values_binary_entropy(a, b):
    keys = np.array([10] * a + [20] * b, dtype=np.uint32)
    p = a / (a + b)
    h = -(p * math.log2(p) + (1 - p) * math.log2(1 - p))
    st, f, _ = O.features(keys)
    assert f.entropy_bits == pytest.approx(h, rel=1e-12)


def test_entropy_matches_scipy_and_bounds():
    scipy_stats = pytest.importorskip("scipy.stats")
    rng = np.random.default_rng(1)
    for n, hi in ((100, 50), (5000, 70000), (20000, 2**32 - 1)):
        keys = rng.integers(0, hi, size=n, dtype=np.uint64).astype(np.uint32)
        st, f, hist = O.features(keys)
        assert f.entropy_bits == pytest.approx(scipy_stats.entropy(hist[hist > 0], base=2), rel=1e-12)
        assert f.entropy_bits <= math.log2(min(n, f.nbins)) + 1e-12
        perm = rng.permutation(keys)
        assert O.features(perm)[1].entropy_bits == f.entropy_bits


@pytest.mark.parametrize("dt,hi", [(np.uint32, 2**32), (np.uint64, 2**64), (np.uint32, 70000), (np.uint32, 65536)])
def test_histogram_bins_by_searchsorted(dt, hi):
    rng = np.random.default_rng(7)
    keys = rng.integers(0, hi, size=30000, dtype=np.uint64 if dt == np.uint64 else np.int64).astype(dt)
    st, f, hist = O.features(keys)
    assert f.min_key == int(keys.min()) and f.max_key == int(keys.max())
    # shift is the smallest giving at most 65,536 bins
    assert (f.span >> f.shift) <= 65535 and (f.shift == 0 or (f.span >> (f.shift - 1)) > 65535)
    # bin b holds keys in [min + b 2^s, min + (b+1) 2^s): count them by binary search
    srt = np.sort(keys.astype(np.uint64))
    edges = [f.min_key + (b << f.shift) for b in range(f.nbins + 1)]
    pos = np.searchsorted(srt, np.array([min(e, 2**64 - 1) for e in edges], dtype=np.uint64), side="left")
    if edges[-1] > 2**64 - 1:
        pos[-1] = srt.size
    assert np.array_equal(np.diff(pos).astype(np.uint32), hist)


def test_float_map_examples():
    st, m, _ = O.map_keys(np.array([-np.inf, -1.0, -0.0, 0.0, 1.0, np.inf], np.float32))
    assert st == O.OK and np.all(np.diff(m.astype(np.int64)) > 0)
    st, m, _ = O.map_keys(np.array([-np.inf, -1e300, -5e-324, -0.0, 0.0, 5e-324, 1e300, np.inf]))
    assert st == O.OK and all(int(m[i]) < int(m[i + 1]) for i in range(m.size - 1))


@pytest.mark.slow
def test_f32_map_exhaustive():
    """Walk the whole 32-bit mapped space in order: NaNs sit exactly at both
    ends; inside, IEEE values increase strictly except -0.0 -> +0.0."""
    lo, hi = 0x007FFFFF, 0xFF800000  # mapped -inf (~0xFF800000) .. mapped +inf
    chunk = 1 << 26
    prev = None
    for start in range(0, 1 << 32, chunk):
        m = np.arange(start, start + chunk, dtype=np.uint64)
        x = O.unmap_keys(m, np.float32)
        isnan = np.isnan(x)
        inside = (m >= lo) & (m <= hi)
        assert np.array_equal(isnan, ~inside)
        xin = x[inside]
        if xin.size:
            if prev is not None:  # across the chunk boundary
                assert prev[0] < xin[0] or (prev[0] == 0 and np.signbit(prev[0]) and not np.signbit(xin[0]))
            d = np.diff(xin)
            assert np.all(d >= 0)
            for t in np.nonzero(d == 0)[0]:  # only -0.0 then +0.0
                assert np.signbit(xin[t]) and not np.signbit(xin[t + 1]) and xin[t] == 0
            prev = xin[-1:]
        # round trip
        st, back, _ = O.map_keys(x[inside])
        assert np.array_equal(back, m[inside])


# ------------------------------------------------------------------ FSM / model
@pytest.mark.parametrize("row", load("fsm_table.json")["rows"])
def test_fsm_golden(row):
    presets = load("fsm_table.json")["presets"]
    f = O.Features(n=row["n"], span=row["span"], nbins=row["nbins"], entropy_bits=row["H"])
    st, s = O.select(f, O.config(presets[row["preset"]]))
    assert st == O.OK and s == STRAT[row["expect"]]


def test_fsm_entropy_boundary():
    cfg = O.config(0)
    B = 65536
    thr = 0.7 * math.log2(B)
    for H, want in ((thr - 1e-9, O.RADIX), (thr, O.QUICK), (thr + 1e-9, O.QUICK)):
        f = O.Features(n=10**6, span=2**32 - 1, nbins=B, entropy_bits=H)
        assert O.select(f, cfg)[1] == want


def test_model_golden():
    cases = load("model_cases.json")
    tiny = O.Model(os.path.join(GOLDEN, "tiny_model.gbt"))
    tie = O.Model(os.path.join(GOLDEN, "tie_model.gbt"))
    for c in cases["tiny_model"]:
        f = O.Features(n=c["n"], span=c["span"], nbins=c["nbins"], entropy_bits=c["H"])
        assert tiny.predict(f) == STRAT[c["expect"]], c
    for c in cases["tie_model"]:
        f = O.Features(n=c["n"], span=c["span"], nbins=c["nbins"], entropy_bits=c["H"])
        assert tie.predict(f) == STRAT[c["expect"]]
    cfg = O.config(0, use_model=1)
    for c in cases["select_with_tiny_model"]:
        f = O.Features(n=c["n"], span=c["span"], nbins=c["nbins"], entropy_bits=c["H"])
        assert O.select(f, cfg, tiny) == (O.OK, STRAT[c["expect"]]), c
    for c in cases["select_with_tie_model_cap"]:
        f = O.Features(n=c["n"], span=c["span"], nbins=c["nbins"], entropy_bits=c["H"])
        assert O.select(f, cfg, tie) == (O.OK, STRAT[c["expect"]]), c
    f = O.Features(n=5000, span=10, nbins=11)
    assert O.select(f, cfg, None)[0] == O.E_NO_MODEL


def test_model_parse_errors(tmp_path):
    bad = tmp_path / "bad.gbt"
    bad.write_text("ahs-gbt 1\nnum_class 3\nbase_score 0 0 0\nnum_trees 1\ntree 0 2\n0 split 1 5 0 1\n1 leaf 1\n")
    with pytest.raises(ValueError):
        O.Model(str(bad))


# ------------------------------------------------------------------ sorts
@pytest.mark.parametrize("case", load("sort_cases.json")["cases"])
def test_sort_golden(case):
    keys = keys_of(case)
    vals = np.arange(keys.size, dtype=np.uint32)
    for s in SORTS + (O.AUTO,):
        st, ko, vo, ch, f = O.sort(keys, vals, s)
        if s == O.COUNTING and f.span >= O.config(0).k_count_cap:
            assert st == O.E_UNSUPPORTED
            continue
        assert st == O.OK
        assert np.array_equal(vo, np.array(case["perm"], np.uint32)), (s, vo)
        assert np.array_equal(bits(ko), bits(keys[np.array(case["perm"])]))
        if "sorted" in case:
            assert np.array_equal(ko, np.array(case["sorted"], dtype=keys.dtype))


def _multisets(n):
    """All value patterns of length n up to relabelling (restricted growth strings)."""
    def rec(prefix, mx):
        if len(prefix) == n:
            yield tuple(prefix)
            return
        for v in range(mx + 2):
            yield from rec(prefix + [v], max(mx, v))
    yield from rec([], -1)


@pytest.mark.parametrize("n", range(0, 7))
def test_bruteforce_all_permutations(n):
    """Every permutation of every multiset pattern of size n, every sort,
    against Python's stable sorted()."""
    cfg = O.config(0)
    scale = np.array([0, 1, 3, 1000, 70000, 2**31, 2**32 - 1], dtype=np.uint64)
    for pat in _multisets(n):
        base = scale[list(pat)].astype(np.uint32)
        for perm in set(itertools.permutations(range(n))):
            keys = base[list(perm)] if n else base
            vals = np.arange(n, dtype=np.uint32)
            want = np.array(stable_reference(keys), dtype=np.int64)
            for s in SORTS:
                st, ko, vo, _, _ = O.sort(keys, vals, s, cfg)
                if s == O.COUNTING and n and int(keys.max()) - int(keys.min()) >= cfg.k_count_cap:
                    assert st == O.E_UNSUPPORTED
                    continue
                assert st == O.OK
                assert np.array_equal(vo, want.astype(np.uint32)), (s, keys, vo, want)
                assert np.array_equal(ko, keys[want] if n else keys)


@pytest.mark.parametrize("n", range(0, 6))
@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_bruteforce_signed_permutations(n, dtype):
    """Signed keys: every permutation of every multiset pattern over values
    that straddle zero and reach both ends of the type, every sort, against
    Python's stable sorted() on the integer values."""
    cfg = O.config(0)
    info = np.iinfo(dtype)
    scale = [int(info.min), int(info.min) + 1, -70000, -1, 0, 1, int(info.max)]
    for pat in _multisets(n):
        base = np.array([scale[p] for p in pat], dtype=dtype)
        for perm in set(itertools.permutations(range(n))):
            keys = base[list(perm)] if n else base
            vals = np.arange(n, dtype=np.uint32)
            want = np.array(sorted(range(n), key=lambda i: int(keys[i])), dtype=np.int64)
            for s in SORTS:
                st, ko, vo, _, _ = O.sort(keys, vals, s, cfg)
                if s == O.COUNTING and n and int(keys.max()) - int(keys.min()) >= cfg.k_count_cap:
                    assert st == O.E_UNSUPPORTED
                    continue
                assert st == O.OK
                assert np.array_equal(vo, want.astype(np.uint32)), (s, keys, vo, want)
                assert np.array_equal(ko, keys[want] if n else keys)


@pytest.mark.parametrize("dtype,udtype", [(np.int32, np.uint32), (np.int64, np.uint64)])
def test_signed_map_is_offset_by_type_minimum(dtype, udtype):
    """The signed map sends v to v - min(type): order preserving and onto the
    unsigned range, so min -> 0, -1 -> 2^(w-1) - 1, 0 -> 2^(w-1), max -> 2^w - 1;
    the features of signed keys equal those of the same values shifted by
    -min(type) into the unsigned type (span, bins and entropy are translation
    invariant)."""
    info = np.iinfo(dtype)
    w = np.dtype(dtype).itemsize * 8
    keys = np.array([info.min, -1, 0, info.max], dtype=dtype)
    st, m, nans = O.map_keys(keys)
    assert st == O.OK and nans == 0
    assert [int(x) for x in m] == [0, 2**(w - 1) - 1, 2**(w - 1), 2**w - 1]
    assert np.array_equal(O.unmap_keys(m, dtype), keys)
    r = np.random.default_rng(7)
    for lo, hi in ((-3000, 1000), (int(info.min), int(info.min) + 5000), (-2**20, 2**20)):
        sk = r.integers(lo, hi, 20000, dtype=np.int64).astype(dtype)
        # shift by -min(type) in Python integers, then into the unsigned type
        uk = np.array([int(v) - int(info.min) for v in sk], dtype=np.uint64).astype(udtype)
        st1, fs, hs = O.features(sk)
        st2, fu, hu = O.features(uk)
        assert st1 == st2 == O.OK
        assert (fs.n, fs.span, fs.nbins, fs.exact) == (fu.n, fu.span, fu.nbins, fu.exact)
        assert fs.span == int(sk.max()) - int(sk.min())
        assert fs.entropy_bits == fu.entropy_bits and np.array_equal(hs, hu)


def _check_sorted_stable(keys, ko, vo):
    srt = np.argsort(keys, kind="stable")  # numpy's stable sort: an independent reference
    if keys.dtype.kind == "f":
        # numpy orders -0.0 == +0.0; the map orders -0.0 first: compare by mapped bits instead
        _, m, _ = O.map_keys(keys)
        srt = np.argsort(m, kind="stable")
    assert np.array_equal(vo, srt.astype(np.uint32))
    assert np.array_equal(bits(ko), bits(keys[srt]))


GEN_CASES = [
    ("u32 small range", lambda r, n: r.integers(0, 1000, n).astype(np.uint32)),
    ("u32 full range", lambda r, n: r.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)),
    ("u32 few distinct", lambda r, n: r.choice(r.integers(0, 2**32, 5, dtype=np.uint64), n).astype(np.uint32)),
    ("u64 full range", lambda r, n: r.integers(0, 2**64, n, dtype=np.uint64)),
    ("u64 narrow", lambda r, n: r.integers(0, 3000, n).astype(np.uint64) + np.uint64(2**63)),
    ("f32 normal", lambda r, n: r.normal(0, 1e3, n).astype(np.float32)),
    ("f64 normal+zeros", lambda r, n: np.where(r.random(n) < 0.1, np.where(r.random(n) < .5, -0.0, 0.0),
                                               r.normal(0, 1, n))),
    ("f32 inf mix", lambda r, n: r.choice(np.array([-np.inf, np.inf, -0.0, 0.0, 1.5, -1.5], np.float32), n)),
    ("i32 mixed sign", lambda r, n: r.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32)),
    ("i32 narrow around zero", lambda r, n: r.integers(-1500, 1500, n).astype(np.int32)),
    ("i32 extremes", lambda r, n: r.choice(np.array([-2**31, -1, 0, 1, 2**31 - 1], np.int32), n)),
    ("i64 mixed sign", lambda r, n: r.integers(-2**63, 2**63 - 1, n, dtype=np.int64)),
    ("i64 narrow negative", lambda r, n: r.integers(-2**40 - 3000, -2**40, n, dtype=np.int64)),
]


@pytest.mark.parametrize("name,make", GEN_CASES, ids=[c[0] for c in GEN_CASES])
@pytest.mark.parametrize("n", [1, 21, 257, 5000])
def test_sorts_agree_and_match_numpy(name, make, n):
    r = np.random.default_rng(n)
    keys = np.ascontiguousarray(make(r, n))
    vals = np.arange(n, dtype=np.uint32)
    cfg = O.config(0)
    outs = []
    for s in SORTS + (O.AUTO,):
        st, ko, vo, ch, f = O.sort(keys, vals, s, cfg)
        if s == O.COUNTING and f.span >= cfg.k_count_cap:
            assert st == O.E_UNSUPPORTED
            continue
        assert st == O.OK, (s, st)
        _check_sorted_stable(keys, ko, vo)
        outs.append((bits(ko).copy(), vo.copy()))
        # idempotent
        st2, ko2, vo2, _, _ = O.sort(ko, vo, s, cfg)
        assert np.array_equal(bits(ko2), bits(ko)) and np.array_equal(vo2, vo)
    for k, v in outs[1:]:
        assert np.array_equal(k, outs[0][0]) and np.array_equal(v, outs[0][1])


def test_paper_edge_cases():
    """Edge patterns of Sec. III-B: uniform values, ascending, descending,
    sawtooth, alternating, empty; closed forms for sorted and reversed."""
    n = 4000
    asc = np.arange(n, dtype=np.uint32) * 7
    cases = {
        "constant": np.full(n, 5, np.uint32),
        "ascending": asc,
        "descending": asc[::-1].copy(),
        "sawtooth": np.tile(np.concatenate([np.arange(50), np.arange(50)[::-1]]), n // 100).astype(np.uint32),
        "alternating": np.tile(np.array([1, 2**31], np.uint32), n // 2),
        "empty": np.array([], np.uint32),
    }
    for name, keys in cases.items():
        vals = np.arange(keys.size, dtype=np.uint32)
        for s in SORTS + (O.AUTO,):
            st, ko, vo, ch, f = O.sort(keys, vals, s)
            if s == O.COUNTING and f.span >= O.config(0).k_count_cap:
                assert st == O.E_UNSUPPORTED
                continue
            assert st == O.OK, (name, s, st)
            _check_sorted_stable(keys, ko, vo)
        if name in ("constant", "ascending"):
            assert np.array_equal(vo, vals)
        if name == "descending":
            assert np.array_equal(vo, vals[::-1])


def test_auto_choices_on_workload_shapes(gen_lib):
    """The FSM's outcomes on the workload families (uniform small range ->
    counting; 256 Zipf values over the full 32-bit range -> radix; uniform
    32-bit -> quicksort), at a size the oracle handles in a second."""
    G = gen_lib
    n = 1 << 18
    want = {"uniform4096": O.COUNTING, "zipf256": O.RADIX, "uniform32": O.QUICK,
            "sorted32": O.QUICK, "reverse32": O.QUICK, "swapped32": O.QUICK}
    for case, s in want.items():
        st, f, _ = O.features(G.strategy_sweep(case, n=n))
        assert O.select(f)[1] == s, case
    st, f, _ = O.features(G.pr1())
    assert O.select(f)[1] == O.COUNTING and f.nbins == 1024 and f.exact == 1
    wide = {"u64uniform": O.QUICK, "u64zipf4096": O.RADIX, "f32normal": O.RADIX, "f64normal": O.RADIX}
    for case, s in wide.items():
        st, f, _ = O.features(G.wide_keys(case, n=n))
        assert O.select(f)[1] == s, case


def test_errors():
    cfg = O.config(0)
    keys = np.array([0, 100000], np.uint32)
    st, *_ = O.sort(keys, None, O.COUNTING, cfg)
    assert st == O.E_UNSUPPORTED
    st, *_ = O.sort(np.array([1.0, np.nan], np.float32), None, O.AUTO, cfg)
    assert st == O.E_NAN
    st, *_ = O.sort(keys, None, 9, cfg)
    assert st == O.E_INVALID_ARG
