"""CPU checks of the seeded workload generators: the core words follow the
published SplitMix64 definition (re-derived here with Python integers and
pinned by the well-known first output of SplitMix64 from state 0), and the
batch generator of concatenated segments composes exactly the documented
primitives."""
import numpy as np

import gen

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def mix64_py(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def test_splitmix64_first_output_from_state_zero():
    # SplitMix64's state advances by GAMMA before mixing; from state 0 its
    # first output is 0xE220A8397B1DCDAF
    assert mix64_py(GAMMA) == 0xE220A8397B1DCDAF


def test_words_follow_the_counter_definition():
    for seed, stream in ((0, 0), (7, 3), (2**40 + 5, 1000)):
        base = mix64_py((seed * GAMMA + mix64_py((stream + GAMMA) & MASK)) & MASK)
        want = [mix64_py((base + (i + 1) * GAMMA) & MASK) for i in range(17)]
        assert gen.words(seed, stream, 17).tolist() == want
        assert gen.u32(seed, stream, 17).tolist() == [w >> 32 for w in want]


def _composed(nseg, seed, sizes):
    kinds = gen.index(seed, 1, nseg, len(gen.SEG_KINDS)).astype(np.int64)
    parts = []
    for i in range(nseg):
        n, st, kind = int(sizes[i]), 1000 + i, gen.SEG_KINDS[kinds[i]]
        if kind == "u256":
            v = gen.u32(seed, st, n, 255)
        elif kind == "u32":
            v = gen.u32(seed, st, n)
        elif kind == "zipf64":
            vals = gen.distinct(seed * 7919 + i, 1, 64, 32)
            v = vals[gen.zipf_index(seed * 7919 + i, 2, n, 1.1, 64)]
        elif kind == "sorted":
            v = np.sort(gen.u32(seed, st, n))
        else:
            v = np.sort(gen.u32(seed, st, n))[::-1]
        parts.append(np.asarray(v, np.uint32))
    return np.concatenate(parts), kinds


def test_segment_batch_composes_the_primitives():
    sizes = gen.segment_sizes(250, 8, cap=1 << 13)
    sizes[:4] = [0, 1, 16, 8193]
    keys, offs, kinds = gen.segments(250, 8, sizes)
    want, wkinds = _composed(250, 8, sizes)
    assert np.array_equal(kinds, wkinds)
    assert np.array_equal(keys, want)
    assert offs[0] == 0 and offs[-1] == keys.size and np.all(np.diff(offs.astype(np.int64)) == sizes)
    assert set(kinds.tolist()) == set(range(len(gen.SEG_KINDS)))


def test_segment_sizes_log_uniform_bounds():
    s = gen.segment_sizes(65536, 8)
    assert s.min() >= 16 and s.max() <= 1 << 20
    # log2 sizes spread evenly over [4, 20): each quarter holds about 1/4
    q = np.histogram(np.log2(s), bins=4, range=(4, 20))[0] / s.size
    assert np.all(np.abs(q - 0.25) < 0.02)


def _value_entropy(x):
    _, c = np.unique(x, return_counts=True)
    p = c / x.size
    return float(-(p * np.log2(p)).sum())


def test_paper_real_dataset_stand_ins_have_the_papers_n_k_h():
    """The synthetic stand-ins carry the range k = max - min + 1 and the value
    entropy H the paper gives for its taxi, sensor and k-mer datasets
    (Sec. III-B); n is the paper's by default (checked on smaller draws)."""
    for case, (n_paper, k_paper, h_paper) in gen.PAPER_REAL.items():
        assert gen.paper_sweep_default_n(case) == n_paper
        x = gen.paper_sweep(case, n=1 << 20)
        k = int(x.max()) - int(x.min()) + 1
        assert k == k_paper, (case, k)
        assert abs(_value_entropy(x) - h_paper) < 0.05, (case, _value_entropy(x))


def test_paper_synthetic_families_shapes():
    n = 1 << 18
    for name, k in (("uniform_k1e2", 100), ("uniform_k1e4", 10**4), ("uniform_k1e6", 10**6)):
        x = gen.paper_sweep(name, n=n)
        assert x.dtype == np.uint32 and x.min() >= 0 and x.max() < k
    for e in range(2, 7):
        x = gen.paper_sweep(f"gauss_k1e{e}", n=n)
        assert x.dtype == np.int32 and (x < 0).any() and (x > 0).any()
        assert abs(float(np.var(x.astype(np.float64))) / (10**e / 4) - 1) < 0.05
    z = gen.paper_sweep("zipf1.5_k1e2", n=n)
    c = np.bincount(z, minlength=100)
    assert c.argmax() == 0 and abs(c[0] / c[1] - 2 ** 1.5) < 0.1 * 2 ** 1.5
    s = gen.paper_sweep("sawtooth", n=1 << 18)
    d = np.diff(s.astype(np.int64))
    assert ((d > 0) | (d < 0) | (np.arange(d.size) % 65536 == 65535)).all()
    a = gen.paper_sweep("alternating", n=1000)
    assert (a[0::2] < a[1::2]).all() and (np.diff(a[0::2].astype(np.int64)) > 0).all()
    assert np.unique(gen.paper_sweep("constant", n=100)).size == 1
    assert gen.paper_sweep("i64_uniform", n=n).dtype == np.int64
