"""Seeded synthetic workloads for Adaptive Hybrid Sort.

Shared by the tests, the benchmark and the smoke check; holds none of the
sorting method's arithmetic.  Raw draws come from ``libahs_gen.so``
(counter-based SplitMix64, see ``ahs_gen.c``); this module composes them
into the workloads used for parity and measurement:

* ``pr1``: 1,000,000 u32 keys uniform on [0, 1023] (seed 0).
* ``strategy_sweep``: u32 arrays, (a) uniform on [0, 4095], (b) 256 distinct
  random 32-bit values drawn with Zipf(1.1) ranks, (c) uniform 32-bit keys,
  the same sorted, reversed, and sorted with n/200 random transpositions.
* ``wide_keys``: u64 uniform; u64 with 4,096 distinct values drawn with
  Zipf(1.0); f32 and f64 Normal(0, sigma=1e3) with 0.1 % duplicates and a few
  +-0.0 values.
* ``segments``: many uneven u32 arrays with sizes log-uniform on [16, 2^20].
* ``request_trace``: Poisson arrivals with log-uniform sizes and mixed types.
* ``paper_sweep``: the paper's synthetic families (uniform over k values,
  rounded Gaussians of variance k/4 as signed keys, Zipf(1.5) over k ranks),
  its edge patterns, full-range signed keys, and synthetic arrays with the
  (n, k, H) of its three real datasets.

The paper's own datasets (taxi timestamps, sensor readings, k-mers) are not
available; these synthetic families stand in for its uniform, skewed and
presorted inputs and its edge cases (Sec. III-B, Sec. IV-A).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libahs_gen.so")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"generator library missing: {LIB_PATH}; run gen/build_gen.py")
        L = C.CDLL(LIB_PATH)
        u64, vp = C.c_uint64, C.c_void_p
        L.gen_words.argtypes = [u64, u64, u64, vp]
        L.gen_u32.argtypes = [u64, u64, u64, C.c_uint32, vp]
        L.gen_u64.argtypes = [u64, u64, u64, u64, vp]
        L.gen_index.argtypes = [u64, u64, u64, u64, vp]
        L.gen_distinct.argtypes = [u64, u64, C.c_uint32, C.c_int, vp]
        L.gen_distinct.restype = u64
        L.gen_zipf_index.argtypes = [u64, u64, u64, C.c_double, C.c_uint32, vp]
        L.gen_zipf_index.restype = C.c_int
        L.gen_normal.argtypes = [u64, u64, u64, C.c_double, vp]
        L.gen_exponential.argtypes = [u64, u64, u64, C.c_double, vp]
        L.gen_unit.argtypes = [u64, u64, u64, vp]
        L.gen_apply_swaps.argtypes = [vp, u64, C.c_uint32, u64, u64, u64]
        L.gen_segments_u32.argtypes = [u64, C.c_uint32, vp, vp, vp, vp]
        L.gen_segments_u32.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- primitives
def words(seed, stream, n):
    out = np.empty(n, np.uint64)
    lib().gen_words(seed, stream, n, _p(out))
    return out


def u32(seed, stream, n, mask=0xFFFFFFFF):
    out = np.empty(n, np.uint32)
    lib().gen_u32(seed, stream, n, mask, _p(out))
    return out


def u64(seed, stream, n, mask=0xFFFFFFFFFFFFFFFF):
    out = np.empty(n, np.uint64)
    lib().gen_u64(seed, stream, n, mask, _p(out))
    return out


def index(seed, stream, n, rng):
    out = np.empty(n, np.uint64)
    lib().gen_index(seed, stream, n, rng, _p(out))
    return out


def distinct(seed, stream, m, bits):
    out = np.empty(m, np.uint64)
    lib().gen_distinct(seed, stream, m, bits, _p(out))
    return out if bits == 64 else out.astype(np.uint32)


def zipf_index(seed, stream, n, s, m):
    out = np.empty(n, np.uint32)
    if lib().gen_zipf_index(seed, stream, n, s, m, _p(out)) != 0:
        raise ValueError("zipf generator failed")
    return out


def normal(seed, stream, n, sigma):
    out = np.empty(n, np.float64)
    lib().gen_normal(seed, stream, n, sigma, _p(out))
    return out


def exponential(seed, stream, n, rate):
    out = np.empty(n, np.float64)
    lib().gen_exponential(seed, stream, n, rate, _p(out))
    return out


def unit(seed, stream, n):
    out = np.empty(n, np.float64)
    lib().gen_unit(seed, stream, n, _p(out))
    return out


def apply_swaps(arr, seed, stream, count):
    assert arr.flags.c_contiguous
    lib().gen_apply_swaps(_p(arr), arr.size, arr.itemsize, seed, stream, count)
    return arr


def zipf_keys(seed, n, m, s, bits):
    """m distinct random values (stream 1), picked with Zipf(s, m) ranks (stream 2)."""
    vals = distinct(seed, 1, m, bits)
    return vals[zipf_index(seed, 2, n, s, m)]


# ---------------------------------------------------------------- workloads
def pr1(n=1_000_000, seed=0):
    """u32 uniform on [0, 1023]."""
    return u32(seed, 0, n, 1023)


SWEEP_CASES = ("uniform4096", "zipf256", "uniform32", "sorted32", "reverse32", "swapped32")


def strategy_sweep(case, n=1 << 28, seed=None):
    """u32 keys of the strategy sweep; default seeds 1 (a), 2 (b), 3 (c)."""
    if case == "uniform4096":
        return u32(1 if seed is None else seed, 0, n, 4095)
    if case == "zipf256":
        return zipf_keys(2 if seed is None else seed, n, 256, 1.1, 32)
    s = 3 if seed is None else seed
    base = u32(s, 0, n)
    if case == "uniform32":
        return base
    base.sort()
    if case == "sorted32":
        return base
    if case == "reverse32":
        return np.ascontiguousarray(base[::-1])
    if case == "swapped32":
        return apply_swaps(base, s, 5, n // 200)
    raise ValueError(case)


WIDE_CASES = ("u64uniform", "u64zipf4096", "f32normal", "f64normal")


def _normal_recipe(seed, n, dtype):
    x = normal(seed, 10, n, 1000.0).astype(dtype)
    ndup = n // 1000
    if ndup:
        dst = index(seed, 11, ndup, n).astype(np.int64)
        src = index(seed, 12, ndup, n).astype(np.int64)
        x[dst] = x[src].copy()
    nz = n // 20000
    if nz:
        x[index(seed, 13, nz, n).astype(np.int64)] = dtype(-0.0)
        x[index(seed, 14, nz, n).astype(np.int64)] = dtype(0.0)
    return x


def wide_keys(case, n=1 << 27, seed=None):
    """Wide and floating keys; default seeds 4..7.  Payload = original index."""
    if case == "u64uniform":
        return u64(4 if seed is None else seed, 0, n)
    if case == "u64zipf4096":
        return zipf_keys(5 if seed is None else seed, n, 4096, 1.0, 64)
    if case == "f32normal":
        return _normal_recipe(6 if seed is None else seed, n, np.float32)
    if case == "f64normal":
        return _normal_recipe(7 if seed is None else seed, n, np.float64)
    raise ValueError(case)


SEG_KINDS = ("u256", "u32", "zipf64", "sorted", "reverse")


def segment_sizes(nseg, seed=8, lo_exp=4, span_exp=16, cap=1 << 20, lo=16):
    u = unit(seed, 0, nseg)
    s = np.floor(np.exp2(lo_exp + span_exp * u)).astype(np.int64)
    return np.clip(s, lo, cap)


def segments(nseg=65536, seed=8, sizes=None):
    """Concatenated u32 segments and their u64 offsets[nseg + 1]; each segment's
    distribution is drawn from SEG_KINDS (stream 1) and its keys from a
    stream of its own (1000 + segment index); see gen_segments_u32."""
    if sizes is None:
        sizes = segment_sizes(nseg, seed)
    sizes = np.ascontiguousarray(sizes, dtype=np.int64)
    nseg = sizes.size
    kinds = (index(seed, 1, nseg, len(SEG_KINDS))).astype(np.int64)
    offs = np.zeros(nseg + 1, np.uint64)
    np.cumsum(sizes, out=offs[1:])
    keys = np.empty(int(offs[-1]), np.uint32)
    if lib().gen_segments_u32(seed, nseg, _p(sizes), _p(kinds), _p(offs), _p(keys)) != 0:
        raise MemoryError("segment generator failed")
    return keys, offs, kinds


POOL_KINDS = ("u32uniform", "u32zipf4096", "u64uniform", "u64zipf4096", "f32normal")


def request_pool(kind, n=1 << 26, seed=10):
    """Device-resident key pools the serving workload draws requests from:
    u32/u64 uniform over the full range, u32/u64 with 4,096 distinct values
    drawn with Zipf(1.0) ranks, f32 Normal(0, 1e3) with duplicates and
    signed zeros (the wide-key recipe)."""
    k = POOL_KINDS.index(kind)
    if kind == "u32uniform":
        return u32(seed + k, 0, n)
    if kind == "u32zipf4096":
        return zipf_keys(seed + k, n, 4096, 1.0, 32).astype(np.uint32)
    if kind == "u64uniform":
        return u64(seed + k, 0, n)
    if kind == "u64zipf4096":
        return zipf_keys(seed + k, n, 4096, 1.0, 64)
    return _normal_recipe(seed + k, n, np.float32)


def request_pool_kind(dtype_code, dist):
    """Pool of a request with key type 0 u32 / 1 u64 / 2 f32 and distribution
    0 uniform / 1 Zipf (f32 requests always use the Normal pool)."""
    if dtype_code == 2:
        return "f32normal"
    return ("u32" if dtype_code == 0 else "u64") + ("uniform" if dist == 0 else "zipf4096")


def request_trace(duration_s=60.0, rate=2000.0, seed=9, lo_exp=10, span_exp=14, max_requests=None):
    """Arrival times, sizes, dtype codes (0 u32, 1 u64, 2 f32), distribution
    flags (0 uniform, 1 Zipf; f32 always Normal) and payload flags."""
    cap = int(duration_s * rate * 2 + 100)
    gaps = exponential(seed, 0, cap, rate)
    t = np.cumsum(gaps)
    keep = t < duration_s
    t = t[keep]
    m = t.size if max_requests is None else min(t.size, max_requests)
    t = t[:m]
    sizes = np.floor(np.exp2(lo_exp + span_exp * unit(seed, 1, m))).astype(np.int64)
    dt = index(seed, 2, m, 3).astype(np.int64)
    dist = index(seed, 3, m, 2).astype(np.int64)
    pay = index(seed, 4, m, 2).astype(np.int64)
    offs = index(seed, 5, m, 1 << 30).astype(np.int64)
    return {"arrival_s": t, "size": sizes, "dtype": dt, "dist": dist, "payload": pay, "offset": offs}


# the paper's dataset families (Sec. III-B) ----------------------------------
PAPER_CASES = (
    "uniform_k1e2", "uniform_k1e4", "uniform_k1e6",
    "gauss_k1e2", "gauss_k1e3", "gauss_k1e4", "gauss_k1e5", "gauss_k1e6",
    "zipf1.5_k1e2", "zipf1.5_k1e4", "zipf1.5_k1e6",
    "constant", "ascending", "descending", "sawtooth", "alternating",
    "i32_uniform", "i64_uniform",
    "taxi_like", "iot_like", "kmer_like",
)

# (n, k, H) the paper gives for its real datasets; the stand-ins match them
PAPER_REAL = {"taxi_like": (10**7, 10**9, 8.2), "iot_like": (10**6, 500, 1.1), "kmer_like": (10**8, 4**30, 3.7)}


def paper_sweep_default_n(case):
    return PAPER_REAL[case][0] if case in PAPER_REAL else 1 << 24


def paper_sweep(case, n=None, seed=None):
    """Keys of one family of the paper's datasets (default seed 20 + the
    case's position in PAPER_CASES):

    * uniform_k*: u32 uniform on [0, k).
    * gauss_k*: Normal(0, variance k/4) rounded to the nearest integer, as
      int32 (negative and positive keys).
    * zipf1.5_k*: u32 Zipf(1.5) ranks 0 .. k-1 (rank r+1 has weight (r+1)^-1.5).
    * constant (one value), ascending / descending (sorted uniform 32-bit
      keys), sawtooth (runs of 2^16 rising then falling keys, spaced 65,537
      apart), alternating (small and large keys in turn).
    * i32_uniform, i64_uniform: the whole signed range.
    * taxi_like: u32, 294 equally likely values over [0, 10^9) with both ends
      present: k = 10^9, H = log2(294) = 8.2 bits.
    * iot_like: u32 over [0, 500): one value with probability 0.92, the other
      499 equally likely: H = 1.1 bits.
    * kmer_like: u64, 13 equally likely 60-bit values (30-mers at 2 bits per
      base) with 0 and 4^30 - 1 present: k = 4^30, H = log2(13) = 3.7 bits.
    """
    if n is None:
        n = paper_sweep_default_n(case)
    s = 20 + PAPER_CASES.index(case) if seed is None else seed
    if case.startswith("uniform_k"):
        return index(s, 0, n, int(float(case[9:]))).astype(np.uint32)
    if case.startswith("gauss_k"):
        k = float(case[7:])
        return np.rint(normal(s, 0, n, float(np.sqrt(k / 4.0)))).astype(np.int32)
    if case.startswith("zipf1.5_k"):
        return zipf_index(s, 0, n, 1.5, int(float(case[9:])))
    if case == "constant":
        return np.full(n, 0x9E3779B9, np.uint32)
    if case in ("ascending", "descending"):
        x = u32(s, 0, n)
        x.sort()
        return x if case == "ascending" else np.ascontiguousarray(x[::-1])
    if case == "sawtooth":
        i = np.arange(n, dtype=np.uint64)
        r = i & np.uint64(0xFFFF)
        up = ((i >> np.uint64(16)) & np.uint64(1)) == 0
        return (np.where(up, r, np.uint64(0xFFFF) - r) * np.uint64(65537)).astype(np.uint32)
    if case == "alternating":
        i = np.arange(n, dtype=np.uint64)
        return np.where(i % np.uint64(2) == 0, i // np.uint64(2), np.uint64(0xFFFFFFFF) - i // np.uint64(2)).astype(
            np.uint32)
    if case == "i32_uniform":
        return u32(s, 0, n).view(np.int32)
    if case == "i64_uniform":
        return u64(s, 0, n).view(np.int64)
    if case == "taxi_like":
        vals = (distinct(s, 1, 294, 32).astype(np.uint64) * np.uint64(10**9)) >> np.uint64(32)
        x = vals[index(s, 2, n, 294).astype(np.int64)].astype(np.uint32)
        if n >= 2:
            x[0], x[n // 2] = 0, 10**9 - 1
        return x
    if case == "iot_like":
        other = index(s, 1, n, 499).astype(np.uint32)
        other += (other >= 250).astype(np.uint32)  # the 499 values besides 250
        return np.where(unit(s, 2, n) < 0.92, np.uint32(250), other).astype(np.uint32)
    if case == "kmer_like":
        vals = distinct(s, 1, 13, 64) >> np.uint64(4)
        x = vals[index(s, 2, n, 13).astype(np.int64)]
        if n >= 2:
            x[0], x[n // 2] = 0, (1 << 60) - 1
        return x
    raise ValueError(case)
