"""Host-only tests of the serving loop's scheduling core: the first-fit
arena that enforces the HBM budget, batch formation (oldest request first,
same key class, limits on keys and requests), the pending order, and the
nearest-rank latency percentiles.  The core is a header without device
calls; a small shim built here with g++ exposes it to ctypes."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
U64 = C.c_uint64


@pytest.fixture(scope="module")
def core_lib(tmp_path_factory):
    out = tmp_path_factory.mktemp("core") / "libcore_shim.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC",
                    "-I", os.path.join(ROOT, "paper_2506_20677_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "core_shim.cpp"), "-o", str(out)], check=True)
    L = C.CDLL(str(out))
    vp = C.c_void_p
    sig = {
        "arena_new": (vp, [U64]), "arena_delete": (None, [vp]), "arena_alloc": (U64, [vp, U64]),
        "arena_release": (C.c_int, [vp, U64]), "arena_used": (U64, [vp]), "arena_largest": (U64, [vp]),
        "arena_ranges": (U64, [vp]),
        "core_new": (vp, [U64, C.c_uint32]), "core_delete": (None, [vp]),
        "core_add": (U64, [vp, C.c_int, C.c_int, U64, C.c_double]),
        "core_plan": (C.c_uint32, [vp, C.POINTER(U64), C.c_uint32, C.POINTER(U64), C.c_int, C.c_int64]),
        "core_offset": (U64, [vp, U64]), "core_pending": (C.c_uint32, [vp, C.POINTER(U64), C.c_uint32]),
        "core_complete": (None, [vp, U64, C.c_int, C.c_double]), "core_percentile": (C.c_double, [vp, C.c_double]),
        "core_completed": (U64, [vp]), "core_failed": (U64, [vp]), "core_keys_done": (U64, [vp]),
    }
    for k, (r, a) in sig.items():
        getattr(L, k).restype = r
        getattr(L, k).argtypes = a
    return L


FAIL = 2**64 - 1


def test_arena_first_fit_alignment_and_coalescing(core_lib):
    L = core_lib
    a = L.arena_new(4096)
    x = L.arena_alloc(a, 1000)   # rounded to 1024
    y = L.arena_alloc(a, 256)
    z = L.arena_alloc(a, 2000)   # rounded to 2048
    assert (x, y, z) == (0, 1024, 1280)
    assert L.arena_used(a) == 1024 + 256 + 2048
    assert L.arena_alloc(a, 1024) == FAIL          # 768 left
    assert L.arena_alloc(a, 768) == 3328
    assert L.arena_release(a, y) == 1
    assert L.arena_release(a, y) == 0              # double free refused
    assert L.arena_alloc(a, 512) == FAIL           # only the 256-byte hole
    assert L.arena_release(a, x) == 1              # coalesces with the hole: 1280 bytes at 0
    assert L.arena_largest(a) == 1280 and L.arena_ranges(a) == 1
    assert L.arena_alloc(a, 1280) == 0
    for off in (0, 1280, 3328):
        assert L.arena_release(a, off) == 1
    assert L.arena_used(a) == 0 and L.arena_largest(a) == 4096 and L.arena_ranges(a) == 1
    L.arena_delete(a)


def test_arena_random_alloc_free_never_overlaps(core_lib):
    L = core_lib
    cap = 1 << 20
    a = L.arena_new(cap)
    rng = np.random.default_rng(5)
    live = {}
    for step in range(3000):
        if live and rng.random() < 0.45:
            off = list(live)[rng.integers(len(live))]
            assert L.arena_release(a, off) == 1
            del live[off]
        else:
            size = int(rng.integers(1, 40_000))
            off = L.arena_alloc(a, size)
            if off == FAIL:
                assert L.arena_largest(a) < (size + 255) // 256 * 256
                continue
            size = (size + 255) // 256 * 256
            assert off % 256 == 0 and off + size <= cap
            for o, s in live.items():
                assert off + size <= o or o + s <= off
            live[off] = size
        assert L.arena_used(a) == sum(live.values())
    L.arena_delete(a)


def plan(L, c, start=False, b=0):
    ids = (U64 * 4096)()
    keys = U64()
    n = L.core_plan(c, ids, 4096, C.byref(keys), 1 if start else 0, b)
    return list(ids[:n]), keys.value


def pending(L, c):
    ids = (U64 * 4096)()
    n = L.core_pending(c, ids, 4096)
    return list(ids[:n])


def test_batches_take_oldest_class_in_arrival_order(core_lib):
    L = core_lib
    c = L.core_new(1000, 3)
    r = [L.core_add(c, dt, pay, n, float(i)) for i, (dt, pay, n) in enumerate(
        [(0, 0, 100), (1, 0, 50), (0, 0, 200), (0, 1, 10), (0, 0, 300), (0, 0, 400), (0, 0, 10)])]
    ids, keys = plan(L, c, start=True, b=7)
    # u32 without payload: r0, r2, r4 (three requests: the request limit)
    assert ids == [r[0], r[2], r[4]] and keys == 600
    assert [L.core_offset(c, i) for i in ids] == [0, 100, 300]
    assert pending(L, c) == [r[1], r[3], r[5], r[6]]
    ids, keys = plan(L, c, start=True)
    assert ids == [r[1]] and keys == 50                  # u64 is now the oldest
    ids, keys = plan(L, c, start=True)
    assert ids == [r[3]]                                 # u32 with payload
    ids, keys = plan(L, c)
    assert ids == [r[5], r[6]] and keys == 410
    L.core_delete(c)


def test_key_limit_stops_the_class_scan_and_head_is_always_taken(core_lib):
    L = core_lib
    c = L.core_new(1000, 100)
    big = L.core_add(c, 2, 0, 5000, 0.0)   # larger than the batch limit: alone
    a = L.core_add(c, 2, 0, 600, 1.0)
    b = L.core_add(c, 2, 0, 500, 2.0)
    d = L.core_add(c, 2, 0, 100, 3.0)
    assert plan(L, c, start=True) == ([big], 5000)
    # a fits, b would exceed 1000: the scan stops there (d waits behind b)
    assert plan(L, c, start=True) == ([a], 600)
    assert plan(L, c) == ([b, d], 600)
    L.core_delete(c)


def test_percentiles_are_nearest_rank(core_lib):
    L = core_lib
    c = L.core_new(1 << 30, 1024)
    rng = np.random.default_rng(3)
    lat = rng.exponential(5.0, 997)
    ids = [L.core_add(c, 0, 0, 10, 0.0) for _ in lat]
    plan(L, c, start=True)
    for i, x in zip(ids, lat):
        L.core_complete(c, i, 0, float(x))
    for q in (50.0, 90.0, 99.0, 100.0):
        assert L.core_percentile(c, q) == np.percentile(lat, q, method="inverted_cdf")
    assert L.core_completed(c) == 997 and L.core_keys_done(c) == 9970
    L.core_complete(c, L.core_add(c, 0, 0, 10, 0.0), -5, 1.0)  # a failure is not a latency sample
    assert L.core_completed(c) == 997 and L.core_failed(c) == 1
    L.core_delete(c)
