"""Python access to the CPU oracle of Adaptive Hybrid Sort.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the product package
never does.  It loads ``liboracle.so`` (built from ``ahs_oracle.c`` by
``oracle/build_oracle.py``) through ctypes and converts numpy arrays.

The passages of the paper each function follows are cited in
``ahs_oracle.h``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

U32, U64, F32, F64, I32, I64 = 0, 1, 2, 3, 4, 5
AUTO, COUNTING, RADIX, QUICK, INSERTION = 0, 1, 2, 3, 4
STRATEGY_NAMES = {AUTO: "auto", COUNTING: "counting", RADIX: "radix",
                  QUICK: "quick", INSERTION: "insertion"}
OK, E_INVALID_ARG, E_UNSUPPORTED, E_NAN, E_OOM, E_NO_MODEL, E_DEPTH, E_PARSE = (
    0, -1, -2, -3, -5, -7, -8, -9)

_DTYPES = {np.dtype(np.uint32): U32, np.dtype(np.uint64): U64,
           np.dtype(np.float32): F32, np.dtype(np.float64): F64,
           np.dtype(np.int32): I32, np.dtype(np.int64): I64}


class Features(C.Structure):
    _fields_ = [("n", C.c_uint64), ("min_key", C.c_uint64), ("max_key", C.c_uint64),
                ("span", C.c_uint64), ("nan_count", C.c_uint64),
                ("shift", C.c_uint32), ("nbins", C.c_uint32), ("exact", C.c_uint32),
                ("reserved", C.c_uint32),
                ("entropy_bits", C.c_double), ("entropy_ratio", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


class Config(C.Structure):
    _fields_ = [("n_small", C.c_uint32), ("use_model", C.c_uint32),
                ("k_count", C.c_uint64), ("k_radix", C.c_uint64),
                ("h_ratio", C.c_double), ("ml_min_n", C.c_uint64),
                ("k_count_cap", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH}; run oracle/build_oracle.py")
        L = C.CDLL(LIB_PATH)
        vp, u64, i32 = C.c_void_p, C.c_uint64, C.c_int
        L.ref_config_init.argtypes = [C.POINTER(Config), i32]
        L.ref_map_keys.argtypes = [i32, vp, u64, vp, C.POINTER(C.c_uint64)]
        L.ref_unmap_keys.argtypes = [i32, vp, u64, vp]
        L.ref_features_compute.argtypes = [i32, vp, u64, vp, C.POINTER(Features)]
        L.ref_select.argtypes = [C.POINTER(Features), C.POINTER(Config), vp, C.POINTER(C.c_int)]
        L.ref_sort.argtypes = [i32, vp, vp, vp, vp, u64, i32, C.POINTER(Config), vp,
                               C.POINTER(C.c_int), C.POINTER(Features)]
        L.ref_model_load.argtypes = [C.c_char_p, C.POINTER(vp)]
        L.ref_model_free.argtypes = [vp]
        L.ref_model_predict.argtypes = [vp, C.POINTER(Features), C.POINTER(C.c_int)]
        for fn in ("ref_config_init", "ref_map_keys", "ref_unmap_keys", "ref_features_compute",
                   "ref_select", "ref_sort", "ref_model_load", "ref_model_predict"):
            getattr(L, fn).restype = C.c_int
        L.ref_model_free.restype = None
        _lib = L
    return _lib


def dtype_code(arr: np.ndarray) -> int:
    try:
        return _DTYPES[arr.dtype]
    except KeyError:
        raise TypeError(f"unsupported key dtype {arr.dtype}") from None


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def config(preset: int = 0, **overrides) -> Config:
    cfg = Config()
    st = lib().ref_config_init(C.byref(cfg), preset)
    if st != OK:
        raise ValueError(f"bad preset {preset}")
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


class Model:
    def __init__(self, path: str):
        h = C.c_void_p()
        st = lib().ref_model_load(path.encode(), C.byref(h))
        if st != OK:
            raise ValueError(f"oracle could not load model {path}: status {st}")
        self._h = h

    @property
    def handle(self):
        return self._h

    def predict(self, feats: Features) -> int:
        out = C.c_int()
        lib().ref_model_predict(self._h, C.byref(feats), C.byref(out))
        return out.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ref_model_free(self._h)
            self._h = None


def map_keys(keys: np.ndarray):
    keys = np.ascontiguousarray(keys)
    out = np.empty(keys.size, dtype=np.uint64)
    nans = C.c_uint64()
    st = lib().ref_map_keys(dtype_code(keys), _ptr(keys), keys.size, _ptr(out), C.byref(nans))
    return st, out, nans.value


def unmap_keys(mapped: np.ndarray, dtype) -> np.ndarray:
    mapped = np.ascontiguousarray(mapped, dtype=np.uint64)
    out = np.empty(mapped.size, dtype=dtype)
    lib().ref_unmap_keys(dtype_code(out), _ptr(mapped), mapped.size, _ptr(out))
    return out


def features(keys: np.ndarray):
    """Returns (status, Features, histogram[nbins] as uint32)."""
    keys = np.ascontiguousarray(keys)
    f = Features()
    hist = np.zeros(65536, dtype=np.uint32)
    st = lib().ref_features_compute(dtype_code(keys), _ptr(keys), keys.size, _ptr(hist), C.byref(f))
    return st, f, hist[: f.nbins].copy()


def select(feats: Features, cfg: Config | None = None, model: Model | None = None):
    cfg = cfg if cfg is not None else config()
    out = C.c_int()
    st = lib().ref_select(C.byref(feats), C.byref(cfg), model.handle if model else None, C.byref(out))
    return st, out.value


def sort(keys: np.ndarray, vals: np.ndarray | None = None, strategy: int = AUTO,
         cfg: Config | None = None, model: Model | None = None):
    """Returns (status, keys_out, vals_out|None, chosen, Features)."""
    keys = np.ascontiguousarray(keys)
    cfg = cfg if cfg is not None else config()
    out = np.empty_like(keys)
    vout = None
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
        assert vals.size == keys.size
        vout = np.empty_like(vals)
    chosen = C.c_int()
    f = Features()
    st = lib().ref_sort(dtype_code(keys), _ptr(keys), _ptr(out), _ptr(vals), _ptr(vout), keys.size,
                        strategy, C.byref(cfg), model.handle if model else None,
                        C.byref(chosen), C.byref(f))
    return st, out, vout, chosen.value, f
