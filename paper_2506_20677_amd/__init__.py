"""MI355X-native Adaptive Hybrid Sort (arXiv 2506.20677): Python binding.

A thin ctypes layer over ``libahs.so`` (the C ABI of ``include/ahs.h``).
It only marshals arguments: torch tensors supply device memory and HIP
streams; every step of the method runs in the library's gfx950 kernels.  If
the library is missing the import of any call fails loudly; there is no
fallback path.

Calls (same names as the C ABI):
    ahs_config_init, ahs_context_create, ahs_workspace_bytes,
    ahs_features, ahs_select, ahs_sort, ahs_sort_static, ahs_model_load, ahs_model_predict,
    ahs_profile_enable / ahs_profile_reset / ahs_profile_query / ahs_profile_dump
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libahs.so")

U32, U64, F32, F64, I32, I64 = 0, 1, 2, 3, 4, 5
AUTO, COUNTING, RADIX, QUICK, INSERTION = 0, 1, 2, 3, 4
STRATEGY_NAMES = {AUTO: "auto", COUNTING: "counting", RADIX: "radix", QUICK: "quick", INSERTION: "insertion"}
STRATEGY_CODES = {v: k for k, v in STRATEGY_NAMES.items()}
OK, E_INVALID_ARG, E_UNSUPPORTED, E_NAN, E_WORKSPACE, E_OOM, E_DEVICE, E_NO_MODEL, E_PARSE = (
    0, -1, -2, -3, -4, -5, -6, -7, -9)
PRESET_GPU, PRESET_PAPER_TEXT, PRESET_PAPER_TABLE2, PRESET_MI355X_CALIBRATED = 0, 1, 2, 3

# signed tensors sort as signed numbers (sign-bit map); pass dtype=U32 / U64
# explicitly to order a signed tensor's raw bits as unsigned
_TORCH_DTYPES = {torch.uint32: U32, torch.int32: I32, torch.uint64: U64, torch.int64: I64,
                 torch.float32: F32, torch.float64: F64}
_KEY_BYTES = {U32: 4, U64: 8, F32: 4, F64: 8, I32: 4, I64: 8}


class AhsError(RuntimeError):
    def __init__(self, status, message, features=None):
        super().__init__(f"ahs status {status}: {message}")
        self.status = status
        self.features = features


class FeatureVector(C.Structure):
    _fields_ = [("n", C.c_uint64), ("min_key", C.c_uint64), ("max_key", C.c_uint64),
                ("span", C.c_uint64), ("nan_count", C.c_uint64),
                ("shift", C.c_uint32), ("nbins", C.c_uint32), ("exact", C.c_uint32),
                ("reserved", C.c_uint32), ("entropy_bits", C.c_double), ("entropy_ratio", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Config(C.Structure):
    _fields_ = [("n_small", C.c_uint32), ("use_model", C.c_uint32), ("k_count", C.c_uint64),
                ("k_radix", C.c_uint64), ("h_ratio", C.c_double), ("ml_min_n", C.c_uint64),
                ("k_count_cap", C.c_uint64)]


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("max_batch_keys", C.c_uint64),
                ("max_batch_requests", C.c_uint32), ("slots", C.c_uint32), ("autotune", C.c_uint32),
                ("lazy_dispatch", C.c_uint32), ("cfg", Config)]


class ServerResult(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int32), ("chosen", C.c_int32), ("n", C.c_uint64),
                ("dtype", C.c_int32), ("reserved", C.c_int32), ("d_keys_out", C.c_void_p),
                ("d_vals_out", C.c_void_p), ("arrival_ms", C.c_double), ("done_ms", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64),
                ("pending", C.c_uint64), ("running_batches", C.c_uint64), ("batches", C.c_uint64),
                ("keys_completed", C.c_uint64), ("mean_batch_requests", C.c_double),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("max_ms", C.c_double), ("mean_ms", C.c_double),
                ("first_arrival_ms", C.c_double), ("last_done_ms", C.c_double), ("gkeys_per_s", C.c_double),
                ("arena_used_bytes", C.c_uint64), ("arena_peak_bytes", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_lock = threading.Lock()


def lib():
    """Loads libahs.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc for gfx950); there is no fallback implementation")
        L = C.CDLL(LIB_PATH)
        vp, u64, u32, i32, sz = C.c_void_p, C.c_uint64, C.c_uint32, C.c_int, C.c_size_t
        sig = {
            "ahs_config_init": (i32, [C.POINTER(Config), i32]),
            "ahs_context_create": (i32, [i32, C.POINTER(vp)]),
            "ahs_context_destroy": (None, [vp]),
            "ahs_context_set_model": (i32, [vp, vp]),
            "ahs_device_cu_count": (u32, [vp]),
            "ahs_workspace_bytes": (sz, [u64, i32, i32, i32]),
            "ahs_features": (i32, [vp, vp, u64, i32, vp, vp, sz, vp, C.POINTER(FeatureVector)]),
            "ahs_select": (i32, [C.POINTER(FeatureVector), C.POINTER(Config), vp, C.POINTER(C.c_int)]),
            "ahs_sort": (i32, [vp, vp, vp, vp, vp, u64, i32, i32, C.POINTER(Config), vp, sz, vp,
                               C.POINTER(C.c_int), C.POINTER(FeatureVector)]),
            "ahs_sort_static": (i32, [vp, vp, vp, vp, vp, u64, i32, i32, C.POINTER(Config), vp,
                                      C.POINTER(C.c_int), C.POINTER(FeatureVector)]),
            "ahs_segmented_workspace_bytes": (sz, [u64, u32, i32, i32]),
            "ahs_sort_segmented": (i32, [vp, vp, vp, vp, vp, vp, u32, u64, i32, i32, C.POINTER(Config), vp, sz,
                                         vp, vp, vp]),
            "ahs_sort_segmented_async": (i32, [vp, vp, vp, vp, vp, vp, u32, u64, u64, i32, i32, C.POINTER(Config),
                                               vp, sz, vp, vp, vp, vp]),
            "ahs_sort_segmented_capture": (i32, [vp, vp, vp, vp, vp, vp, u32, u64, u64, i32, i32,
                                                 C.POINTER(Config), vp, sz, vp, vp, vp, C.POINTER(vp)]),
            "ahs_graph_launch": (i32, [vp, vp]),
            "ahs_graph_destroy": (None, [vp]),
            "ahs_segmented_autotune": (i32, [vp, i32, i32, vp, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
            "ahs_segmented_get_variants": (i32, [vp, i32, i32, C.POINTER(C.c_int)]),
            "ahs_segmented_set_variants": (i32, [vp, i32, i32, C.POINTER(C.c_int)]),
            "ahs_segmented_get_radix_tile": (i32, [vp, i32, i32, C.POINTER(C.c_uint32)]),
            "ahs_segmented_set_radix_tile": (i32, [vp, i32, i32, u32]),
            "ahs_server_config_init": (None, [C.POINTER(ServerConfig)]),
            "ahs_server_create": (i32, [i32, C.POINTER(ServerConfig), C.POINTER(vp)]),
            "ahs_server_now_ms": (C.c_double, [vp]),
            "ahs_server_submit": (i32, [vp, i32, u64, vp, vp, vp, C.c_double, C.POINTER(C.c_uint64)]),
            "ahs_server_poll": (i32, [vp, C.POINTER(ServerResult), u32, C.POINTER(C.c_uint32), C.c_double]),
            "ahs_server_release": (i32, [vp, u64]),
            "ahs_server_stats": (i32, [vp, C.POINTER(ServerStats)]),
            "ahs_server_destroy": (None, [vp]),
            "ahs_model_load": (i32, [C.c_char_p, C.POINTER(vp)]),
            "ahs_model_free": (None, [vp]),
            "ahs_model_predict": (i32, [vp, C.POINTER(FeatureVector), C.POINTER(C.c_int)]),
            "ahs_profile_enable": (i32, [vp, i32]),
            "ahs_profile_reset": (i32, [vp]),
            "ahs_profile_query": (i32, [vp, C.c_char_p, C.POINTER(C.c_uint64), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]),
            "ahs_profile_dump": (sz, [vp, C.c_char_p, sz]),
            "ahs_status_str": (C.c_char_p, [i32]),
            "ahs_last_error": (C.c_char_p, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        return _lib


def _raise(status, ctx=None, features=None):
    msg = lib().ahs_last_error(ctx.handle).decode() if ctx is not None else lib().ahs_status_str(status).decode()
    raise AhsError(status, msg, features)


def ahs_config_init(preset: int = PRESET_GPU, **overrides) -> Config:
    cfg = Config()
    st = lib().ahs_config_init(C.byref(cfg), preset)
    if st != OK:
        _raise(st)
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


class Model:
    """Tree-ensemble strategy predictor (Sec. III-H) loaded by the library."""

    def __init__(self, path: str):
        h = C.c_void_p()
        st = lib().ahs_model_load(os.fsencode(path), C.byref(h))
        if st != OK:
            raise AhsError(st, f"cannot load model {path}")
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ahs_model_free(self.handle)
            self.handle = None


SELECTOR_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models", "mi355x_selector.gbt")


def default_model() -> "Model":
    """The selector trained on MI355X measurements (models/mi355x_selector.gbt)."""
    return ahs_model_load(SELECTOR_MODEL)


def ahs_model_load(path: str) -> Model:
    return Model(path)


def ahs_model_predict(model: Model, f: FeatureVector) -> int:
    out = C.c_int()
    st = lib().ahs_model_predict(model.handle, C.byref(f), C.byref(out))
    if st != OK:
        _raise(st)
    return out.value


class Context:
    """Host-side library state bound to one HIP device, plus a cached
    device workspace per stream allocated through torch.

    A sort returns with its kernels still enqueued on its stream, so each
    stream gets its own workspace, allocated on that stream: torch's caching
    allocator then never hands a grown-out buffer to another stream while
    the old one's kernels may still run.  Like the C context, one Context is
    driven by one host thread."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        st = lib().ahs_context_create(device, C.byref(h))
        if st != OK:
            raise AhsError(st, f"cannot create a context on device {device}")
        self.handle = h
        self.device = device
        self._ws = {}
        self._model = None

    def workspace(self, nbytes: int, stream=None) -> torch.Tensor:
        dev = torch.device("cuda", self.device)
        s = torch.cuda.current_stream(dev) if stream is None else stream
        ws = self._ws.get(s.cuda_stream)
        if ws is None or ws.numel() < nbytes:
            self._ws.pop(s.cuda_stream, None)
            del ws
            with torch.cuda.stream(s):
                ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
            self._ws[s.cuda_stream] = ws
        return ws

    def set_model(self, model: Model | None):
        self._model = model
        st = lib().ahs_context_set_model(self.handle, model.handle if model else None)
        if st != OK:
            _raise(st, self)

    @property
    def cu_count(self) -> int:
        return lib().ahs_device_cu_count(self.handle)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ahs_context_destroy(self.handle)
            self.handle = None


def ahs_context_create(device: int = 0) -> Context:
    return Context(device)


_default_ctx = {}


def default_context(device: int | None = None) -> Context:
    d = torch.cuda.current_device() if device is None else device
    if d not in _default_ctx:
        _default_ctx[d] = Context(d)
    return _default_ctx[d]


def dtype_code(t: torch.Tensor, dtype: int | None = None) -> int:
    if dtype is not None:
        return dtype
    try:
        return _TORCH_DTYPES[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported key dtype {t.dtype}") from None


def ahs_workspace_bytes(n: int, dtype: int, with_payload: bool, strategy: int = AUTO) -> int:
    return lib().ahs_workspace_bytes(n, dtype, 1 if with_payload else 0, strategy)


def _stream_handle(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _check_keys(keys: torch.Tensor, code: int):
    if not keys.is_cuda or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous device tensor")
    if keys.element_size() != _KEY_BYTES[code]:
        raise ValueError("key tensor element size does not match the dtype")


def ahs_features(keys: torch.Tensor, hist: torch.Tensor | None = None, dtype: int | None = None,
                 ctx: Context | None = None, stream=None) -> FeatureVector:
    """Feature vector of a device key array (Sec. III-A).  ``hist`` (optional,
    >= 65,536 uint32/int32 elements) receives the nbins counts."""
    code = dtype_code(keys, dtype)
    _check_keys(keys, code)
    ctx = ctx or default_context(keys.device.index)
    n = keys.numel()
    if hist is not None and (not hist.is_cuda or hist.numel() < 65536 or hist.element_size() != 4):
        raise ValueError("hist must be a device tensor of at least 65,536 32-bit elements")
    wsb = ahs_workspace_bytes(n, code, False, AUTO)
    ws = ctx.workspace(wsb, stream)
    f = FeatureVector()
    st = lib().ahs_features(ctx.handle, C.c_void_p(keys.data_ptr()), n, code,
                            C.c_void_p(hist.data_ptr()) if hist is not None else None,
                            C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream), C.byref(f))
    if st != OK:
        _raise(st, ctx, f)
    return f


def ahs_select(f: FeatureVector, cfg: Config | None = None, model: Model | None = None) -> int:
    cfg = cfg or ahs_config_init()
    out = C.c_int()
    st = lib().ahs_select(C.byref(f), C.byref(cfg), model.handle if model else None, C.byref(out))
    if st != OK:
        _raise(st)
    return out.value


def ahs_sort(keys: torch.Tensor, values: torch.Tensor | None = None, strategy: int | str = AUTO,
             cfg: Config | None = None, out: torch.Tensor | None = None,
             out_values: torch.Tensor | None = None, dtype: int | None = None,
             ctx: Context | None = None, stream=None, want_features: bool = False):
    """Sorts device keys (and an optional uint32 payload) ascending and stably.

    Returns (keys_out, values_out or None, chosen strategy, FeatureVector or
    None).  ``out``/``out_values`` may alias the inputs (in place)."""
    if isinstance(strategy, str):
        strategy = STRATEGY_CODES[strategy]
    code = dtype_code(keys, dtype)
    _check_keys(keys, code)
    ctx = ctx or default_context(keys.device.index)
    n = keys.numel()
    if out is None:
        out = torch.empty_like(keys)
    if values is not None:
        if values.numel() != n or values.element_size() != 4 or not values.is_cuda or not values.is_contiguous():
            raise ValueError("values must be a contiguous device tensor of n 32-bit elements")
        if out_values is None:
            out_values = torch.empty_like(values)
    elif out_values is not None:
        raise ValueError("out_values given without values")
    wsb = ahs_workspace_bytes(n, code, values is not None, strategy)
    ws = ctx.workspace(wsb, stream)
    chosen = C.c_int()
    f = FeatureVector()
    vp = (lambda t: C.c_void_p(t.data_ptr()) if t is not None else None)
    st = lib().ahs_sort(ctx.handle, vp(keys), vp(out), vp(values), vp(out_values), n, code, strategy,
                        C.byref(cfg) if cfg is not None else None, C.c_void_p(ws.data_ptr()), ws.numel(),
                        _stream_handle(stream), C.byref(chosen), C.byref(f) if want_features else None)
    if st != OK:
        _raise(st, ctx, f if want_features else None)
    return out, out_values, chosen.value, (f if want_features else None)


STATIC_SCRATCH_BYTES = 64 << 20  # AHS_STATIC_SCRATCH_BYTES


def ahs_sort_static(keys: torch.Tensor, out: torch.Tensor, values: torch.Tensor | None = None,
                    out_values: torch.Tensor | None = None, strategy: int | str = AUTO, cfg: Config | None = None,
                    dtype: int | None = None, ctx: Context | None = None, stream=None, want_features: bool = False):
    """ahs_sort with the library's fixed per-device scratch instead of a
    workspace: the call allocates nothing, so the caller passes the outputs.
    Returns (chosen strategy, FeatureVector or None)."""
    if isinstance(strategy, str):
        strategy = STRATEGY_CODES[strategy]
    code = dtype_code(keys, dtype)
    _check_keys(keys, code)
    ctx = ctx or default_context(keys.device.index)
    n = keys.numel()
    if out.numel() != n or out.element_size() != keys.element_size() or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous device tensor shaped like keys")
    if (values is None) != (out_values is None):
        raise ValueError("values and out_values must be given together")
    for t in (values, out_values):
        if t is not None and (t.numel() != n or t.element_size() != 4 or not t.is_cuda or not t.is_contiguous()):
            raise ValueError("payloads must be contiguous device tensors of n 32-bit elements")
    chosen = C.c_int()
    f = FeatureVector()
    vp = (lambda t: C.c_void_p(t.data_ptr()) if t is not None else None)
    st = lib().ahs_sort_static(ctx.handle, vp(keys), vp(out), vp(values), vp(out_values), n, code, strategy,
                               C.byref(cfg) if cfg is not None else None, _stream_handle(stream), C.byref(chosen),
                               C.byref(f) if want_features else None)
    if st != OK:
        _raise(st, ctx, f if want_features else None)
    return chosen.value, (f if want_features else None)


SEG_NAN = 0xFD  # per-segment decision code of a segment that holds NaN keys


def ahs_segmented_workspace_bytes(n_total: int, nseg: int, dtype: int, with_payload: bool) -> int:
    return lib().ahs_segmented_workspace_bytes(n_total, nseg, dtype, 1 if with_payload else 0)


SEG_ERR_OFFSETS, SEG_ERR_OVERFLOW, SEG_ERR_LEVELS, SEG_ERR_HINT = 1, 2, 4, 8  # bits of the enqueue-only status word


def _seg_prepare(keys, offsets, values, strategy, out, out_values, dtype, ctx, want_chosen, want_features):
    if isinstance(strategy, str):
        strategy = STRATEGY_CODES[strategy]
    code = dtype_code(keys, dtype)
    _check_keys(keys, code)
    if not offsets.is_cuda or not offsets.is_contiguous() or offsets.element_size() != 8 or offsets.dim() != 1:
        raise ValueError("offsets must be a contiguous 1-D device tensor of 64-bit elements")
    nseg = offsets.numel() - 1
    if nseg < 0:
        raise ValueError("offsets needs at least one element")
    ctx = ctx or default_context(keys.device.index)
    n = keys.numel()
    if out is None:
        out = torch.empty_like(keys)
    if values is not None:
        if values.numel() != n or values.element_size() != 4 or not values.is_cuda or not values.is_contiguous():
            raise ValueError("values must be a contiguous device tensor of n 32-bit elements")
        if out_values is None:
            out_values = torch.empty_like(values)
    elif out_values is not None:
        raise ValueError("out_values given without values")
    chosen = torch.empty(nseg, dtype=torch.uint8, device=keys.device) if want_chosen else None
    feats = (torch.empty(nseg * C.sizeof(FeatureVector), dtype=torch.uint8, device=keys.device)
             if want_features else None)
    return strategy, code, nseg, n, ctx, out, out_values, chosen, feats


def ahs_sort_segmented(keys: torch.Tensor, offsets: torch.Tensor, values: torch.Tensor | None = None,
                       strategy: int | str = AUTO, cfg: Config | None = None, out: torch.Tensor | None = None,
                       out_values: torch.Tensor | None = None, dtype: int | None = None,
                       ctx: Context | None = None, stream=None, want_chosen: bool = True,
                       want_features: bool = False):
    """Sorts nseg independent segments of one device array in one call.

    ``offsets`` is a device int64/uint64 tensor of nseg + 1 non-decreasing
    boundaries ending at keys.numel().  Returns (keys_out, values_out or None,
    chosen (device uint8 tensor of nseg decisions) or None, features (device
    tensor of nseg FeatureVector records, viewed as bytes) or None)."""
    strategy, code, nseg, n, ctx, out, out_values, chosen, feats = _seg_prepare(
        keys, offsets, values, strategy, out, out_values, dtype, ctx, want_chosen, want_features)
    wsb = ahs_segmented_workspace_bytes(n, nseg, code, values is not None)
    ws = ctx.workspace(wsb, stream)
    vp = (lambda t: C.c_void_p(t.data_ptr()) if t is not None else None)
    st = lib().ahs_sort_segmented(ctx.handle, vp(keys), vp(out), vp(values), vp(out_values), vp(offsets), nseg, n,
                                  code, strategy, C.byref(cfg) if cfg is not None else None,
                                  C.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream), vp(chosen),
                                  vp(feats))
    if st != OK:
        _raise(st, ctx)
    return out, out_values, chosen, feats


def ahs_sort_segmented_async(keys: torch.Tensor, offsets: torch.Tensor, values: torch.Tensor | None = None,
                             strategy: int | str = AUTO, cfg: Config | None = None, out: torch.Tensor | None = None,
                             out_values: torch.Tensor | None = None, dtype: int | None = None,
                             ctx: Context | None = None, stream=None, max_seg_hint: int = 0,
                             want_chosen: bool = True, want_features: bool = False, ws: torch.Tensor | None = None):
    """Enqueue-only batched sort (no host synchronisation).  Returns (keys_out,
    values_out, chosen, features, status) where status is a device uint32
    tensor of one element: 0 on success, else SEG_ERR_* bits.  ``ws`` (a
    device byte tensor of at least ahs_segmented_workspace_bytes) keeps the
    workspace fixed across calls; by default the context's is used."""
    strategy, code, nseg, n, ctx, out, out_values, chosen, feats = _seg_prepare(
        keys, offsets, values, strategy, out, out_values, dtype, ctx, want_chosen, want_features)
    wsb = ahs_segmented_workspace_bytes(n, nseg, code, values is not None)
    if ws is None:
        ws = ctx.workspace(wsb, stream)
    status = torch.empty(1, dtype=torch.int32, device=keys.device)
    vp = (lambda t: C.c_void_p(t.data_ptr()) if t is not None else None)
    st = lib().ahs_sort_segmented_async(ctx.handle, vp(keys), vp(out), vp(values), vp(out_values), vp(offsets), nseg,
                                        n, max_seg_hint, code, strategy,
                                        C.byref(cfg) if cfg is not None else None, C.c_void_p(ws.data_ptr()),
                                        ws.numel(), _stream_handle(stream), vp(chosen), vp(feats), vp(status))
    if st != OK:
        _raise(st, ctx)
    return out, out_values, chosen, feats, status


class SegmentedGraph:
    """hipGraph of one enqueue-only batched sort over fixed buffers.  The
    object keeps every buffer the graph uses alive; launch() replays it."""

    def __init__(self, keys, offsets, values=None, strategy=AUTO, cfg=None, out=None, out_values=None, dtype=None,
                 ctx=None, max_seg_hint=0, want_chosen=True, want_features=False):
        strategy, code, nseg, n, ctx, out, out_values, chosen, feats = _seg_prepare(
            keys, offsets, values, strategy, out, out_values, dtype, ctx, want_chosen, want_features)
        self.ws = torch.empty(ahs_segmented_workspace_bytes(n, nseg, code, values is not None), dtype=torch.uint8,
                              device=keys.device)
        self.status = torch.zeros(1, dtype=torch.int32, device=keys.device)
        self.keys, self.offsets, self.values, self.out, self.out_values = keys, offsets, values, out, out_values
        self.chosen, self.feats, self.ctx, self.cfg = chosen, feats, ctx, cfg
        torch.cuda.synchronize(keys.device)
        vp = (lambda t: C.c_void_p(t.data_ptr()) if t is not None else None)
        h = C.c_void_p()
        st = lib().ahs_sort_segmented_capture(ctx.handle, vp(keys), vp(out), vp(values), vp(out_values),
                                              vp(offsets), nseg, n, max_seg_hint, code, strategy,
                                              C.byref(cfg) if cfg is not None else None,
                                              C.c_void_p(self.ws.data_ptr()), self.ws.numel(), vp(chosen),
                                              vp(feats), vp(self.status), C.byref(h))
        if st != OK:
            _raise(st, ctx)
        self.handle = h

    def launch(self, stream=None):
        st = lib().ahs_graph_launch(self.handle, _stream_handle(stream))
        if st != OK:
            _raise(st)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ahs_graph_destroy(self.handle)
            self.handle = None


def ahs_segmented_autotune(dtype: int, with_payload: bool = False, ctx: Context | None = None, stream=None):
    """Times every admissible LDS kernel variant per size class and keeps the
    fastest in the context.  Returns ([capacity per class], [ms per class])."""
    ctx = ctx or default_context()
    caps = (C.c_int * 4)()
    ms = (C.c_double * 4)()
    st = lib().ahs_segmented_autotune(ctx.handle, dtype, 1 if with_payload else 0, _stream_handle(stream), caps, ms)
    if st != OK:
        _raise(st, ctx)
    return list(caps), list(ms)


def ahs_segmented_get_variants(dtype: int, with_payload: bool = False, ctx: Context | None = None):
    ctx = ctx or default_context()
    caps = (C.c_int * 4)()
    st = lib().ahs_segmented_get_variants(ctx.handle, dtype, 1 if with_payload else 0, caps)
    if st != OK:
        _raise(st, ctx)
    return list(caps)


def ahs_segmented_set_variants(dtype: int, caps, with_payload: bool = False, ctx: Context | None = None):
    ctx = ctx or default_context()
    arr = (C.c_int * 4)(*caps)
    st = lib().ahs_segmented_set_variants(ctx.handle, dtype, 1 if with_payload else 0, arr)
    if st != OK:
        _raise(st, ctx)


def ahs_segmented_get_radix_tile(dtype: int, with_payload: bool = False, ctx: Context | None = None) -> int:
    """Keys per tile of the batched sort's segmented radix passes."""
    ctx = ctx or default_context()
    out = C.c_uint32()
    st = lib().ahs_segmented_get_radix_tile(ctx.handle, dtype, 1 if with_payload else 0, C.byref(out))
    if st != OK:
        _raise(st, ctx)
    return out.value


def ahs_segmented_set_radix_tile(dtype: int, keys_per_tile: int, with_payload: bool = False,
                                 ctx: Context | None = None):
    ctx = ctx or default_context()
    st = lib().ahs_segmented_set_radix_tile(ctx.handle, dtype, 1 if with_payload else 0, keys_per_tile)
    if st != OK:
        _raise(st, ctx)


class Server:
    """The serving loop (continuous batching under an HBM budget).  Results
    are device tensors viewing the server's arena, valid until release()."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int | None = None, max_batch_keys: int | None = None,
                 max_batch_requests: int | None = None, slots: int | None = None, autotune: bool = False,
                 lazy_dispatch: bool = False, cfg: Config | None = None):
        c = ServerConfig()
        lib().ahs_server_config_init(C.byref(c))
        if hbm_budget_bytes is not None:
            c.hbm_budget_bytes = hbm_budget_bytes
        if max_batch_keys is not None:
            c.max_batch_keys = max_batch_keys
        if max_batch_requests is not None:
            c.max_batch_requests = max_batch_requests
        if slots is not None:
            c.slots = slots
        c.autotune = 1 if autotune else 0
        c.lazy_dispatch = 1 if lazy_dispatch else 0
        if cfg is not None:
            c.cfg = cfg
        h = C.c_void_p()
        st = lib().ahs_server_create(device, C.byref(c), C.byref(h))
        if st != OK:
            _raise(st)
        self.handle = h
        self.device = device
        self._inputs = {}  # id -> tensors kept alive until completion

    def now_ms(self) -> float:
        return lib().ahs_server_now_ms(self.handle)

    def submit(self, keys: torch.Tensor, values: torch.Tensor | None = None, dtype: int | None = None,
               arrival_ms: float = -1.0, stream=None) -> int:
        code = dtype_code(keys, dtype)
        _check_keys(keys, code)
        if values is not None and (values.numel() != keys.numel() or values.element_size() != 4
                                   or not values.is_contiguous()):
            raise ValueError("values must be a contiguous device tensor of n 32-bit elements")
        rid = C.c_uint64()
        st = lib().ahs_server_submit(self.handle, code, keys.numel(), C.c_void_p(keys.data_ptr()),
                                     C.c_void_p(values.data_ptr()) if values is not None else None,
                                     _stream_handle(stream), arrival_ms, C.byref(rid))
        if st != OK:
            _raise(st)
        self._inputs[rid.value] = (keys, values)
        return rid.value

    def poll(self, max_results: int = 256, wait_ms: float = 0.0) -> list:
        """Finished requests as dicts: id, status, chosen, n, dtype, keys and
        values (device tensors viewing the arena), arrival_ms, done_ms."""
        arr = (ServerResult * max_results)()
        cnt = C.c_uint32()
        st = lib().ahs_server_poll(self.handle, arr, max_results, C.byref(cnt), wait_ms)
        if st != OK:
            _raise(st)
        out = []
        for i in range(cnt.value):
            r = arr[i]
            keys = vals = None
            if r.status == OK:
                keys = _device_view(r.d_keys_out, r.n, _KEY_TORCH[r.dtype], self.device)
                if r.dtype == U32:
                    keys = keys.view(torch.uint32)
                elif r.dtype == U64:
                    keys = keys.view(torch.uint64)
                if r.d_vals_out:
                    vals = _device_view(r.d_vals_out, r.n, torch.int32, self.device).view(torch.uint32)
            self._inputs.pop(r.id, None)
            out.append({"id": r.id, "status": r.status, "chosen": r.chosen, "n": r.n, "dtype": r.dtype,
                        "keys": keys, "values": vals, "arrival_ms": r.arrival_ms, "done_ms": r.done_ms})
        return out

    def release(self, rid: int):
        st = lib().ahs_server_release(self.handle, rid)
        if st != OK:
            _raise(st)

    def stats(self) -> dict:
        s = ServerStats()
        st = lib().ahs_server_stats(self.handle, C.byref(s))
        if st != OK:
            _raise(st)
        return s.as_dict()

    def close(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ahs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


_KEY_TORCH = {U32: torch.int32, U64: torch.int64, F32: torch.float32, F64: torch.float64, I32: torch.int32,
              I64: torch.int64}


class _DevBuf:
    """Minimal __cuda_array_interface__ holder for memory owned by the library."""

    def __init__(self, ptr, n, typestr, device):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False), "version": 3,
                                         "strides": None, "stream": None}
        self.device = device


def _device_view(ptr: int, n: int, tdtype, device: int) -> torch.Tensor:
    """A torch tensor aliasing n elements at a device address the library owns."""
    typestr = {torch.int32: "<i4", torch.int64: "<i8", torch.float32: "<f4", torch.float64: "<f8"}[tdtype]
    if n == 0:
        return torch.empty(0, dtype=tdtype, device=f"cuda:{device}")
    with torch.cuda.device(device):
        return torch.as_tensor(_DevBuf(ptr, n, typestr, device), device=f"cuda:{device}")


def feature_records(feats: torch.Tensor) -> list:
    """Host list of FeatureVector from the byte tensor ahs_sort_segmented returns."""
    raw = feats.cpu().numpy().tobytes()
    sz = C.sizeof(FeatureVector)
    return [FeatureVector.from_buffer_copy(raw[i:i + sz]) for i in range(0, len(raw), sz)]


def ahs_profile_enable(ctx: Context, on: bool = True):
    lib().ahs_profile_enable(ctx.handle, 1 if on else 0)


def ahs_profile_reset(ctx: Context):
    lib().ahs_profile_reset(ctx.handle)


def ahs_profile_query(ctx: Context, kernel: str):
    """(launches, total_ms, algorithmic_bytes) of one kernel family."""
    n = C.c_uint64()
    ms = C.c_double()
    b = C.c_double()
    lib().ahs_profile_query(ctx.handle, kernel.encode(), C.byref(n), C.byref(ms), C.byref(b))
    return n.value, ms.value, b.value


def ahs_profile_dump(ctx: Context) -> dict:
    """{kernel: (launches, total_ms, algorithmic_bytes)} for every kernel seen."""
    need = lib().ahs_profile_dump(ctx.handle, None, 0)
    buf = C.create_string_buffer(need)
    lib().ahs_profile_dump(ctx.handle, buf, need)
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms, nbytes = line.split()
        out[name] = (int(cnt), float(ms), float(nbytes))
    return out
