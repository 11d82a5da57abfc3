"""ctypes binding of libbinar.so (argument marshalling only).

The library must have been built (``python paper_0811_3448_amd/build.py``);
importing this module without it raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbinar.so")

BINAR_OK, BINAR_EINVAL, BINAR_ERANGE, BINAR_ENOMEM, BINAR_EDEVICE = 0, -1, -2, -3, -4
MAX_KEYS = (1 << 30) - 1


class _Params(ctypes.Structure):
    _fields_ = [("digit_bits", ctypes.c_uint32), ("tile_keys", ctypes.c_uint32),
                ("finish_max", ctypes.c_uint32), ("offsets", ctypes.c_uint32),
                ("key_bits", ctypes.c_uint32), ("key_kind", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 2)]


class _Stats(ctypes.Structure):
    _fields_ = [("moved", ctypes.c_uint64 * 16), ("hist_keys", ctypes.c_uint64 * 16),
                ("finish_keys", ctypes.c_uint64), ("finish_segments", ctypes.c_uint64),
                ("passes", ctypes.c_uint32), ("status", ctypes.c_int32),
                ("finish_class_keys", ctypes.c_uint64 * 4), ("finish_class_segments", ctypes.c_uint64 * 4),
                ("copyback_keys", ctypes.c_uint64), ("sorted_keys", ctypes.c_uint64),
                ("finish_small_keys", ctypes.c_uint64), ("finish_small_segments", ctypes.c_uint64)]


class _LaunchTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("pass_", ctypes.c_int32), ("ms", ctypes.c_float)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbinar.so is not built (%s); run python paper_0811_3448_amd/build.py" % LIB_PATH)
    # torch brings its own HIP runtime; load it first so that the library's
    # HIP runtime dependency resolves to the copy torch's tensors and streams
    # live in.  Loaded the other way round, the library's runtime has been
    # seen to find no device in a process where torch finds one.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, sz, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int
    P = ctypes.POINTER(_Params)
    L.binar_sort.argtypes = [vp, u32, u64, vp]
    L.binar_sort_async.argtypes = [vp, u32, u64, vp, vp, vp, sz]
    L.binar_sort_static.argtypes = [vp, u32, u64, vp, vp]
    L.binar_stream_copy.argtypes = [vp, vp, sz, u32, u32, vp]
    L.binar_stream_read.argtypes = [vp, sz, vp, u32, u32, vp]
    L.binar_sort_segmented.argtypes = [vp, u32, vp, u32, u64, vp, vp, vp, sz]
    L.binar_sort_ex.argtypes = [vp, u32, u64, vp, vp, u32, P, vp, vp, sz]
    L.binar_workspace_bytes.argtypes = [u32, u64, i32, u32, P]
    L.binar_workspace_bytes.restype = sz
    L.binar_stats_read.argtypes = [vp, vp, ctypes.POINTER(_Stats)]
    L.binar_get_default_params.argtypes = [u32, i32, P]
    L.binar_set_default_params.argtypes = [u32, i32, P]
    L.binar_resolve_params.argtypes = [u32, i32, P, P]
    L.binar_profile_enable.argtypes = [i32]
    L.binar_profile_read.argtypes = [ctypes.POINTER(_LaunchTime), u32, ctypes.POINTER(u32)]
    L.binar_plan_create.argtypes = [ctypes.POINTER(vp), u32, u64, u32, i32, P]
    L.binar_plan_sort.argtypes = [vp, vp, vp, vp, u32, u64, vp]
    L.binar_plan_stats.argtypes = [vp, vp, ctypes.POINTER(_Stats)]
    L.binar_plan_graphs.argtypes = [vp]
    L.binar_plan_status_async.argtypes = [vp, vp, vp]
    L.binar_plan_workspace_bytes.argtypes = [vp]
    L.binar_plan_workspace_bytes.restype = sz
    L.binar_plan_destroy.argtypes = [vp]
    L.binar_plan_destroy.restype = None
    L.binar_strerror.argtypes = [i32]
    L.binar_strerror.restype = ctypes.c_char_p
    L.binar_sort_strings.argtypes = [vp, u64, vp, u64, vp, vp, vp, sz]
    L.binar_sort_strings.restype = i32
    L.binar_strings_workspace_bytes.argtypes = [u64]
    L.binar_strings_workspace_bytes.restype = sz
    L.binar_sort_inplace.argtypes = [vp, u32, u64, vp, P, vp, vp, sz]
    L.binar_inplace_workspace_bytes.argtypes = [u32, u64, i32, P]
    L.binar_inplace_workspace_bytes.restype = sz
    L.binar_last_error.argtypes = []
    L.binar_last_error.restype = ctypes.c_char_p
    for f in ("binar_sort", "binar_sort_async", "binar_sort_static", "binar_stream_copy", "binar_stream_read",
              "binar_sort_segmented", "binar_sort_ex",
              "binar_stats_read", "binar_get_default_params", "binar_set_default_params", "binar_resolve_params",
              "binar_profile_enable", "binar_profile_read", "binar_plan_create", "binar_plan_sort",
              "binar_plan_stats", "binar_plan_graphs", "binar_plan_status_async"):
        getattr(L, f).restype = i32
    return L


lib = _load()


class BinarError(RuntimeError):
    def __init__(self, status: int):
        self.status = status
        detail = lib.binar_last_error().decode() if status == BINAR_EDEVICE else ""
        super().__init__("binar: %s (status %d)%s" % (strerror(status), status, "; " + detail if detail else ""))


def strerror(status: int) -> str:
    return lib.binar_strerror(status).decode()


def _check(rc: int) -> None:
    if rc != BINAR_OK:
        raise BinarError(rc)


OFFSETS_CHUNKED, OFFSETS_LOOKBACK = 1, 2
KEY_UNSIGNED, KEY_SIGNED, KEY_FLOAT = 0, 1, 2


@dataclass
class Params:
    """Tuning knobs (0 = library default) and the key kind; see binar_params
    in binar.h."""
    digit_bits: int = 0
    tile_keys: int = 0
    finish_max: int = 0
    offsets: int = 0
    key_bits: int = 0
    key_kind: int = 0

    def c(self):
        return _Params(self.digit_bits, self.tile_keys, self.finish_max, self.offsets, self.key_bits,
                       self.key_kind)


def key_bytes_of(keys) -> int:
    """4 / 8 for 1-D tensors of 4- / 8-byte elements, 16 for uint8 (n, 16)."""
    import torch
    if keys.dim() == 1 and keys.element_size() in (4, 8):
        return keys.element_size()
    if keys.dim() == 2 and keys.dtype == torch.uint8 and keys.shape[1] == 16:
        return 16
    raise ValueError("keys must be 1-D with 4- or 8-byte elements, or uint8 of shape (n, 16)")


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def key_kind_of(keys, params: "Params | None", key_kind: int | None) -> "Params | None":
    """Params carrying the key kind: the explicit key_kind, else the one in
    params, else KEY_FLOAT for floating-point tensors (their bits read as
    unsigned integers would not be in numeric order).  Integer tensors are
    read as unsigned unless told otherwise (torch has no uint32 tensors, so
    int32 storage often holds unsigned keys)."""
    import torch
    if key_kind is None:
        if params is not None and params.key_kind:
            return params
        if keys.dtype in (torch.float32, torch.float64):
            key_kind = KEY_FLOAT
        else:
            return params
    p = Params() if params is None else Params(**vars(params))
    p.key_kind = key_kind
    return p


_TUNED = {"cache": None, "loaded": False}


def tuned_params(key_bytes: int, has_payload: bool, n: int, batched: bool = False) -> "Params | None":
    """Parameters the autotune cache holds for this case (nearest size bucket
    within one), for this device; None without a matching cache or when the
    environment sets BINAR_AUTOTUNE=0."""
    if os.environ.get("BINAR_AUTOTUNE", "1") == "0":
        return None
    if not _TUNED["loaded"]:
        _TUNED["loaded"] = True
        try:
            from . import tune
            c = tune.TuneCache(arch=tune.device_arch())
            _TUNED["cache"] = c if c.entries else None
        except Exception:  # no readable cache for this device: library defaults
            _TUNED["cache"] = None
    c = _TUNED["cache"]
    return None if c is None else c.lookup(key_bytes, has_payload, n, batched, max_distance=1)


def _with_tuning(params, key_bytes, has_payload, n, batched):
    """params as given, or the tuned ones for this case (keeping any key kind)."""
    if params is not None and (params.digit_bits or params.tile_keys or params.finish_max or params.offsets):
        return params
    t = tuned_params(key_bytes, has_payload, n, batched)
    if t is None:
        return params
    if params is not None:
        t.key_bits, t.key_kind = params.key_bits, params.key_kind
    return t


def _check_tensors(keys, payload):
    if not keys.is_cuda or not keys.is_contiguous():
        raise ValueError("keys must be a contiguous device tensor")
    if payload is not None:
        if not payload.is_cuda or not payload.is_contiguous() or payload.element_size() != 4 \
                or payload.dim() != 1 or payload.shape[0] != keys.shape[0]:
            raise ValueError("payload must be a contiguous 1-D 4-byte device tensor of the keys' length")


class Workspace:
    """Caller-owned scratch: a device uint8 tensor of the required size."""

    def __init__(self, nbytes: int, device=None):
        import torch
        self.nbytes = int(nbytes)
        self.tensor = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device or "cuda")

    @property
    def ptr(self):
        return ctypes.c_void_p(self.tensor.data_ptr())


def workspace_bytes(key_bytes: int, n: int, has_payload: bool, num_segments: int = 1,
                    params: Params | None = None) -> int:
    p = None if params is None else ctypes.byref(params.c())
    return int(lib.binar_workspace_bytes(key_bytes, n, 1 if has_payload else 0, num_segments, p))


def sort(keys, payload=None, stream=None, workspace: Workspace | None = None,
         params: Params | None = None, key_kind: int | None = None):
    """Sort keys (and payload) in place on `stream` (default: torch's current
    stream).  Returns keys.  Asynchronous like any torch op.  key_kind: see
    key_kind_of."""
    _check_tensors(keys, payload)
    params = key_kind_of(keys, params, key_kind)
    kb = key_bytes_of(keys)
    n = keys.shape[0]
    if workspace is None:
        # the library's pool grows to fit: tuned parameters are safe to use
        params = _with_tuning(params, kb, payload is not None, n, False)
    ws = (None, 0) if workspace is None else (workspace.ptr, workspace.nbytes)
    pp = None if params is None else ctypes.byref(params.c())
    _check(lib.binar_sort_ex(_dev_ptr(keys), kb, n, _dev_ptr(payload), None, 0, pp,
                             _stream_ptr(stream), ws[0], ws[1]))
    return keys


def sort_segmented(keys, seg_offsets, payload=None, stream=None, workspace: Workspace | None = None,
                   params: Params | None = None, key_kind: int | None = None):
    """Sort every segment [off[s], off[s+1]) of keys independently, in place.
    seg_offsets: device int32/uint32 tensor of S + 1 nondecreasing offsets."""
    _check_tensors(keys, payload)
    params = key_kind_of(keys, params, key_kind)
    if not seg_offsets.is_cuda or seg_offsets.element_size() != 4 or seg_offsets.dim() != 1 \
            or not seg_offsets.is_contiguous():
        raise ValueError("seg_offsets must be a contiguous 1-D 4-byte device tensor")
    kb = key_bytes_of(keys)
    n = keys.shape[0]
    nseg = seg_offsets.shape[0] - 1
    if nseg < 0:
        raise ValueError("seg_offsets needs at least one entry")
    ws = (None, 0) if workspace is None else (workspace.ptr, workspace.nbytes)
    pp = None if params is None else ctypes.byref(params.c())
    _check(lib.binar_sort_ex(_dev_ptr(keys), kb, n, _dev_ptr(payload), _dev_ptr(seg_offsets), nseg, pp,
                             _stream_ptr(stream), ws[0], ws[1]))
    return keys


def sort_inplace(keys, payload=None, stream=None, workspace: Workspace | None = None,
                 params: Params | None = None, key_kind: int | None = None):
    """Stable sort like sort(), with no scratch copy of the keys: the passes
    permute inside keys and payload themselves.  params: digit_bits 0/4/8,
    tile_keys 0/4096, offsets 0/1.  Returns keys."""
    _check_tensors(keys, payload)
    params = key_kind_of(keys, params, key_kind)
    kb = key_bytes_of(keys)
    ws = (None, 0) if workspace is None else (workspace.ptr, workspace.nbytes)
    pp = None if params is None else ctypes.byref(params.c())
    _check(lib.binar_sort_inplace(_dev_ptr(keys), kb, keys.shape[0], _dev_ptr(payload), pp,
                                  _stream_ptr(stream), ws[0], ws[1]))
    return keys


def inplace_workspace_bytes(key_bytes: int, n: int, has_payload: bool, params: Params | None = None) -> int:
    pp = None if params is None else ctypes.byref(params.c())
    return int(lib.binar_inplace_workspace_bytes(key_bytes, n, 1 if has_payload else 0, pp))


def strings_workspace_bytes(n: int) -> int:
    return int(lib.binar_strings_workspace_bytes(n))


def sort_strings(data, offsets, payload, stream=None, workspace: Workspace | None = None):
    """Sort n variable-length byte strings -- string i is
    data[offsets[i]:offsets[i+1]] -- in memcmp order (a proper prefix
    first, equal strings in input order) and permute payload with them in
    place.  data: device uint8 tensor; offsets: device 4-byte tensor of
    n + 1 offsets; payload: device 4-byte tensor of n entries (pass
    0..n-1 to receive the sorting permutation).  Blocks until done."""
    import torch
    if not data.is_cuda or data.dtype != torch.uint8 or data.dim() != 1 or not data.is_contiguous():
        raise ValueError("data must be a contiguous 1-D uint8 device tensor")
    if not offsets.is_cuda or offsets.element_size() != 4 or offsets.dim() != 1 or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous 1-D 4-byte device tensor")
    n = offsets.shape[0] - 1
    if n < 0:
        raise ValueError("offsets needs at least one entry")
    if not payload.is_cuda or payload.element_size() != 4 or payload.dim() != 1 or payload.shape[0] != n \
            or not payload.is_contiguous():
        raise ValueError("payload must be a contiguous 1-D 4-byte device tensor of n entries")
    ws = (None, 0) if workspace is None else (workspace.ptr, workspace.nbytes)
    _check(lib.binar_sort_strings(_dev_ptr(data), data.shape[0], _dev_ptr(offsets), n, _dev_ptr(payload),
                                  _stream_ptr(stream), ws[0], ws[1]))
    return payload


def stats(workspace: Workspace | None = None, stream=None) -> dict:
    """Counters of the last call on `workspace` (None: this device's pool)."""
    s = _Stats()
    _check(lib.binar_stats_read(None if workspace is None else workspace.ptr, _stream_ptr(stream),
                                ctypes.byref(s)))
    return _stats_dict(s)


def profile_enable(on: bool = True) -> None:
    """Bracket every library kernel launch with HIP events on its stream."""
    _check(lib.binar_profile_enable(1 if on else 0))


def profile_read(cap: int = 1 << 16) -> list:
    """[(name, pass, ms)] of the launches timed since the last read."""
    buf = (_LaunchTime * cap)()
    cnt = ctypes.c_uint32(0)
    _check(lib.binar_profile_read(buf, cap, ctypes.byref(cnt)))
    return [(buf[i].name.decode(), buf[i].pass_, float(buf[i].ms)) for i in range(cnt.value)]


def _stats_dict(s: "_Stats") -> dict:
    return {"moved": list(s.moved), "hist_keys": list(s.hist_keys), "finish_keys": s.finish_keys,
            "finish_segments": s.finish_segments, "passes": s.passes, "status": s.status,
            "finish_class_keys": list(s.finish_class_keys),
            "finish_class_segments": list(s.finish_class_segments), "copyback_keys": s.copyback_keys,
            "sorted_keys": s.sorted_keys, "finish_small_keys": s.finish_small_keys,
            "finish_small_segments": s.finish_small_segments}


def status_of_words(error: int, overflow: int) -> int:
    """Status code of a sort from its two device status words (the error
    flags and the list-overflow flag, see binar_plan_status_async)."""
    if error & 1:
        return BINAR_EINVAL
    return BINAR_EDEVICE if (error or overflow) else BINAR_OK


class Plan:
    """Reusable sort plan on resident buffers: the first sort with a given
    set of buffers captures a HIP graph, later sorts replay it (see
    binar_plan_* in binar.h)."""

    def __init__(self, key_bytes: int, max_keys: int, max_segments: int = 1, has_payload: bool = True,
                 params: Params | None = None):
        self._h = ctypes.c_void_p()
        pp = None if params is None else ctypes.byref(params.c())
        _check(lib.binar_plan_create(ctypes.byref(self._h), key_bytes, max_keys, max_segments,
                                     1 if has_payload else 0, pp))
        self.key_bytes, self.max_keys, self.max_segments = key_bytes, max_keys, max_segments

    def sort(self, keys, payload=None, seg_offsets=None, n_total: int | None = None, stream=None):
        """Sort on the plan's graph.  Single array (seg_offsets None): n_total
        keys (default: all of keys).  Segmented: keys and payload must hold the
        plan's max_keys entries; n_total is then ignored."""
        _check_tensors(keys, payload)
        if key_bytes_of(keys) != self.key_bytes:
            raise ValueError("key width differs from the plan's")
        n = keys.shape[0] if n_total is None else n_total
        nseg = 0
        if seg_offsets is not None:
            # segmented: the buffers must hold the plan's whole capacity (the
            # device checks the offsets against it, not against n_total)
            if keys.shape[0] < self.max_keys:
                raise ValueError("segmented plan sort: keys hold %d entries, the plan's capacity is %d"
                                 % (keys.shape[0], self.max_keys))
            if not seg_offsets.is_cuda or seg_offsets.element_size() != 4 or not seg_offsets.is_contiguous():
                raise ValueError("seg_offsets must be a contiguous 4-byte device tensor")
            nseg = seg_offsets.shape[0] - 1
            n = keys.shape[0]
        _check(lib.binar_plan_sort(self._h, _dev_ptr(keys), _dev_ptr(payload), _dev_ptr(seg_offsets), nseg, n,
                                   _stream_ptr(stream)))
        return keys

    def stats(self, stream=None) -> dict:
        s = _Stats()
        _check(lib.binar_plan_stats(self._h, _stream_ptr(stream), ctypes.byref(s)))
        return _stats_dict(s)

    def status_async(self, host_words, stream=None) -> None:
        """Enqueue on `stream` a copy of the last sort's two status words
        into `host_words` (a pinned int32 CPU tensor of two elements); read
        them with status_of_words once the stream has passed the copy."""
        if (host_words.is_cuda or host_words.element_size() != 4 or host_words.numel() < 2
                or not host_words.is_contiguous()):
            raise ValueError("host_words must be a contiguous 4-byte host tensor of two elements")
        _check(lib.binar_plan_status_async(self._h, _stream_ptr(stream), ctypes.c_void_p(host_words.data_ptr())))

    @property
    def graphs(self) -> int:
        return int(lib.binar_plan_graphs(self._h))

    @property
    def workspace_bytes(self) -> int:
        return int(lib.binar_plan_workspace_bytes(self._h))

    def close(self):
        if self._h:
            lib.binar_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_params(key_bytes: int, has_payload: bool) -> Params:
    p = _Params()
    _check(lib.binar_get_default_params(key_bytes, 1 if has_payload else 0, ctypes.byref(p)))
    return Params(p.digit_bits, p.tile_keys, p.finish_max, p.offsets)


def resolve_params(key_bytes: int, has_payload: bool, params: Params | None = None) -> Params:
    """The parameters a call with `params` would run with, all fields set."""
    p = _Params()
    _check(lib.binar_resolve_params(key_bytes, 1 if has_payload else 0,
                                    None if params is None else ctypes.byref(params.c()), ctypes.byref(p)))
    return Params(p.digit_bits, p.tile_keys, p.finish_max, p.offsets, p.key_bits, p.key_kind)


def set_default_params(key_bytes: int, has_payload: bool, params: Params) -> None:
    _check(lib.binar_set_default_params(key_bytes, 1 if has_payload else 0, ctypes.byref(params.c())))
