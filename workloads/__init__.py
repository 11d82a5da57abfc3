"""Seeded synthetic inputs for the binar sort workloads.

The arrays come from counter-based SplitMix64 streams in ``gen.c`` (built
with gcc into ``libbinar_workloads.so`` next to it).  This module draws keys,
sizes and arrival times only; it holds none of the sorting arithmetic.

The workloads follow the paper's experiment (random 32-bit integers, section
"Performance of Algorithm") widened to the key widths and distributions the
GPU path is measured on: uniform, low-entropy (AND of four words), heavy
duplicates, nearly sorted, Zipf, batched lognormal segments and a mixed
serving stream.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

BASE_SEED = 0x08113448

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libbinar_workloads.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile gen.c with gcc (seconds); returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        u64, u32, dbl, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p
        sig = {
            "wl_u64_stream": (None, [u64, u64, u64, vp]),
            "wl_u32_uniform": (None, [u64, u64, vp]),
            "wl_u32_and4": (None, [u64, u64, vp]),
            "wl_u32_dup": (ctypes.c_int, [u64, u64, u32, vp]),
            "wl_u64_uniform": (None, [u64, u64, vp]),
            "wl_u64_nearly_sorted": (ctypes.c_int, [u64, u64, dbl, vp]),
            "wl_u64_zipf": (ctypes.c_int, [u64, u64, u32, dbl, vp]),
            "wl_lognormal_sizes": (None, [u64, u64, dbl, dbl, u64, u64, vp]),
            "wl_exponential": (None, [u64, u64, dbl, vp]),
            "wl_str16": (None, [u64, u64, u32, vp]),
            "wl_below": (None, [u64, u64, u64, vp]),
            "wl_iota_u32": (None, [u64, u64, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _check(rc: int) -> None:
    if rc != 0:
        raise RuntimeError("workload generator failed with status %d" % rc)


# ----------------------------------------------------------------- primitives
def stream_u64(seed: int, n: int, start: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _L().wl_u64_stream(seed, start, n, _ptr(out))
    return out


def u32_uniform(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    _L().wl_u32_uniform(seed, n, _ptr(out))
    return out


def u32_and4(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    _L().wl_u32_and4(seed, n, _ptr(out))
    return out


def u32_dup(n: int, seed: int, npool: int = 256) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    _check(_L().wl_u32_dup(seed, n, npool, _ptr(out)))
    return out


def u64_uniform(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _L().wl_u64_uniform(seed, n, _ptr(out))
    return out


def u64_nearly_sorted(n: int, seed: int, frac: float = 0.01) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _check(_L().wl_u64_nearly_sorted(seed, n, frac, _ptr(out)))
    return out


def u64_zipf(n: int, seed: int, npool: int = 1 << 20, s: float = 1.1) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _check(_L().wl_u64_zipf(seed, n, npool, s, _ptr(out)))
    return out


def lognormal_sizes(count: int, seed: int, median: float, sigma: float, lo: int, hi: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _L().wl_lognormal_sizes(seed, count, median, sigma, lo, hi, _ptr(out))
    return out


def exponential(count: int, seed: int, mean: float) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _L().wl_exponential(seed, count, mean, _ptr(out))
    return out


def str16(n: int, seed: int, prefix_len: int) -> np.ndarray:
    """n fixed 16-byte lowercase strings, shape (n, 16) uint8."""
    out = np.empty((n, 16), dtype=np.uint8)
    _L().wl_str16(seed, n, prefix_len, _ptr(out))
    return out


def below(n: int, seed: int, m: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _L().wl_below(seed, n, m, _ptr(out))
    return out


def iota_u32(n: int, start: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    _L().wl_iota_u32(start, n, _ptr(out))
    return out


def small_alphabet_u32(n: int, seed: int, alphabet) -> np.ndarray:
    """Keys drawn uniformly from a given small alphabet (forces ties)."""
    alphabet = np.asarray(alphabet, dtype=np.uint32)
    return alphabet[below(n, seed, len(alphabet)).astype(np.int64)]


def f32_normal(n: int, seed: int) -> np.ndarray:
    """float32 draws from N(0, 1) (Box-Muller on two uniform streams), as
    uint32 bit patterns."""
    u1 = (stream_u64(seed, n) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    u2 = (stream_u64(seed + 1, n) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
    return z.astype(np.float32).view(np.uint32)


# ------------------------------------------------------------ named workloads
# Each entry: name -> (key_bytes, n, has_payload, description).  Seeds are
# BASE_SEED + the workload's index in this table.
SINGLE = {
    "u32_2e16_uniform_keys": (4, 1 << 16, False, "2^16 uniform u32, keys only"),
    "u32_2e28_uniform": (4, 1 << 28, True, "2^28 uniform u32 + u32 index payload"),
    "u32_2e28_and4": (4, 1 << 28, True, "2^28 u32 = AND of 4 uniform words + index payload"),
    "u32_2e28_dup256": (4, 1 << 28, True, "2^28 u32 drawn from 256 distinct values + index payload"),
    "u64_2e27_uniform": (8, 1 << 27, True, "2^27 uniform u64 + u32 index payload"),
    "u64_2e27_nearly_sorted": (8, 1 << 27, True, "2^27 sorted u64 with 1% positions swapped + index"),
    "u64_2e27_zipf": (8, 1 << 27, True, "2^27 u64 Zipf(1.1) over 2^20 distinct values + index"),
    "f32_2e28_normal": (4, 1 << 28, True, "2^28 float32 N(0, 1) values (IEEE-754 order) + index payload"),
}


def single_keys(name: str, n: int | None = None) -> np.ndarray:
    """Keys of a named single-array workload (optionally at a smaller n)."""
    kb, n_full, _, _ = SINGLE[name]
    n = n_full if n is None else n
    seed = BASE_SEED + list(SINGLE).index(name)
    dist = name.split("_", 2)[2]
    if name.startswith("f32"):
        return f32_normal(n, seed)
    if kb == 4:
        if dist.startswith("uniform"):
            return u32_uniform(n, seed)
        if dist == "and4":
            return u32_and4(n, seed)
        if dist == "dup256":
            return u32_dup(n, seed, 256)
    else:
        if dist == "uniform":
            return u64_uniform(n, seed)
        if dist == "nearly_sorted":
            return u64_nearly_sorted(n, seed, 0.01)
        if dist == "zipf":
            return u64_zipf(n, seed, 1 << 20, 1.1)
    raise KeyError(name)


BATCHED_SEGMENTS = 100_000
BATCHED_MEDIAN = 1024.0
BATCHED_SIGMA = 0.7356


def batched_u32(num_segments: int = BATCHED_SEGMENTS, seed: int = BASE_SEED + 3,
                median: float = BATCHED_MEDIAN, sigma: float = BATCHED_SIGMA,
                max_len: int = 1 << 20):
    """Batched workload: lognormal segment sizes, uniform u32 keys per segment,
    global index payload.  Returns (keys u32, seg_offsets u64 of length S+1)."""
    sizes = lognormal_sizes(num_segments, seed, median, sigma, 1, max_len)
    offsets = np.zeros(num_segments + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offsets[1:])
    keys = u32_uniform(int(offsets[-1]), seed + 1000)
    return keys, offsets


def var_strings(n: int, seed: int, mean_len: float = 20.0, alphabet: int = 26, shared_prefix: int = 0):
    """n variable-length strings: lognormal lengths (median mean_len / e^0.18,
    sigma 0.6, at most 200), lowercase letters from an alphabet of the given
    size, optionally a prefix of shared_prefix bytes common to all.
    Returns (data uint8, offsets uint32 of n + 1 entries)."""
    lens = lognormal_sizes(n, seed, mean_len / np.exp(0.18), 0.6, 0, 200).astype(np.int64)
    offs = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(lens + shared_prefix, out=offs[1:])
    total = int(offs[-1])
    letters = (ord("a") + below(total, seed + 1, alphabet)).astype(np.uint8)
    if shared_prefix:
        pre = (ord("a") + below(shared_prefix, seed + 2, 26)).astype(np.uint8)
        starts = offs[:-1].astype(np.int64)
        for j in range(shared_prefix):
            letters[starts + j] = pre[j]
    return letters, offs.astype(np.uint32)


SERVE_KINDS = ((4, 0.5), (8, 0.3), (16, 0.2))


def serve_requests(count: int, seed: int = BASE_SEED + 4, rate_per_s: float = 1000.0,
                   median: float = 65536.0, sigma: float = 2.0 * np.log(2.0),
                   lo: int = 1 << 8, hi: int = 1 << 24):
    """Serving stream: Poisson arrival times (s), lognormal sizes, key widths
    mixed 50/30/20 over 4/8/16 bytes, and a prefix length U{0..12} per string
    request.  Keys are drawn lazily by request_keys()."""
    gaps = exponential(count, seed, 1.0 / rate_per_s)
    arrivals = np.cumsum(gaps)
    sizes = lognormal_sizes(count, seed + 1, median, sigma, lo, hi)
    u = below(count, seed + 2, 100)
    kinds = np.where(u < 50, 4, np.where(u < 80, 8, 16)).astype(np.int64)
    prefix = below(count, seed + 3, 13).astype(np.int64)
    return [
        {"id": i, "arrival_s": float(arrivals[i]), "n": int(sizes[i]), "key_bytes": int(kinds[i]),
         "prefix_len": int(prefix[i]), "seed": int(seed + 10_000 + i)}
        for i in range(count)
    ]


def request_keys(req) -> np.ndarray:
    """Keys of one serving request: u32 / u64 uniform, or (n, 16) strings."""
    kb, n, s = req["key_bytes"], req["n"], req["seed"]
    if kb == 4:
        return u32_uniform(n, s)
    if kb == 8:
        return u64_uniform(n, s)
    return str16(n, s, req["prefix_len"])
