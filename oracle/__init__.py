"""CPU oracle for binar sort -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_0811_3448_amd``) and never imports it.

Contents
--------
* ``binar_ref.c`` (built with gcc into ``libbinar_oracle.so``): the paper's
  recursive binar partition, one bit per level, MSB first, made stable
  (sections "Operation of Algorithm" and "Optimize the Algorithm").  Wrapped
  here as :func:`sort`, :func:`partition`, :func:`sort_bits` and
  :func:`sort_segmented`.
* ``definition.py``: the plain definition of the result (section "Sorting
  Formalism" with a stability tie-break), written with Python's sort.
* ``swap_partition.py``: the paper's own unstable exchange partition, written
  from its prose, used to check the printed worked example.
* ``baselines.cpp`` (built with g++ together with ``binar_ref.c`` into
  ``libbinar_baselines.so``): two CPU reference timings for the benchmark,
  :func:`stable_sort_ref` (``std::stable_sort`` on one thread) and
  :func:`parallel_sort_ref` (the paper's parallel variant: one stable
  partition on the leading byte, then the buckets on several threads).

Key arrays: ``uint32`` (4-byte keys), ``uint64`` (8-byte keys) or ``uint8``
of shape (n, 16) (16-byte strings in memcmp order).  Payloads are ``uint32``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "binar_ref.c")
_LIB = os.path.join(_HERE, "libbinar_oracle.so")
_BSRC = os.path.join(_HERE, "baselines.cpp")
_BLIB = os.path.join(_HERE, "libbinar_baselines.so")
_lib = None
_blib = None


def _stale(lib, *srcs):
    return not os.path.exists(lib) or any(os.path.getmtime(lib) < os.path.getmtime(s) for s in srcs)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc and the CPU baselines with g++ (seconds);
    returns the oracle library's path."""
    if force or _stale(_LIB, _SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    if force or _stale(_BLIB, _SRC, _BSRC):
        tmp = _BLIB + ".tmp%d" % os.getpid()
        obj = tmp + ".o"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-c", "-o", obj, _SRC])
        try:
            subprocess.check_call(["g++", "-O2", "-std=c++17", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
                                   "-o", tmp, _BSRC, obj])
        finally:
            os.remove(obj)
        os.replace(tmp, _BLIB)
    return _LIB


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        lib.binar_sort_ref.argtypes = [vp, u32, u64, vp, vp]
        lib.binar_partition_ref.argtypes = [vp, u32, u64, vp, u32, vp]
        lib.binar_sort_bits_ref.argtypes = [vp, u32, u64, vp, u32, vp]
        lib.binar_sort_segmented_ref.argtypes = [vp, u32, vp, u64, vp]
        for f in (lib.binar_sort_ref, lib.binar_partition_ref, lib.binar_sort_bits_ref,
                  lib.binar_sort_segmented_ref):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def key_bytes_of(keys: np.ndarray) -> int:
    if keys.dtype == np.uint32 and keys.ndim == 1:
        return 4
    if keys.dtype == np.uint64 and keys.ndim == 1:
        return 8
    if keys.dtype == np.uint8 and keys.ndim == 2 and keys.shape[1] == 16:
        return 16
    raise TypeError("keys must be uint32[n], uint64[n] or uint8[n, 16]")


def _prep(keys, payload):
    k = np.ascontiguousarray(keys).copy()
    p = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint32).copy()
    if p is not None and p.shape[0] != k.shape[0]:
        raise ValueError("payload length differs from key count")
    return k, p


def _pp(p):
    return None if p is None else p.ctypes.data


def _check(rc):
    if rc != 0:
        raise RuntimeError("oracle failed with status %d" % rc)


def sort(keys: np.ndarray, payload: np.ndarray | None = None, with_steps: bool = False):
    """Stable binar sort; returns (keys, payload) copies (payload None if not given)."""
    k, p = _prep(keys, payload)
    steps = ctypes.c_uint64(0)
    _check(_L().binar_sort_ref(k.ctypes.data, key_bytes_of(k), k.shape[0], _pp(p),
                               ctypes.byref(steps)))
    return (k, p, steps.value) if with_steps else (k, p)


def partition(keys: np.ndarray, payload: np.ndarray | None, nbits: int):
    """State after stable partitions on the leading ``nbits`` bits only."""
    k, p = _prep(keys, payload)
    _check(_L().binar_partition_ref(k.ctypes.data, key_bytes_of(k), k.shape[0], _pp(p),
                                    nbits, None))
    return k, p


def sort_bits(keys: np.ndarray, key_bits: int, payload: np.ndarray | None = None,
              nbits: int | None = None, with_steps: bool = False):
    """Stable binar sort of unsigned ``key_bits``-wide keys held in uint64."""
    k, p = _prep(np.asarray(keys, dtype=np.uint64), payload)
    steps = ctypes.c_uint64(0)
    _check(_L().binar_sort_bits_ref(k.ctypes.data, key_bits, k.shape[0], _pp(p),
                                    key_bits if nbits is None else nbits, ctypes.byref(steps)))
    return (k, p, steps.value) if with_steps else (k, p)


def sort_segmented(keys: np.ndarray, seg_offsets: np.ndarray, payload: np.ndarray | None = None):
    """Every segment [off[s], off[s+1]) sorted on its own."""
    k, p = _prep(keys, payload)
    off = np.ascontiguousarray(seg_offsets, dtype=np.uint64)
    _check(_L().binar_sort_segmented_ref(k.ctypes.data, key_bytes_of(k), off.ctypes.data,
                                         off.shape[0] - 1, _pp(p)))
    return k, p


def _B():
    global _blib
    if _blib is None:
        build()
        lib = ctypes.CDLL(_BLIB)
        vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        lib.ref_stable_sort.argtypes = [vp, u32, u64, vp]
        lib.ref_parallel_binar.argtypes = [vp, u32, u64, vp, ctypes.c_int]
        lib.ref_stable_sort.restype = ctypes.c_int
        lib.ref_parallel_binar.restype = ctypes.c_int
        _blib = lib
    return _blib


def stable_sort_ref(keys: np.ndarray, payload: np.ndarray | None = None):
    """CPU baseline: std::stable_sort of (key, payload) pairs on one thread."""
    k, p = _prep(keys, payload)
    _check(_B().ref_stable_sort(k.ctypes.data, key_bytes_of(k), k.shape[0], _pp(p)))
    return k, p


def parallel_sort_ref(keys: np.ndarray, payload: np.ndarray | None = None, threads: int = 1):
    """CPU baseline: the paper's parallel variant (one stable partition on the
    leading byte, then each bucket by the oracle's binar sort, on ``threads``
    threads)."""
    k, p = _prep(keys, payload)
    _check(_B().ref_parallel_binar(k.ctypes.data, key_bytes_of(k), k.shape[0], _pp(p), int(threads)))
    return k, p
