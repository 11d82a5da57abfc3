"""GPU parity of the small-sub-array path: sub-arrays of 2..64 keys are
ranked inside one 64-lane wave, many packed into a wave at once.  Segment
length mixes that straddle the 64-key limit and a wave's 64-entry window,
heavy ties (stability), every key width with and without payload, partial
key bits, signed and float keys, and the counters that split the work
between the small path and the LDS classes."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import gpu_sort, gpu_sort_segmented, need_gpu
from oracle import orders

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def P(**kw):
    from paper_0811_3448_amd import Params
    return Params(**kw)


def iota(n):
    return np.arange(n, dtype=np.uint32)


def small_offsets(nseg, seed, hi=70):
    """Segment table of nseg segments, lengths uniform on 0..hi (empty and
    one-key segments included), with a run of 64-key and 65-key segments."""
    lens = workloads.below(nseg, seed, hi + 1).astype(np.int64)
    lens[5:40] = 64
    lens[40:60] = 65
    lens[60:70] = 1
    off = np.zeros(nseg + 1, dtype=np.uint32)
    off[1:] = np.cumsum(lens)
    return off


def keys_of(kb, n, seed, distinct):
    """n keys of kb bytes drawn from `distinct` values (ties inside segments)."""
    pick = workloads.below(n, seed, distinct).astype(np.int64)
    pool = {4: lambda: workloads.u32_uniform(distinct, seed + 1),
            8: lambda: workloads.u64_uniform(distinct, seed + 1),
            16: lambda: workloads.str16(distinct, seed + 1, 3)}[kb]()
    return pool[pick]


@pytest.mark.parametrize("kb", [4, 8, 16])
@pytest.mark.parametrize("pay", [True, False])
@pytest.mark.parametrize("distinct", [3, 1 << 20])
def test_segmented_small(kb, pay, distinct):
    off = small_offsets(5000, 900 + kb, 70)
    n = int(off[-1])
    keys = keys_of(kb, n, 910 + kb, distinct)
    print("small segmented kb=%d pay=%d distinct=%d n=%d" % (kb, pay, distinct, n), flush=True)
    gk, gp = gpu_sort_segmented(keys, off, iota(n) if pay else None)
    rk, rp = oracle.sort_segmented(keys, off, iota(n) if pay else None)
    assert np.array_equal(gk, rk)
    if pay:
        assert np.array_equal(gp, rp)


@pytest.mark.parametrize("kb", [4, 8, 16])
def test_small_after_passes(kb):
    """finish_max 64: every sub-array a pass leaves with 2..64 keys is ranked
    by a wave, and none goes to an LDS class."""
    import paper_0811_3448_amd as binar
    n = 300_007
    keys = {4: lambda: workloads.u32_uniform(n, 920), 8: lambda: workloads.u64_zipf(n, 921, 1 << 14, 1.1),
            16: lambda: workloads.str16(n, 922, 4)}[kb]()
    print("small after passes kb=%d n=%d" % (kb, n), flush=True)
    gk, gp = gpu_sort(keys, iota(n), params=P(finish_max=64))
    st = binar.stats()
    rk, rp = oracle.sort(keys, iota(n))
    assert np.array_equal(gk, rk) and np.array_equal(gp, rp)
    assert sum(st["finish_class_segments"]) == 0
    assert st["finish_small_segments"] == st["finish_segments"] > 0


def test_small_counts_split_from_classes():
    import paper_0811_3448_amd as binar
    off = small_offsets(3000, 930, 200)
    n = int(off[-1])
    lens = np.diff(off.astype(np.int64))
    keys = workloads.u32_uniform(n, 931)
    gk, gp = gpu_sort_segmented(keys, off, iota(n))
    st = binar.stats()
    rk, rp = oracle.sort_segmented(keys, off, iota(n))
    assert np.array_equal(gk, rk) and np.array_equal(gp, rp)
    small = (lens >= 2) & (lens <= 64)
    assert st["finish_small_segments"] == int(small.sum())
    assert st["finish_small_keys"] == int(lens[small].sum())
    assert st["finish_class_segments"][0] == int((lens > 64).sum())
    assert st["finish_keys"] == int(lens[lens >= 2].sum())


@pytest.mark.parametrize("nbits", [3, 12, 20])
def test_small_partial_bits(nbits):
    """Keys equal on the leading nbits bits keep input order in the small
    path too."""
    n = 100_003
    keys = workloads.u32_uniform(n, 940 + nbits)
    pay = iota(n)
    gk, gp = gpu_sort(keys, pay, params=P(key_bits=nbits, finish_max=64, digit_bits=4, tile_keys=4096))
    rk, rp = oracle.partition(keys, pay, nbits)
    assert np.array_equal(gp, rp) and np.array_equal(gk, rk)


@pytest.mark.parametrize("kind", [orders.SIGNED, orders.FLOAT])
def test_small_kinds(kind):
    off = small_offsets(3000, 950, 70)
    n = int(off[-1])
    rng = np.random.default_rng(951)
    if kind == orders.FLOAT:
        v = (rng.standard_normal(n) * 10.0 ** rng.integers(-5, 5, n)).astype(np.float32)
        v[rng.integers(0, n, n // 20)] = np.float32(-0.0)
        v[rng.integers(0, n, n // 20)] = np.float32(np.inf)
        keys = v.view(np.uint32).copy()
    else:
        keys = rng.integers(-50, 50, n, dtype=np.int32).view(np.uint32)
    pay = iota(n)
    gk, gp = gpu_sort_segmented(keys, off, pay, params=P(key_kind=kind))
    rk, rp = orders.sort_segmented(keys, off, pay, kind)
    assert np.array_equal(gp, rp) and np.array_equal(gk, rk)


@pytest.mark.parametrize("kb", [4, 8, 16])
def test_wave_finish_long_tied_runs(kb):
    """Sub-arrays of 65..1024 keys (one wave each for 4- and 8-byte keys)
    whose keys share their leading varying bits in two or three long runs:
    the ranking of tied runs gives way to passes over every varying bit.
    Full-key ties too (stability)."""
    rng = np.random.default_rng(980 + kb)
    lens = rng.integers(65, 1025, 300)
    off = np.zeros(lens.shape[0] + 1, dtype=np.uint32)
    off[1:] = np.cumsum(lens)
    n = int(off[-1])
    seg = np.repeat(np.arange(lens.shape[0]), lens)
    leads = rng.integers(0, 1 << 16, (lens.shape[0], 3), dtype=np.uint64)
    lead = leads[seg, rng.integers(0, 3, n)]
    low = rng.integers(0, 1 << 20, n, dtype=np.uint64)
    low[rng.random(n) < 0.2] = 5
    if kb == 4:
        keys = ((lead << np.uint64(16)) | (low & np.uint64(0xFFFF))).astype(np.uint32)
    elif kb == 8:
        keys = ((lead << np.uint64(48)) | low).astype(np.uint64)
    else:
        words = np.stack([(lead << np.uint64(48)) | low, low * np.uint64(0x9E3779B97F4A7C15)], axis=1)
        keys = words.astype(">u8").view(np.uint8).reshape(n, 16).copy()
    print("wave finish long runs kb=%d n=%d" % (kb, n), flush=True)
    gk, gp = gpu_sort_segmented(keys, off, iota(n))
    rk, rp = oracle.sort_segmented(keys, off, iota(n))
    assert np.array_equal(gk, rk)
    assert np.array_equal(gp, rp)
