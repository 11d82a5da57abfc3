"""GPU per-pass parity: sorting by the leading B bits only must reproduce the
oracle's state after partitioning on the first B bits (stable by those bits,
input order among keys equal in them), for every B at a pass boundary and
in between."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import gpu_sort, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def P(**kw):
    from paper_0811_3448_amd import Params
    return Params(**kw)


def check_partial(keys, nbits, **kw):
    n = keys.shape[0]
    pay = np.arange(n, dtype=np.uint32)
    print("partial n=%d kb=%d nbits=%d %s" % (n, oracle.key_bytes_of(keys), nbits, kw), flush=True)
    gk, gp = gpu_sort(keys, pay, params=P(key_bits=nbits, **kw))
    rk, rp = oracle.partition(keys, pay, nbits)
    assert np.array_equal(gp, rp), "permutation differs after %d bits" % nbits
    assert np.array_equal(gk, rk)


@pytest.mark.parametrize("offsets", [1, 2])
@pytest.mark.parametrize("dist", ["uniform", "and4"])
@pytest.mark.parametrize("T", [0, 1, 64])
def test_u32_after_each_pass(offsets, dist, T):
    n = 100_003
    keys = workloads.u32_uniform(n, 5) if dist == "uniform" else workloads.u32_and4(n, 6)
    for nbits in (8, 16, 24, 32, 5, 13):
        check_partial(keys, nbits, finish_max=T, offsets=offsets)


@pytest.mark.parametrize("k", [1, 4, 5, 7])
def test_u32_binary_steps(k):
    """k = 1 is the paper's one-bit partition, made stable."""
    n = 50_001
    keys = workloads.u32_and4(n, 7)
    for nbits in (1, 2, 3, 7, 12, 32):
        check_partial(keys, nbits, digit_bits=k, finish_max=100)


@pytest.mark.parametrize("kb", [8, 16])
def test_wide_keys_partial(kb):
    n = 70_001
    keys = workloads.u64_zipf(n, 8, 1 << 10, 1.1) if kb == 8 else workloads.str16(n, 9, 6)
    for nbits in (8, 20, 48, 64, 8 * kb):
        check_partial(keys, min(nbits, 8 * kb), finish_max=200)


@pytest.mark.parametrize("kb,nbits", [(8, 48), (8, 33), (16, 72), (16, 100)])
def test_partial_ties_inside_finish(kb, nbits):
    """One sub-array finished on chip whose keys vary over many leading bits,
    in groups that agree on all nbits leading bits and differ after them:
    the tied runs left by the on-chip digit passes must be ordered by the
    leading nbits bits only, equal keys there keeping input order."""
    rng = np.random.default_rng(nbits)
    n = 4001
    pool = rng.integers(0, 1 << 63, (250, kb // 8), dtype=np.uint64)
    rows = pool[rng.integers(0, 250, n)]
    # bits from nbits on are noise
    noise = rng.integers(0, 1 << 63, (n, kb // 8), dtype=np.uint64)
    lead = nbits
    for wd in range(kb // 8):
        hi_bits = min(max(lead - 64 * wd, 0), 64)
        keep = np.uint64(0) if hi_bits == 0 else np.uint64(((1 << 64) - 1) ^ ((1 << (64 - hi_bits)) - 1))
        rows[:, wd] = (rows[:, wd] & keep) | (noise[:, wd] & ~keep)
    if kb == 8:
        keys = rows[:, 0].copy()
    else:
        keys = rows.astype(">u8").view(np.uint8).reshape(n, 16).copy()
    check_partial(keys, nbits)
    check_partial(keys, nbits, finish_max=64)
