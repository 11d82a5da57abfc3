"""Signed and IEEE-754 keys on the GPU against the oracle's by-value orders
(oracle.orders): keys bit-exact (the caller's bits come back unchanged) and
permutation exact."""
import numpy as np
import pytest

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


def float_bits(n, seed, width):
    """Floats of many magnitudes and both signs, with zeros of both signs,
    infinities, NaNs of both signs and several payloads, subnormals, and
    repeated values, as uint bit patterns."""
    rng = np.random.default_rng(seed)
    ft = np.float32 if width == 32 else np.float64
    ut = np.uint32 if width == 32 else np.uint64
    v = (rng.standard_normal(n) * 10.0 ** rng.integers(-20, 20, n)).astype(ft)
    bits = v.view(ut).copy()
    sb = 1 << (width - 1)
    expo = ((1 << (8 if width == 32 else 11)) - 1) << (23 if width == 32 else 52)
    special = [0, sb, expo, expo | sb, expo | 1, expo | (1 << (22 if width == 32 else 51)),
               sb | expo | 5, sb | expo | (1 << (22 if width == 32 else 51)), 1, sb | 1, sb | 7]
    idx = rng.integers(0, n, n // 10)
    bits[idx] = np.array(special, dtype=ut)[rng.integers(0, len(special), idx.shape[0])]
    dup = rng.integers(0, n, n // 10)
    bits[dup] = bits[rng.integers(0, n, dup.shape[0])]
    return bits


def int_bits(n, seed, width):
    rng = np.random.default_rng(seed)
    it = np.int32 if width == 32 else np.int64
    info = np.iinfo(it)
    v = rng.integers(info.min, info.max, n, dtype=it, endpoint=True)
    v[rng.integers(0, n, n // 10)] = rng.choice(np.array([info.min, info.max, -1, 0, 1], dtype=it), n // 10)
    v[rng.integers(0, n, n // 10)] = rng.integers(-300, 300, n // 10).astype(it)
    return v.view(np.uint32 if width == 32 else np.uint64)


def check(keys, kind, **kw):
    n = keys.shape[0]
    pay = np.arange(n, dtype=np.uint32)
    print("kind=%d n=%d width=%d %s" % (kind, n, keys.dtype.itemsize * 8, kw), flush=True)
    gk, gp = gpu_sort(keys, pay, params=P(key_kind=kind, **kw))
    rk, rp = orders.sort(keys, pay, kind)
    assert np.array_equal(gp, rp), "permutation differs"
    assert np.array_equal(gk, rk), "keys differ"


@pytest.mark.parametrize("width", [32, 64])
@pytest.mark.parametrize("kind", [orders.SIGNED, orders.FLOAT])
@pytest.mark.parametrize("T", [0, 300])
def test_kinds(width, kind, T):
    n = 200_003
    keys = float_bits(n, 11 + width, width) if kind == orders.FLOAT else int_bits(n, 12 + width, width)
    check(keys, kind, finish_max=T)


@pytest.mark.parametrize("kind", [orders.SIGNED, orders.FLOAT])
def test_kinds_lookback_and_narrow_digits(kind):
    keys = float_bits(150_001, 21, 32) if kind == orders.FLOAT else int_bits(150_001, 22, 32)
    check(keys, kind, finish_max=100, offsets=2)
    check(keys, kind, finish_max=100, digit_bits=5, tile_keys=4096)


@pytest.mark.parametrize("kind", [orders.SIGNED, orders.FLOAT])
def test_kinds_segmented(kind):
    _, off = workloads.batched_u32(400, seed=31, median=400, sigma=1.0, max_len=20_000)
    n = int(off[-1])
    keys = float_bits(n, 32, 64) if kind == orders.FLOAT else int_bits(n, 33, 64)
    pay = np.arange(n, dtype=np.uint32)
    gk, gp = gpu_sort_segmented(keys, off, pay, params=P(key_kind=kind))
    rk, rp = orders.sort_segmented(keys, off, pay, kind)
    assert np.array_equal(gp, rp) and np.array_equal(gk, rk)


def test_float_tensors_sort_by_value():
    """A float tensor is read as IEEE-754 without being told."""
    import torch
    import paper_0811_3448_amd as binar
    bits = float_bits(50_000, 41, 32)
    t = torch.from_numpy(bits.view(np.float32)).cuda()
    p = torch.arange(50_000, dtype=torch.int32, device="cuda")
    binar.sort(t, p)
    torch.cuda.synchronize()
    rk, rp = orders.sort(bits, np.arange(50_000, dtype=np.uint32), orders.FLOAT)
    assert np.array_equal(t.cpu().numpy().view(np.uint32), rk)
    assert np.array_equal(p.cpu().numpy().view(np.uint32), rp)


def test_plan_with_kind():
    import torch
    import paper_0811_3448_amd as binar
    _, off = workloads.batched_u32(100, seed=51, median=300, sigma=1.0, max_len=5000)
    n = int(off[-1])
    keys = int_bits(n, 52, 32)
    kd = torch.from_numpy(keys.view(np.int32)).cuda()
    pd = torch.arange(n, dtype=torch.int32, device="cuda")
    od = torch.from_numpy(off.astype(np.uint32).view(np.int32)).cuda()
    plan = binar.Plan(4, n, 100, True, binar.Params(key_kind=binar.KEY_SIGNED))
    plan.sort(kd, pd, od)
    torch.cuda.synchronize()
    rk, rp = orders.sort_segmented(keys, off, np.arange(n, dtype=np.uint32), orders.SIGNED)
    assert np.array_equal(kd.cpu().numpy().view(np.uint32), rk)
    assert np.array_equal(pd.cpu().numpy().view(np.uint32), rp)
    plan.close()
