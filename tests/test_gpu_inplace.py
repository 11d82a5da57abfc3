"""GPU parity of the in-place variant: each pass sorts every tile by its
digit in LDS, writes it back over itself and applies the pass's permutation
by following its cycles, with no scratch copy of the keys.  The result must
equal the oracle's stable sort exactly, for every key width, with and
without payload, on uniform, duplicate-heavy, sorted, reversed, all-equal
and tiny inputs, partial key bits and signed / float keys; the workspace is
a small fraction of the ping-pong one."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import need_gpu, to_dev, to_host
from oracle import orders

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def P(**kw):
    from paper_0811_3448_amd import Params
    return Params(**kw)


def ip_sort(keys, payload=None, params=None):
    import torch
    import paper_0811_3448_amd as binar
    kd, pd = to_dev(keys), to_dev(payload)
    binar.sort_inplace(kd, pd, params=params)
    torch.cuda.synchronize()
    st = binar.stats()
    if keys.shape[0] >= 2:
        assert st["status"] == 0
    return to_host(kd, keys), (None if payload is None else to_host(pd, payload)), st


def compare(keys, with_payload=True, **kw):
    n = keys.shape[0]
    pay = np.arange(n, dtype=np.uint32) if with_payload else None
    print("inplace n=%d kb=%d pay=%d %s" % (n, oracle.key_bytes_of(keys), with_payload, kw), flush=True)
    gk, gp, st = ip_sort(keys, pay, params=P(**kw) if kw else None)
    rk, rp = oracle.sort(keys, pay)
    assert np.array_equal(gk, rk)
    if with_payload:
        assert np.array_equal(gp, rp)
    return st


@pytest.mark.parametrize("n", [2, 63, 64, 65, 300, 4095, 4097, 70_001])
def test_sizes_u32(n):
    compare(workloads.u32_uniform(n, 700 + n))


@pytest.mark.parametrize("dist", ["uniform", "and4", "dup", "sorted", "reversed", "equal"])
def test_u32_distributions(dist):
    n = 1_000_003
    base = workloads.u32_uniform(n, 710)
    keys = {"uniform": lambda: base, "and4": lambda: workloads.u32_and4(n, 711),
            "dup": lambda: base[workloads.below(n, 712, 64).astype(np.int64)],
            "sorted": lambda: np.sort(base), "reversed": lambda: np.sort(base)[::-1].copy(),
            "equal": lambda: np.full(n, 12345, dtype=np.uint32)}[dist]()
    st = compare(keys)
    if dist == "uniform":
        assert st["passes"] >= 1 and st["moved"][0] == n


@pytest.mark.parametrize("kb", [4, 8, 16])
@pytest.mark.parametrize("pay", [True, False])
def test_widths(kb, pay):
    n = 600_001
    keys = {4: lambda: workloads.u32_uniform(n, 720), 8: lambda: workloads.u64_zipf(n, 721, 1 << 16, 1.1),
            16: lambda: workloads.str16(n, 722, 4)}[kb]()
    compare(keys, with_payload=pay)


@pytest.mark.parametrize("T", [0, 256, 1000])
def test_finish_max(T):
    compare(workloads.u64_uniform(400_009, 730 + T), finish_max=T)


@pytest.mark.parametrize("nbits", [5, 16, 40])
def test_partial_bits(nbits):
    n = 300_007
    keys = workloads.u64_uniform(n, 740 + nbits)
    pay = np.arange(n, dtype=np.uint32)
    gk, gp, _ = ip_sort(keys, pay, params=P(key_bits=nbits))
    rk, rp = oracle.partition(keys, pay, nbits)
    assert np.array_equal(gp, rp) and np.array_equal(gk, rk)


@pytest.mark.parametrize("kind", [orders.SIGNED, orders.FLOAT])
def test_kinds(kind):
    n = 250_001
    rng = np.random.default_rng(750 + kind)
    if kind == orders.FLOAT:
        v = (rng.standard_normal(n) * 10.0 ** rng.integers(-10, 10, n)).astype(np.float32)
        v[rng.integers(0, n, n // 50)] = np.float32(-0.0)
        v[rng.integers(0, n, n // 50)] = np.float32(np.inf)
        keys = v.view(np.uint32).copy()
    else:
        keys = rng.integers(-(1 << 31), (1 << 31) - 1, n, dtype=np.int64).astype(np.int32).view(np.uint32)
    pay = np.arange(n, dtype=np.uint32)
    gk, gp, _ = ip_sort(keys, pay, params=P(key_kind=kind))
    rk, rp = orders.sort(keys, pay, kind)
    assert np.array_equal(gp, rp) and np.array_equal(gk, rk)


def test_rejects_other_shapes():
    import torch
    import paper_0811_3448_amd as binar
    k = torch.zeros(1000, dtype=torch.int32, device="cuda")
    for bad in (P(digit_bits=5), P(digit_bits=1), P(tile_keys=8192), P(offsets=2)):
        with pytest.raises(binar.BinarError):
            binar.sort_inplace(k, params=bad)


def test_workspace_is_small():
    import paper_0811_3448_amd as binar
    n = 1 << 28
    ip = binar.inplace_workspace_bytes(4, n, True)
    pp = binar.workspace_bytes(4, n, True)
    assert ip < 0.25 * 8 * n < pp


@pytest.mark.parametrize("k", [4, 8])
@pytest.mark.parametrize("kb", [4, 8, 16])
def test_digit_widths(k, kb):
    """4-bit digits: twice the passes, runs of one digit sixteen times longer."""
    n = 500_003
    keys = {4: lambda: workloads.u32_and4(n, 760), 8: lambda: workloads.u64_uniform(n, 761),
            16: lambda: workloads.str16(n, 762, 5)}[kb]()
    compare(keys, digit_bits=k)
    compare(keys, with_payload=False, digit_bits=k, finish_max=300)


def test_digit_4_partial_and_kinds():
    n = 200_003
    keys = workloads.u64_uniform(n, 770)
    pay = np.arange(n, dtype=np.uint32)
    gk, gp, _ = ip_sort(keys, pay, params=P(key_bits=22, digit_bits=4))
    rk, rp = oracle.partition(keys, pay, 22)
    assert np.array_equal(gp, rp) and np.array_equal(gk, rk)
    rng = np.random.default_rng(771)
    ik = rng.integers(-1000, 1000, n, dtype=np.int64).astype(np.int32).view(np.uint32)
    gk, gp, _ = ip_sort(ik, pay, params=P(key_kind=orders.SIGNED, digit_bits=4))
    rk, rp = orders.sort(ik, pay, orders.SIGNED)
    assert np.array_equal(gp, rp) and np.array_equal(gk, rk)


@pytest.mark.parametrize("nbits", [12, 40, 100])
def test_partial_bits_16_bytes(nbits):
    """16-byte keys in place, sorted by their leading nbits bits only (the
    walk's digits come from the leading bits of each key's first bytes)."""
    n = 150_001
    keys = workloads.str16(n, 780 + nbits, 3)
    pay = np.arange(n, dtype=np.uint32)
    gk, gp, _ = ip_sort(keys, pay, params=P(key_bits=nbits))
    rk, rp = oracle.partition(keys, pay, nbits)
    assert np.array_equal(gp, rp) and np.array_equal(gk, rk)
