"""GPU parity of the allocation-free entry point binar_sort_static (scratch
in a fixed per-device array of the library) against binar_sort_async with a
workspace of the caller's, called through the C ABI with raw device
pointers: keys and permutation bit-exact, on two calls in a row, the second
smaller, so the second runs on the array the first left behind."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import need_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 << 20  # BINAR_STATIC_SCRATCH_BYTES


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def keys_for(kb, n, seed):
    return {4: lambda: workloads.u32_uniform(n, seed), 8: lambda: workloads.u64_uniform(n, seed),
            16: lambda: workloads.str16(n, seed, 3)}[kb]()


def ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def largest_fitting(lib, kb, pay):
    """Largest n whose workspace fits the static array (bisection on the
    library's own size function)."""
    lo, hi = 2, 1 << 24
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if int(lib.binar_workspace_bytes(kb, mid, 1 if pay else 0, 1, None)) <= STATIC_BYTES:
            lo = mid
        else:
            hi = mid - 1
    return lo


@pytest.mark.parametrize("kb", [4, 8, 16])
@pytest.mark.parametrize("pay", [True, False])
def test_static_matches_async_two_calls(kb, pay):
    import torch
    from paper_0811_3448_amd.binar import lib
    s = torch.cuda.current_stream()
    sp = ctypes.c_void_p(s.cuda_stream)
    nmax = largest_fitting(lib, kb, pay)
    # the largest input that fits, then a smaller ragged one
    for n, seed in ((nmax, 1400 + kb), (70_001, 1410 + kb)):
        keys = keys_for(kb, n, seed)
        p = np.arange(n, dtype=np.uint32)
        ka, pa = to_dev(keys), (to_dev(p) if pay else None)
        kz, pz = to_dev(keys), (to_dev(p) if pay else None)
        nb = int(lib.binar_workspace_bytes(kb, n, 1 if pay else 0, 1, None))
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        print("binar_sort_static kb=%d pay=%d n=%d" % (kb, pay, n), flush=True)
        assert lib.binar_sort_static(ptr(kz), kb, n, ptr(pz), sp) == 0
        assert lib.binar_sort_async(ptr(ka), kb, n, ptr(pa), sp, ptr(ws), nb) == 0
        torch.cuda.synchronize()
        gk = to_host(kz, keys)
        assert np.array_equal(gk, to_host(ka, keys)), "keys differ from binar_sort_async"
        if pay:
            assert np.array_equal(to_host(pz, p), to_host(pa, p)), "permutation differs from binar_sort_async"
        # sampled against the oracle as well: the first and last 4096 positions
        rk, rp = oracle.sort(keys, p)
        assert np.array_equal(gk[:4096], rk[:4096]) and np.array_equal(gk[-4096:], rk[-4096:])
        if pay:
            gp = to_host(pz, p)
            assert np.array_equal(gp, rp)
        del ws


def test_static_stats_and_limit():
    """binar_stats_read(NULL) reads the static call's counters; an input whose
    workspace exceeds the array is refused with BINAR_ENOMEM before any work."""
    import torch
    from paper_0811_3448_amd.binar import lib
    import paper_0811_3448_amd as binar
    n = 300_007
    keys = workloads.u32_uniform(n, 1420)
    kd, pd = to_dev(keys), to_dev(np.arange(n, dtype=np.uint32))
    assert lib.binar_sort_static(ptr(kd), 4, n, ptr(pd), None) == 0
    st = binar.stats()
    assert st["status"] == 0 and sum(st["moved"]) + st["finish_keys"] >= n
    big = largest_fitting(lib, 4, True) + 1
    kb_ = torch.zeros(big, dtype=torch.int32, device="cuda")
    pb_ = torch.arange(big, dtype=torch.int32, device="cuda")
    before = pb_.clone()
    assert lib.binar_sort_static(ptr(kb_), 4, big, ptr(pb_), None) == binar.BINAR_ENOMEM
    torch.cuda.synchronize()
    assert torch.equal(pb_, before)
    assert lib.binar_sort_static(ptr(kd), 3, n, ptr(pd), None) == binar.BINAR_EINVAL
    assert lib.binar_sort_static(ptr(kd), 4, 1, ptr(pd), None) == 0
