"""GPU parity of the two plain entry points of the C ABI, called directly
through ctypes with raw device pointers: binar_sort(keys, key_bytes, n,
payload) (the problem statement of section "Sorting Formalism": the keys
in nondecreasing bit order, the permutation carried in the payload) and
binar_sort_async on a side stream, with the library's pool and with a
workspace of the caller's."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import need_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def keys_for(kb, n, seed):
    return {4: lambda: workloads.u32_uniform(n, seed), 8: lambda: workloads.u64_uniform(n, seed),
            16: lambda: workloads.str16(n, seed, 3)}[kb]()


def ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("kb", [4, 8, 16])
@pytest.mark.parametrize("pay", [True, False])
@pytest.mark.parametrize("n", [1, 2, 4097, 300_007])
def test_binar_sort_direct(kb, pay, n):
    """binar_sort blocks until the result is in place."""
    from paper_0811_3448_amd.binar import lib
    keys = keys_for(kb, n, 1200 + kb + n % 97)
    p = np.arange(n, dtype=np.uint32)
    kd, pd = to_dev(keys), (to_dev(p) if pay else None)
    print("binar_sort kb=%d pay=%d n=%d" % (kb, pay, n), flush=True)
    assert lib.binar_sort(ptr(kd), kb, n, ptr(pd)) == 0
    rk, rp = oracle.sort(keys, p if pay else None)
    assert np.array_equal(to_host(kd, keys), rk)
    if pay:
        assert np.array_equal(to_host(pd, p), rp)


@pytest.mark.parametrize("kb", [4, 8, 16])
@pytest.mark.parametrize("own_workspace", [False, True])
def test_binar_sort_async_side_stream(kb, own_workspace):
    """binar_sort_async enqueues on the caller's stream; the result is there
    once that stream has been synchronised.  Two sorts in a row on the same
    stream and workspace, the second smaller."""
    import torch
    from paper_0811_3448_amd.binar import lib
    s = torch.cuda.Stream()
    ws = None
    if own_workspace:
        nb = int(lib.binar_workspace_bytes(kb, 500_003, 1, 1, None))
        assert nb > 0
        ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    for n, seed in ((500_003, 1300 + kb), (70_001, 1310 + kb)):
        keys = keys_for(kb, n, seed)
        p = np.arange(n, dtype=np.uint32)
        kd, pd = to_dev(keys), to_dev(p)
        torch.cuda.synchronize()
        print("binar_sort_async kb=%d own_ws=%d n=%d" % (kb, own_workspace, n), flush=True)
        rc = lib.binar_sort_async(ptr(kd), kb, n, ptr(pd), ctypes.c_void_p(s.cuda_stream),
                                  ptr(ws), 0 if ws is None else ws.numel())
        assert rc == 0
        s.synchronize()
        rk, rp = oracle.sort(keys, p)
        assert np.array_equal(to_host(kd, keys), rk)
        assert np.array_equal(to_host(pd, p), rp)


def test_binar_sort_async_small_workspace_rejected():
    """A workspace below binar_workspace_bytes is refused with BINAR_ENOMEM
    before any work."""
    import torch
    from paper_0811_3448_amd.binar import lib
    n = 100_000
    nb = int(lib.binar_workspace_bytes(4, n, 1, 1, None))
    ws = torch.empty(nb - 256, dtype=torch.uint8, device="cuda")
    keys = workloads.u32_uniform(n, 1320)
    kd, pd = to_dev(keys), to_dev(np.arange(n, dtype=np.uint32))
    before = kd.clone()
    rc = lib.binar_sort_async(ptr(kd), 4, n, ptr(pd), None, ptr(ws), ws.numel())
    torch.cuda.synchronize()
    assert rc == -3
    assert torch.equal(kd, before)
