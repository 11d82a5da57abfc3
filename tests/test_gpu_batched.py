"""Batched segmented sorts and their HIP-graph replay (through the C ABI),
against the oracle and against the eager call."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import check_segmented, need_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def dev_offsets(off):
    import torch
    return torch.from_numpy(np.asarray(off, dtype=np.uint32).view(np.int32)).cuda()


def test_plan_replays_match_oracle_and_eager():
    """One plan, one set of resident buffers: the graph is captured once and
    replayed on fresh data several times, with eager sorts and syncs in
    between; every replay must equal the oracle and the eager result."""
    import torch
    import paper_0811_3448_amd as binar
    S, cap = 400, 600_000
    plan = binar.Plan(4, cap, S, True)
    kbuf = torch.empty(cap, dtype=torch.int32, device="cuda")
    pbuf = torch.empty(cap, dtype=torch.int32, device="cuda")
    obuf = torch.empty(S + 1, dtype=torch.int32, device="cuda")
    for rep in range(4):
        keys, off = workloads.batched_u32(S, seed=500 + rep, median=700, sigma=1.0, max_len=30_000)
        n = int(off[-1])
        assert n <= cap
        print("replay %d n=%d" % (rep, n), flush=True)
        kbuf[:n] = to_dev(keys)
        pbuf[:n] = torch.arange(n, dtype=torch.int32, device="cuda")
        obuf.copy_(dev_offsets(off))
        plan.sort(kbuf, pbuf, obuf)
        torch.cuda.synchronize()
        assert plan.stats()["status"] == 0
        gk = kbuf[:n].cpu().numpy().view(np.uint32)
        gp = pbuf[:n].cpu().numpy().view(np.uint32)
        rk, rp = oracle.sort_segmented(keys, off, np.arange(n, dtype=np.uint32))
        assert np.array_equal(gk, rk) and np.array_equal(gp, rp), rep
        # the eager segmented call on a copy gives the same
        ek, ep = to_dev(keys), torch.arange(n, dtype=torch.int32, device="cuda")
        binar.sort_segmented(ek, dev_offsets(off), ep)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(ek, keys), gk) and np.array_equal(ep.cpu().numpy().view(np.uint32), gp)
    assert plan.graphs == 1, "the replays must reuse one captured graph"
    plan.close()


def test_plan_single_array_and_changed_layout():
    import torch
    import paper_0811_3448_amd as binar
    cap = 300_000
    plan = binar.Plan(8, cap, 50, True)
    kbuf = torch.empty(cap, dtype=torch.int64, device="cuda")
    pbuf = torch.empty(cap, dtype=torch.int32, device="cuda")
    for rep in range(3):
        keys = workloads.u64_zipf(cap, 600 + rep, 1 << 12, 1.1)
        kbuf.copy_(to_dev(keys))
        pbuf.copy_(torch.arange(cap, dtype=torch.int32, device="cuda"))
        plan.sort(kbuf, pbuf)
        torch.cuda.synchronize()
        rk, rp = oracle.sort(keys, np.arange(cap, dtype=np.uint32))
        assert np.array_equal(to_host(kbuf, keys), rk) and np.array_equal(pbuf.cpu().numpy().view(np.uint32), rp)
    # segmented layouts change between replays of one graph (same buffers)
    obuf = torch.empty(51, dtype=torch.int32, device="cuda")
    for rep in range(3):
        keys = workloads.u64_uniform(cap, 700 + rep)
        cuts = np.sort(workloads.below(49, 800 + rep, cap).astype(np.int64))
        off = np.concatenate([[0], cuts, [cap]]).astype(np.uint32)
        kbuf.copy_(to_dev(keys))
        pbuf.copy_(torch.arange(cap, dtype=torch.int32, device="cuda"))
        obuf.copy_(dev_offsets(off))
        plan.sort(kbuf, pbuf, obuf)
        torch.cuda.synchronize()
        rk, rp = oracle.sort_segmented(keys, off, np.arange(cap, dtype=np.uint32))
        assert np.array_equal(to_host(kbuf, keys), rk) and np.array_equal(pbuf.cpu().numpy().view(np.uint32), rp)
    assert plan.graphs == 2
    plan.close()


@pytest.mark.parametrize("params_from", ["library defaults", "autotune cache"])
def test_batched_100k_segments_full_size(params_from):
    """The batched workload at its full size: 100,000 lognormal segments,
    about 2^27 keys, checked completely by per-segment properties plus the
    oracle on a sample of segments; once with the library's defaults and
    once with the parameters the autotune cache holds for this case (the
    ones the batched benchmark runs)."""
    import torch
    import paper_0811_3448_amd as binar
    from paper_0811_3448_amd import tune
    keys, off = workloads.batched_u32()
    n, S = int(off[-1]), off.shape[0] - 1
    params = None
    if params_from == "autotune cache":
        params = tune.TuneCache(arch=tune.device_arch()).lookup(4, True, n, True, max_distance=1)
        assert params is not None, "no batched entry in the autotune cache"
    print("batched n=%d S=%d params=%s" % (n, S, params), flush=True)
    plan = binar.Plan(4, n, S, True, params)
    kd, pd = to_dev(keys), torch.arange(n, dtype=torch.int32, device="cuda")
    plan.sort(kd, pd, dev_offsets(off))
    torch.cuda.synchronize()
    assert plan.stats()["status"] == 0
    gk, gp = to_host(kd, keys), pd.cpu().numpy().view(np.uint32)
    check_segmented(keys, off, gk, gp)
    for s in workloads.below(64, 900, S).astype(np.int64).tolist() + [int(np.argmax(np.diff(off)))]:
        a, b = int(off[s]), int(off[s + 1])
        rk, rp = oracle.sort(keys[a:b], np.arange(a, b, dtype=np.uint32))
        assert np.array_equal(gk[a:b], rk) and np.array_equal(gp[a:b], rp), s
    plan.close()


def test_plan_segmented_short_buffers_refused_by_the_library():
    """Through the C ABI: a segmented plan sort whose n_total (the caller's
    buffer length) is below the plan's capacity returns BINAR_EINVAL before
    any device work, and the keys stay as they were."""
    import ctypes
    import torch
    import paper_0811_3448_amd as binar
    plan = binar.Plan(4, 5000, 4, True)
    keys = torch.arange(4000, 0, -1, dtype=torch.int32, device="cuda")
    pay = torch.arange(4000, dtype=torch.int32, device="cuda")
    off = dev_offsets([0, 1000, 2000, 3000, 4000])
    before = keys.clone()
    vp = ctypes.c_void_p
    rc = binar.lib.binar_plan_sort(plan._h, vp(keys.data_ptr()), vp(pay.data_ptr()), vp(off.data_ptr()), 4, 4000,
                                   None)
    assert rc == binar.BINAR_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(keys, before)
    plan.close()
