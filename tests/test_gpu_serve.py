"""Serving loop on the device: every request's result in a mixed, batched,
multi-stream run equals the same request sorted alone (keys and permutation,
tolerance 0), and small ones equal the oracle."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def make_requests(count, seed, max_log2=17):
    import torch
    rng = np.random.default_rng(seed)
    host = []
    sizes = [0, 1, 2, 3, 255, 256, 4097] + [int(2 ** rng.uniform(8, max_log2)) for _ in range(count - 7)]
    for i, n in enumerate(sizes):
        w = rng.choice([4, 8, 16], p=[0.5, 0.3, 0.2])
        s = 1000 * seed + i
        a = {4: lambda: workloads.u32_uniform(n, s), 8: lambda: workloads.u64_zipf(n, s, 1 << 10, 1.1),
             16: lambda: workloads.str16(n, s, 5)}[w]()
        host.append(a)
    dev = []
    for a in host:
        t = torch.from_numpy(a.view(np.int32) if a.dtype == np.uint32 else
                             (a.view(np.int64) if a.dtype == np.uint64 else a))
        dev.append(t.cuda())
    return host, dev


def alone(t):
    import torch
    import paper_0811_3448_amd as binar
    k = t.clone()
    p = torch.arange(t.shape[0], dtype=torch.int32, device=t.device)
    if t.shape[0]:
        binar.sort(k, p)
    return k, p


def check_against_alone(host, dev, results, oracle_every=10):
    import torch
    for i, (a, t, r) in enumerate(zip(host, dev, results)):
        k, p = alone(t)
        torch.cuda.synchronize()
        assert torch.equal(r.keys, k), "request %d: keys differ from the sort alone" % i
        assert torch.equal(r.perm, p), "request %d: permutation differs from the sort alone" % i
        if i % oracle_every == 0 and a.shape[0] <= 20000:
            rk, rp = oracle.sort(a, np.arange(a.shape[0], dtype=np.uint32))
            assert np.array_equal(r.keys.cpu().numpy().view(rk.dtype).reshape(rk.shape), rk)
            assert np.array_equal(r.perm.cpu().numpy().view(np.uint32), rp)


def test_alone_equals_in_mix():
    from paper_0811_3448_amd.serve import Server
    host, dev = make_requests(160, 1)
    print("serve mix: %d requests, %d keys" % (len(dev), sum(t.shape[0] for t in dev)), flush=True)
    # every third request comes from pinned host memory and is uploaded by its batch
    subs = [t.cpu().pin_memory() if i % 3 == 1 else t for i, t in enumerate(dev)]
    with Server(budget_bytes=1 << 30, streams=2, max_batch_keys=1 << 20, max_batch_requests=32,
                check_status=True) as srv:
        futs = [srv.submit(t) for t in subs]
        res = [f.result(timeout=120) for f in futs]
        rep = srv.report()
    assert rep["requests"] == len(dev)
    assert rep["batches"] < len(dev)
    assert max(r.batch_requests for r in res) > 1
    check_against_alone(host, dev, res)


def test_tight_budget_queues_on_device():
    from paper_0811_3448_amd.serve import Server, request_cost
    host, dev = make_requests(40, 2, max_log2=15)
    budget = 3 * max(request_cost(4 if a.dtype == np.uint32 else (8 if a.dtype == np.uint64 else 16), a.shape[0])
                     for a in host)
    print("serve tight budget %d bytes" % budget, flush=True)
    with Server(budget_bytes=budget, streams=2, max_batch_keys=1 << 18, check_status=True) as srv:
        futs = [srv.submit(t) for t in dev]
        res = [f.result(timeout=120) for f in futs]
        assert srv.admission.peak <= budget
        assert srv.max_waiting > 0
    check_against_alone(host, dev, res)


def test_one_request_per_launch_matches():
    from paper_0811_3448_amd.serve import Server
    host, dev = make_requests(20, 3, max_log2=14)
    with Server(budget_bytes=1 << 30, streams=3, max_batch_keys=1 << 16, batching=False,
                check_status=True) as srv:
        res = [f.result(timeout=120) for f in [srv.submit(t) for t in dev]]
    assert all(r.batch_requests == 1 for r in res)
    check_against_alone(host, dev, res, oracle_every=5)


def test_key_kinds_in_the_mix():
    """Float and signed requests share the server with unsigned ones; each
    result equals the same request sorted alone and the oracle's order."""
    import torch
    import paper_0811_3448_amd as binar
    from oracle import orders
    from paper_0811_3448_amd.serve import Server
    rng = np.random.default_rng(9)
    reqs = []
    for i in range(30):
        n = int(rng.integers(1, 20_000))
        kind = i % 3
        if kind == 0:
            t = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
            reqs.append((t, None, orders.FLOAT))
        elif kind == 1:
            t = torch.from_numpy(rng.integers(-1000, 1000, n).astype(np.int64)).cuda()
            reqs.append((t, binar.KEY_SIGNED, orders.SIGNED))
        else:
            t = torch.from_numpy((rng.standard_normal(n) * 1e300).astype(np.float64)).cuda()
            reqs.append((t, None, orders.FLOAT))
    with Server(budget_bytes=1 << 28, streams=2, max_batch_keys=1 << 18, check_status=True) as srv:
        res = [f.result(timeout=120) for f in [srv.submit(t, key_kind=k) for t, k, _ in reqs]]
    for (t, k, ok), r in zip(reqs, res):
        a = t.clone()
        p = torch.arange(t.shape[0], dtype=torch.int32, device="cuda")
        binar.sort(a, p, key_kind=k)
        torch.cuda.synchronize()
        assert r.keys.dtype == t.dtype
        assert torch.equal(r.keys.view(torch.uint8), a.view(torch.uint8))
        assert torch.equal(r.perm, p)
        bits = t.cpu().numpy().view(np.uint32 if t.element_size() == 4 else np.uint64)
        rk, rp = orders.sort(bits, np.arange(t.shape[0], dtype=np.uint32), ok)
        assert np.array_equal(r.perm.cpu().numpy().view(np.uint32), rp)
