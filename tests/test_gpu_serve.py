"""Serving loop on the device: every request's result in a mixed, batched,
multi-stream run equals the same request sorted alone (keys and permutation,
tolerance 0), and small ones equal the oracle; the serving mix at its real
shape is checked completely on the device plus sampled oracle ranks; the
device memory the server allocates stays within its budget."""
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
    with Server(budget_bytes=1 << 30, streams=2, max_batch_keys=1 << 20, max_batch_requests=32) as srv:
        futs = [srv.submit(t) for t in subs]
        res = [f.result(timeout=120) for f in futs]
        rep = srv.report()
    assert rep["requests"] == len(dev)
    assert rep["batches"] < len(dev)
    assert max(r.batch_requests for r in res) > 1
    check_against_alone(host, dev, res)


def test_first_batch_while_the_default_stream_is_busy():
    """A lane is made, and its first batch runs, while the default stream
    (which the thread that makes the lane would use) still has queued work:
    the lane fills its resident buffers on its own stream, so the answer is
    right.  (Filled on the default stream, the permutation buffer could be
    read by the batch before it was written.)"""
    import torch
    from paper_0811_3448_amd.serve import Server
    a = workloads.u32_uniform(200_000, 4321)
    t = torch.from_numpy(a.view(np.int32)).pin_memory()
    with Server(budget_bytes=4 << 30, streams=1, max_batch_keys=1 << 21) as srv:
        torch.cuda._sleep(50_000_000)   # a bounded spin queued on the default stream
        r = srv.submit(t).result(timeout=120)
    order = np.argsort(a, kind="stable")
    assert np.array_equal(r.perm.cpu().numpy(), order.astype(np.int32))
    assert np.array_equal(r.keys.cpu().numpy().view(np.uint32), a[order])


def kb_of(a):
    return 4 if a.dtype == np.uint32 else (8 if a.dtype == np.uint64 else 16)


def test_tight_budget_queues_on_device():
    """Room for one lane per key class and three of the largest requests:
    requests queue, and the device memory the server allocates (torch's
    allocations plus the plans' workspaces) never passes the budget.  Each
    answer is moved to the host as it completes, so the caller holds no
    device memory; every answer equals the oracle's."""
    import torch
    from paper_0811_3448_amd.serve import DeviceBackend, Server, request_cost
    host, dev = make_requests(40, 2, max_log2=15)
    cap, segs = 1 << 18, 64
    be = DeviceBackend(2, cap, segs)
    lanes = sum(be.lane_cost((kb, 0)) for kb in (4, 8, 16))
    budget = lanes + 3 * max(request_cost(kb_of(a), a.shape[0]) for a in host)
    print("serve tight budget %d bytes (%d for lanes)" % (budget, lanes), flush=True)
    subs = [t.cpu().pin_memory() if i % 2 else t for i, t in enumerate(dev)]
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    got = [None] * len(subs)

    def to_host(i):
        def cb(f):
            r = f.result()
            got[i] = (r.keys.cpu().numpy(), r.perm.cpu().numpy().view(np.uint32))
            r.keys = r.perm = None        # the caller keeps no device memory
        return cb
    with Server(budget_bytes=budget, streams=2, max_batch_keys=cap, max_batch_requests=segs) as srv:
        futs = [srv.submit(t) for t in subs]
        for i, f in enumerate(futs):
            f.add_done_callback(to_host(i))
        for f in futs:
            assert f.exception(timeout=120) is None
    # closed: every callback has run
    torch.cuda.synchronize()
    grew = torch.cuda.max_memory_allocated() - base
    ws = sum(ln.plan.workspace_bytes for q in srv.backend.lanes.values() for ln in q)
    made = {cls: len(q) for cls, q in srv.backend.lanes.items()}
    for cls, q in srv.backend.lanes.items():
        for ln in q:
            assert ln.plan.workspace_bytes + ln.resident_bytes(cls[0], cap, segs) < srv.backend.lane_cost(cls)
    assert srv.admission.peak <= budget
    assert srv.max_waiting > 0
    rep = srv.report()
    print("  torch growth %d + plan workspaces %d = %d of %d; lanes %s; batches %d"
          % (grew, ws, grew + ws, budget, made, rep["batches"]), flush=True)
    assert grew + ws <= budget
    assert rep["failed_batches"] == 0
    for i, (a, g) in enumerate(zip(host, got)):
        rk, rp = oracle.sort(a, np.arange(a.shape[0], dtype=np.uint32))
        assert np.array_equal(g[0].view(rk.dtype).reshape(rk.shape), rk), i
        assert np.array_equal(g[1], rp), i


def string_words(t):
    """(n, 16) uint8 device strings as two int64 words each whose signed
    order is the strings' byte order (big-endian halves, top bit flipped)."""
    import torch
    n = t.shape[0]
    b = t.view(torch.uint8).reshape(n, 16).to(torch.int64)
    sh = torch.arange(56, -8, -8, device=t.device)
    w = torch.stack([(b[:, h * 8:(h + 1) * 8] << sh).sum(1) for h in range(2)], 1)
    return w ^ (-(1 << 63))


def check_served(a, kin, r, samples=3):
    """Complete device check of one answer (nondecreasing, the permutation a
    permutation, keys following it, ties in input order) plus the oracle's
    stable rank at sampled inputs, the first and the last."""
    import torch
    from oracle.definition import stable_rank_bytes, stable_rank_u
    from test_gpu_fullsize import device_checks
    n = a.shape[0]
    if n == 0:
        assert r.keys.shape[0] == 0 and r.perm.shape[0] == 0
        return
    if a.ndim == 2:
        w, wo = string_words(kin), string_words(r.keys)
        p = r.perm.to(torch.int64)
        less = (wo[1:, 0] > wo[:-1, 0]) | ((wo[1:, 0] == wo[:-1, 0]) & (wo[1:, 1] >= wo[:-1, 1]))
        assert bool(less.all()), "strings not sorted"
        assert bool(((p >= 0) & (p < n)).all()), "permutation out of range"
        seen = torch.zeros(n, dtype=torch.int8, device=p.device)
        seen[p] = 1
        assert bool(seen.all()), "not a permutation"
        assert torch.equal(w[p], wo), "strings do not follow the permutation"
        tie = (wo[1:] == wo[:-1]).all(1)
        assert bool((p[1:][tie] > p[:-1][tie]).all()), "unstable on ties"
        rank = stable_rank_bytes
    else:
        device_checks(kin, r.keys, r.perm, kb_of(a))
        rank = stable_rank_u
    js = sorted(set(workloads.below(samples, n + 17, n).astype(np.int64).tolist() + [0, n - 1]))
    rs = [rank(a, j) for j in js]
    ix = torch.tensor(rs, device=r.keys.device)
    kh = r.keys[ix].cpu().numpy().view(a.dtype).reshape((len(rs),) + a.shape[1:])
    ph = r.perm[ix].cpu().numpy().view(np.uint32)
    for j, rk, k, p in zip(js, rs, kh, ph):
        assert p == j and np.array_equal(k, a[j]), "input %d should sit at output %d" % (j, rk)


def test_serving_mix_at_real_shape():
    """About 200 requests of the serving workload (lognormal sizes, key
    widths 4/8/16 bytes at 50/30/20 %, strings with 0..12-byte shared
    prefixes) plus one request of the largest size, 2^24 keys, per width,
    from pinned host memory through the server configured as the serving
    benchmark runs it; every answer checked."""
    import torch
    from paper_0811_3448_amd.serve import Server
    trace = workloads.serve_requests(200)
    big = [{"id": 200 + i, "n": 1 << 24, "key_bytes": kb, "prefix_len": 12, "seed": 777_000 + kb}
           for i, kb in enumerate((4, 8, 16))]
    trace = trace[:70] + big[:1] + trace[70:140] + big[1:2] + trace[140:] + big[2:]
    host = [workloads.request_keys(t) for t in trace]
    print("serve real shape: %d requests, %d keys, largest %d" % (len(host), sum(a.shape[0] for a in host),
                                                                  max(a.shape[0] for a in host)), flush=True)
    subs = []
    for a in host:
        t = torch.from_numpy(a.view(np.int32) if a.dtype == np.uint32 else
                             (a.view(np.int64) if a.dtype == np.uint64 else a))
        subs.append(t.pin_memory())
    with Server(budget_bytes=32 << 30, streams=2, max_batch_keys=1 << 25, max_batch_requests=1024) as srv:
        futs = [srv.submit(t) for t in subs]
        for i, (a, t, f) in enumerate(zip(host, subs, futs)):
            r = f.result(timeout=300)
            check_served(a, t.cuda(), r)
            futs[i] = None
            if i % 50 == 0:
                print("  checked %d/%d" % (i + 1, len(host)), flush=True)
        rep = srv.report()
    assert rep["requests"] == len(host) and rep["failed_batches"] == 0
    assert rep["batches"] < len(host)
    print("  batches %d, peak admitted %.2f GiB (lanes %.2f GiB)"
          % (rep["batches"], rep["peak_admitted_bytes"] / 2 ** 30, rep["lane_bytes"] / 2 ** 30), flush=True)


def test_one_request_per_launch_matches():
    from paper_0811_3448_amd.serve import Server
    host, dev = make_requests(20, 3, max_log2=14)
    with Server(budget_bytes=1 << 30, streams=3, max_batch_keys=1 << 16, batching=False) as srv:
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
    with Server(budget_bytes=1 << 28, streams=2, max_batch_keys=1 << 18) as srv:
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
