"""Serving-loop policy on the host: admission against a tiny budget queues
instead of failing, oversize requests get ENOMEM at submit, cancelled
requests free their budget, batches hold one key width in admission order.
The device is replaced by a host backend that sorts with numpy."""
import threading
import time

import numpy as np
import pytest
import torch

from paper_0811_3448_amd import BinarError
from paper_0811_3448_amd.binar import BINAR_ENOMEM
from paper_0811_3448_amd.serve import META_BYTES, Admission, Server, request_cost


def np_stable(keys):
    a = keys.numpy()
    if a.ndim == 2:
        perm = np.lexsort(a.T[::-1])
    else:
        perm = np.argsort(a.view(np.uint32 if a.dtype == np.int32 else np.uint64), kind="stable")
    return torch.from_numpy(a[perm].copy()), torch.from_numpy(perm.astype(np.int32))


class HostBackend:
    """Lanes that finish only when `gate` is set (or at once if gate is None);
    each lane costs `lane_bytes` of the budget."""

    def __init__(self, lanes=1, gate=None, lane_bytes=0):
        self.lanes, self.gate, self.lane_bytes = lanes, gate, lane_bytes
        self.busy = {}
        self.created = {}
        self.batches = []
        self.lane_block = threading.Event()
        self.lane_block.set()

    def thread_init(self):
        pass

    def mark_ready(self, keys):
        return None

    def lane_cost(self, cls):
        return self.lane_bytes

    def free_lane(self, cls, may_create):
        if not self.lane_block.is_set():
            return None
        if self.busy.get(cls, 0) >= self.created.get(cls, 0):
            if self.created.get(cls, 0) >= self.lanes or not may_create():
                return None
            self.created[cls] = self.created.get(cls, 0) + 1
        self.busy[cls] = self.busy.get(cls, 0) + 1
        return cls

    def release_lane(self, cls):
        self.busy[cls] -= 1

    def launch(self, cls, reqs):
        self.batches.append((cls[0], [r.id for r in reqs]))
        return [np_stable(r.keys) for r in reqs]

    def poll(self, h):
        return self.gate is None or self.gate.is_set()

    def collect(self, h):
        return h


def u32(n, seed):
    return torch.from_numpy(np.random.default_rng(seed).integers(0, 1 << 32, n, dtype=np.uint64)
                            .astype(np.uint32).view(np.int32))


def u64(n, seed):
    return torch.from_numpy(np.random.default_rng(seed).integers(0, 1 << 63, n, dtype=np.int64))


def s16(n, seed):
    return torch.from_numpy(np.random.default_rng(seed).integers(0, 4, (n, 16), dtype=np.uint8))


def test_cost_formula():
    assert request_cost(4, 1000) == 2 * 8 * 1000 + META_BYTES
    assert request_cost(16, 0) == META_BYTES


def test_admission_fifo_and_release():
    class R:
        def __init__(self, cost):
            from concurrent.futures import Future
            self.cost, self.future = cost, Future()
    a = Admission(100)
    rs = [R(60), R(30), R(20), R(10)]
    for r in rs:
        a.offer(r)
    got = a.admit(0.0)
    assert got == rs[:2] and a.in_use == 90            # 20 does not fit behind: FIFO, no overtaking
    a.release(60)
    assert a.admit(1.0) == rs[2:] and a.in_use == 60
    with pytest.raises(BinarError) as e:
        a.offer(R(101))
    assert e.value.status == BINAR_ENOMEM


def test_tiny_budget_queues_and_all_complete():
    reqs = [u32(1000 + 37 * i, i) for i in range(12)] + [u64(500, 99), s16(300, 98)]
    budget = max(request_cost(4 if t.dim() == 1 and t.element_size() == 4 else (8 if t.dim() == 1 else 16),
                              t.shape[0]) for t in reqs) + 64
    be = HostBackend(lanes=2)
    peak = []
    with Server(budget, backend=be) as srv:
        futs = [srv.submit(t) for t in reqs]
        res = [f.result(timeout=10) for f in futs]
        peak.append(srv.admission.peak)
        rep = srv.report()
    assert peak[0] <= budget
    assert rep["requests"] == len(reqs)
    for t, r in zip(reqs, res):
        k, p = np_stable(t)
        assert torch.equal(r.keys, k) and torch.equal(r.perm, p)
    # each admitted request nearly fills the budget: one at a time
    assert all(len(ids) == 1 for _, ids in be.batches)


def test_oversize_gets_enomem_up_front():
    be = HostBackend()
    with Server(request_cost(4, 100), backend=be, max_batch_keys=1 << 20) as srv:
        with pytest.raises(BinarError) as e:
            srv.submit(u32(101, 1))
        assert e.value.status == BINAR_ENOMEM
        with pytest.raises(BinarError):
            srv.submit(torch.zeros((1 << 20) + 1, dtype=torch.int32))
        assert not srv.admission.waiting and srv.admission.in_use == 0
        assert srv.submit(u32(100, 2)).result(timeout=10).keys.shape[0] == 100


def test_cancel_frees_budget():
    gate = threading.Event()
    be = HostBackend(lanes=1, gate=gate)
    cost = request_cost(4, 1000)
    with Server(cost, backend=be) as srv:
        f1 = srv.submit(u32(1000, 1))         # admitted and launched, held in flight by the gate
        f2 = srv.submit(u32(1000, 2))         # waits for budget
        f3 = srv.submit(u32(1000, 3))
        time.sleep(0.05)
        assert f2.cancel()                    # cancelled while waiting: never charged
        gate.set()
        assert f1.result(timeout=10) and f3.result(timeout=10)
        assert f2.cancelled()
    assert [ids for _, ids in be.batches] == [[0], [2]]


def test_cancel_after_admission_releases():
    be = HostBackend(lanes=1)
    be.lane_block.clear()                     # no lane free: admitted requests wait in the ready queue
    cost = request_cost(4, 1000)
    with Server(cost, backend=be) as srv:
        f1 = srv.submit(u32(1000, 1))
        f2 = srv.submit(u32(1000, 2))
        deadline = time.time() + 5
        while srv.admission.in_use != cost and time.time() < deadline:
            time.sleep(0.001)
        assert srv.admission.in_use == cost    # f1 admitted, f2 waiting
        assert f1.cancel()
        deadline = time.time() + 5
        while len(srv.admission.waiting) and time.time() < deadline:
            time.sleep(0.001)
        assert not srv.admission.waiting       # f1's budget went to f2
        be.lane_block.set()
        assert f2.result(timeout=10).keys.shape[0] == 1000
    assert [ids for _, ids in be.batches] == [[1]]


def test_batches_one_width_in_admission_order():
    be = HostBackend(lanes=1)
    be.lane_block.clear()
    kinds = [u32, u64, s16]
    with Server(1 << 30, backend=be, max_batch_requests=5) as srv:
        futs = [srv.submit(kinds[i % 3](50 + i, i)) for i in range(30)]
        time.sleep(0.05)
        be.lane_block.set()
        for f in futs:
            f.result(timeout=10)
    width_of = {i: (4, 8, 16)[i % 3] for i in range(30)}
    seen = []
    for kb, ids in be.batches:
        assert len(ids) <= 5
        assert all(width_of[i] == kb for i in ids)
        seen.extend(ids)
    for kb in (4, 8, 16):
        order = [i for i in seen if width_of[i] == kb]
        assert order == sorted(order)
    assert sorted(seen) == list(range(30))


def test_no_batching_is_one_request_per_launch():
    be = HostBackend(lanes=2)
    with Server(1 << 30, backend=be, batching=False) as srv:
        futs = [srv.submit(u32(10 + i, i)) for i in range(10)]
        for f in futs:
            assert f.result(timeout=10).batch_requests == 1
    assert all(len(ids) == 1 for _, ids in be.batches)


def test_backend_failure_fails_pending_requests():
    class Broken(HostBackend):
        def launch(self, cls, reqs):
            raise RuntimeError("device lost")
    srv = Server(1 << 30, backend=Broken())
    f = srv.submit(u32(10, 1))
    with pytest.raises(RuntimeError):
        f.result(timeout=10)
    with pytest.raises(RuntimeError):
        srv.close()


def test_report_percentiles():
    be = HostBackend(lanes=4)
    with Server(1 << 30, backend=be) as srv:
        for i in range(50):
            srv.submit(u32(100, i)).result(timeout=10)
        rep = srv.report()
    assert rep["requests"] == 50 and rep["keys"] == 5000
    assert 0 <= rep["p50_s"] <= rep["p99_s"] <= rep["max_s"]
    assert rep["throughput_keys_s"] > 0


def test_key_kinds_batch_apart():
    """Float and integer requests of one width never share a batch."""
    be = HostBackend(lanes=1)
    be.lane_block.clear()
    with Server(1 << 30, backend=be) as srv:
        fi = [srv.submit(u32(10, i)) for i in range(3)]
        ff = [srv.submit(torch.randn(10)) for _ in range(3)]
        fs = [srv.submit(u32(10, 9), key_kind=1)]
        time.sleep(0.05)
        be.lane_block.set()
        for f in fi + ff + fs:
            f.result(timeout=10)
    groups = [sorted(ids) for _, ids in be.batches]
    assert sorted(groups) == [[0, 1, 2], [3, 4, 5], [6]]
    with pytest.raises(ValueError):
        Server(1 << 30, backend=HostBackend()).submit(torch.zeros((4, 16), dtype=torch.uint8), key_kind=2)


def test_admission_lane_accounting():
    class R:
        def __init__(self, cost, cls):
            from concurrent.futures import Future
            self.cost, self.cls, self.future = cost, cls, Future()
    a = Admission(1000)
    cost = {"x": 300, "y": 400}.get
    r1, r2, r3 = R(100, "x"), R(100, "x"), R(250, "y")
    for r in (r1, r2, r3):
        a.offer(r, cost)
    # r1 reserves x's first lane (300 + 100), r2 needs no lane (100); r3
    # needs y's first lane as well (400 + 250): 500 + 650 > 1000, it waits
    assert a.admit(0.0, cost) == [r1, r2]
    assert (a.in_use, a.fixed, a.reserved["x"], a.lanes["x"]) == (500, 300, 1, 1)
    assert a.take_lane("x", 300)                 # the reserved lane: nothing more charged
    assert (a.in_use, a.reserved["x"]) == (500, 0)
    a.release(100)
    a.release(100)
    assert a.admit(1.0, cost) == [r3]            # 300 + 400 + 250 = 950
    assert (a.in_use, a.fixed, a.peak) == (950, 700, 950)
    assert not a.take_lane("x", 300)             # a second x lane would pass the budget
    a.release(250)
    assert a.take_lane("x", 300) and (a.in_use, a.fixed, a.lanes["x"]) == (1000, 1000, 2)
    with pytest.raises(AssertionError):
        a.release(1)                             # lanes are never released
    # with every byte held by lanes, a new request can never fit: refused at offer
    with pytest.raises(BinarError) as e:
        a.offer(R(1, "x"), cost)
    assert e.value.status == BINAR_ENOMEM


def test_request_left_without_room_fails_instead_of_waiting():
    """A request that fit when offered but not beside lanes charged later
    (for a class that reached the head of the queue first) fails with
    BINAR_ENOMEM rather than waiting forever."""
    class R:
        def __init__(self, cost, cls):
            from concurrent.futures import Future
            self.cost, self.cls, self.future = cost, cls, Future()
    a = Admission(1000)
    cost = {"x": 500, "y": 500}.get
    rx, ry = R(100, "x"), R(450, "y")
    a.offer(rx, cost)
    a.offer(ry, cost)                            # 500 + 450 <= 1000 when offered
    assert a.admit(0.0, cost) == [rx]            # x's lane is now held: 500 + 500 + 450 > 1000
    a.release(100)
    assert a.admit(1.0, cost) == []
    assert not a.waiting
    with pytest.raises(BinarError) as e:
        ry.future.result(timeout=1)
    assert e.value.status == BINAR_ENOMEM


def test_lanes_within_budget_end_to_end():
    """Lane bytes count against the budget: with room for one lane per class
    plus one request, the server still answers everything, never holds more
    than the budget, and creates a second lane only when it fits."""
    reqs = [u32(1000 + 37 * i, i) for i in range(12)] + [u64(500, 99), s16(300, 98)]
    lane = 1 << 20
    budget = 3 * lane + request_cost(16, 1400) + request_cost(4, 1500)
    be = HostBackend(lanes=2, lane_bytes=lane)
    with Server(budget, backend=be) as srv:
        res = [f.result(timeout=10) for f in [srv.submit(t) for t in reqs]]
        assert srv.admission.peak <= budget
        assert srv.admission.fixed == lane * sum(be.created.values())
        assert srv.report()["lane_bytes"] == srv.admission.fixed
    for t, r in zip(reqs, res):
        k, p = np_stable(t)
        assert torch.equal(r.keys, k) and torch.equal(r.perm, p)


def test_failed_batch_fails_only_its_requests():
    class Failing(HostBackend):
        def collect(self, h):
            if any(k.shape[0] == 13 for k, _ in h):
                raise BinarError(-4)
            return h
    be = Failing(lanes=1)
    with Server(1 << 30, backend=be, batching=False) as srv:
        good = srv.submit(u32(12, 1))
        bad = srv.submit(u32(13, 2))
        after = srv.submit(u32(14, 3))
        assert good.result(timeout=10).keys.shape[0] == 12
        with pytest.raises(BinarError) as e:
            bad.result(timeout=10)
        assert e.value.status == -4
        assert after.result(timeout=10).keys.shape[0] == 14
        assert srv.report()["failed_batches"] == 1
