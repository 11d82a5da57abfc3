"""Serving loop for sort requests on one GPU.

Requests (tensors of keys: 4-byte, 8-byte or 16-byte, see ``key_bytes_of``;
on the device, or in pinned host memory, which the batch uploads) arrive over
time through ``Server.submit`` and are answered
through a ``concurrent.futures.Future`` with the sorted keys and the stable
sorting permutation (int32 holding uint32 indices into the request).

* Budget: every byte of device memory the server allocates is charged to one
  HBM budget.  A lane (one stream and key class) holds resident buffers and a
  plan workspace for ``max_batch_keys`` keys; it is charged when it is
  created and held until the server closes (``DeviceBackend.lane_cost``).
  A request costs ``2 * (key_bytes + 4) * n + META_BYTES`` while it is in
  flight (the batch's output keys and permutation and the temporaries that
  make them); the outputs handed to the caller are the caller's.
* Admission: requests are admitted in arrival order while the charged bytes
  stay within the budget; otherwise they wait.  The first request of a key
  class also reserves that class's first lane, so every admitted request has
  a lane to run on; further lanes of a class (up to ``streams``) are created
  only while the budget has room for them.  A request that could never fit
  beside the lanes already held is refused with BINAR_ENOMEM (at submit, or
  when lanes created later leave it no room).
* Batching: admitted requests of one key class are packed, in admission
  order, into the resident buffers of a lane and sorted as the segments of
  one segmented sort: one replay of the lane's captured HIP graph.  Lanes run
  on separate streams, so batches overlap.  A lane takes up to
  ``max_batch_keys`` keys and ``max_batch_requests`` requests; whatever has
  been admitted when a lane frees up goes in.
* Completion: every batch copies the plan's device status words to pinned
  host memory behind its sort; when the batch has finished they are read,
  and a batch whose sort reported an error fails its Futures with that
  BinarError (the server carries on).  Otherwise each request's results are
  views of that batch's output tensors (keys, permutation); its budget is
  released and its Future set.
* Cancelling a Future before its batch starts frees its budget.
* Streams: a lane's resident buffers are made and filled on the lane's own
  stream, and a batch's outputs are allocated there.  A Future is set only
  once its batch has finished on the device, so its tensors can be read on
  any stream; a caller that reads them asynchronously on another stream and
  then drops them calls ``record_stream`` for that stream first (torch's
  caching allocator hands freed memory back to the lane's stream at once).

One scheduler thread does admission, packing, launches and completion; the
device work lives in a backend object (``DeviceBackend``), so the policy can
be exercised with a host-only backend.
"""
from __future__ import annotations

import threading
import time
from collections import defaultdict, deque
from concurrent.futures import Future
from dataclasses import dataclass

from .binar import BINAR_ENOMEM, KEY_FLOAT, KEY_UNSIGNED, BinarError, key_bytes_of

META_BYTES = 256


def request_cost(key_bytes: int, n: int) -> int:
    return 2 * (key_bytes + 4) * n + META_BYTES


@dataclass
class SortResult:
    keys: object          # sorted keys, same shape and dtype as the request
    perm: object          # int32 tensor: perm[i] = input index of keys[i]
    submitted: float
    admitted: float
    launched: float
    done: float
    batch_requests: int

    @property
    def latency(self) -> float:
        return self.done - self.submitted


@dataclass
class _Req:
    id: int
    keys: object
    kb: int
    n: int
    cost: int
    future: Future
    submitted: float
    ready_event: object = None
    admitted: float = 0.0
    launched: float = 0.0
    kind: int = 0

    @property
    def cls(self):
        """Requests batch together when their key width and kind agree."""
        return (self.kb, self.kind)


class Admission:
    """HBM-budget accounting with a FIFO wait queue (no device work).

    ``in_use`` counts the bytes of admitted, unfinished requests plus the
    bytes of every lane charged so far (``fixed``, never released).  A class
    (key width and kind) holds ``lanes[cls]`` charged lanes, of which
    ``reserved[cls]`` are charged but not yet created."""

    def __init__(self, budget: int):
        if budget <= 0:
            raise ValueError("budget must be positive")
        self.budget = int(budget)
        self.in_use = 0
        self.fixed = 0
        self.peak = 0
        self.waiting: deque = deque()
        self.lanes = defaultdict(int)
        self.reserved = defaultdict(int)

    def _lane_need(self, r, lane_cost) -> int:
        return lane_cost(r.cls) if lane_cost is not None and self.lanes[r.cls] == 0 else 0

    def offer(self, req: _Req, lane_cost=None) -> None:
        """Queue a request; BINAR_ENOMEM if it can never fit (its cost, plus
        its class's first lane if none is charged yet, beside the lanes
        already held)."""
        if self.fixed + req.cost + self._lane_need(req, lane_cost) > self.budget:
            raise BinarError(BINAR_ENOMEM)
        self.waiting.append(req)

    def _charge(self, nbytes: int) -> None:
        self.in_use += nbytes
        self.peak = max(self.peak, self.in_use)

    def admit(self, now: float, lane_cost=None) -> list:
        """Admit from the head of the queue while the budget allows.  The
        first admitted request of a class without a lane also reserves the
        class's first lane.  Requests cancelled while waiting are dropped
        without being charged; a head request that lanes charged since its
        offer leave no room for fails with BINAR_ENOMEM."""
        out = []
        while self.waiting:
            r = self.waiting[0]
            if r.future.cancelled():
                self.waiting.popleft()
                continue
            need = self._lane_need(r, lane_cost)
            if self.fixed + r.cost + need > self.budget:
                self.waiting.popleft()
                if r.future.set_running_or_notify_cancel():
                    r.future.set_exception(BinarError(BINAR_ENOMEM))
                continue
            if self.in_use + r.cost + need > self.budget:
                break
            self.waiting.popleft()
            if need:
                self.fixed += need
                self.lanes[r.cls] += 1
                self.reserved[r.cls] += 1
            self._charge(r.cost + need)
            r.admitted = now
            out.append(r)
        return out

    def take_lane(self, cls, nbytes: int) -> bool:
        """May a new lane of `cls` be created?  Uses a reserved lane, else
        charges `nbytes` if the budget has room for them."""
        if self.reserved[cls] > 0:
            self.reserved[cls] -= 1
            return True
        if self.in_use + nbytes > self.budget:
            return False
        self.fixed += nbytes
        self.lanes[cls] += 1
        self._charge(nbytes)
        return True

    def release(self, cost: int) -> None:
        self.in_use -= cost
        assert self.in_use >= self.fixed


class Server:
    """Continuous-batching sort server; see the module docstring."""

    def __init__(self, budget_bytes: int = 8 << 30, backend=None, streams: int = 2,
                 max_batch_keys: int = 1 << 25, max_batch_requests: int = 1024, batching: bool = True,
                 params_lookup=None, clock=time.perf_counter):
        self.max_batch_keys = int(max_batch_keys)
        self.max_batch_requests = int(max_batch_requests) if batching else 1
        self.clock = clock
        self.admission = Admission(budget_bytes)
        self.backend = backend if backend is not None else DeviceBackend(
            streams, self.max_batch_keys, self.max_batch_requests, params_lookup)
        self._cv = threading.Condition()
        self._ready = defaultdict(deque)   # (key width, key kind) -> admitted requests
        self._inflight: list = []
        self._next_id = 0
        self._running = True
        self._error = None
        self.records: list = []            # (n, submitted, admitted, launched, done, batch size) per request
        self.batches = 0
        self.failed_batches = 0
        self.max_waiting = 0
        self._thread = threading.Thread(target=self._loop, name="binar-serve", daemon=True)
        self._thread.start()

    # ------------------------------------------------------------ client side
    def submit(self, keys, key_kind: int | None = None) -> Future:
        """Queue one request.  `keys` is not modified; the caller must not
        modify it either until the Future is done.  key_kind: KEY_* of
        binar.py; default KEY_FLOAT for floating-point tensors, else
        KEY_UNSIGNED."""
        kb = key_bytes_of(keys)
        n = int(keys.shape[0])
        if key_kind is None:
            key_kind = KEY_FLOAT if keys.is_floating_point() else KEY_UNSIGNED
        if kb == 16 and key_kind != KEY_UNSIGNED:
            raise ValueError("16-byte keys are byte strings: key_kind must be KEY_UNSIGNED")
        if n > self.max_batch_keys:
            raise BinarError(BINAR_ENOMEM)
        fut: Future = Future()
        with self._cv:
            if not self._running:
                raise RuntimeError("server is closed")
            if self._error is not None:
                raise RuntimeError("server failed") from self._error
            req = _Req(self._next_id, keys, kb, n, request_cost(kb, n), fut, self.clock(), kind=key_kind)
            req.ready_event = self.backend.mark_ready(keys)
            self.admission.offer(req, self.backend.lane_cost)   # BINAR_ENOMEM if it can never fit
            self._next_id += 1
            self.max_waiting = max(self.max_waiting, len(self.admission.waiting))
            self._cv.notify()
        return fut

    def close(self, wait: bool = True) -> None:
        with self._cv:
            self._running = False
            self._cv.notify()
        if wait:
            self._thread.join()
        if self._error is not None:
            raise RuntimeError("server failed") from self._error

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def report(self) -> dict:
        """Latency percentiles (seconds), throughput and counters over the
        requests finished so far."""
        recs = list(self.records)
        lat = sorted(r[4] - r[1] for r in recs)
        keys = sum(r[0] for r in recs)
        span = (max(r[4] for r in recs) - min(r[1] for r in recs)) if recs else 0.0

        def pct(p):
            if not lat:
                return None
            return lat[min(len(lat) - 1, int(round(p / 100.0 * (len(lat) - 1))))]
        return {"requests": len(lat), "keys": keys, "batches": self.batches, "failed_batches": self.failed_batches,
                "p50_s": pct(50), "p99_s": pct(99), "max_s": lat[-1] if lat else None,
                "throughput_keys_s": keys / span if span > 0 else None,
                "peak_admitted_bytes": self.admission.peak, "lane_bytes": self.admission.fixed,
                "max_waiting": self.max_waiting}

    # ------------------------------------------------------------- scheduler
    def _loop(self):
        try:
            self.backend.thread_init()
            while True:
                progressed = False
                with self._cv:
                    now = self.clock()
                    for r in self.admission.admit(now, self.backend.lane_cost):
                        self._ready[r.cls].append(r)
                        progressed = True
                    self._drop_cancelled()
                    batches = self._form_batches()
                    idle = (not self._running and not self.admission.waiting and not self._inflight
                            and not any(self._ready.values()) and not batches)
                if idle:
                    return
                for i, (lane, reqs) in enumerate(batches):
                    t = self.clock()
                    for r in reqs:
                        r.launched = t
                    try:
                        h = self.backend.launch(lane, reqs)
                    except BaseException:
                        # these requests are in no queue any more: fail them here
                        self._inflight += [(None, ln, rq) for ln, rq in batches[i:]]
                        raise
                    self._inflight.append((h, lane, reqs))
                    self.batches += 1
                    progressed = True
                still = []
                for item in self._inflight:
                    if self.backend.poll(item[0]):
                        self._complete(*item)
                        progressed = True
                    else:
                        still.append(item)
                self._inflight = still
                # hold no finished batch's outputs here: they are the callers' now
                h = item = batches = lane = reqs = None
                if not progressed:
                    with self._cv:
                        if self._running or self.admission.waiting or any(self._ready.values()):
                            self._cv.wait(timeout=0.0002 if self._inflight else 0.01)
        except BaseException as e:  # fail every pending request rather than hang the callers
            self._error = e
            with self._cv:
                pending = list(self.admission.waiting) + [r for q in self._ready.values() for r in q]
                pending += [r for _, _, reqs in self._inflight for r in reqs]
                self.admission.waiting.clear()
                for q in self._ready.values():
                    q.clear()
            for r in pending:
                if not r.future.done():
                    r.future.set_exception(e)

    def _drop_cancelled(self):
        for cls, q in self._ready.items():
            if any(r.future.cancelled() for r in q):
                keep = deque()
                for r in q:
                    if r.future.cancelled():
                        self.admission.release(r.cost)
                    else:
                        keep.append(r)
                self._ready[cls] = keep

    def _form_batches(self) -> list:
        out = []
        for cls, q in self._ready.items():
            while q:
                lane = self.backend.free_lane(
                    cls, lambda c=cls: self.admission.take_lane(c, self.backend.lane_cost(c)))
                if lane is None:
                    break
                reqs, keys = [], 0
                while q and len(reqs) < self.max_batch_requests and keys + q[0].n <= self.max_batch_keys:
                    r = q.popleft()
                    if not r.future.set_running_or_notify_cancel():
                        self.admission.release(r.cost)
                        continue
                    reqs.append(r)
                    keys += r.n
                if not reqs:
                    self.backend.release_lane(lane)
                    continue
                out.append((lane, reqs))
        return out

    def _complete(self, handle, lane, reqs):
        try:
            outs = self.backend.collect(handle)
        except BinarError as e:         # the batch's sort reported an error: fail its requests only
            outs = e
        t = self.clock()
        with self._cv:
            for r in reqs:
                self.admission.release(r.cost)
            self._cv.notify()
        self.backend.release_lane(lane)
        if isinstance(outs, BinarError):
            self.failed_batches += 1
            for r in reqs:
                r.future.set_exception(outs)
            return
        for r, (k, p) in zip(reqs, outs):
            self.records.append((r.n, r.submitted, r.admitted, r.launched, t, len(reqs)))
            r.future.set_result(SortResult(k, p, r.submitted, r.admitted, r.launched, t, len(reqs)))


ALLOC_SLACK = 9 << 20
"""Bytes charged per lane beyond its buffers' sizes: the caching allocator
may hand out a block up to 1 MiB larger than asked for, and a lane makes up
to nine live allocations (four resident buffers, four batch outputs and
temporaries, one spare)."""


class _Lane:
    """Resident buffers of one stream and key class: keys, permutation,
    segment table (device and pinned host copy), pinned status words, and a
    plan whose graph is captured on the first batch and replayed for every
    later one."""

    def __init__(self, kb: int, kind: int, cap: int, max_segments: int, device, params):
        import torch
        from .binar import Plan
        self.kb, self.kind, self.cap, self.max_segments = kb, kind, cap, max_segments
        self.stream = torch.cuda.Stream(device=device)
        # allocated and filled on the lane's own stream, which every batch
        # runs on: the stream of the thread that makes the lane is not
        # ordered with it (filled there, the first batch could copy the
        # permutation's start from memory arange had not written yet)
        with torch.cuda.stream(self.stream):
            if kb == 16:
                self.keys = torch.empty((cap, 16), dtype=torch.uint8, device=device)
            else:
                self.keys = torch.empty(cap, dtype=torch.int32 if kb == 4 else torch.int64, device=device)
            self.pay = torch.empty(cap, dtype=torch.int32, device=device)
            self.iota = torch.arange(cap, dtype=torch.int32, device=device)
            self.off_dev = torch.zeros(max_segments + 1, dtype=torch.int32, device=device)
        self.off_host = torch.zeros(max_segments + 1, dtype=torch.int32, pin_memory=True)
        self.status = torch.zeros(2, dtype=torch.int32, pin_memory=True)
        self.plan = Plan(kb, cap, max_segments, True, params)
        self.done = torch.cuda.Event()
        self.busy = False

    @staticmethod
    def resident_bytes(kb: int, cap: int, max_segments: int) -> int:
        """Device bytes of the buffers above (the plan's workspace aside)."""
        return cap * (kb + 4 + 4) + 4 * (max_segments + 1)


class DeviceBackend:
    """Runs batches on the GPU: lanes are created on first use, up to
    `streams` per key class, each only once the server has charged it."""

    def __init__(self, streams: int, cap: int, max_segments: int, params_lookup=None, device=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.streams, self.cap, self.max_segments = streams, cap, max_segments
        self.params_lookup = params_lookup
        self.lanes = defaultdict(list)     # (key width, key kind) -> lanes
        self._params = {}
        self._cost = {}

    def thread_init(self):
        self.torch.cuda.set_device(self.device)

    def _lane_params(self, cls):
        if cls not in self._params:
            from .binar import Params
            kb, kind = cls
            base = None if self.params_lookup is None else self.params_lookup(kb, self.cap)
            self._params[cls] = Params(**{**(vars(base) if base is not None else {}), "key_kind": kind})
        return self._params[cls]

    def lane_cost(self, cls) -> int:
        """Device bytes one lane of `cls` holds: its resident buffers, its
        plan's workspace and the allocator slack."""
        if cls not in self._cost:
            from .binar import workspace_bytes
            kb = cls[0]
            ws = workspace_bytes(kb, self.cap, True, self.max_segments, self._lane_params(cls))
            self._cost[cls] = _Lane.resident_bytes(kb, self.cap, self.max_segments) + ws + ALLOC_SLACK
        return self._cost[cls]

    def mark_ready(self, keys):
        """Device keys: an event on the submitting thread's current stream,
        which the lane waits for before reading them.  Host keys (pinned
        memory, for an asynchronous upload) need none."""
        if not keys.is_contiguous():
            raise ValueError("keys must be contiguous")
        if not keys.is_cuda:
            return None
        if keys.device != self.device:
            raise ValueError("keys must live on %s or in host memory" % self.device)
        ev = self.torch.cuda.Event()
        ev.record()
        return ev

    def free_lane(self, cls, may_create):
        """An idle lane of `cls` (marked busy), or a new one when fewer than
        `streams` exist and may_create() agrees (it charges the lane)."""
        kb, kind = cls
        for lane in self.lanes[cls]:
            if not lane.busy:
                lane.busy = True
                return lane
        if len(self.lanes[cls]) < self.streams and may_create():
            lane = _Lane(kb, kind, self.cap, self.max_segments, self.device, self._lane_params(cls))
            self.lanes[cls].append(lane)
            lane.busy = True
            return lane
        return None

    def release_lane(self, lane):
        lane.busy = False

    def launch(self, lane, reqs):
        torch = self.torch
        outs = []
        with torch.cuda.stream(lane.stream):
            pos = 0
            offs = lane.off_host.numpy()
            offs[0] = 0
            for i, r in enumerate(reqs):
                if r.ready_event is not None:
                    lane.stream.wait_event(r.ready_event)
                if r.n:
                    # bits, not values: a float request lands in the integer lane unchanged
                    lane.keys[pos:pos + r.n].copy_(r.keys.view(lane.keys.dtype), non_blocking=True)
                    if r.keys.is_cuda:
                        r.keys.record_stream(lane.stream)
                pos += r.n
                offs[i + 1] = pos
            m = len(reqs)
            offs[m + 1:] = pos              # the unused segments are empty
            lane.off_dev.copy_(lane.off_host, non_blocking=True)
            lane.pay[:pos].copy_(lane.iota[:pos], non_blocking=True)
            lane.plan.sort(lane.keys, lane.pay, lane.off_dev, stream=lane.stream)
            lane.plan.status_async(lane.status, stream=lane.stream)
            # one output pair per batch; each request gets views of its range,
            # its permutation made request-local by subtracting its start
            out_keys = lane.keys[:pos].clone()
            starts = lane.off_dev[:m]
            lens = lane.off_dev[1:m + 1] - starts
            out_perm = lane.pay[:pos] - torch.repeat_interleave(starts, lens, output_size=pos)
            start = 0
            for r in reqs:
                outs.append((out_keys[start:start + r.n].view(r.keys.dtype), out_perm[start:start + r.n]))
                start += r.n
            lane.done.record(lane.stream)
        return (lane, outs)

    def poll(self, handle) -> bool:
        return handle[0].done.query()

    def collect(self, handle):
        """The batch's per-request outputs, once its status words (copied
        behind the sort, complete with the batch) show no error; otherwise
        BinarError with the sort's status."""
        from .binar import status_of_words
        lane, outs = handle
        err, ovf = (int(w) & 0xFFFFFFFF for w in lane.status.tolist())
        st = status_of_words(err, ovf)
        if st != 0:
            raise BinarError(st)
        return outs
