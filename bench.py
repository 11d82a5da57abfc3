#!/usr/bin/env python3
"""Benchmark of the gfx950 stable binar sort on one MI355X.

One step = one complete sort (every global pass + the LDS finish) of one
batch of 2^28 uniform uint32 keys carrying a uint32 index payload, already
resident in HBM.  Each step sorts its own unsorted copy (prepared before the
timed region), so no step sorts sorted data.

Prints ONE JSON line: Gkeys/s over the timed steps, the roofline of the
kernel that takes the most time (algorithmic bytes / its average launch time,
from HIP events recorded on the kernel's own stream inside the timed
region), and the CPU oracle timed on a bounded sample on one host core.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gkeys/s and % HBM peak, 2^28 uint32+u32 payload; p50/p99 batched-serve latency"
HBM_PEAK_GBS = 8000.0
INPLACE_DEFAULT_DIGIT_BITS = 4  # the in-place variant's digit width when none is given
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_0811_3448_amd", "csrc")


# the sources the fixed-width sort's kernels and launches are built from
# (the string and in-place paths live in files of their own)
TRAFFIC_SOURCES = ("binar_api.hip", "binar_host.h", "binar_keys.h", "binar_kernels.h", "binar_launch_4p.hip",
                   "binar_launch_4k.hip", "binar_launch_8p.hip", "binar_launch_8k.hip", "binar_launch_16p.hip",
                   "binar_launch_16k.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources (else None)."""
    path = os.path.join(PROFILES, "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256") != kernel_source_hash():
        return None
    return t.get("traffic_bytes_per_launch")


def copy_ceiling(torch, dev, nbytes: int = 2 << 30, reps: int = 5):
    """Achievable bandwidth on the day, timed with HIP events (median of
    reps): torch's device-to-device copy of nbytes, and the library's own
    streaming copy (read + write bytes) and read-only pass over the same
    buffer, each at its best of a few launch shapes (blocks per CU x 16-byte
    vectors in flight per thread)."""
    import ctypes
    import paper_0811_3448_amd as binar
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty_like(src)
    out = torch.zeros(1 << 14, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    vp = ctypes.c_void_p

    def median_ms(fn):
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2]

    def check(rc):
        if rc != 0:
            raise RuntimeError("stream kernel status %d" % rc)

    res = {"torch_copy_gbs": round(2 * nbytes / (median_ms(lambda: dst.copy_(src)) * 1e-3) / 1e9, 1)}
    best_c, best_r = (0.0, None), (0.0, None)
    for bpc, unroll in ((1, 4), (2, 4), (2, 8), (4, 8)):
        c = median_ms(lambda: check(binar.lib.binar_stream_copy(vp(dst.data_ptr()), vp(src.data_ptr()), nbytes, bpc,
                                                                unroll, sp)))
        r = median_ms(lambda: check(binar.lib.binar_stream_read(vp(src.data_ptr()), nbytes, vp(out.data_ptr()), bpc,
                                                                unroll, sp)))
        best_c = max(best_c, (2 * nbytes / (c * 1e-3) / 1e9, (bpc, unroll)))
        best_r = max(best_r, (nbytes / (r * 1e-3) / 1e9, (bpc, unroll)))
    if not torch.equal(dst[:1 << 20], src[:1 << 20]):
        raise RuntimeError("stream copy check failed")
    del src, dst, out
    torch.cuda.empty_cache()
    res.update({"gbs": round(best_c[0], 1), "read_gbs": round(best_r[0], 1),
                "copy_shape": {"blocks_per_cu": best_c[1][0], "vectors_per_thread": best_c[1][1]},
                "read_shape": {"blocks_per_cu": best_r[1][0], "vectors_per_thread": best_r[1][1]},
                "bytes": nbytes,
                "what": "2 GiB: torch copy_; the library's streaming copy (read + write bytes, 'gbs') and "
                        "read-only pass ('read_gbs'), best launch shape, median of %d" % reps})
    return res


def cpu_baseline(keys_np, log2_sample: int):
    """The oracle (recursive stable binar partition in C) on one host core,
    on the first 2^log2_sample keys of the workload with an index payload."""
    import numpy as np
    import oracle
    n = min(keys_np.shape[0], 1 << log2_sample)
    k = keys_np[:n].copy()
    p = np.arange(n, dtype=np.uint32)
    oracle.build()
    t0 = time.perf_counter()
    oracle.sort(k, p)
    dt = time.perf_counter() - t0
    return {"value": n / dt / 1e9, "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": "first 2^%d keys (+ index payload) of the same workload, recursive stable binar "
                      "partition in C on one host core, %.1f s" % (log2_sample, dt)}


def cpu_more_baselines(keys_np, log2_sample: int) -> dict:
    """Two more host references on the same sample: std::stable_sort on one
    core, and the paper's parallel variant (one stable partition on the
    leading byte, then the buckets by the oracle on every core this process
    may use, at most 16)."""
    import numpy as np
    import oracle
    n = min(keys_np.shape[0], 1 << log2_sample)
    k = keys_np[:n].copy()
    p = np.arange(n, dtype=np.uint32)
    t0 = time.perf_counter()
    oracle.stable_sort_ref(k, p)
    dt_s = time.perf_counter() - t0
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    oracle.parallel_sort_ref(k, p, cores)
    dt_p = time.perf_counter() - t0
    return {"cpu_stable_sort": {"value": n / dt_s / 1e9, "unit": "Gkeys/s", "cores": 1, "kind": "std::stable_sort",
                                "sample": "first 2^%d keys (+ index payload), %.1f s" % (log2_sample, dt_s)},
            "cpu_parallel_variant": {"value": n / dt_p / 1e9, "unit": "Gkeys/s", "cores": cores,
                                     "kind": "leading-byte partition, then the oracle per bucket on %d threads"
                                             % cores,
                                     "sample": "first 2^%d keys (+ index payload), %.1f s" % (log2_sample, dt_p)}}


def choose_params(binar, args, kb, has_pay, n, batched):
    """Command-line knobs if any is given, else the autotune cache's entry
    for this case (tuned on the device), else the library defaults."""
    if args.digit_bits or args.tile_keys or args.finish_max or args.offsets:
        return binar.Params(args.digit_bits, args.tile_keys, args.finish_max, args.offsets), "command line"
    if not args.untuned:
        from paper_0811_3448_amd import tune
        p = tune.TuneCache(arch=tune.device_arch()).lookup(kb, has_pay, n, batched, max_distance=1)
        if p is not None:
            return p, "autotune cache"
    return binar.Params(), "library defaults"


def describe_params(binar, kb, has_pay, params, source):
    r = binar.resolve_params(kb, has_pay, params)
    return {"digit_bits": r.digit_bits, "tile_keys": r.tile_keys, "finish_max": r.finish_max,
            "offsets": "decoupled look-back" if r.offsets == 2 else "chunk prefixes", "params_from": source}


def per_array_calls(binar, torch, kbuf, pbuf, restore, offs, S, params, stream, np):
    """The same arrays sorted by one library call each, all enqueued on the
    stream with one workspace: (GPU ms between events, host seconds)."""
    ws = binar.Workspace(binar.workspace_bytes(4, int(max(b - a for a, b in zip(offs, offs[1:]))), True, 1,
                                               params))
    restore()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for s in range(S):
        a, b = offs[s], offs[s + 1]
        if b - a > 1:
            binar.sort(kbuf[a:b], pbuf[a:b], workspace=ws, params=params)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), time.perf_counter() - t0


def offs_of(off_np):
    return off_np.astype("int64").tolist()


def measure_batched(args, per_array: bool = True) -> dict:
    """Batched workload: 100,000 lognormal segments of u32 keys (+ global
    index payload), about 2^27 keys.  One HIP-graph replay of the segmented
    sort (median of the timed replays) against one plain library call per
    array on the same GPU (measured once)."""
    import numpy as np
    import torch
    import paper_0811_3448_amd as binar
    import workloads

    keys_np, off_np = workloads.batched_u32()
    n, S = int(off_np[-1]), off_np.shape[0] - 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pristine = torch.from_numpy(keys_np.view(np.int32)).to(dev)
    pay0 = torch.arange(n, dtype=torch.int32, device=dev)
    kbuf, pbuf = pristine.clone(), pay0.clone()
    off = torch.from_numpy(off_np.astype(np.uint32).view(np.int32)).to(dev)
    params, source = choose_params(binar, args, 4, True, n, batched=True)
    plan = binar.Plan(4, n, S, True, params)
    stream = torch.cuda.current_stream()

    def restore():
        kbuf.copy_(pristine)
        pbuf.copy_(pay0)

    for _ in range(args.warmup):
        restore()
        plan.sort(kbuf, pbuf, off)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        restore()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.sort(kbuf, pbuf, off)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    st = plan.stats()
    if st["status"] != 0:
        raise RuntimeError("batched sort status %d" % st["status"])
    # the last replay's output, checked on the device: every segment sorted,
    # its payload a permutation of its own indices, ties in index order
    seg = torch.repeat_interleave(torch.arange(S, device=dev), torch.diff(off.to(torch.int64)), output_size=n)
    u = kbuf.to(torch.int64) & 0xFFFFFFFF
    same = seg[1:] == seg[:-1]
    p = pbuf.to(torch.int64)
    ok = bool((u[1:] >= u[:-1])[same].all()) and bool((p[1:] > p[:-1])[same & (u[1:] == u[:-1])].all())
    ok = ok and torch.equal(torch.sort(p).values, torch.arange(n, device=dev)) and torch.equal(
        pristine.to(torch.int64)[p] & 0xFFFFFFFF, u) and bool((seg[p] == seg).all())
    if not ok:
        raise RuntimeError("batched output check failed")
    del seg, u, same, p
    graph_ms = float(np.median(times))

    # per-kernel breakdown: one eager call of the same sort, each launch
    # bracketed by events (outside the timed replays)
    restore()
    ws_b = binar.Workspace(binar.workspace_bytes(4, n, True, S, params))
    torch.cuda.synchronize()
    binar.profile_enable(True)
    binar.profile_read()
    binar.sort_segmented(kbuf, off, pbuf, workspace=ws_b, params=params)
    torch.cuda.synchronize()
    prof = binar.profile_read()
    binar.profile_enable(False)
    kernels = {}
    for nm, _p, ms in prof:
        kernels[nm] = round(kernels.get(nm, 0.0) + ms, 4)
    st_e = binar.stats(ws_b)
    del ws_b

    per_array_ms = per_array_wall = None
    if per_array:
        per_array_ms, per_array_wall = per_array_calls(binar, torch, kbuf, pbuf, restore, offs_of(off_np),
                                                       S, params, stream, np)
    plan.close()
    return {
        "graph_ms": round(graph_ms, 4), "gkeys_s": round(n / (graph_ms * 1e-3) / 1e9, 3),
        "segments": S, "n": n, **describe_params(binar, 4, True, params, source),
        "per_array_calls": None if per_array_ms is None else {
            "ms": round(per_array_ms, 2), "gkeys_s": round(n / (per_array_ms * 1e-3) / 1e9, 3),
            "host_wall_s": round(per_array_wall, 2), "measured": "once, every array by one library call"},
        "speedup_vs_per_array": None if per_array_ms is None else round(per_array_ms / graph_ms, 2),
        "finish_segments": st["finish_segments"], "passes": st["passes"],
        "eager_kernels_ms": kernels,
        "finish_class_segments": st_e["finish_class_segments"], "finish_class_keys": st_e["finish_class_keys"],
        "finish_small_segments": st_e["finish_small_segments"],
    }


def bench_batched(args) -> int:
    r = measure_batched(args, per_array=not args.no_per_array)
    result = {
        "metric": "Gkeys/s, batched segmented sort of 100,000 arrays in one graph replay",
        "value": r["gkeys_s"], "unit": "Gkeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["graph_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "batched_u32_100k: %d lognormal segments (median 1024, sigma 0.7356), %d u32 keys "
                               "+ u32 index payload" % (r["segments"], r["n"]), "segments": r["segments"],
                   "n": r["n"], "digit_bits": r["digit_bits"], "tile_keys": r["tile_keys"],
                   "finish_max": r["finish_max"], "offsets": r["offsets"], "params_from": r["params_from"]},
        **{k: v for k, v in r.items() if k not in ("graph_ms", "gkeys_s", "segments", "n", "digit_bits",
                                                     "tile_keys", "finish_max", "offsets", "params_from")},
    }
    print(json.dumps(result), flush=True)
    return 0


def measure_serve(args, R: int) -> dict:
    """Serving workload: R sort requests with Poisson arrivals, sizes
    lognormal (median 2^16, sigma 2 ln 2, clipped to [2^8, 2^24]), key widths
    u32 / u64 / 16-byte strings = 50 / 30 / 20 % (strings: a lowercase prefix
    of 0..12 bytes shared by the request, the rest lowercase), each answered
    with sorted keys and permutation.  Keys start in pinned host memory, so
    latency (arrival to the batch's completion event) includes the upload.
    A saturating run (all requests at once) calibrates the rate: the timed
    runs use 0.7 of its request rate, once with continuous batching
    (segmented graph replays, two streams per width) and once with one
    request per launch in arrival order.  A last, untimed run of the same
    requests checks every answer on the device (sorted, the permutation a
    permutation, keys following it, ties in input order)."""
    import numpy as np
    import torch
    import workloads
    from paper_0811_3448_amd import tune
    from paper_0811_3448_amd.serve import Server

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    trace = workloads.serve_requests(R, rate_per_s=1.0)     # unit rate: arrival times scale with 1/rate
    print("bench: serve pools", file=sys.stderr, flush=True)
    pool_n = 1 << 24
    pools = {(4, 0): torch.from_numpy(workloads.u32_uniform(pool_n, 401).view(np.int32)).pin_memory(),
             (8, 0): torch.from_numpy(workloads.u64_uniform(pool_n, 402).view(np.int64)).pin_memory()}
    for L in range(13):
        pools[(16, L)] = torch.from_numpy(workloads.str16(pool_n, 410 + L, L)).pin_memory()
    rng = np.random.default_rng(0x5E7E)
    reqs = []
    for t in trace:
        key = (t["key_bytes"], t["prefix_len"] if t["key_bytes"] == 16 else 0)
        start = int(rng.integers(0, pool_n - t["n"] + 1))
        reqs.append(pools[key][start:start + t["n"]])
    unit_arrivals = np.array([t["arrival_s"] for t in trace])
    unit_arrivals -= unit_arrivals[0]
    total_keys = int(sum(t["n"] for t in trace))
    cache = tune.TuneCache(arch=tune.device_arch())

    def lookup(kb, cap):
        return cache.lookup(kb, True, cap, True, max_distance=4)

    def make_server(batching):
        return Server(budget_bytes=args.serve_budget_gib << 30, streams=2, max_batch_keys=1 << 25,
                      max_batch_requests=1024, batching=batching, params_lookup=lookup)

    def run(batching, rate):
        srv = make_server(batching)
        warm = [srv.submit(pools[k][:4096]) for k in ((4, 0), (8, 0), (16, 0)) for _ in range(2)]
        for f in warm:
            f.result()
        srv.records.clear()
        srv.batches = 0
        t0 = time.perf_counter()
        for i in range(R):
            if rate is not None:
                delay = t0 + unit_arrivals[i] / rate - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            srv.submit(reqs[i])
            if i % 2000 == 0:
                print("bench: serve %s rate %s: submitted %d/%d" % ("batched" if batching else "one-per-launch",
                                                                    rate, i, R), file=sys.stderr, flush=True)
        srv.close()
        return srv.report()

    def check_all():
        """Every request once more through the batching server (untimed),
        each answer checked on the device as it completes."""
        srv = make_server(True)
        futs = [srv.submit(r) for r in reqs]
        bad = 0
        for i, r in enumerate(reqs):
            res = futs[i].result()
            futs[i] = None    # each answer is dropped once checked
            kin = r.to(dev, non_blocking=True)
            p = res.perm.to(torch.int64)
            n = kin.shape[0]
            if kin.dim() == 2:       # 16-byte strings: compare as two big-endian 64-bit halves
                be = kin.view(torch.uint8).reshape(n, 16).to(torch.int64)
                w = torch.stack([(be[:, i * 8:(i + 1) * 8] << torch.arange(56, -8, -8, device=dev)).sum(1)
                                 for i in range(2)], 1)
                ko = res.keys.view(torch.uint8).reshape(n, 16).to(torch.int64)
                wo = torch.stack([(ko[:, i * 8:(i + 1) * 8] << torch.arange(56, -8, -8, device=dev)).sum(1)
                                  for i in range(2)], 1)
                flip = -(1 << 63)
                a, b = wo[:-1] ^ flip, wo[1:] ^ flip
                order = (a[:, 0] < b[:, 0]) | ((a[:, 0] == b[:, 0]) & (a[:, 1] <= b[:, 1]))
                tie = (a[:, 0] == b[:, 0]) & (a[:, 1] == b[:, 1])
                follows = torch.equal(w[p], wo)
            else:
                u_in = kin.to(torch.int64) & 0xFFFFFFFF if kin.dtype == torch.int32 else kin ^ (-(1 << 63))
                u_out = res.keys.to(torch.int64) & 0xFFFFFFFF if kin.dtype == torch.int32 else res.keys ^ (-(1 << 63))
                order = u_out[1:] >= u_out[:-1]
                tie = u_out[1:] == u_out[:-1]
                follows = torch.equal(u_in[p], u_out)
            ok = bool(order.all()) and follows and torch.equal(torch.sort(p).values, torch.arange(n, device=dev))
            ok = ok and bool((p[1:] > p[:-1])[tie].all())
            bad += 0 if ok else 1
        srv.close()
        return bad

    sat = run(True, None)
    # requests per second of the saturating run (first submission to last completion)
    rate = 0.7 * sat["throughput_keys_s"] / (total_keys / R)
    batched = run(True, rate)
    fifo = run(False, rate)
    print("bench: serve: checking every answer", file=sys.stderr, flush=True)
    bad = check_all()
    if bad:
        raise RuntimeError("serving: %d of %d answers failed the check" % (bad, R))

    def fmt(rep):
        return {"p50_ms": round(rep["p50_s"] * 1e3, 3), "p99_ms": round(rep["p99_s"] * 1e3, 3),
                "max_ms": round(rep["max_s"] * 1e3, 3),
                "throughput_gkeys_s": round(rep["throughput_keys_s"] / 1e9, 3),
                "requests_per_s": round(rep["requests"] * rep["throughput_keys_s"] / rep["keys"], 1),
                "batches": rep["batches"], "requests": rep["requests"],
                "peak_admitted_gib": round(rep["peak_admitted_bytes"] / 2 ** 30, 3),
                "lanes_gib": round(rep["lane_bytes"] / 2 ** 30, 3), "failed_batches": rep["failed_batches"],
                "max_waiting": rep["max_waiting"]}
    del pools, reqs
    torch.cuda.empty_cache()
    return {"requests": R, "keys": total_keys, "rate_req_s": round(rate, 1), "budget_gib": args.serve_budget_gib,
            "saturated": fmt(sat), "batched": fmt(batched), "one_request_per_launch": fmt(fifo),
            "answers_checked": R}


def bench_serve(args) -> int:
    r = measure_serve(args, args.serve_requests)
    b = r["batched"]
    result = {
        "metric": "serving throughput (Gkeys/s) with p50/p99 latency, Poisson sort requests",
        "value": b["throughput_gkeys_s"], "unit": "Gkeys/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(r["keys"] / (b["throughput_gkeys_s"] * 1e9) * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32/u64/u8x16",
        "data": "synthetic",
        "config": {"workload": "serve_c5: %d requests, Poisson at 0.7 x saturated rate, sizes lognormal "
                               "(median 2^16, sigma 2 ln 2) in [2^8, 2^24], u32/u64/16 B = 50/30/20 %%, "
                               "keys in pinned host memory, u32 index payload" % r["requests"],
                   "requests": r["requests"], "keys": r["keys"], "rate_req_s": r["rate_req_s"],
                   "budget_gib": r["budget_gib"]},
        "saturated": r["saturated"], "batched": r["batched"],
        "one_request_per_launch": r["one_request_per_launch"], "answers_checked": r["answers_checked"],
    }
    print(json.dumps(result), flush=True)
    return 0


def measure_small(args) -> dict:
    """Single array of 2^16 uniform u32 keys, keys only: the library's plain
    call (events around each call on the stream, the host's launches
    included) and a plan's graph replay on the same buffers; medians."""
    import numpy as np
    import torch
    import paper_0811_3448_amd as binar
    import workloads
    n = 1 << 16
    keys = workloads.single_keys("u32_2e16_uniform_keys")
    dev = torch.device("cuda:0")
    pristine = torch.from_numpy(keys.view(np.int32)).to(dev)
    kd = pristine.clone()
    stream = torch.cuda.current_stream()
    ws = binar.Workspace(binar.workspace_bytes(4, n, False, 1), device=dev)
    plan = binar.Plan(4, n, 1, False)

    def timed(fn, reps=30):
        for _ in range(3):
            kd.copy_(pristine)
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            kd.copy_(pristine)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))
    eager = timed(lambda: binar.sort(kd, workspace=ws))
    replay = timed(lambda: plan.sort(kd))
    ok = bool(((kd.to(torch.int64) & 0xFFFFFFFF).diff() >= 0).all())
    plan.close()
    if not ok:
        raise RuntimeError("small sort output not sorted")
    return {"n": n, "eager_us": round(eager * 1e3, 1), "plan_replay_us": round(replay * 1e3, 1),
            "what": "2^16 uniform u32 keys only; median of 30 sorts, events on the stream"}


def linear_fit(xs, ys):
    """Least-squares line y = a + b x: (a, b, R^2, largest relative residual)."""
    import numpy as np
    x, y = np.asarray(xs, dtype=np.float64), np.asarray(ys, dtype=np.float64)
    b, a = np.polyfit(x, y, 1)
    pred = a + b * x
    ss_res = float(((y - pred) ** 2).sum())
    ss_tot = float(((y - y.mean()) ** 2).sum())
    return float(a), float(b), 1.0 - ss_res / ss_tot if ss_tot > 0 else 1.0, float(np.max(np.abs(y - pred) / y))


def bench_linearity(args) -> int:
    """The paper's performance experiment (section "Performance of
    Algorithm"): 32-bit integers from a Mersenne Twister, sizes from 1 to 10
    million by a fixed step, each timed as the mean of 10 sorts, to show that
    time grows linearly with N.  Keys only.  The GPU runs every size; the CPU
    oracle every millionth (one sort each)."""
    import numpy as np
    import torch
    import paper_0811_3448_amd as binar

    lo, hi, step, iters = 1_000_000, 10_000_000, args.lin_step, 10
    mt = np.random.RandomState(0x0811)          # MT19937
    full = mt.randint(0, 1 << 32, size=hi, dtype=np.uint64).astype(np.uint32)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pristine = torch.from_numpy(full.view(np.int32)).to(dev)
    work = torch.empty_like(pristine)
    from paper_0811_3448_amd import tune as _tune
    ws = binar.Workspace(max([binar.workspace_bytes(4, hi, False, 1, c) for c in _tune.candidates(4, False)]
                             + [binar.workspace_bytes(4, hi, False)]), device=dev)
    stream = torch.cuda.current_stream()
    sizes = list(range(lo, hi + 1, step))
    gpu_ms, passes = [], []
    cache = None
    if not args.untuned:
        from paper_0811_3448_amd import tune
        cache = tune.TuneCache(arch=tune.device_arch())

    def params_for(n):
        p = None if cache is None else cache.lookup(4, False, n, False, max_distance=0)
        return p if p is not None else binar.Params()
    for _ in range(3):                          # first launches load the code objects
        work[:lo].copy_(pristine[:lo])
        binar.sort(work[:lo], workspace=ws)
    torch.cuda.synchronize()
    for k, n in enumerate(sizes):
        tot = 0.0
        prm = params_for(n)
        for _ in range(iters):
            work[:n].copy_(pristine[:n])
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            binar.sort(work[:n], workspace=ws, params=prm)
            e1.record(stream)
            e1.synchronize()
            tot += e0.elapsed_time(e1)
        gpu_ms.append(tot / iters)
        passes.append(binar.stats(ws)["passes"])
        if k % max(1, len(sizes) // 10) == 0:
            print("bench: linearity n=%d %.4f ms" % (n, gpu_ms[-1]), file=sys.stderr, flush=True)
    u = work[:hi].to(torch.int64) & 0xFFFFFFFF
    if not bool((u[1:] >= u[:-1]).all().item()):
        raise RuntimeError("output not sorted")
    if args.lin_dump:
        with open(args.lin_dump, "w") as f:
            f.write("n,ms,passes\n")
            for n, m, q in zip(sizes, gpu_ms, passes):
                f.write("%d,%.5f,%d\n" % (n, m, q))
    cpu_sizes, cpu_ms = [], []
    if not args.no_cpu_baseline:
        import oracle
        for n in range(lo, hi + 1, 1_000_000):
            t0 = time.perf_counter()
            oracle.sort(full[:n].copy())
            cpu_ms.append((time.perf_counter() - t0) * 1e3)
            cpu_sizes.append(n)
            print("bench: linearity oracle n=%d %.1f ms" % (n, cpu_ms[-1]), file=sys.stderr, flush=True)
    ga, gb, gr2, gdev = linear_fit(sizes, gpu_ms)
    # the breadth-first passes come in whole numbers: time is a line per
    # number of global passes, with a step where N / 2^k first exceeds the
    # LDS-finish threshold
    by_passes = {}
    for pc in sorted(set(passes)):
        xs = [n for n, q in zip(sizes, passes) if q == pc]
        ys = [m for m, q in zip(gpu_ms, passes) if q == pc]
        if len(xs) >= 3:
            a, b, r2, dv = linear_fit(xs, ys)
            by_passes[str(pc)] = {"sizes": [xs[0], xs[-1]], "intercept_ms": round(a, 4), "ns_per_key": round(b * 1e6, 5),
                                  "r2": round(r2, 6), "max_rel_residual": round(dv, 4)}
    result = {
        "metric": "sort time vs N, MT19937 u32 keys, 1M..10M (linearity)", "value": round(gr2, 6),
        "unit": "R^2 of a straight-line fit of GPU time to N", "n_gpus": 1, "steps": iters,
        "warmup": 0, "ms_per_step": round(gpu_ms[-1], 4), "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "linearity: MT19937 u32 keys only, N = %d..%d step %d, mean of %d sorts per N"
                               % (lo, hi, step, iters), "sizes": len(sizes),
                   "params_from": "autotune cache per size bucket" if cache is not None else "library defaults"},
        "gpu": {"intercept_ms": round(ga, 4), "ns_per_key": round(gb * 1e6, 5), "r2": round(gr2, 6),
                "max_rel_residual": round(gdev, 4),
                "ms_at_millions": [round(gpu_ms[sizes.index(n)], 4) for n in range(lo, hi + 1, 1_000_000)
                                   if n in sizes],
                "gkeys_s_at_10M": round(hi / (gpu_ms[-1] * 1e-3) / 1e9, 3),
                "by_global_passes": by_passes},
    }
    if cpu_ms:
        ca, cb, cr2, cdev = linear_fit(cpu_sizes, cpu_ms)
        result["cpu_oracle"] = {"intercept_ms": round(ca, 2), "ns_per_key": round(cb * 1e6, 2), "r2": round(cr2, 6),
                                "max_rel_residual": round(cdev, 4), "ms_at_millions": [round(x, 1) for x in cpu_ms],
                                "cores": 1}
    print(json.dumps(result), flush=True)
    return 0


def bench_strings(args) -> int:
    """Variable-length byte strings: 2^24 strings of lowercase letters,
    lognormal lengths (mean 20 bytes), with no shared prefix and with a
    shared 40-byte prefix (several 15-byte rounds), sorted into memcmp order
    with an index payload (the permutation)."""
    import numpy as np
    import torch
    import paper_0811_3448_amd as binar
    import workloads

    n = 1 << args.str_log2
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    out = {}
    for label, prefix in (("no_prefix", 0), ("prefix40", 40)):
        data, offs = workloads.var_strings(n, 0x5771 + prefix, 20.0, 26, prefix)
        dd = torch.from_numpy(data).to(dev)
        od = torch.from_numpy(offs.view(np.int32)).to(dev)
        iota = torch.arange(n, dtype=torch.int32, device=dev)
        pay = iota.clone()
        ws = binar.Workspace(binar.strings_workspace_bytes(n), device=dev)
        for _ in range(args.warmup):
            pay.copy_(iota)
            binar.sort_strings(dd, od, pay, workspace=ws)
        times = []
        for _ in range(args.steps):
            pay.copy_(iota)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            binar.sort_strings(dd, od, pay, workspace=ws)
            e1.record(stream)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        # sanity: adjacent strings in order (sampled)
        p = pay.cpu().numpy().view(np.uint32)
        o = offs.astype(np.int64)
        for i in np.random.default_rng(1).integers(0, n - 1, 2000):
            a, b = int(p[i]), int(p[i + 1])
            sa, sb = data[o[a]:o[a + 1]].tobytes(), data[o[b]:o[b + 1]].tobytes()
            if sa > sb or (sa == sb and a > b):
                raise RuntimeError("strings out of order")
        out[label] = {"ms": round(ms, 3), "gstrings_s": round(n / (ms * 1e-3) / 1e9, 3),
                      "string_gbytes_s": round(int(offs[-1]) / (ms * 1e-3) / 1e9, 2),
                      "mean_len": round(int(offs[-1]) / n, 1)}
        del dd, od, pay, iota, ws
    result = {
        "metric": "variable-length string sort throughput (Gstrings/s)", "value": out["no_prefix"]["gstrings_s"],
        "unit": "Gstrings/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": out["no_prefix"]["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8 strings", "data": "synthetic",
        "config": {"workload": "str_var: 2^%d lowercase strings, lognormal lengths (mean 20 B), u32 index payload"
                               % args.str_log2, "n": n},
        "cases": out,
    }
    print(json.dumps(result), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="u32_2e28_uniform")
    ap.add_argument("--cpu-sample-log2", type=int, default=25)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: skip the 2^16-key, batched and serving measurements")
    ap.add_argument("--digit-bits", type=int, default=0)
    ap.add_argument("--tile-keys", type=int, default=0)
    ap.add_argument("--finish-max", type=int, default=0)
    ap.add_argument("--offsets", type=int, default=0, help="1 = chunk prefixes, 2 = decoupled look-back")
    ap.add_argument("--untuned", action="store_true", help="ignore the autotune cache: library defaults")
    ap.add_argument("--no-per-array", action="store_true", help="batched workload: skip the per-array comparison")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--lin-step", type=int, default=1000, help="linearity workload: size step")
    ap.add_argument("--str-log2", type=int, default=24, help="str_var workload: log2 of the string count")
    ap.add_argument("--lin-dump", default="", help="linearity workload: write n,ms,passes CSV here")
    ap.add_argument("--serve-budget-gib", type=int, default=32)
    ap.add_argument("--no-copy-ceiling", action="store_true",
                    help="skip the 2 GiB copy (counter runs calibrate on the bench's 1 GiB copies alone)")
    ap.add_argument("--inplace", action="store_true",
                    help="single-array workloads: the in-place variant (no scratch copy of the keys)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the sort runs on a single MI355X and has no "
              "multi-GPU path; run it with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    lib_path = os.path.join(ROOT, "paper_0811_3448_amd", "libbinar.so")
    if not os.path.exists(lib_path):
        sys.path.insert(0, os.path.join(ROOT, "paper_0811_3448_amd"))
        import build as _b  # noqa: E402
        _b.build()
    import paper_0811_3448_amd as binar
    import workloads

    if args.workload == "batched_u32_100k":
        return bench_batched(args)
    if args.workload == "serve_c5":
        return bench_serve(args)
    if args.workload == "linearity":
        return bench_linearity(args)
    if args.workload == "str_var":
        return bench_strings(args)

    name = args.workload
    kb, n, has_pay, desc = workloads.SINGLE[name]
    print("bench: generating %s (%s)" % (name, desc), file=sys.stderr, flush=True)
    keys_np = workloads.single_keys(name)
    if kb == 4:
        keys_t = torch.from_numpy(keys_np.view(np.int32))
    else:
        keys_t = torch.from_numpy(keys_np.view(np.int64))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pristine = keys_t.to(dev)
    pay0 = torch.arange(n, dtype=torch.int32, device=dev) if has_pay else None
    K, W = args.steps, args.warmup
    P = max(1, min(K, 3))  # sorts of the separate, profiled run (per-kernel times)
    bufs = [(pristine.clone(), None if pay0 is None else pay0.clone()) for _ in range(K + W + P)]
    params, source = choose_params(binar, args, kb, has_pay, n, batched=False)
    if args.inplace:
        # fixed pass shape (8-bit digits, 4096-key tiles, chunk prefixes)
        params, source = binar.Params(digit_bits=args.digit_bits, finish_max=args.finish_max), "in-place pass shape"
    if name.startswith("f32"):
        # IEEE-754 keys: same kernels, keys read through the order-preserving view
        params = binar.Params(**{**vars(params), "key_kind": binar.KEY_FLOAT})
    pp_ws_bytes = binar.workspace_bytes(kb, n, has_pay, 1, params)
    # the in-place variant has its own pass shape: size it with that
    ip_params = params if args.inplace else binar.Params(key_kind=params.key_kind)
    ip_ws_bytes = binar.inplace_workspace_bytes(kb, n, has_pay, ip_params)
    ws = binar.Workspace(ip_ws_bytes if args.inplace else pp_ws_bytes, device=dev)
    sort_fn = binar.sort_inplace if args.inplace else binar.sort
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    print("bench: warmup %d" % W, file=sys.stderr, flush=True)
    for i in range(W):
        sort_fn(bufs[i][0], bufs[i][1], workspace=ws, params=params)
    torch.cuda.synchronize()
    st = binar.stats(ws)
    if st["status"] != 0:
        raise RuntimeError("sort reported status %d" % st["status"])

    print("bench: timing %d steps" % K, file=sys.stderr, flush=True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    # one event between consecutive sorts (same stream, no sync): per-step
    # times for the median / min / max beside the total
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    t0 = time.perf_counter()
    ev0.record(stream)
    marks[0].record(stream)
    for i in range(W, W + K):
        sort_fn(bufs[i][0], bufs[i][1], workspace=ws, params=params)
        marks[i - W + 1].record(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = sorted(marks[j].elapsed_time(marks[j + 1]) for j in range(K))
    gpu_ms = ev0.elapsed_time(ev1)
    st = binar.stats(ws)
    if st["status"] != 0:
        raise RuntimeError("sort reported status %d" % st["status"])
    last = bufs[W + K - 1][0]

    # per-kernel times from a separate run of P more sorts with every launch
    # bracketed by HIP events on the launch stream (outside the timed steps,
    # so the headline carries no profiling events)
    print("bench: profiled run of %d sorts" % P, file=sys.stderr, flush=True)
    binar.profile_enable(True)
    binar.profile_read()
    for i in range(W + K, W + K + P):
        sort_fn(bufs[i][0], bufs[i][1], workspace=ws, params=params)
    torch.cuda.synchronize()
    launches = binar.profile_read()
    binar.profile_enable(False)
    if binar.stats(ws)["status"] != 0:
        raise RuntimeError("profiled sort reported a nonzero status")

    # the last timed batch must be sorted (in its key order) -- a cheap sanity check
    if name.startswith("f32"):
        v = last.view(torch.float32)
        ok = bool((v[1:] >= v[:-1]).all().item())
    elif kb == 4:
        u = last.to(torch.int64) & 0xFFFFFFFF
        ok = bool((u[1:] >= u[:-1]).all().item())
    else:
        s = last ^ (-(1 << 63))
        ok = bool((s[1:] >= s[:-1]).all().item())
    if not ok:
        raise RuntimeError("output not sorted")

    # algorithmic bytes per sort, per kernel kind (exact counters from the
    # device): the first-digit count reads the keys once; the digit counts of
    # later passes re-read keys the scatter has just moved, which is overhead
    # of this design (reported apart, not credited)
    pb = 4 if has_pay else 0
    per_kernel = {"k_hist": kb * st["hist_keys"][0]}
    count_overhead = sum(kb * x for x in st["hist_keys"][1:])
    if args.inplace:
        # each partitioned key is read and written by the tile sort, then
        # picked up and put down once by the cycle walk
        per_kernel["k_local"] = sum(2 * (kb + pb) * x for x in st["moved"])
        per_kernel["k_cycle"] = sum(2 * (kb + pb) * x for x in st["moved"])
    else:
        per_kernel["k_scatter"] = sum(2 * (kb + pb) * x for x in st["moved"])
    for c in range(4):
        per_kernel["k_finish%d" % c] = 2 * (kb + pb) * st["finish_class_keys"][c]
    per_kernel["k_finish_small"] = 2 * (kb + pb) * st["finish_small_keys"]
    total_bytes = sum(per_kernel.values())

    agg = {}
    for nm, _pass, ms in launches:
        a = agg.setdefault(nm, [0.0, 0])
        a[0] += ms
        a[1] += 1
    ranked = sorted(((v[0], nm) for nm, v in agg.items() if per_kernel.get(nm, 0) > 0), reverse=True)
    dom = ranked[0][1]
    dom_ms, dom_launches = agg[dom]
    bytes_per_launch = per_kernel[dom] * P / dom_launches
    avg_ms = dom_ms / dom_launches
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9

    # per global pass: digit count + offsets + scatter, against the pass's
    # algorithmic bytes (keys read by the count, keys + payload moved); then
    # the LDS finish as the last stage
    per_pass = []
    for j in range(16):
        ms = sum(m for nm, ps, m in launches if ps == j and nm in (
            "k_hist", "k_pscan", "k_plan", "k_scatter", "k_ip_clear", "k_local", "k_cycle", "k_small_pairs")) / P
        b = (kb * st["hist_keys"][0] if j == 0 else 0) + 2 * (kb + pb) * st["moved"][j] * (2 if args.inplace else 1)
        if b == 0:
            continue
        per_pass.append({"pass": j, "ms": round(ms, 4), "bytes": int(b),
                         "count_overhead_bytes": int(kb * st["hist_keys"][j]) if j else 0,
                         "gbs": round(b / (ms * 1e-3) / 1e9, 1),
                         "frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
    fin_ms = sum(m for nm, ps, m in launches if nm.startswith("k_finish")) / P
    fin_b = 2 * (kb + pb) * st["finish_keys"]
    if fin_b:
        per_pass.append({"pass": "finish", "ms": round(fin_ms, 4), "bytes": int(fin_b),
                         "gbs": round(fin_b / (fin_ms * 1e-3) / 1e9, 1),
                         "frac": round(fin_b / (fin_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})

    ms_per_step = gpu_ms / K
    value = n * K / (gpu_ms * 1e-3) / 1e9
    result = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 4),
        "step_ms": {"median": round(step_ms[K // 2], 4), "min": round(step_ms[0], 4), "max": round(step_ms[-1], 4)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if name.startswith("f32") else ("u32" if kb == 4 else ("u64" if kb == 8 else "u8x16")),
        "data": "synthetic",
        "config": {"workload": "%s%s: %s" % (name, " in place" if args.inplace else "", desc), "n": n,
                   "key_bytes": kb, "payload_bytes": pb, "variant": "in place" if args.inplace else "ping-pong",
                   **describe_params(binar, kb, has_pay, params, source),
                   "parallelism": "single GPU"},
        "workspace_bytes": {"used": int(ip_ws_bytes if args.inplace else pp_ws_bytes),
                            "in_place": int(ip_ws_bytes), "ping_pong": int(pp_ws_bytes),
                            "data": int((kb + pb) * n)},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom, name),
                     "bytes_per_launch": int(bytes_per_launch), "avg_launch_ms": round(avg_ms, 4),
                     "launches_per_step": dom_launches // P},
        "sort_roofline": {"algorithmic_bytes_per_step": int(total_bytes),
                          "count_overhead_bytes_per_step": int(count_overhead),
                          "achieved_gbs": round(total_bytes / (ms_per_step * 1e-3) / 1e9, 1),
                          "frac": round(total_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels_ms_per_step": {nm: round(v[0] / P, 4) for nm, v in sorted(agg.items())},
        "kernel_timing": "separate run of %d sorts after the timed steps, HIP events around every launch" % P,
        "passes": st["passes"],
        "per_pass": per_pass,
        "moved_per_pass": [x for x in st["moved"] if x],
        "wall_s": round(wall, 4),
    }
    if args.inplace:
        result["config"].update(digit_bits=args.digit_bits or INPLACE_DEFAULT_DIGIT_BITS, tile_keys=4096,
                                offsets="chunk prefixes",
                                finish_max=max(result["config"]["finish_max"], 256))
    del bufs
    torch.cuda.empty_cache()
    if not args.no_copy_ceiling:
        cc = copy_ceiling(torch, dev)
        result["copy_ceiling"] = cc
        result["roofline"]["frac_of_copy"] = round(achieved / cc["gbs"], 4)
        result["sort_roofline"]["frac_of_copy"] = round(total_bytes / (ms_per_step * 1e-3) / 1e9 / cc["gbs"], 4)
    if not args.no_extras and not args.inplace and name == "u32_2e28_uniform":
        # the other configurations, measured in the same run
        print("bench: 2^16 keys", file=sys.stderr, flush=True)
        result["c1_small"] = measure_small(args)
        print("bench: 100,000 arrays", file=sys.stderr, flush=True)
        result["c4_batched"] = measure_batched(args, per_array=not args.no_per_array)
        print("bench: serving", file=sys.stderr, flush=True)
        result["c5_serve"] = measure_serve(args, args.serve_requests)
    if not args.no_cpu_baseline:
        print("bench: CPU oracle sample", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(keys_np, args.cpu_sample_log2)
        print("bench: CPU library and parallel-variant samples", file=sys.stderr, flush=True)
        result.update(cpu_more_baselines(keys_np, args.cpu_sample_log2))
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
