"""Autotuner for libbinar.so on the device it runs on.

For one case -- key width, payload or not, size bucket (ceil log2 n), one
array or a batch of segments -- it times every built combination of

  * digit width k (1 = the one-bit partition step, 4 .. 8),
  * scatter tile (which fixes the scatter workgroup: 2048 keys -> 256
    threads, 4096 -> 512, 6144 -> 768, 8192 -> 1024),
  * LDS-finish threshold T (the largest sub-array one workgroup finishes
    on chip),
  * offset scheme (per-chunk counts, or decoupled look-back),

on synthetic keys of that case, and keeps the fastest.  Results live in a
JSON cache keyed by the device's architecture; ``install`` makes the cached
choice the library's default for plain calls, and the serving loop looks
parameters up per batch.

Timing uses HIP events on the current stream around the sort only; the
input is restored from a pristine copy before every timed call.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict
from typing import Callable

from .binar import Params, resolve_params, set_default_params, workspace_bytes

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.environ.get("BINAR_TUNE_CACHE", os.path.join(_HERE, "tuned_gfx950.json"))
FORMAT = 1

DIGIT_BITS = (1, 4, 5, 6, 7, 8)
TILE_THREADS = {2048: 256, 4096: 512, 6144: 768, 8192: 1024}


def bucket(n: int) -> int:
    """Size bucket: ceil(log2 n), 0 for n <= 1."""
    return max(0, int(n) - 1).bit_length()


def case_key(key_bytes: int, has_payload: bool, n: int, batched: bool) -> str:
    return "kb%d/pay%d/n%d/%s" % (key_bytes, 1 if has_payload else 0, bucket(n), "seg" if batched else "one")


def candidates(key_bytes: int, has_payload: bool) -> list:
    """Every built (k, tile, T, offsets) combination for this key width.
    The finish thresholds are the library's largest (its default) and two
    smaller ones that move more sub-arrays through the global passes."""
    tmax = resolve_params(key_bytes, has_payload, Params(finish_max=0xFFFFFFFF)).finish_max
    finish = sorted({tmax, (tmax * 5) // 8, (tmax * 3) // 8}, reverse=True)
    out = []
    for k in DIGIT_BITS:
        for tile in TILE_THREADS:
            for T in finish:
                for offsets in (1, 2):
                    p = Params(digit_bits=k, tile_keys=tile, finish_max=T, offsets=offsets)
                    if workspace_bytes(key_bytes, 1 << 16, has_payload, 1, p) > 0:
                        out.append(p)
    return out


def lognormal_offsets(n: int, median: float = 1024.0, sigma: float = 0.7356, seed: int = 1):
    """Segment table of lognormal lengths (clipped to [1, 2^20]) summing to
    exactly n, as uint32 numpy offsets."""
    import numpy as np
    rng = np.random.default_rng(seed)
    sizes = []
    total = 0
    while total < n:
        s = np.clip(np.rint(rng.lognormal(math.log(median), sigma, 4096)), 1, 1 << 20).astype(np.int64)
        sizes.append(s)
        total += int(s.sum())
    sizes = np.concatenate(sizes)
    cs = np.cumsum(sizes)
    m = int(np.searchsorted(cs, n)) + 1
    sizes = sizes[:m]
    sizes[-1] -= int(cs[m - 1]) - n
    off = np.zeros(m + 1, dtype=np.uint32)
    off[1:] = np.cumsum(sizes)
    return off


def synth_keys(key_bytes: int, n: int, seed: int = 1, device="cuda"):
    """Uniform random keys of the given width, generated on the device."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    if key_bytes == 4:
        return torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int32, device=device, generator=g)
    if key_bytes == 8:
        hi = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int32, device=device, generator=g)
        lo = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int32, device=device, generator=g)
        return (hi.to(torch.int64) << 32) | (lo.to(torch.int64) & 0xFFFFFFFF)
    if key_bytes == 16:
        return torch.randint(0, 256, (n, 16), dtype=torch.uint8, device=device, generator=g)
    raise ValueError("key_bytes must be 4, 8 or 16")


class DeviceTimer:
    """Times one sort configuration on resident synthetic data (median of
    `reps` event-timed calls after `warmup` untimed ones)."""

    def __init__(self, key_bytes: int, has_payload: bool, n: int, batched: bool = False, sample=None,
                 seg_offsets=None, reps: int = 3, warmup: int = 1, device="cuda"):
        import numpy as np
        import torch
        self.torch = torch
        self.key_bytes, self.has_payload, self.n, self.batched = key_bytes, has_payload, n, batched
        self.reps, self.warmup = reps, warmup
        self.pristine = synth_keys(key_bytes, n, device=device) if sample is None else sample.clone()
        self.keys = self.pristine.clone()
        self.pay0 = torch.arange(n, dtype=torch.int32, device=device) if has_payload else None
        self.pay = None if self.pay0 is None else self.pay0.clone()
        self.off = None
        if batched:
            off = lognormal_offsets(n) if seg_offsets is None else np.asarray(seg_offsets, dtype=np.uint32)
            self.nseg = off.shape[0] - 1
            self.off = torch.from_numpy(off.view(np.int32)).to(device)

    def _restore(self):
        self.keys.copy_(self.pristine)
        if self.pay is not None:
            self.pay.copy_(self.pay0)

    def __call__(self, params: Params) -> float:
        from .binar import Plan, Workspace, sort, stats
        torch = self.torch
        if self.batched:
            plan = Plan(self.key_bytes, self.n, self.nseg, self.has_payload, params)
            run = lambda: plan.sort(self.keys, self.pay, self.off)  # noqa: E731
        else:
            ws = Workspace(workspace_bytes(self.key_bytes, self.n, self.has_payload, 1, params),
                           device=self.keys.device)
            run = lambda: sort(self.keys, self.pay, workspace=ws, params=params)  # noqa: E731
        stream = torch.cuda.current_stream()
        times = []
        for i in range(self.warmup + self.reps):
            self._restore()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run()
            e1.record(stream)
            e1.synchronize()
            if i >= self.warmup:
                times.append(e0.elapsed_time(e1))
        # a configuration whose kernels bailed out (wait limit, list overflow)
        # returns early and would time as the fastest: read the device status
        # and check the last output (outside the timed calls) before trusting
        # the time
        st = plan.stats() if self.batched else stats(ws)
        ok = st["status"] == 0 and self._output_ok()
        if self.batched:
            plan.close()
        if not ok:
            return math.inf
        times.sort()
        return times[len(times) // 2]

    def _output_ok(self) -> bool:
        """The last sort's output is a sort of the input: keys nondecreasing
        inside every segment, payload a permutation that carries the keys."""
        torch = self.torch
        k = self.keys
        if self.key_bytes == 16:
            be = k.to(torch.int64)
            hi = torch.zeros(k.shape[0], dtype=torch.int64, device=k.device)
            lo = torch.zeros_like(hi)
            for b in range(8):
                hi = (hi << 8) | be[:, b]
                lo = (lo << 8) | be[:, 8 + b]
            hi, lo = hi ^ (-(1 << 63)), lo ^ (-(1 << 63))     # unsigned order as signed
            bad = (hi[1:] < hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] < lo[:-1]))
        elif self.key_bytes == 8:
            u = k ^ (-(1 << 63))
            bad = u[1:] < u[:-1]
        else:
            u = k.to(torch.int64) & 0xFFFFFFFF
            bad = u[1:] < u[:-1]
        if self.off is not None:
            cut = self.off.to(torch.int64)
            cut = cut[(cut > 0) & (cut < k.shape[0])] - 1       # pair (i, i+1) crosses a segment end
            bad[cut] = False
        if bool(bad.any().item()):
            return False
        if self.pay is None:
            return True
        p = self.pay.to(torch.int64)
        if not torch.equal(torch.sort(p).values, torch.arange(p.shape[0], device=p.device)):
            return False
        return bool(torch.equal(self.pristine[p], k))


TIE = 0.02  # candidates within this fraction of the fastest count as tied


def choose(table: list) -> int:
    """Index of the winning row of a timing table ([k, tile, T, offsets, ms],
    ms None for a failed candidate): among the rows within TIE of the
    fastest, the one with the largest LDS-finish threshold T, then the
    fastest of those.  A larger T that costs nothing measurable on the tuning
    keys finishes the larger sub-arrays of other distributions (nearly
    sorted, skewed) on chip instead of sending them through another global
    pass.  TIE is about the spread of the median of three timings between
    thresholds that do the same work on uniform keys."""
    timed = [i for i in range(len(table)) if table[i][4] is not None]
    fastest = min(table[i][4] for i in timed)
    tied = [i for i in timed if table[i][4] <= fastest * (1.0 + TIE)]
    return min(tied, key=lambda i: (-table[i][2], table[i][4], i))


def autotune(key_bytes: int, has_payload: bool, n: int, batched: bool = False,
             timer: Callable[[Params], float] | None = None, cands: list | None = None,
             log: Callable[[str], None] | None = None, **timer_kw) -> dict:
    """Time every candidate for one case and return the cache entry
    {"params", "ms", "gkeys_s", "n", "batched", "table"}; `timer` maps
    Params to milliseconds (default: DeviceTimer on synthetic keys)."""
    if n < 2:
        raise ValueError("nothing to tune for n < 2")
    cands = candidates(key_bytes, has_payload) if cands is None else cands
    timer = DeviceTimer(key_bytes, has_payload, n, batched, **timer_kw) if timer is None else timer
    table = []
    t0 = time.perf_counter()
    for p in cands:
        ms = float(timer(p))
        # a candidate that failed its status or output check is listed with
        # no time and never chosen
        table.append([p.digit_bits, p.tile_keys, p.finish_max, p.offsets,
                      round(ms, 5) if math.isfinite(ms) else None])
        if log:
            log("k=%d tile=%d T=%d offsets=%d: %s" % (p.digit_bits, p.tile_keys, p.finish_max, p.offsets,
                                                      "%.4f ms" % ms if math.isfinite(ms) else "FAILED"))
    timed = [i for i in range(len(table)) if table[i][4] is not None]
    if not timed:
        raise RuntimeError("autotune: every candidate failed its status or output check")
    best = choose(table)
    k, tile, T, off, ms = table[best]
    return {"params": {"digit_bits": k, "tile_keys": tile, "finish_max": T, "offsets": off},
            "ms": ms, "gkeys_s": round(n / (ms * 1e-3) / 1e9, 4) if ms > 0 else None, "n": n,
            "batched": batched, "workgroup": TILE_THREADS[tile], "tune_seconds": round(time.perf_counter() - t0, 2),
            "table": table}


class TuneCache:
    """JSON cache {"format", "arch", "entries": {case_key: entry}}."""

    def __init__(self, path: str = DEFAULT_CACHE, arch: str | None = None):
        self.path = path
        self.arch = arch
        self.entries: dict = {}
        if os.path.exists(path):
            with open(path) as f:
                data = json.load(f)
            if data.get("format") != FORMAT:
                raise ValueError("%s: unknown tune cache format %r" % (path, data.get("format")))
            if self.arch is None or data.get("arch") == self.arch:
                self.arch = data.get("arch")
                self.entries = dict(data.get("entries", {}))

    def put(self, key_bytes: int, has_payload: bool, n: int, batched: bool, entry: dict) -> None:
        self.entries[case_key(key_bytes, has_payload, n, batched)] = entry

    def save(self, path: str | None = None) -> None:
        path = path or self.path
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump({"format": FORMAT, "arch": self.arch, "entries": self.entries}, f, indent=1,
                      sort_keys=True)
            f.write("\n")
        os.replace(tmp, path)

    def lookup(self, key_bytes: int, has_payload: bool, n: int, batched: bool = False,
               max_distance: int = 2) -> Params | None:
        """Params of this case's bucket, else of the nearest tuned bucket of
        the same width/payload/batching within max_distance buckets (ties go
        to the larger bucket), else None."""
        want = bucket(n)
        prefix = "kb%d/pay%d/" % (key_bytes, 1 if has_payload else 0)
        suffix = "/seg" if batched else "/one"
        best = None
        for k, e in self.entries.items():
            if not (k.startswith(prefix) and k.endswith(suffix)):
                continue
            b = int(k[len(prefix):-len(suffix)].lstrip("n"))
            d = abs(b - want)
            if d <= max_distance and (best is None or (d, -b) < best[0]):
                best = ((d, -b), e)
        return None if best is None else Params(**best[1]["params"])

    def install(self) -> list:
        """Make the entry of the largest tuned single-array bucket of every
        (key width, payload) the library's default; returns what was set."""
        chosen = {}
        for k, e in self.entries.items():
            kb, pay, nb, kind = k.split("/")
            if kind != "one":
                continue
            cur = chosen.get((kb, pay))
            if cur is None or int(nb[1:]) > cur[0]:
                chosen[(kb, pay)] = (int(nb[1:]), e)
        done = []
        for (kb, pay), (_, e) in sorted(chosen.items()):
            p = Params(**e["params"])
            set_default_params(int(kb[2:]), pay == "pay1", p)
            done.append((int(kb[2:]), pay == "pay1", asdict(p)))
        return done


def device_arch() -> str:
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", "unknown").split(":")[0]


def main(argv=None) -> int:
    import argparse
    ap = argparse.ArgumentParser(description="Time libbinar.so configurations and cache the fastest.")
    ap.add_argument("--key-bytes", type=int, default=4, choices=(4, 8, 16))
    ap.add_argument("--no-payload", action="store_true")
    ap.add_argument("--log2n", type=int, nargs="+", default=[28])
    ap.add_argument("--batched", action="store_true", help="lognormal segments (median 1024) in one plan")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args(argv)
    cache = TuneCache(a.cache, arch=device_arch())
    cache.arch = device_arch()
    for lg in a.log2n:
        n = 1 << lg
        e = autotune(a.key_bytes, not a.no_payload, n, a.batched, reps=a.reps,
                     log=(lambda s: print(s, flush=True)) if a.verbose else None)
        cache.put(a.key_bytes, not a.no_payload, n, a.batched, e)
        cache.save()
        print(json.dumps({"case": case_key(a.key_bytes, not a.no_payload, n, a.batched),
                          "best": e["params"], "ms": e["ms"], "gkeys_s": e["gkeys_s"],
                          "candidates": len(e["table"]), "tune_seconds": e["tune_seconds"]}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
