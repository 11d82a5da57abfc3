"""Full-size parity: the 2^28 u32 and 2^27 u64 workloads (with index
payload, every distribution) sorted in the configuration bench.py times,
then checked completely on the device (nondecreasing, payload a
permutation, keys follow the payload, ties in input order: together these
fix the unique stable sort) and at sampled inputs against the oracle's
stable rank computed one element at a time."""
import numpy as np
import pytest

import workloads
from gpu_util import need_gpu
from oracle.definition import stable_rank_u

pytestmark = pytest.mark.gpu

SAMPLES = 12


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def bench_params(kb, n):
    """The parameters bench.py runs with: the autotune cache's entry for
    this case when there is one, else the library defaults."""
    from paper_0811_3448_amd import Params, tune
    p = tune.TuneCache(arch=tune.device_arch()).lookup(kb, True, n, False, max_distance=1)
    return p if p is not None else Params()


def device_checks(kin, kout, pout, kb):
    import torch
    n = kin.shape[0]
    if kb == 4:
        u = kout.to(torch.int64) & 0xFFFFFFFF
    else:
        u = kout ^ torch.tensor(-(1 << 63), dtype=torch.int64, device=kout.device)   # unsigned order as signed
    assert bool((u[1:] >= u[:-1]).all()), "not sorted"
    del u
    p = pout.to(torch.int64)
    assert bool(((p >= 0) & (p < n)).all()), "payload out of range"
    seen = torch.zeros(n, dtype=torch.int8, device=kout.device)
    seen[p] = 1
    assert bool(seen.all()), "payload is not a permutation"
    del seen
    assert torch.equal(kin[p], kout), "keys do not follow the payload"
    tie = kout[1:] == kout[:-1]
    assert bool((p[1:][tie] > p[:-1][tie]).all()), "unstable on ties"


@pytest.mark.parametrize("name", [k for k in workloads.SINGLE if k.endswith(("2e28_uniform", "2e28_and4",
                                                                              "2e28_dup256", "2e27_uniform",
                                                                              "2e27_nearly_sorted", "2e27_zipf"))])
def test_full_size(name):
    import torch
    import paper_0811_3448_amd as binar
    kb, n, has_pay, desc = workloads.SINGLE[name]
    print("full size %s: %s" % (name, desc), flush=True)
    keys = workloads.single_keys(name)
    dt = np.int32 if kb == 4 else np.int64
    kin = torch.from_numpy(keys.view(dt)).cuda()
    kout = kin.clone()
    pout = torch.arange(n, dtype=torch.int32, device="cuda")
    params = bench_params(kb, n)
    binar.sort(kout, pout, params=params)
    torch.cuda.synchronize()
    assert binar.stats()["status"] == 0
    print("  sorted with %s; device checks" % params, flush=True)
    device_checks(kin, kout, pout, kb)
    del kin
    rng = np.random.default_rng(n + kb)
    js = rng.integers(0, n, SAMPLES).tolist() + [0, n - 1]
    ranks = [stable_rank_u(keys, j) for j in js]
    kh = kout[torch.tensor(ranks, device="cuda")].cpu().numpy().view(keys.dtype)
    ph = pout[torch.tensor(ranks, device="cuda")].cpu().numpy()
    for j, r, k, p in zip(js, ranks, kh, ph):
        assert k == keys[j] and p == j, "input %d should sit at output %d" % (j, r)


@pytest.mark.parametrize("name", ["u32_2e28_uniform", "u32_2e28_and4", "u32_2e28_dup256", "u64_2e27_uniform",
                                  "u64_2e27_nearly_sorted", "u64_2e27_zipf"])
def test_full_size_inplace(name):
    """The in-place variant at full size, in the configuration
    `bench.py --inplace` times (library defaults: 4-bit digits)."""
    import torch
    import paper_0811_3448_amd as binar
    kb, n, has_pay, desc = workloads.SINGLE[name]
    print("full size in place %s: %s" % (name, desc), flush=True)
    keys = workloads.single_keys(name)
    dt = np.int32 if kb == 4 else np.int64
    kin = torch.from_numpy(keys.view(dt)).cuda()
    kout = kin.clone()
    pout = torch.arange(n, dtype=torch.int32, device="cuda")
    binar.sort_inplace(kout, pout, params=binar.Params())
    torch.cuda.synchronize()
    assert binar.stats()["status"] == 0
    print("  sorted in place; device checks", flush=True)
    device_checks(kin, kout, pout, kb)
    del kin
    rng = np.random.default_rng(n + kb + 1)
    js = rng.integers(0, n, SAMPLES).tolist() + [0, n - 1]
    ranks = [stable_rank_u(keys, j) for j in js]
    kh = kout[torch.tensor(ranks, device="cuda")].cpu().numpy().view(keys.dtype)
    ph = pout[torch.tensor(ranks, device="cuda")].cpu().numpy()
    for j, r, k, p in zip(js, ranks, kh, ph):
        assert k == keys[j] and p == j, "input %d should sit at output %d" % (j, r)


@pytest.mark.parametrize("prefix", [0, 40])
def test_full_size_strings(prefix):
    """2^24 variable-length strings as `bench.py --workload str_var` sorts
    them: every adjacent pair of outputs in order (bytes, then input index
    on equal strings: together with a permutation check this is the unique
    stable order), checked on the host."""
    import torch
    import paper_0811_3448_amd as binar
    n = 1 << 24
    data, offs = workloads.var_strings(n, 0x5771 + prefix, 20.0, 26, prefix)
    print("full size strings prefix=%d n=%d bytes=%d" % (prefix, n, data.shape[0]), flush=True)
    dd = torch.from_numpy(data).cuda()
    od = torch.from_numpy(offs.view(np.int32)).cuda()
    pd = torch.arange(n, dtype=torch.int32, device="cuda")
    binar.sort_strings(dd, od, pd)
    torch.cuda.synchronize()
    p = pd.cpu().numpy().view(np.uint32).astype(np.int64)
    seen = np.zeros(n, dtype=bool)
    seen[p] = True
    assert seen.all(), "not a permutation"
    # adjacent pairs: compare the strings byte-wise, vectorised over pairs by
    # a zero-padded fixed-width copy plus the lengths (the letters are never
    # zero, so padding never hides a difference)
    o = offs.astype(np.int64)
    lens = o[1:] - o[:-1]
    width = int(lens.max())
    pad = np.zeros((n, width), dtype=np.uint8)
    idx = np.arange(width)[None, :]
    for lo in range(0, n, 1 << 20):
        hi = min(n, lo + (1 << 20))
        ln = lens[lo:hi, None]
        src = np.minimum(o[lo:hi, None] + np.minimum(idx, np.maximum(ln - 1, 0)), data.shape[0] - 1)
        pad[lo:hi] = np.where(idx < ln, data[src], 0)
    a, b = p[:-1], p[1:]
    for lo in range(0, n - 1, 1 << 20):
        hi = min(n - 1, lo + (1 << 20))
        pa, pb = pad[a[lo:hi]], pad[b[lo:hi]]
        ne = pa != pb
        first = np.where(ne.any(axis=1), ne.argmax(axis=1), width)
        rows = np.arange(hi - lo)
        ca = np.where(first < width, pa[rows, np.minimum(first, width - 1)], 0).astype(np.int64)
        cb = np.where(first < width, pb[rows, np.minimum(first, width - 1)], 0).astype(np.int64)
        la, lb = lens[a[lo:hi]], lens[b[lo:hi]]
        # differing byte decides; else the shorter (a prefix) first; else input order
        less = np.where(first < np.minimum(la, lb), ca < cb,
                        np.where(la != lb, la < lb, a[lo:hi] < b[lo:hi]))
        assert less.all(), "pair %d out of order" % (lo + int(np.argmin(less)))
