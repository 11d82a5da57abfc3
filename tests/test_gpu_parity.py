"""GPU parity: libbinar.so (through the C ABI) against the CPU oracle,
element by element, keys and permutation bit-exact."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import gpu_sort, gpu_sort_segmented, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def iota(n):
    return np.arange(n, dtype=np.uint32)


def P(k=0, tile=0, T=0, offsets=0):
    from paper_0811_3448_amd import Params
    return Params(digit_bits=k, tile_keys=tile, finish_max=T, offsets=offsets)


def compare(keys, with_payload=True, params=None):
    n = keys.shape[0]
    pay = iota(n) if with_payload else None
    print("case n=%d kb=%d payload=%s params=%s" % (n, oracle.key_bytes_of(keys), with_payload, params),
          flush=True)
    gk, gp = gpu_sort(keys, pay, params=params)
    rk, rp = oracle.sort(keys, pay)
    assert np.array_equal(gk, rk), "keys differ"
    if with_payload:
        assert np.array_equal(gp, rp), "permutation differs"


EDGE = [0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF, 0x80000001, 0x00010000, 0xFF]


@pytest.mark.parametrize("n", [0, 1, 2, 3, 64, 65, 1000, 8192, 8193, 50_000])
def test_u32_uniform_sizes(n):
    compare(workloads.u32_uniform(n, 1000 + n))


def test_u32_keys_only_2e16():
    compare(workloads.single_keys("u32_2e16_uniform_keys"), with_payload=False)


@pytest.mark.parametrize("dist", ["and4", "dup256", "edge", "equal", "sorted", "reversed"])
def test_u32_distributions(dist):
    n = 300_000
    keys = {"and4": lambda: workloads.u32_and4(n, 7),
            "dup256": lambda: workloads.u32_dup(n, 8, 256),
            "edge": lambda: workloads.small_alphabet_u32(n, 9, EDGE),
            "equal": lambda: np.full(n, 0x12345678, dtype=np.uint32),
            "sorted": lambda: np.sort(workloads.u32_uniform(n, 10)),
            "reversed": lambda: np.sort(workloads.u32_uniform(n, 11))[::-1].copy()}[dist]()
    compare(keys)


@pytest.mark.parametrize("offsets", [1, 2])
@pytest.mark.parametrize("k,tile,T", [(8, 4096, 64), (8, 2048, 300), (4, 4096, 100), (4, 2048, 1000),
                                      (1, 4096, 64), (1, 2048, 5000), (8, 4096, 1)])
def test_u32_global_passes(k, tile, T, offsets):
    """Small LDS threshold: many tiles per segment, several global passes,
    chunk prefixes or look-back across tiles, ragged last tiles."""
    n = 100_003
    compare(workloads.u32_uniform(n, 20 + k), params=P(k, tile, T, offsets))
    compare(workloads.u32_and4(n, 21 + k), params=P(k, tile, T, offsets))
    compare(workloads.u32_dup(n, 22 + k, 256), params=P(k, tile, T, offsets))


@pytest.mark.parametrize("k", [5, 6, 7])
@pytest.mark.parametrize("kb", [4, 8, 16])
def test_odd_digit_widths(k, kb):
    """Digits of 5, 6 or 7 bits straddle byte (and, for 16-byte keys, word)
    boundaries, and the last pass takes fewer than k bits."""
    n = 90_001
    keys = {4: lambda: workloads.u32_uniform(n, 60 + k), 8: lambda: workloads.u64_zipf(n, 61 + k, 1 << 12, 1.1),
            16: lambda: workloads.str16(n, 62 + k, 7)}[kb]()
    for T, offsets in ((0, 1), (150, 1), (150, 2)):
        compare(keys, params=P(k, 4096, T, offsets))
    if kb == 4:
        compare(workloads.u32_and4(n, 63 + k), params=P(k, 4096, 1, 1))


@pytest.mark.parametrize("offsets", [1, 2])
def test_u32_many_chunks(offsets):
    """Several million keys: every chunk holds many tiles, pieces of many
    segments, both offset schemes."""
    n = 3_000_017
    compare(workloads.u32_uniform(n, 90), params=P(offsets=offsets))
    compare(workloads.u32_and4(n, 91), params=P(T=2000, offsets=offsets))


@pytest.mark.parametrize("offsets", [1, 2])
@pytest.mark.parametrize("n", [6143, 6145, 3 * 6144 + 1, 100_003])
def test_u64_6144_tile(n, offsets):
    """The 6144-key tile of 8-byte keys (768 threads): ragged last tiles,
    both offset schemes, several global passes."""
    compare(workloads.u64_uniform(n, 70), params=P(8, 6144, 64, offsets))
    compare(workloads.u64_nearly_sorted(n, 71, 0.01), params=P(8, 6144, 64, offsets))


@pytest.mark.parametrize("dist", ["uniform", "nearly", "zipf", "dup"])
@pytest.mark.parametrize("T", [0, 200])
def test_u64(dist, T):
    n = 200_001
    keys = {"uniform": lambda: workloads.u64_uniform(n, 31),
            "nearly": lambda: workloads.u64_nearly_sorted(n, 32, 0.01),
            "zipf": lambda: workloads.u64_zipf(n, 33, 1 << 12, 1.1),
            "dup": lambda: workloads.u64_uniform(16, 34)[workloads.below(n, 35, 16).astype(np.int64)]}[dist]()
    compare(keys, params=P(T=T))


@pytest.mark.parametrize("prefix", [0, 5, 12, 16])
@pytest.mark.parametrize("T", [0, 100])
def test_str16(prefix, T):
    n = 60_000
    compare(workloads.str16(n, 40 + prefix, prefix), params=P(T=T))


@pytest.mark.parametrize("kb", [4, 8, 16])
def test_keys_only_widths(kb):
    n = 77_777
    keys = {4: lambda: workloads.u32_uniform(n, 51), 8: lambda: workloads.u64_uniform(n, 52),
            16: lambda: workloads.str16(n, 53, 3)}[kb]()
    compare(keys, with_payload=False, params=P(T=500))


def test_determinism():
    keys = workloads.u32_and4(500_000, 61)
    a = gpu_sort(keys, iota(keys.shape[0]))
    b = gpu_sort(keys, iota(keys.shape[0]))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("T", [0, 50])
def test_segmented_small(T):
    keys, off = workloads.batched_u32(300, seed=71, median=200, sigma=1.2, max_len=20_000)
    off = off.copy()
    off[10] = off[9]            # empty segment
    off[20] = off[19] + 1       # one-key segment
    off = np.maximum.accumulate(off)
    n = keys.shape[0]
    print("segmented n=%d S=%d T=%d" % (n, 300, T), flush=True)
    gk, gp = gpu_sort_segmented(keys, off, iota(n), params=P(T=T))
    rk, rp = oracle.sort_segmented(keys, off, iota(n))
    assert np.array_equal(gk, rk)
    assert np.array_equal(gp, rp)


@pytest.mark.parametrize("offsets", [1, 2])
def test_segmented_u64_6144_tile(offsets):
    """Segments of 8-byte keys through the 6144-key tile: lognormal sizes up
    to several tiles, an empty and a one-key segment, chunk prefixes or
    look-back across a segment's tiles, several global passes (T = 64)."""
    _, off = workloads.batched_u32(200, seed=73, median=3000, sigma=1.0, max_len=40_000)
    n = int(off[-1])
    keys = workloads.u64_uniform(n, 74)
    off = off.copy()
    off[10] = off[9]            # empty segment
    off[20] = off[19] + 1       # one-key segment
    off = np.maximum.accumulate(off)
    print("segmented u64 tile 6144 n=%d offsets=%d" % (n, offsets), flush=True)
    gk, gp = gpu_sort_segmented(keys, off, iota(n), params=P(8, 6144, 64, offsets))
    rk, rp = oracle.sort_segmented(keys, off, iota(n))
    assert np.array_equal(gk, rk)
    assert np.array_equal(gp, rp)


@pytest.mark.parametrize("kb", [4, 8, 16])
def test_finish_class_boundaries(kb):
    """Segments exactly at and just past every LDS-finish class capacity
    (4-byte keys 1024, 2048, 5120, 8192; 8-byte keys 1024, 2304, 5120, 8192;
    16-byte keys 1024, 2048, 3072, 5120), at unaligned offsets, each
    finished by its class or split by a pass."""
    caps = {4: [1024, 2048, 5120, 8192], 8: [1024, 2304, 5120, 8192], 16: [1024, 2048, 3072, 5120]}[kb]
    lens = []
    for c in caps:
        lens += [c - 1, c, c + 1]
    lens += [1, 2, 3, 63, 65]
    off = np.zeros(len(lens) + 1, dtype=np.uint32)
    off[1:] = np.cumsum(lens)
    n = int(off[-1])
    keys = {4: lambda: workloads.u32_uniform(n, 300), 8: lambda: workloads.u64_uniform(n, 301),
            16: lambda: workloads.str16(n, 302, 2)}[kb]()
    print("class boundaries kb=%d n=%d segments=%d" % (kb, n, len(lens)), flush=True)
    gk, gp = gpu_sort_segmented(keys, off, iota(n))
    rk, rp = oracle.sort_segmented(keys, off, iota(n))
    assert np.array_equal(gk, rk)
    assert np.array_equal(gp, rp)


@pytest.mark.parametrize("runlen", [1, 2, 63, 64, 65, 200])
def test_tied_runs_after_leading_bits(runlen):
    """The LDS finish sorts by the leading 16 varying bits and then orders
    each run of keys tied on them: runs of up to 64 keys by ranking inside
    one wave, longer ones by passes over every varying bit.  Segments whose
    keys share their leading bits in runs of a chosen length, the rest random,
    with ties in the full key as well."""
    rng = np.random.default_rng(runlen)
    lens = [int(x) for x in rng.integers(100, 5000, 40)]
    off = np.zeros(len(lens) + 1, dtype=np.uint32)
    off[1:] = np.cumsum(lens)
    n = int(off[-1])
    groups = max(1, n // runlen)
    lead = rng.integers(0, 1 << 16, groups, dtype=np.uint64)[rng.integers(0, groups, n)]
    low = rng.integers(0, 1 << 20, n, dtype=np.uint64)
    low[rng.random(n) < 0.2] = 7                           # full-key ties too
    keys = ((lead << np.uint64(48)) | low).astype(np.uint64)
    print("tied runs len=%d n=%d" % (runlen, n), flush=True)
    gk, gp = gpu_sort_segmented(keys, off, iota(n))
    rk, rp = oracle.sort_segmented(keys, off, iota(n))
    assert np.array_equal(gk, rk)
    assert np.array_equal(gp, rp)
    k32 = (lead.astype(np.uint32) << np.uint32(16)) | (low & np.uint64(0xFFFF)).astype(np.uint32)
    gk, gp = gpu_sort_segmented(k32, off, iota(n))
    rk, rp = oracle.sort_segmented(k32, off, iota(n))
    assert np.array_equal(gk, rk)
    assert np.array_equal(gp, rp)


def mixed_runs(n, seed, kb=4):
    """Runs of equal keys (whole waves on one digit), runs drawn from two or
    three values (waves with a few digits), and stretches of random keys, in
    random order and lengths: the digit count's wave-step peeling switches
    on and off inside one segment, and its miss counter restarts."""
    rng = np.random.default_rng(seed)
    top = (1 << 32) if kb == 4 else (1 << 64)
    dt = np.uint32 if kb == 4 else np.uint64
    parts, left = [], n
    while left > 0:
        ln = int(min(left, rng.integers(1, 3000)))
        kind = rng.integers(0, 3)
        if kind == 0:
            part = np.full(ln, rng.integers(0, top, dtype=np.uint64), dtype=np.uint64)
        elif kind == 1:
            vals = rng.integers(0, top, int(rng.integers(2, 4)), dtype=np.uint64)
            part = vals[rng.integers(0, vals.shape[0], ln)]
        else:
            part = rng.integers(0, top, ln, dtype=np.uint64)
        parts.append(part.astype(dt))
        left -= ln
    return np.concatenate(parts)


@pytest.mark.parametrize("kb", [4, 8])
@pytest.mark.parametrize("k,tile,T", [(8, 8192, 5120), (8, 4096, 64), (4, 2048, 300)])
def test_mixed_runs(kb, k, tile, T):
    if kb == 8 and tile == 8192:
        tile = 6144         # 8-byte keys: the largest tile is 6144 keys
    compare(mixed_runs(200_003, 40 + kb + k, kb), params=P(k, tile, T, 1))


@pytest.mark.parametrize("kb", [4, 8])
def test_sorted_runs_first_pass_pairs(kb):
    """2^26 keys in long sorted runs: the first pass of one large array counts
    digit pairs, and its waves hold one pair bin for long stretches (peeled
    pairs, bins that pass 65535 inside a block); the result is checked on
    the device completely and at sampled oracle ranks."""
    import torch
    import paper_0811_3448_amd as binar
    from oracle.definition import stable_rank_u
    from test_gpu_fullsize import device_checks
    n = 1 << 26
    base = workloads.u32_uniform(n, 4242) if kb == 4 else workloads.u64_uniform(n, 4243)
    keys = base.copy()
    runs = 64
    for r in range(runs):       # sorted runs of n / 64 keys each
        lo, hi = r * (n // runs), (r + 1) * (n // runs)
        keys[lo:hi] = np.sort(base[lo:hi])
    print("sorted runs kb=%d n=%d" % (kb, n), flush=True)
    kin = torch.from_numpy(keys.view(np.int32 if kb == 4 else np.int64)).cuda()
    kd = kin.clone()
    pd = torch.arange(n, dtype=torch.int32, device="cuda")
    binar.sort(kd, pd, params=P(8, 8192 if kb == 4 else 4096, 5120, 1))
    torch.cuda.synchronize()
    assert binar.stats()["status"] == 0
    device_checks(kin, kd, pd, kb)
    gk = kd.cpu().numpy().view(keys.dtype)
    gp = pd.cpu().numpy().view(np.uint32)
    for i in workloads.below(12, 4244 + kb, n).astype(np.int64).tolist() + [0, n - 1]:
        r = stable_rank_u(keys, i)
        assert gp[r] == i and gk[r] == keys[i], i
