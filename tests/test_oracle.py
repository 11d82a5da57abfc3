"""Pins for the CPU oracle (no GPU).

The oracle (recursive stable binar partition) is checked against things it
does not share code with: the paper's printed worked example, brute force over
all orderings, Python's and numpy's stable sorts (library special cases),
invariants written separately below, closed forms, and the bit-step bound of
the time analysis.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import definition
from oracle.swap_partition import binar_swap_sort
import workloads

HEX = "0123456789ABCDEF"


def nyb(xs):
    return [HEX.index(x) for x in xs]


# ---------------------------------------------------------------- invariants
def check_invariants(keys_in, keys_out, pay_out):
    """Permutation + gather + nondecreasing + stable; together these fix the
    stable sort uniquely.  Comparison is on big-endian bytes (the encoding)."""
    n = keys_in.shape[0]
    assert keys_out.shape == keys_in.shape
    seen = np.zeros(n, dtype=bool)
    seen[pay_out.astype(np.int64)] = True
    assert seen.all(), "payload is not a permutation"
    assert np.array_equal(keys_in[pay_out.astype(np.int64)], keys_out), "keys_out != keys_in[p]"
    for i in range(n - 1):
        a = definition.bit_string(keys_out, i)
        b = definition.bit_string(keys_out, i + 1)
        assert a <= b, "not nondecreasing at %d" % i
        if a == b:
            assert pay_out[i] < pay_out[i + 1], "unstable tie at %d" % i


def iota(n):
    return np.arange(n, dtype=np.uint32)


# ------------------------------------------------------ paper's worked example
@pytest.fixture(scope="module")
def example(golden_dir):
    with open(os.path.join(golden_dir, "worked_example.json")) as f:
        return json.load(f)


def test_swap_partition_reproduces_printed_configurations(example):
    trace = []
    out = binar_swap_sort(nyb(example["input"]), example["key_bits"], trace)
    assert out == nyb(example["sorted"])
    calls = {(b, lo, hi): states for (b, lo, hi, states) in trace}
    for name, bit in (("first_pass_bit1", 0), ("lower_subarray_bit2", 1), ("upper_subarray_bit2", 1)):
        t = example["traces"][name]
        lo, hi = t["bounds"]
        got = calls[(bit, lo, hi)]
        want = [tuple(nyb(part) for part in st) for st in t["states"]]
        assert [tuple(list(p) for p in st) for st in got] == [tuple(list(p) for p in st) for st in want]


def test_oracle_sorts_worked_example(example):
    keys = np.array(nyb(example["input"]), dtype=np.uint64)
    k, p, steps = oracle.sort_bits(keys, 4, iota(8), with_steps=True)
    assert k.tolist() == nyb(example["sorted"])
    # the two 0s keep input order (indices 2 then 3): the stable permutation
    assert p.tolist() == [2, 3, 1, 4, 5, 0, 6, 7]
    assert steps <= 4 * 8


def groups_after(keys_u64, nbits, width):
    """Split a partially partitioned array into runs of equal top-nbits prefix."""
    out, cur, prev = [], [], None
    for v in keys_u64.tolist():
        pre = v >> (width - nbits)
        if prev is not None and pre != prev:
            out.append(cur)
            cur = []
        cur.append(v)
        prev = pre
    if cur:
        out.append(cur)
    return out


def test_oracle_partial_states_match_printed_summary(example):
    keys = np.array(nyb(example["input"]), dtype=np.uint64)
    for b in (1, 2, 3, 4):
        k, _ = oracle.sort_bits(keys, 4, iota(8), nbits=b)
        got = [sorted(g) for g in groups_after(k, b, 4)]
        want = [sorted(nyb(g)) for g in example["reading_of_summary"]["bit%d" % b]]
        assert got == want, b
        if b <= 2:  # the printed rows for bits 1 and 2 agree with the bits
            printed = [sorted(nyb(g)) for g in example["printed_summary"]["bit%d" % b]]
            assert got == printed
    # stable order inside the groups after bit 1: input order of each group
    k, p = oracle.sort_bits(keys, 4, iota(8), nbits=1)
    assert [HEX[v] for v in k.tolist()] == list("4007BACE")
    assert p.tolist() == [1, 2, 3, 4, 0, 5, 6, 7]


def test_pins_detect_unstable_partition(example):
    """The paper's exchange partition swaps the two equal 0s; the stability
    invariant must reject it (a planted mistake, on the CPU)."""
    vals = nyb(example["input"])
    a = list(vals)
    idx = list(range(8))
    binar_swap_sort(a, 4, payload=idx)
    keys_in = np.array(vals, dtype=np.uint32)
    with pytest.raises(AssertionError):
        check_invariants(keys_in, np.array(a, dtype=np.uint32), np.array(idx, dtype=np.uint32))
    assert idx == [3, 2, 1, 4, 5, 0, 6, 7]


# ------------------------------------------------------------- brute force
def brute_force_stable(keys):
    """Enumerate every ordering; keep those that are nondecreasing and keep
    equal keys in input order.  Exactly one must survive."""
    n = keys.shape[0]
    enc = [definition.bit_string(keys, i) for i in range(n)]
    found = []
    for perm in itertools.permutations(range(n)):
        ok = True
        for a, b in zip(perm, perm[1:]):
            if enc[a] > enc[b] or (enc[a] == enc[b] and a > b):
                ok = False
                break
        if ok:
            found.append(perm)
    assert len(found) == 1
    return list(found[0])


U32_EDGE = [0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF, 0x80000001, 0x00010000]


@pytest.mark.parametrize("n,seed", [(0, 1), (1, 2), (2, 3), (3, 4), (5, 5), (6, 6), (7, 7), (8, 8)])
def test_brute_force_u32(n, seed):
    keys = workloads.small_alphabet_u32(n, seed, U32_EDGE[: 3 + seed % 5])
    want = brute_force_stable(keys) if n else []
    k, p = oracle.sort(keys, iota(n))
    assert p.tolist() == want
    assert k.tolist() == keys[np.array(want, dtype=np.int64)].tolist()


@pytest.mark.parametrize("n,seed", [(4, 11), (6, 12), (7, 13)])
def test_brute_force_u64(n, seed):
    alphabet = np.array([0, 1 << 63, (1 << 63) - 1, 0xFFFFFFFF, 1 << 32, (1 << 64) - 1], dtype=np.uint64)
    keys = alphabet[workloads.below(n, seed, len(alphabet)).astype(np.int64)]
    want = brute_force_stable(keys)
    k, p = oracle.sort(keys, iota(n))
    assert p.tolist() == want


@pytest.mark.parametrize("n,seed", [(5, 21), (7, 22)])
def test_brute_force_str16(n, seed):
    base = np.frombuffer(b"abcdefghijklmnop", dtype=np.uint8)
    alphabet = np.stack([base.copy() for _ in range(5)])
    alphabet[1, 0] = ord("b") - 1   # differs in the first byte
    alphabet[2, 15] = ord("a")      # differs in the last byte
    alphabet[3, 0] = 0xFF           # high bit of the first byte
    alphabet[4, 15] = 0x80
    keys = alphabet[workloads.below(n, seed, 5).astype(np.int64)]
    want = brute_force_stable(keys)
    k, p = oracle.sort(keys, iota(n))
    assert p.tolist() == want


# ------------------------------------------------- library special cases
@pytest.mark.parametrize("n,seed", [(1000, 31), (4097, 32), (100_000, 33)])
def test_matches_numpy_stable_argsort_u32(n, seed):
    keys = workloads.u32_uniform(n, seed)
    m = keys[::11].shape[0]
    keys[: 7 * m : 7] = keys[::11]  # inject ties
    k, p = oracle.sort(keys, iota(n))
    ref = np.argsort(keys, kind="stable")
    assert np.array_equal(p, ref.astype(np.uint32))
    assert np.array_equal(k, keys[ref])


@pytest.mark.parametrize("gen", ["uniform", "dup", "zipf", "nearly"])
def test_matches_numpy_stable_argsort_u64(gen):
    n = 20_000
    keys = {"uniform": lambda: workloads.u64_uniform(n, 41),
            "dup": lambda: workloads.u64_uniform(64, 42)[workloads.below(n, 43, 64).astype(np.int64)],
            "zipf": lambda: workloads.u64_zipf(n, 44, 1 << 10, 1.1),
            "nearly": lambda: workloads.u64_nearly_sorted(n, 45, 0.01)}[gen]()
    k, p = oracle.sort(keys, iota(n))
    ref = np.argsort(keys, kind="stable")
    assert np.array_equal(p, ref.astype(np.uint32))


def test_matches_stable_lexsort_str16():
    n = 5000
    keys = workloads.str16(n, 51, 6)
    m = keys[1::3].shape[0]
    keys[: 3 * m : 3] = keys[1::3]
    k, p = oracle.sort(keys, iota(n))
    ref = np.lexsort(tuple(keys[:, c] for c in range(15, -1, -1)))  # byte 0 is the primary key
    assert np.array_equal(p, ref.astype(np.uint32))


@pytest.mark.parametrize("kind,seed", [("u32", 61), ("u64", 62), ("str", 63), ("u32ties", 64)])
def test_matches_plain_definition(kind, seed):
    n = 1500
    keys = {"u32": lambda: workloads.u32_uniform(n, seed),
            "u64": lambda: workloads.u64_uniform(n, seed),
            "str": lambda: workloads.str16(n, seed, 10),
            "u32ties": lambda: workloads.small_alphabet_u32(n, seed, U32_EDGE)}[kind]()
    k, p = oracle.sort(keys, iota(n))
    dk, dp = definition.sort(keys, iota(n))
    assert np.array_equal(p, dp)
    assert np.array_equal(k, dk)
    check_invariants(keys, k, p)


# ---------------------------------------------------------- closed forms
def test_closed_forms():
    n = 777
    same = np.full(n, 0xDEADBEEF, dtype=np.uint32)
    _, p = oracle.sort(same, iota(n))
    assert np.array_equal(p, iota(n))                         # all equal -> identity
    inc = np.arange(n, dtype=np.uint32) * 3 + 5
    _, p = oracle.sort(inc, iota(n))
    assert np.array_equal(p, iota(n))                         # increasing -> identity
    dec = inc[::-1].copy()
    k, p = oracle.sort(dec, iota(n))
    assert np.array_equal(p, iota(n)[::-1])                   # decreasing distinct -> reversal
    assert np.array_equal(k, inc)


@pytest.mark.parametrize("bit", [0, 1, 15, 31])
def test_one_bit_difference_splits_at_that_bit(bit):
    n = 300
    base = np.uint32(0x5A5A5A5A) & ~np.uint32(1 << (31 - bit))
    sel = workloads.below(n, 70 + bit, 2).astype(bool)
    keys = np.where(sel, base | np.uint32(1 << (31 - bit)), base).astype(np.uint32)
    # before partitioning bit `bit` nothing moves; after it the zeros lead
    k0, p0 = oracle.partition(keys, iota(n), bit)
    assert np.array_equal(p0, iota(n))
    k1, p1 = oracle.partition(keys, iota(n), bit + 1)
    zeros = np.flatnonzero(~sel).astype(np.uint32)
    ones = np.flatnonzero(sel).astype(np.uint32)
    assert np.array_equal(p1, np.concatenate([zeros, ones]))


def test_partial_partition_equals_stable_sort_by_prefix():
    n = 50_000
    keys = workloads.u32_uniform(n, 81)
    for nbits in (1, 4, 8, 13, 16, 24, 32):
        k, p = oracle.partition(keys, iota(n), nbits)
        prefix = keys >> np.uint32(32 - nbits) if nbits < 32 else keys
        ref = np.argsort(prefix, kind="stable")
        assert np.array_equal(p, ref.astype(np.uint32)), nbits


def test_bit_step_bound():
    """Section "Recursion Analysis": at most (bits per key) visits per element."""
    for kb, keys in ((4, workloads.u32_uniform(30_000, 91)), (8, workloads.u64_uniform(30_000, 92)),
                     (16, workloads.str16(30_000, 93, 0))):
        n = keys.shape[0]
        _, _, steps = oracle.sort(keys, None, with_steps=True)
        assert 0 < steps <= 8 * kb * n
    # distinct keys with all bits examined: uniform u32 needs ~log2(n) levels each
    _, _, steps = oracle.sort(workloads.u32_uniform(1 << 14, 94), None, with_steps=True)
    assert steps >= 14 * (1 << 14) * 0.9


def test_small_and_empty():
    for n in (0, 1, 2):
        keys = workloads.u32_uniform(n, 100 + n)
        k, p = oracle.sort(keys, iota(n))
        assert sorted(keys.tolist()) == k.tolist()
    k, p = oracle.sort(np.array([5, 5], dtype=np.uint32), iota(2))
    assert p.tolist() == [0, 1]
    k, p = oracle.sort(np.array([0x80000000, 0x7FFFFFFF], dtype=np.uint32), iota(2))
    assert p.tolist() == [1, 0]


def test_segmented_is_per_segment():
    keys, off = workloads.batched_u32(200, seed=7, median=64, sigma=1.0, max_len=4000)
    n = keys.shape[0]
    off[5] = off[4]  # an empty segment
    k, p = oracle.sort_segmented(keys, off, iota(n))
    for s in range(200):
        a, b = int(off[s]), int(off[s + 1])
        if b < a:
            continue
        ref = np.argsort(keys[a:b], kind="stable").astype(np.uint32) + np.uint32(a)
        assert np.array_equal(p[a:b], ref), s


def test_appendix_exchange_sort_agrees_on_keys():
    """The paper's unstable exchange partition yields the same key order."""
    for seed in range(5):
        vals = workloads.u32_uniform(3000, 200 + seed)
        vals = (vals >> np.uint32(20)).astype(np.uint64)  # 12-bit keys: many ties
        out = binar_swap_sort(vals.tolist(), 12)
        k, _ = oracle.sort_bits(vals, 12)
        assert out == k.tolist()


# ---------------------------------------------------------------- key kinds
# The orders of signed and IEEE-754 keys (oracle.orders), pinned against
# numpy's own comparisons and against hand-written special-value orders.

def _f32_bits(x):
    return np.asarray(x, dtype=np.float32).view(np.uint32)


def _f64_bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


@pytest.mark.parametrize("width", [32, 64])
def test_kind_signed_matches_numpy(width):
    from oracle import orders
    rng = np.random.default_rng(width)
    it = np.int32 if width == 32 else np.int64
    ut = np.uint32 if width == 32 else np.uint64
    info = np.iinfo(it)
    v = rng.integers(info.min, info.max, 5000, dtype=it, endpoint=True)
    v[:6] = [info.min, info.max, -1, 0, 1, info.min + 1]
    v[6:400] = v[rng.integers(0, 6, 394)]                  # ties
    keys = v.view(ut)
    p = orders.stable_order(keys, orders.SIGNED)
    assert np.array_equal(p, np.argsort(v, kind="stable"))


@pytest.mark.parametrize("width", [32, 64])
def test_kind_float_matches_numpy_without_zero_or_nan(width):
    """numpy orders floats numerically (and keeps -0 == +0, NaN last), so
    the comparison leaves out zeros and NaNs; they are pinned below."""
    from oracle import orders
    rng = np.random.default_rng(100 + width)
    ft = np.float32 if width == 32 else np.float64
    v = (rng.standard_normal(5000) * 10.0 ** rng.integers(-30, 30, 5000)).astype(ft)
    v[:4] = [np.inf, -np.inf, np.finfo(ft).max, -np.finfo(ft).tiny / 4]  # infinities, max, a subnormal
    v[4:300] = v[rng.integers(0, 4, 296)]
    v[v == 0] = 1
    bits = v.view(np.uint32 if width == 32 else np.uint64)
    p = orders.stable_order(bits, orders.FLOAT)
    assert np.array_equal(p, np.argsort(v, kind="stable"))


def test_kind_float_special_values_order():
    from oracle import orders
    qnan = 0x7FC00000
    vals = [0x7F800000 | 1, qnan, 0xFFC00000, 0xFF800001,  # +sNaN, +qNaN, -qNaN, -sNaN
            0x7F800000, 0xFF800000,                          # +inf, -inf
            0x80000000, 0x00000000,                          # -0, +0
            0x00000001, 0x80000001,                          # +/- smallest subnormal
            _f32_bits(1.0), _f32_bits(-1.0), _f32_bits(2.5), _f32_bits(-2.5)]
    keys = np.array([int(x) for x in vals], dtype=np.uint32)
    p = orders.stable_order(keys, orders.FLOAT)
    expect = [0xFFC00000, 0xFF800001, 0xFF800000, _f32_bits(-2.5), _f32_bits(-1.0), 0x80000001,
              0x80000000, 0x00000000, 0x00000001, _f32_bits(1.0), _f32_bits(2.5), 0x7F800000,
              0x7F800000 | 1, qnan]
    # total order: -qNaN (payload 0x400000) is below -sNaN (payload 1), and
    # +sNaN below +qNaN
    assert [int(x) for x in keys[p]] == [int(x) for x in expect]


def test_kind_unsigned_matches_oracle():
    from oracle import orders
    keys = np.random.default_rng(5).integers(0, 1 << 32, 3000, dtype=np.uint64).astype(np.uint32)
    keys[100:800] = keys[:700] & 0xFF
    rk, rp = oracle.sort(keys, np.arange(3000, dtype=np.uint32))
    ok, op = orders.sort(keys, np.arange(3000, dtype=np.uint32), orders.UNSIGNED)
    assert np.array_equal(ok, rk) and np.array_equal(op, rp)


def test_kind_planted_mistake_fails():
    """A float order that forgets to reverse negative magnitudes must fail
    the numpy pin (the check can catch a wrong formula)."""
    rng = np.random.default_rng(7)
    v = rng.standard_normal(200).astype(np.float32)
    bits = v.view(np.uint32)
    wrong = np.where(bits >> 31, -(bits & 0x7FFFFFFF).astype(np.int64), (bits & 0x7FFFFFFF).astype(np.int64))
    wrong = np.where(bits >> 31, -wrong - 1, wrong)   # magnitude order kept for negatives: wrong
    assert not np.array_equal(np.argsort(wrong, kind="stable"), np.argsort(v, kind="stable"))


# ---------------------------------------------------- variable-length strings

def test_strings_brute_force():
    """Every ordering of up to 6 strings over a small alphabet (prefixes,
    empty strings, equal strings, a zero byte): exactly one is nondecreasing
    with ties in index order, and the oracle returns it."""
    from oracle import strings
    pool = [b"", b"a", b"ab", b"a\x00", b"b", b"ab", b"\x00", b"aa"]
    rng = np.random.default_rng(3)
    for trial in range(40):
        k = int(rng.integers(1, 7))
        s = [pool[int(i)] for i in rng.integers(0, len(pool), k)]
        data, offs = strings.pack(s)
        got = [int(x) for x in strings.stable_order(data, offs)]
        good = [p for p in itertools.permutations(range(k))
                if all(s[p[i]] < s[p[i + 1]] or (s[p[i]] == s[p[i + 1]] and p[i] < p[i + 1]) for i in range(k - 1))]
        assert good == [tuple(got)]


def test_strings_prefix_and_zero_bytes():
    from oracle import strings
    s = [b"abc", b"ab", b"ab\x00", b"", b"abc\x00\x00", b"b", b"ab"]
    data, offs = strings.pack(s)
    p = [int(x) for x in strings.stable_order(data, offs)]
    assert [s[i] for i in p] == [b"", b"ab", b"ab", b"ab\x00", b"abc", b"abc\x00\x00", b"b"]
    assert p[1:3] == [1, 6]                      # equal strings keep input order


def test_strings_fixed_length_match_lexsort():
    """Strings of one length: numpy's lexsort over byte columns (stable, last
    key primary) gives the same order."""
    from oracle import strings
    rng = np.random.default_rng(11)
    a = rng.integers(0, 3, (3000, 7)).astype(np.uint8)
    data, offs = strings.pack([bytes(r) for r in a])
    assert np.array_equal(strings.stable_order(data, offs), np.lexsort(a.T[::-1]))


# ------------------------------------- pins of the helpers the GPU tests use
# definition.stable_rank_u gives the expected positions in the full-size
# parity tests; orders.sort_segmented the expected result of segmented signed
# and float sorts; strings.sort the direction in which the payload follows the
# strings.  Each is checked against code it does not share, and a planted
# mistake (written here, on the CPU) must fail the same check.

def _ranks_from_oracle(keys):
    """Output position of every input element under the C oracle: the
    inverse of the permutation it carries in an index payload."""
    _, p = oracle.sort(keys, iota(keys.shape[0]))
    inv = np.empty(keys.shape[0], dtype=np.int64)
    inv[p.astype(np.int64)] = np.arange(keys.shape[0])
    return inv


def _rank_le_mistake(keys, j):
    """stable_rank_u with `<=` for `<` (a plausible slip)."""
    kj = keys[j]
    return int(np.count_nonzero(keys <= kj)) + int(np.count_nonzero(keys[:j] == kj))


def _rank_tie_mistake(keys, j):
    """stable_rank_u counting equal keys after j instead of before it."""
    kj = keys[j]
    return int(np.count_nonzero(keys < kj)) + int(np.count_nonzero(keys[j + 1:] == kj))


@pytest.mark.parametrize("dtype,seed", [(np.uint32, 71), (np.uint64, 72)])
def test_stable_rank_matches_oracle_positions(dtype, seed):
    """Heavy ties (eight values) plus the extremes of the key range; every
    element, including the first and the last index."""
    rng = np.random.default_rng(seed)
    top = np.iinfo(dtype).max
    pool = np.array([0, 1, 7, top // 2, top // 2 + 1, top - 1, top, 12345], dtype=dtype)
    keys = pool[rng.integers(0, pool.shape[0], 3000)]
    keys[0], keys[-1] = pool[3], pool[3]           # first and last tie with each other
    ranks = _ranks_from_oracle(keys)
    got = [definition.stable_rank_u(keys, j) for j in range(keys.shape[0])]
    assert got == ranks.tolist()
    assert got[0] < got[-1]                        # the tie keeps input order


def test_stable_rank_brute_force_small():
    """Against the brute-force stable permutation on tiny inputs."""
    rng = np.random.default_rng(73)
    for _ in range(30):
        n = int(rng.integers(1, 8))
        keys = rng.integers(0, 3, n).astype(np.uint32)
        perm = brute_force_stable(keys)
        want = [perm.index(j) for j in range(n)]
        assert [definition.stable_rank_u(keys, j) for j in range(n)] == want


def test_stable_rank_planted_mistakes_fail():
    keys = np.array([5, 3, 5, 5, 0, 3, 9, 5], dtype=np.uint32)
    ranks = _ranks_from_oracle(keys).tolist()
    assert [definition.stable_rank_u(keys, j) for j in range(8)] == ranks
    assert [_rank_le_mistake(keys, j) for j in range(8)] != ranks
    assert [_rank_tie_mistake(keys, j) for j in range(8)] != ranks


def _rank_bytes_last_diff_mistake(keys, j):
    """stable_rank_bytes deciding at the last differing byte instead of the
    first (a plausible slip)."""
    kj = keys[j]
    ne = keys != kj[None, :]
    differs = ne.any(axis=1)
    last = keys.shape[1] - 1 - ne[:, ::-1].argmax(axis=1)
    smaller = differs & (keys[np.arange(keys.shape[0]), last] < kj[last])
    return int(np.count_nonzero(smaller)) + int(np.count_nonzero(~differs[:j]))


def test_stable_rank_bytes_matches_oracle_positions():
    """16-byte strings from a four-letter alphabet with a shared prefix
    (long common runs, many equal rows), every element, against the C
    oracle's positions; and brute force on tiny inputs."""
    rng = np.random.default_rng(74)
    keys = rng.integers(0, 4, (3000, 16)).astype(np.uint8)
    keys[:, :10] = 7
    keys[1::3] = keys[0]
    ranks = _ranks_from_oracle(keys)
    assert [definition.stable_rank_bytes(keys, j) for j in range(keys.shape[0])] == ranks.tolist()
    for _ in range(30):
        n = int(rng.integers(1, 7))
        small = rng.integers(0, 2, (n, 16)).astype(np.uint8)
        perm = brute_force_stable(small)
        assert [definition.stable_rank_bytes(small, j) for j in range(n)] == [perm.index(j) for j in range(n)]


def test_stable_rank_bytes_planted_mistake_fails():
    keys = np.zeros((6, 16), dtype=np.uint8)
    keys[:, 0] = [2, 1, 2, 1, 0, 2]
    keys[:, 15] = [0, 9, 5, 0, 1, 0]
    ranks = _ranks_from_oracle(keys).tolist()
    assert [definition.stable_rank_bytes(keys, j) for j in range(6)] == ranks
    assert [_rank_bytes_last_diff_mistake(keys, j) for j in range(6)] != ranks


def _segments_with_edges(n_seg, seed, total_hint):
    """Offsets with empty and one-key segments among random lengths."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 2 * total_hint // n_seg, n_seg)
    lens[:6] = [0, 1, 0, 2, 1, 0]
    lens[-1] = 0
    off = np.zeros(n_seg + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    return off


def _per_segment_numpy(values, off):
    """Per segment, numpy's stable argsort of the values, as global indices."""
    p = np.arange(values.shape[0], dtype=np.int64)
    for s in range(off.shape[0] - 1):
        a, b = int(off[s]), int(off[s + 1])
        p[a:b] = a + np.argsort(values[a:b], kind="stable")
    return p


def test_orders_segmented_unsigned_matches_c_oracle():
    from oracle import orders
    off = _segments_with_edges(60, 74, 3000)
    n = int(off[-1])
    keys = workloads.u32_uniform(n, 75) >> np.uint32(24)         # ties
    pay = (np.arange(n, dtype=np.uint32) * np.uint32(7919)) ^ np.uint32(0xABC)
    ok, op = orders.sort_segmented(keys, off, pay, orders.UNSIGNED)
    rk, rp = oracle.sort_segmented(keys, off, pay)
    assert np.array_equal(ok, rk) and np.array_equal(op, rp)


@pytest.mark.parametrize("width", [32, 64])
def test_orders_segmented_signed_float_match_numpy(width):
    from oracle import orders
    off = _segments_with_edges(80, 76 + width, 4000)
    n = int(off[-1])
    rng = np.random.default_rng(78 + width)
    it, ut, ft = (np.int32, np.uint32, np.float32) if width == 32 else (np.int64, np.uint64, np.float64)
    pay = rng.permutation(n).astype(np.uint32)                  # not the identity
    # signed: ties, both extremes, values of both signs
    v = rng.integers(-50, 50, n).astype(it)
    v[::97] = np.iinfo(it).min
    v[1::89] = np.iinfo(it).max
    ok, op = orders.sort_segmented(v.view(ut), off, pay, orders.SIGNED)
    p = _per_segment_numpy(v, off)
    assert np.array_equal(op, pay[p]) and np.array_equal(ok.view(it), v[p])
    # float, numerically ordered by numpy (zeros and NaNs are pinned apart)
    f = (rng.standard_normal(n) * 10.0 ** rng.integers(-5, 5, n)).astype(ft)
    f[::53] = f[0]
    f[f == 0] = 1
    ok, op = orders.sort_segmented(f.view(ut), off, pay, orders.FLOAT)
    p = _per_segment_numpy(f, off)
    assert np.array_equal(op, pay[p]) and np.array_equal(ok.view(ft), f[p])


def test_orders_segmented_bounds_mistake_fails():
    """Segments that leak into their neighbours (one key too far) must fail
    the same per-segment check."""
    from oracle import orders
    off = np.array([0, 5, 5, 6, 12], dtype=np.int64)
    v = np.array([9, 1, 8, 2, 7, 3, 6, 0, 5, 4, 4, 1], dtype=np.int32)
    pay = np.arange(12, dtype=np.uint32)
    ok, op = orders.sort_segmented(v.view(np.uint32), off, pay, orders.SIGNED)
    assert np.array_equal(op, pay[_per_segment_numpy(v, off)])
    leaky = off.copy()
    leaky[1] += 1
    _, bad = orders.sort_segmented(v.view(np.uint32), leaky, pay, orders.SIGNED)
    assert not np.array_equal(bad, pay[_per_segment_numpy(v, off)])


def _lexsort_strings(data, offs):
    """Stable order of variable-length strings by numpy's lexsort: zero-padded
    byte columns (byte 0 primary), then the length (a proper prefix first,
    also before its extensions by zero bytes), then the input index."""
    o = np.asarray(offs, dtype=np.int64)
    n = o.shape[0] - 1
    lens = o[1:] - o[:-1]
    width = int(lens.max()) if n else 0
    cols = np.zeros((n, max(width, 1)), dtype=np.uint8)
    for i in range(n):
        cols[i, :lens[i]] = data[o[i]:o[i + 1]]
    keys = [np.arange(n), lens] + [cols[:, c] for c in range(cols.shape[1] - 1, -1, -1)]
    return np.lexsort(keys)


def test_strings_sort_payload_direction():
    """strings.sort returns payload[p] (output i carries the payload of the
    i-th smallest string), checked with a payload that is not the identity;
    the inverse permutation (a plausible slip) must fail."""
    from oracle import strings
    rng = np.random.default_rng(79)
    alpha = np.frombuffer(b"ab\x00", dtype=np.uint8)
    s = [bytes(alpha[rng.integers(0, 3, int(rng.integers(0, 6)))]) for _ in range(400)]
    data, offs = strings.pack(s)
    pay = (rng.permutation(400).astype(np.uint32) * np.uint32(3)) + np.uint32(11)
    order = _lexsort_strings(data, offs)
    got = strings.sort(data, offs, pay)
    assert np.array_equal(got, pay[order])
    inv = np.empty_like(order)
    inv[order] = np.arange(order.shape[0])
    assert not np.array_equal(pay[inv], pay[order])
    # and the strings the payload points at are in order
    srt = [s[int(i)] for i in order]
    assert all(srt[i] <= srt[i + 1] for i in range(len(srt) - 1))
