"""The benchmark's two extra CPU baselines (std::stable_sort on one thread,
and the paper's parallel variant: one stable partition on the leading
byte, then the buckets on several threads) give the oracle's result byte
for byte: keys and permutation, every key width, tie-heavy inputs, the
empty and one-key cases, and more threads than buckets with keys."""
import numpy as np
import pytest

import oracle
import workloads


def inputs(kb, n, seed):
    if kb == 4:
        return workloads.u32_uniform(n, seed) & np.uint32(0xC00000F0)   # few distinct keys, many ties
    if kb == 8:
        return workloads.u64_uniform(n, seed) & np.uint64(0xFF000000000000FF)
    return workloads.str16(n, seed, 14)


@pytest.mark.parametrize("kb", [4, 8, 16])
@pytest.mark.parametrize("n", [0, 1, 2, 3000, 70001])
def test_baselines_match_oracle(kb, n):
    keys = inputs(kb, n, 900 + kb + n % 13)
    pay = (np.arange(n, dtype=np.uint32) * np.uint32(7)) ^ np.uint32(0x5A5A)   # not the identity
    rk, rp = oracle.sort(keys, pay)
    sk, sp = oracle.stable_sort_ref(keys, pay)
    assert np.array_equal(sk, rk) and np.array_equal(sp, rp)
    for threads in (1, 3, 300):
        pk, pp = oracle.parallel_sort_ref(keys, pay, threads)
        assert np.array_equal(pk, rk) and np.array_equal(pp, rp), threads


def test_baselines_keys_only():
    keys = inputs(4, 5000, 77)
    rk, _ = oracle.sort(keys)
    assert np.array_equal(oracle.stable_sort_ref(keys)[0], rk)
    assert np.array_equal(oracle.parallel_sort_ref(keys, None, 4)[0], rk)
