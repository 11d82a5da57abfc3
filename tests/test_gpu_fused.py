"""The second pass's digit counts taken from the first pass's digit-pair
counts (one array of at least 2^26 keys): the counters show that the second
pass read no key, and the result is checked completely on the device
(nondecreasing, payload a permutation, keys follow it, ties in input order)
and at sampled inputs against the oracle's stable rank.  An input whose
blocks hold more than 65535 keys of one leading digit (so that a 16-bit
pair bin could overflow) falls back to counting the second pass's digits
from the keys, with the same checks."""
import numpy as np
import pytest

import workloads
from gpu_util import need_gpu
from oracle.definition import stable_rank_u
from test_gpu_fullsize import device_checks

pytestmark = pytest.mark.gpu

N = 1 << 26


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def sort_and_check(keys, kb, params):
    import torch
    import paper_0811_3448_amd as binar
    n = keys.shape[0]
    kin = torch.from_numpy(keys.view(np.int32 if kb == 4 else np.int64)).cuda()
    kd = kin.clone()
    pd = torch.arange(n, dtype=torch.int32, device="cuda")
    binar.sort(kd, pd, params=params)
    torch.cuda.synchronize()
    st = binar.stats()
    assert st["status"] == 0
    device_checks(kin, kd, pd, kb)
    gk = kd.cpu().numpy().view(keys.dtype)
    gp = pd.cpu().numpy().view(np.uint32)
    for i in workloads.below(16, 7070 + kb, n).astype(np.int64).tolist():
        r = stable_rank_u(keys, i)
        assert gp[r] == i and gk[r] == keys[i], i
    return st


@pytest.mark.parametrize("kb", [4, 8])
def test_second_pass_counts_from_pairs(kb):
    from paper_0811_3448_amd import Params
    keys = workloads.u32_uniform(N, 7001) if kb == 4 else workloads.u64_uniform(N, 7002)
    tile = 8192 if kb == 4 else 6144
    print("fused pass counts kb=%d n=%d" % (kb, N), flush=True)
    st = sort_and_check(keys, kb, Params(digit_bits=8, tile_keys=tile, offsets=1))
    assert st["passes"] >= 2
    assert st["hist_keys"][0] == N and st["hist_keys"][1] == 0, st["hist_keys"][:3]
    assert st["moved"][0] == N and st["moved"][1] == N


def test_pair_bins_overflow_falls_back():
    """Each block's chunk holds one leading byte and two second bytes (0 and
    128), so a pair bin passes 65535 in every block; bit 8 varies and the
    256 children are even, so only the overflow guard stops the pair
    counts."""
    from paper_0811_3448_amd import Params
    i = np.arange(N, dtype=np.uint64)
    rnd = workloads.u32_uniform(N, 7003)
    keys = ((((i * 256) // N) << 24).astype(np.uint32) | ((rnd >> np.uint32(31)) << np.uint32(23))
            | (rnd & np.uint32(0xFFFF)))
    print("pair overflow n=%d" % N, flush=True)
    st = sort_and_check(keys, 4, Params(digit_bits=8, tile_keys=8192, offsets=1))
    assert st["passes"] >= 2
    assert st["hist_keys"][0] == N and st["hist_keys"][1] == N, st["hist_keys"][:3]
