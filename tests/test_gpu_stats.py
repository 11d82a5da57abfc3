"""The library's device counters (moved / read keys per pass, keys and
sub-arrays finished in LDS, copy-back) against counts derived from the input
with numpy; the bench's algorithmic bytes are built from these counters."""
import numpy as np
import pytest

import workloads
from gpu_util import need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def run(keys, params, offsets=None):
    import torch
    import paper_0811_3448_amd as binar
    kd, pd = to_dev(keys), torch.arange(keys.shape[0], dtype=torch.int32, device="cuda")
    if offsets is None:
        binar.sort(kd, pd, params=params)
    else:
        binar.sort_segmented(kd, to_dev(np.asarray(offsets, dtype=np.uint32)), pd, params=params)
    torch.cuda.synchronize()
    st = binar.stats()
    assert st["status"] == 0
    return st


def test_one_pass_then_finish():
    from paper_0811_3448_amd import Params
    n = 1 << 20
    keys = workloads.u32_uniform(n, 4242)
    st = run(keys, Params(digit_bits=8, finish_max=8192))
    top = np.bincount(keys >> 24, minlength=256)
    assert st["passes"] == 1
    assert st["hist_keys"][0] == n and st["moved"][0] == n
    assert st["finish_segments"] == int((top >= 2).sum())
    assert st["finish_keys"] == int(top[top >= 2].sum())
    assert st["copyback_keys"] == 0


@pytest.mark.parametrize("k", [6, 7])
def test_many_tiny_finish_segments(k):
    """Two global passes leave ~2^(20 - 2k) keys per sub-array: hundreds of
    thousands of tiny LDS finishes."""
    from paper_0811_3448_amd import Params
    n = 1 << 20
    keys = workloads.u32_uniform(n, 4343 + k)
    st = run(keys, Params(digit_bits=k, tile_keys=4096, finish_max=(n >> k) // 2))
    pre = np.bincount(keys >> (32 - 2 * k), minlength=1 << (2 * k))
    assert st["passes"] == 2
    assert st["hist_keys"][:2] == [n, n] and st["moved"][:2] == [n, n]
    assert st["finish_segments"] == int((pre >= 2).sum())
    assert st["finish_keys"] == int(pre[pre >= 2].sum())
    assert st["copyback_keys"] == 0


def test_batched_all_small_segments():
    from paper_0811_3448_amd import Params
    keys, off = workloads.batched_u32(5000, seed=17, median=300, sigma=0.5, max_len=8000)
    lens = np.diff(off.astype(np.int64))
    st = run(keys, Params(finish_max=8192), offsets=off)
    assert st["passes"] == 0 and sum(st["hist_keys"]) == 0 and sum(st["moved"]) == 0
    assert st["finish_segments"] == int((lens >= 2).sum())
    assert st["finish_keys"] == int(lens[lens >= 2].sum())
