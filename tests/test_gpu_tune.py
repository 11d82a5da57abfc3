"""Autotuner on the device: it times the built configurations, and the
configuration it picks sorts bit-exactly like the oracle (one array and a
batch of segments)."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import gpu_sort, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def test_autotune_single_then_sort_matches_oracle(tmp_path):
    from paper_0811_3448_amd import Params, tune
    n = 1 << 18
    print("autotune kb=4 payload n=%d" % n, flush=True)
    e = tune.autotune(4, True, n, reps=2)
    assert len(e["table"]) == len(tune.candidates(4, True))
    assert all(row[4] > 0 for row in e["table"])
    c = tune.TuneCache(str(tmp_path / "t.json"), arch="gfx950")
    c.put(4, True, n, False, e)
    c.save()
    p = tune.TuneCache(str(tmp_path / "t.json")).lookup(4, True, n)
    assert p == Params(**e["params"])
    keys = workloads.u32_uniform(n + 17, 1234)
    pay = np.arange(n + 17, dtype=np.uint32)
    gk, gp = gpu_sort(keys, pay, params=p)
    rk, rp = oracle.sort(keys, pay)
    assert np.array_equal(gk, rk) and np.array_equal(gp, rp)


def test_autotune_batched_plan_matches_oracle():
    import torch
    from paper_0811_3448_amd import Params, Plan, tune
    n = 1 << 18
    cands = [p for p in tune.candidates(8, True) if p.digit_bits in (4, 8) and p.offsets == 1]
    print("autotune batched kb=8 n=%d candidates=%d" % (n, len(cands)), flush=True)
    e = tune.autotune(8, True, n, batched=True, cands=cands, reps=2)
    p = Params(**e["params"])
    off = tune.lognormal_offsets(n, seed=5)
    keys = workloads.u64_uniform(n, 77)
    pay = np.arange(n, dtype=np.uint32)
    dev = torch.device("cuda:0")
    kd = torch.from_numpy(keys.view(np.int64)).to(dev)
    pd = torch.from_numpy(pay.view(np.int32)).to(dev)
    od = torch.from_numpy(off.view(np.int32)).to(dev)
    plan = Plan(8, n, off.shape[0] - 1, True, p)
    plan.sort(kd, pd, od)
    torch.cuda.synchronize()
    assert plan.stats()["status"] == 0
    rk, rp = oracle.sort_segmented(keys, off, pay)
    assert np.array_equal(kd.cpu().numpy().view(np.uint64), rk)
    assert np.array_equal(pd.cpu().numpy().view(np.uint32), rp)
    plan.close()
