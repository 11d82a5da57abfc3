"""Autotuner host logic (no device): candidate grid, selection, JSON cache,
nearest-bucket lookup, installing library defaults."""
import json

import numpy as np
import pytest

from paper_0811_3448_amd import Params, default_params, resolve_params, set_default_params, tune


def test_bucket_and_key():
    assert [tune.bucket(n) for n in (0, 1, 2, 3, 4, 5, 1 << 20, (1 << 20) + 1)] == [0, 0, 1, 2, 2, 3, 20, 21]
    assert tune.case_key(4, True, 1 << 28, False) == "kb4/pay1/n28/one"
    assert tune.case_key(16, False, 1000, True) == "kb16/pay0/n10/seg"


@pytest.mark.parametrize("kb", [4, 8, 16])
def test_candidates_are_built_and_complete(kb):
    c = tune.candidates(kb, True)
    ks = sorted({p.digit_bits for p in c})
    assert ks == [1, 4, 5, 6, 7, 8]
    tiles = {p.tile_keys for p in c}
    assert tiles == {4: {2048, 4096, 8192}, 8: {2048, 4096, 6144}, 16: {2048, 4096}}[kb]
    assert {p.offsets for p in c} == {1, 2}
    assert len({(p.digit_bits, p.tile_keys, p.finish_max, p.offsets) for p in c}) == len(c)
    tmax = resolve_params(kb, True, Params(finish_max=1 << 30)).finish_max
    assert max(p.finish_max for p in c) == tmax
    for p in c:
        r = resolve_params(kb, True, p)   # every candidate is a built combination
        assert (r.digit_bits, r.tile_keys, r.finish_max, r.offsets) == \
            (p.digit_bits, p.tile_keys, p.finish_max, p.offsets)


def test_autotune_picks_fastest_with_stable_ties():
    cands = tune.candidates(4, True)
    cost = {id(p): 10.0 + i for i, p in enumerate(cands)}
    target = cands[17]
    cost[id(target)] = 1.5
    # a tie with the same finish threshold: the earlier candidate wins
    twin = next(p for p in cands[18:] if p.finish_max == target.finish_max)
    cost[id(twin)] = 1.5
    e = tune.autotune(4, True, 1 << 20, timer=lambda p: cost[id(p)], cands=cands)
    assert e["params"] == {"digit_bits": target.digit_bits, "tile_keys": target.tile_keys,
                           "finish_max": target.finish_max, "offsets": target.offsets}
    assert e["ms"] == 1.5 and len(e["table"]) == len(cands)
    assert e["gkeys_s"] == pytest.approx((1 << 20) / 1.5e-3 / 1e9, rel=1e-3)
    assert e["workgroup"] == tune.TILE_THREADS[target.tile_keys]
    with pytest.raises(ValueError):
        tune.autotune(4, True, 1, timer=lambda p: 1.0)


def test_ties_within_the_band_prefer_the_larger_finish_threshold():
    # [k, tile, T, offsets, ms]
    t = [[8, 4096, 3072, 1, 1.000], [8, 4096, 5120, 1, 1.018], [8, 4096, 8192, 1, 1.03],
         [8, 2048, 5120, 1, 1.005], [8, 4096, 8192, 2, None]]
    assert tune.TIE == 0.02
    assert tune.choose(t) == 3          # tied: T = 5120 beats 3072; of the two 5120 rows the faster
    t[3][4] = 1.2
    assert tune.choose(t) == 1
    t[1][4] = 1.021                     # past the band: the fastest stands
    assert tune.choose(t) == 0
    cands = tune.candidates(8, True)
    big = max(p.finish_max for p in cands)
    fast = next(p for p in cands if p.finish_max < big)
    slow = next(p for p in cands if p.finish_max == big)
    cost = {id(p): 10.0 for p in cands}
    cost[id(fast)], cost[id(slow)] = 2.0, 2.015
    assert tune.autotune(8, True, 1 << 20, timer=lambda p: cost[id(p)], cands=cands)["params"]["finish_max"] == big


def test_cache_roundtrip_and_lookup(tmp_path):
    path = str(tmp_path / "cache.json")
    c = tune.TuneCache(path, arch="gfx950")
    mk = lambda k: {"params": {"digit_bits": k, "tile_keys": 4096, "finish_max": 3072, "offsets": 1},  # noqa: E731
                    "ms": 1.0, "gkeys_s": 1.0, "n": 0, "batched": False, "table": []}
    c.put(4, True, 1 << 20, False, mk(4))
    c.put(4, True, 1 << 24, False, mk(6))
    c.put(4, True, 1 << 24, True, mk(7))
    c.save()
    d = tune.TuneCache(path)
    assert d.arch == "gfx950" and set(d.entries) == set(c.entries)
    assert json.load(open(path))["format"] == tune.FORMAT
    assert d.lookup(4, True, 1 << 20).digit_bits == 4
    assert d.lookup(4, True, (1 << 20) + 5).digit_bits == 4      # bucket 21: nearest is 20
    assert d.lookup(4, True, 1 << 22).digit_bits == 6            # tie 20/24 at distance 2 -> larger
    assert d.lookup(4, True, 1 << 24, batched=True).digit_bits == 7
    assert d.lookup(4, True, 1 << 10) is None                    # too far from any tuned bucket
    assert d.lookup(8, True, 1 << 20) is None
    assert d.lookup(4, False, 1 << 20) is None
    # another architecture's cache is not used
    assert tune.TuneCache(path, arch="gfx942").entries == {}


def test_install_sets_library_defaults(tmp_path):
    before = default_params(8, True)
    c = tune.TuneCache(str(tmp_path / "c.json"), arch="gfx950")
    c.put(8, True, 1 << 20, False, {"params": {"digit_bits": 4, "tile_keys": 2048, "finish_max": 3072,
                                               "offsets": 2}})
    c.put(8, True, 1 << 27, False, {"params": {"digit_bits": 6, "tile_keys": 4096, "finish_max": 5120,
                                               "offsets": 1}})
    try:
        done = c.install()
        assert done == [(8, True, {"digit_bits": 6, "tile_keys": 4096, "finish_max": 5120, "offsets": 1,
                                   "key_bits": 0, "key_kind": 0})]
        p = default_params(8, True)
        assert (p.digit_bits, p.tile_keys, p.finish_max, p.offsets) == (6, 4096, 5120, 1)
    finally:
        set_default_params(8, True, before)
    p = default_params(8, True)
    assert (p.digit_bits, p.tile_keys, p.offsets) == (before.digit_bits, before.tile_keys, before.offsets)


def test_set_default_rejects_unbuilt_pairs():
    from paper_0811_3448_amd import BinarError
    before = default_params(4, True)
    with pytest.raises(BinarError):
        set_default_params(4, True, Params(digit_bits=6, tile_keys=2048))
    with pytest.raises(BinarError):
        set_default_params(8, True, Params(tile_keys=8192))
    after = default_params(4, True)
    assert (after.digit_bits, after.tile_keys) == (before.digit_bits, before.tile_keys)


@pytest.mark.parametrize("n", [1, 1000, 1 << 20, 3_000_017])
def test_lognormal_offsets(n):
    off = tune.lognormal_offsets(n)
    assert off[0] == 0 and int(off[-1]) == n
    d = np.diff(off.astype(np.int64))
    assert (d >= 1).all() and d.max() <= 1 << 20
    if n >= 1 << 20:
        assert 700 < np.median(d) < 1400


def test_autotune_never_picks_a_failed_candidate():
    """A candidate whose status or output check failed (the timer reports
    inf) is listed without a time and never chosen, however fast it looked;
    if every candidate failed, tuning fails."""
    import math
    cands = tune.candidates(4, True)
    cost = {id(p): 10.0 + i for i, p in enumerate(cands)}
    cost[id(cands[3])] = math.inf
    cost[id(cands[9])] = 2.0
    e = tune.autotune(4, True, 1 << 20, timer=lambda p: cost[id(p)], cands=cands)
    assert e["params"]["digit_bits"] == cands[9].digit_bits and e["ms"] == 2.0
    assert e["table"][3][4] is None
    with pytest.raises(RuntimeError):
        tune.autotune(4, True, 1 << 20, timer=lambda p: math.inf, cands=cands[:4])
