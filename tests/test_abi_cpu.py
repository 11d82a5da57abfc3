"""The C ABI library: it loads, exports every symbol include/binar.h
declares, and rejects bad arguments before touching a device (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "binar.h")


@pytest.fixture(scope="module")
def lib():
    from paper_0811_3448_amd import binar
    return binar.lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(binar_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "binar_sort" in names and "binar_sort_segmented" in names
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings(lib):
    from paper_0811_3448_amd import binar
    for code in (0, -1, -2, -3, -4):
        assert binar.strerror(code)
    assert "unknown" in binar.strerror(42)


def test_argument_errors_before_device_work(lib):
    vp = ctypes.c_void_p
    fake = vp(0x10000)  # never dereferenced: validation fails first
    assert lib.binar_sort_ex(fake, 3, 100, None, None, 0, None, None, None, 0) == -1   # key width
    assert lib.binar_sort_ex(fake, 4, 1 << 30, None, None, 0, None, None, None, 0) == -2  # too many
    assert lib.binar_sort_ex(None, 4, 100, None, None, 0, None, None, None, 0) == -1  # NULL keys
    assert lib.binar_sort_ex(vp(0x10002), 4, 100, None, None, 0, None, None, None, 0) == -1  # misaligned
    assert lib.binar_sort_ex(vp(0x10008), 16, 100, None, None, 0, None, None, None, 0) == -1  # 16 B align
    assert lib.binar_sort_segmented(fake, 4, None, 3, 100, None, None, None, 0) == -1  # NULL table
    # base cases: nothing to order, no device needed
    for n in (0, 1):
        assert lib.binar_sort_ex(None, 4, n, None, None, 0, None, None, None, 0) == 0
        assert lib.binar_sort(None, 8, n, None) == 0
    assert lib.binar_sort_segmented(fake, 4, fake, 0, 0, None, None, None, 0) == 0


def test_bad_tuning_knobs(lib):
    from paper_0811_3448_amd import binar
    bad = binar.Params(digit_bits=3).c()
    assert lib.binar_sort_ex(ctypes.c_void_p(0x10000), 4, 100, None, None, 0, ctypes.byref(bad),
                             None, None, 0) == -1
    with pytest.raises(binar.BinarError):
        binar.set_default_params(4, True, binar.Params(tile_keys=1000))
    # built digit/tile pairs: every digit width at 4096; 2048 only for 1, 4, 8
    for k in (2, 3, 9):
        assert binar.workspace_bytes(4, 1000, True, params=binar.Params(digit_bits=k)) == 0
    for k in (1, 4, 5, 6, 7, 8):
        assert binar.workspace_bytes(8, 1000, True, params=binar.Params(digit_bits=k, tile_keys=4096)) > 0
    for k in (5, 6, 7):
        assert binar.workspace_bytes(4, 1000, True, params=binar.Params(digit_bits=k, tile_keys=2048)) == 0
        assert binar.workspace_bytes(4, 1000, True, params=binar.Params(digit_bits=k, tile_keys=8192)) == 0
    # the 6144-key tile: 8-byte keys with 8-bit digits only
    assert binar.workspace_bytes(8, 1000, True, params=binar.Params(digit_bits=8, tile_keys=6144)) > 0
    assert binar.workspace_bytes(8, 1000, False, params=binar.Params(digit_bits=8, tile_keys=6144)) > 0
    for kb, k in ((4, 8), (16, 8), (8, 4), (8, 1), (8, 7)):
        assert binar.workspace_bytes(kb, 1000, True, params=binar.Params(digit_bits=k, tile_keys=6144)) == 0


def test_workspace_bytes(lib):
    from paper_0811_3448_amd import binar
    n = 1 << 28
    wb = binar.workspace_bytes(4, n, True)
    assert wb >= 8 * n                     # the ping-pong key + payload buffers
    # plus worst-case work lists: LDS-finish and copy-back entries (8 B each,
    # at most n/2 of each) and per-tile digit counts
    assert wb < 18 * n
    assert binar.workspace_bytes(4, n, False) < wb
    assert binar.workspace_bytes(3, 100, True) == 0
    assert binar.workspace_bytes(4, 1 << 30, True) == 0
    assert binar.workspace_bytes(16, 1000, True) > binar.workspace_bytes(4, 1000, True)
    p = binar.default_params(4, True)
    assert p.digit_bits == 8 and p.tile_keys in (2048, 4096, 8192) and p.finish_max > 0
    assert binar.default_params(8, True).tile_keys in (2048, 4096, 6144)


def test_key_kind_params(lib):
    from paper_0811_3448_amd import KEY_FLOAT, KEY_SIGNED, BinarError, Params, default_params, resolve_params
    for kb in (4, 8):
        for kind in (0, KEY_SIGNED, KEY_FLOAT):
            assert resolve_params(kb, True, Params(key_kind=kind)).key_kind == kind
    with pytest.raises(BinarError):
        resolve_params(16, True, Params(key_kind=KEY_SIGNED))       # byte strings have one order
    with pytest.raises(BinarError):
        resolve_params(4, True, Params(key_kind=3))
    assert default_params(4, True).key_kind == 0                    # never part of the defaults


def test_inplace_parameters_and_workspace(lib):
    """The in-place entry point's pass shape is checked before any device
    work, and its workspace is a small fraction of the data (no second copy
    of the keys), against the ping-pong sort's."""
    from paper_0811_3448_amd import binar
    n = 1 << 28
    ip = binar.inplace_workspace_bytes(4, n, True)
    assert 0 < ip < 0.1 * 8 * n < 8 * n < binar.workspace_bytes(4, n, True)
    assert binar.inplace_workspace_bytes(4, n, True, binar.Params(digit_bits=8)) > ip  # 256-way tables
    for kb in (4, 8, 16):
        assert binar.inplace_workspace_bytes(kb, 1000, False) > 0
    for bad in (binar.Params(digit_bits=5), binar.Params(digit_bits=1), binar.Params(tile_keys=8192),
                binar.Params(offsets=2)):
        assert binar.inplace_workspace_bytes(4, 1000, True, bad) == 0
        p = bad.c()
        assert lib.binar_sort_inplace(ctypes.c_void_p(0x10000), 4, 1000, None, ctypes.byref(p),
                                      None, None, 0) == -1
    assert lib.binar_sort_inplace(ctypes.c_void_p(0x10000), 3, 1000, None, None, None, None, 0) == -1
    assert lib.binar_sort_inplace(None, 4, 1, None, None, None, None, 0) == 0  # base case
    assert lib.binar_sort_inplace(ctypes.c_void_p(0x10000), 4, 1 << 30, None, None, None, None, 0) == -2


def test_strings_argument_errors(lib):
    from paper_0811_3448_amd import binar
    assert binar.strings_workspace_bytes(1000) > 0
    vp = ctypes.c_void_p
    assert lib.binar_sort_strings(None, 0, None, 1, None, None, None, 0) == 0      # one string: nothing to do
    assert lib.binar_sort_strings(vp(0x10000), 10, None, 5, vp(0x20000), None, None, 0) == -1  # NULL offsets
    assert lib.binar_sort_strings(vp(0x10000), 10, vp(0x20000), 5, None, None, None, 0) == -1  # NULL payload
    assert lib.binar_sort_strings(vp(0x10000), 10, vp(0x20000), 1 << 30, vp(0x30000), None, None, 0) == -2


def test_build_tracks_every_source():
    """The library is rebuilt when any of its sources changes: every file
    under csrc and the public header are dependencies of the build."""
    from paper_0811_3448_amd import build
    csrc = os.path.join(os.path.dirname(build.__file__), "csrc")
    deps = {os.path.abspath(p) for p in build.DEPS}
    for f in os.listdir(csrc):
        assert os.path.abspath(os.path.join(csrc, f)) in deps, f
    assert any(p.endswith(os.path.join("include", "binar.h")) for p in deps)


def test_plan_segmented_refuses_short_buffers(monkeypatch):
    """A segmented plan sort whose buffers are shorter than the plan's
    capacity is refused before the library is called: a segment table that
    is valid for the capacity would reach past them."""
    import torch
    from paper_0811_3448_amd import binar
    plan = binar.Plan.__new__(binar.Plan)
    plan._h = ctypes.c_void_p()          # never reaches the library
    plan.key_bytes, plan.max_keys, plan.max_segments = 4, 1000, 10
    monkeypatch.setattr(binar, "_check_tensors", lambda k, p: None)
    keys = torch.zeros(999, dtype=torch.int32)
    off = torch.zeros(11, dtype=torch.int32)
    with pytest.raises(ValueError, match="capacity"):
        plan.sort(keys, torch.zeros(999, dtype=torch.int32), off)
