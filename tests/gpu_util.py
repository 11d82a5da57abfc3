"""Helpers shared by the GPU tests: device round trips and checks."""
import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_dev(a):
    import torch
    if a is None:
        return None
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32)).cuda()
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64)).cuda()
    return torch.from_numpy(a).cuda()


def to_host(t, like):
    a = t.cpu().numpy()
    return a.view(like.dtype).reshape(like.shape)


def gpu_sort(keys, payload=None, params=None, workspace=None):
    import torch
    import paper_0811_3448_amd as binar
    kd, pd = to_dev(keys), to_dev(payload)
    binar.sort(kd, pd, params=params, workspace=workspace)
    torch.cuda.synchronize()
    if keys.shape[0] >= 2:
        assert binar.stats(workspace)["status"] == 0
    return to_host(kd, keys), (None if payload is None else to_host(pd, payload))


def gpu_sort_segmented(keys, offsets, payload=None, params=None):
    import torch
    import paper_0811_3448_amd as binar
    kd, pd = to_dev(keys), to_dev(payload)
    od = torch.from_numpy(np.asarray(offsets, dtype=np.uint32).view(np.int32)).cuda()
    binar.sort_segmented(kd, od, pd, params=params)
    torch.cuda.synchronize()
    assert binar.stats()["status"] == 0
    return to_host(kd, keys), (None if payload is None else to_host(pd, payload))


def check_sorted_permutation(keys_in, keys_out, pay_out):
    """Complete check of a stable sort of unsigned integer keys: nondecreasing,
    payload a permutation, keys_out == keys_in[payload], ties in index order."""
    n = keys_in.shape[0]
    if n == 0:
        return
    assert np.all(keys_out[1:] >= keys_out[:-1]), "not sorted"
    seen = np.zeros(n, dtype=bool)
    seen[pay_out] = True
    assert seen.all(), "payload is not a permutation"
    assert np.array_equal(keys_in[pay_out], keys_out), "keys do not follow payload"
    tie = keys_out[1:] == keys_out[:-1]
    assert np.all(pay_out[1:][tie] > pay_out[:-1][tie]), "unstable on ties"


def check_segmented(keys_in, offsets, keys_out, pay_out):
    """Complete check of per-segment stable sorts of unsigned integer keys
    with a global-index payload: each segment's payload is a permutation of
    its own indices, keys follow the payload, keys are nondecreasing inside
    each segment and ties keep index order."""
    offsets = np.asarray(offsets, dtype=np.int64)
    n = int(offsets[-1])
    if n == 0:
        return
    sizes = np.diff(offsets)
    seg = np.repeat(np.arange(sizes.shape[0]), sizes)
    p = pay_out[:n].astype(np.int64)
    assert np.all(p >= offsets[seg]) and np.all(p < offsets[seg + 1]), "payload leaves its segment"
    seen = np.zeros(n, dtype=bool)
    seen[p] = True
    assert seen.all(), "payload is not a permutation"
    assert np.array_equal(keys_in[p], keys_out[:n]), "keys do not follow payload"
    same = seg[1:] == seg[:-1]
    k0, k1 = keys_out[:n - 1], keys_out[1:n]
    assert np.all(k1[same] >= k0[same]), "not sorted inside a segment"
    tie = same & (k1 == k0)
    assert np.all(p[1:][tie] > p[:-1][tie]), "unstable on ties"
