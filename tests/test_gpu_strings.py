"""Variable-length byte strings on the GPU against the oracle's plain
definition: the permutation (payload) exact."""
import numpy as np
import pytest

import workloads
from gpu_util import need_gpu
from oracle import strings

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def gpu_sort_strings(data, offs, payload=None):
    import torch
    import paper_0811_3448_amd as binar
    n = offs.shape[0] - 1
    pay = np.arange(n, dtype=np.uint32) if payload is None else payload
    dd = torch.from_numpy(np.asarray(data, dtype=np.uint8)).cuda()
    od = torch.from_numpy(np.asarray(offs, dtype=np.uint32).view(np.int32)).cuda()
    pd = torch.from_numpy(pay.view(np.int32)).cuda()
    binar.sort_strings(dd, od, pd)
    torch.cuda.synchronize()
    return pd.cpu().numpy().view(np.uint32), pay


def check(data, offs, label):
    print("strings %s n=%d bytes=%d" % (label, offs.shape[0] - 1, data.shape[0]), flush=True)
    got, pay = gpu_sort_strings(data, offs)
    assert np.array_equal(got, strings.sort(data, offs, pay)), label


@pytest.mark.parametrize("n", [0, 1, 2, 3, 1000, 65_537])
def test_random_lengths(n):
    data, offs = workloads.var_strings(n, 100 + n, 20.0, 26, 0)
    check(data, offs, "random")


@pytest.mark.parametrize("alphabet,prefix", [(2, 0), (2, 14), (3, 15), (2, 16), (4, 31), (26, 45)])
def test_long_ties_and_shared_prefixes(alphabet, prefix):
    """Small alphabets and shared prefixes around the 15-byte round width:
    many rounds, long tied runs, equal strings."""
    data, offs = workloads.var_strings(40_000, 7 * alphabet + prefix, 12.0, alphabet, prefix)
    check(data, offs, "alphabet=%d prefix=%d" % (alphabet, prefix))


def test_prefixes_zero_bytes_and_empty():
    rng = np.random.default_rng(9)
    base = [b"", b"a", b"ab", b"a\x00", b"ab\x00", b"\x00", b"\x00\x00", b"x" * 15, b"x" * 16, b"x" * 30,
            b"x" * 15 + b"\x00", b"x" * 31, b"y"]
    s = [base[int(i)] for i in rng.integers(0, len(base), 5000)]
    data, offs = strings.pack(s)
    check(data, offs, "special")


def test_arbitrary_payload():
    """Any payload is carried (payload_out[i] = payload_in[p(i)])."""
    data, offs = workloads.var_strings(3000, 55, 10.0, 4, 0)
    n = offs.shape[0] - 1
    pay = ((np.arange(n, dtype=np.uint64) * 7919) ^ 0x5A5A5A5A).astype(np.uint32)
    got, _ = gpu_sort_strings(data, offs, pay)
    assert np.array_equal(got, strings.sort(data, offs, pay))


def test_bad_offsets_rejected():
    import torch
    import paper_0811_3448_amd as binar
    dd = torch.zeros(100, dtype=torch.uint8, device="cuda")
    od = torch.tensor([0, 10, 5, 20], dtype=torch.int32, device="cuda")     # out of order
    pd = torch.arange(3, dtype=torch.int32, device="cuda")
    with pytest.raises(binar.BinarError):
        binar.sort_strings(dd, od, pd)
    od = torch.tensor([0, 10, 50, 200], dtype=torch.int32, device="cuda")   # past the buffer
    with pytest.raises(binar.BinarError):
        binar.sort_strings(dd, od, pd)


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_unaligned_byte_buffer(shift):
    """The byte buffer starts 1..3 bytes past a 4-byte boundary and ends
    inside a word: the key build reads whole words only inside the buffer."""
    import torch
    import paper_0811_3448_amd as binar
    data, offs = workloads.var_strings(20_000, 300 + shift, 9.0, 5, 0)
    n = offs.shape[0] - 1
    backing = torch.zeros(data.shape[0] + shift, dtype=torch.uint8, device="cuda")
    backing[shift:] = torch.from_numpy(data).cuda()
    dd = backing[shift:]
    assert dd.data_ptr() % 4 == shift
    od = torch.from_numpy(offs.view(np.int32)).cuda()
    pay = np.arange(n, dtype=np.uint32)
    pd = torch.from_numpy(pay.view(np.int32)).cuda()
    print("strings unaligned shift=%d n=%d" % (shift, n), flush=True)
    binar.sort_strings(dd, od, pd)
    torch.cuda.synchronize()
    assert np.array_equal(pd.cpu().numpy().view(np.uint32), strings.sort(data, offs, pay))
