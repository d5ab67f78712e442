"""Host logic of the Python binding that needs no GPU: packed descriptor arrays."""
import pytest
import torch

from paper_2102_00319_amd import fhe


def _cts(n):
    return [fhe.Ciphertext(torch.zeros(2, 3, 8, dtype=torch.int64), 2.0 ** 30) for _ in range(n)]


def test_packed_array_is_a_read_only_list():
    cts = _cts(5)
    a = fhe.CtArray(cts)
    assert len(a) == 5 and a[2] is cts[2] and list(a) == cts
    assert (a + cts[:1])[-1] is cts[0] and (cts[:1] + a)[0] is cts[0]
    assert [a.arr[i].d for i in range(5)] == [c.data.data_ptr() for c in cts]
    assert a.arr[0].limbs == 3 and a.arr[0].polys == 2 and a.arr[0].scale == 2.0 ** 30
    assert fhe.Context._arr(a) is a.arr


def test_stale_packed_array_is_refused_until_refreshed():
    cts = _cts(3)
    a = fhe.CtArray(cts)
    for c in cts:   # the data moves (as an eviction to host and back does)
        c.data = c.data.clone()
    with pytest.raises(fhe.FheError):
        fhe.Context._arr(a)
    a.refresh()
    assert fhe.Context._arr(a)[2].d == cts[2].data.data_ptr()
