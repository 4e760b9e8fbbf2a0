"""The Python binding refuses inputs the library would misread, before any
library call: wrong element type (an int64 batch read as int32 pairs),
non-contiguous memory, and host memory given to a context whose inputs are
device memory or the other way round (a host pointer read on the GPU, a
device pointer copied on the host).  CPU only: the library is never loaded."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2607_20211_amd import drsf


@pytest.fixture(autouse=True)
def _no_library(monkeypatch):
    def refuse():
        raise AssertionError("the library was called")
    monkeypatch.setattr(drsf, "load", refuse)


class FakeGpuTensor:
    """Stands for a torch tensor in device memory (there is no GPU here)."""

    def __init__(self, dtype="torch.int32", n=8, contiguous=True):
        self.dtype, self._n, self._c = dtype, n, contiguous
        self.is_cuda = True

    def data_ptr(self):
        return 0x1000

    def numel(self):
        return self._n

    def is_contiguous(self):
        return self._c


def _ctx(cls=drsf.Forest, on_device=False, G=None):
    f = object.__new__(cls)
    f.on_device = on_device
    f.ctx = None
    if G is not None:
        f.G = G
    return f


def _refused(fn, *args, **kw):
    with pytest.raises(drsf.DrsfError) as e:
        fn(*args, **kw)
    assert e.value.code == drsf.DRSF_E_ARG
    return str(e.value)


def test_int64_tensor_batch_is_refused():
    f = _ctx()
    msg = _refused(f.apply, torch.zeros((4, 2), dtype=torch.int64), drsf.DRSF_INSERT)
    assert "int64" in msg
    g = _ctx(on_device=True)
    _refused(g.apply, FakeGpuTensor(dtype="torch.int64"), drsf.DRSF_INSERT)


def test_host_batch_on_device_context_is_refused():
    f = _ctx(on_device=True)
    msg = _refused(f.apply, np.zeros((3, 2), np.int32), drsf.DRSF_DELETE)
    assert "device memory" in msg
    _refused(f.apply, torch.zeros((3, 2), dtype=torch.int32), drsf.DRSF_DELETE)  # CPU tensor
    _refused(f.apply_async, np.zeros((3, 2), np.int32), drsf.DRSF_DELETE)


def test_device_batch_on_host_context_is_refused():
    f = _ctx(on_device=False)
    msg = _refused(f.apply, FakeGpuTensor(), drsf.DRSF_INSERT)
    assert "GPU tensor" in msg


def test_non_contiguous_and_odd_batches_are_refused():
    f = _ctx()
    t = torch.zeros((4, 4), dtype=torch.int32)[:, ::2]
    assert not t.is_contiguous()
    _refused(f.apply, t, drsf.DRSF_INSERT)
    _refused(_ctx(on_device=True).apply, FakeGpuTensor(contiguous=False), drsf.DRSF_INSERT)
    _refused(f.apply, torch.zeros(5, dtype=torch.int32), drsf.DRSF_INSERT)  # not pairs


def test_numpy_batch_of_a_host_context_is_converted_by_value():
    arr, b = drsf._batch(np.array([[1, 2], [3, 4]], np.int64), False)
    assert arr.dtype == np.int32 and b == 2 and arr.tolist() == [[1, 2], [3, 4]]


def test_create_inputs_are_checked():
    # wrong dtype / too short / wrong memory, all before drsf_create
    rp = np.array([0, 1, 2], np.int64)
    col = np.array([1, 0], np.int32)
    par = np.array([0, 0], np.int32)
    _refused(drsf.Forest, 2, torch.from_numpy(rp).to(torch.int32), col, par)
    _refused(drsf.Forest, 3, rp, col, np.array([0, 0, 0], np.int32))  # row_ptr too short for n
    _refused(drsf.Forest, 2, rp, col[:1], par)  # col shorter than row_ptr[n]
    _refused(drsf.Forest, 2, rp, col, par, inputs_on_device=True)  # numpy on a device context
    _refused(drsf.Forest, 2, FakeGpuTensor("torch.int64", 3), FakeGpuTensor(n=2), FakeGpuTensor(n=1),
             inputs_on_device=True)  # parent too short


def test_multi_batch_offsets_are_checked():
    f = _ctx(drsf.MultiForest, G=2)
    e = np.zeros((4, 2), np.int32)
    _refused(f.apply_multi, e, [0, 2], [0, 1])             # b_off too short
    _refused(f.apply_multi, e, [0, 2, 5], [0, 1])          # more edges than given
    _refused(f.apply_multi, torch.zeros((4, 2), dtype=torch.int64), [0, 2, 4], [0, 1])
