"""Host-side argument checks of the ctypes binding (no GPU needed): media sizes,
and the dtype / shape / overlap checks that every vector passes before a
pointer reaches the library, which has no sizes to check them against."""
import numpy as np
import pytest
import torch

from paper_1806_11277_amd import ehh


class _FakeDeviceTensor:
    """Stands in for a contiguous device tensor: dtype, shape and an address
    range, which is all the checks read."""

    def __init__(self, shape, dtype=torch.float64, ptr=4096):
        self.shape = tuple(shape)
        self.dtype = dtype
        self.is_cuda = True
        self._ptr = ptr

    def is_contiguous(self):
        return True

    def dim(self):
        return len(self.shape)

    def numel(self):
        return int(np.prod(self.shape))

    def element_size(self):
        return torch.empty((), dtype=self.dtype).element_size()

    def data_ptr(self):
        return self._ptr


def test_host_media_must_match_the_grid():
    a, addr = ehh._media(np.ones((4, 6)), 24, "mu")
    assert a.dtype == np.float64 and a.flags.c_contiguous and a.size == 24 and addr == a.ctypes.data
    assert ehh._media(torch.ones(24, dtype=torch.float32), 24, "rho")[0].dtype == np.float64
    with pytest.raises(ValueError, match="mu has 20 entries"):
        ehh._media(np.ones(20), 24, "mu")


def test_vectors_need_the_right_dtype_shape_and_device():
    good = _FakeDeviceTensor((2, 10))
    ehh._check_vectors([("x", good)], torch.float64, 2, 10)
    with pytest.raises(ValueError, match="must be torch.float64"):
        ehh._check_vectors([("x", _FakeDeviceTensor((2, 10), torch.float32))], torch.float64, 2, 10)
    with pytest.raises(ValueError, match="shape"):
        ehh._check_vectors([("x", _FakeDeviceTensor((2, 12)))], torch.float64, 2, 10)
    with pytest.raises(ValueError, match="shape"):
        ehh._check_vectors([("x", _FakeDeviceTensor((3, 10)))], torch.float64, 2, 10)
    with pytest.raises(ValueError, match="device tensor"):
        ehh._check_vectors([("x", torch.zeros(2, 10, dtype=torch.float64))], torch.float64, 2, 10)


def test_outputs_must_not_overlap_inputs():
    x = _FakeDeviceTensor((2, 10), ptr=1000)             # bytes [1000, 1160)
    y_over = _FakeDeviceTensor((2, 10), ptr=1080)
    y_apart = _FakeDeviceTensor((2, 10), ptr=1160)
    ehh._check_vectors([("x", x), ("y", y_apart)], torch.float64, 2, 10, ("y",))
    with pytest.raises(ValueError, match="y must not overlap x"):
        ehh._check_vectors([("x", x), ("y", y_over)], torch.float64, 2, 10, ("y",))
    # two inputs may share memory
    ehh._check_vectors([("b", x), ("e", x), ("out", y_apart)], torch.float64, 2, 10, ("out",))
