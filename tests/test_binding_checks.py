"""Host-side argument checks of the Python binding (no GPU).

The kernels touch rows 0 .. n - 1 of every output and auxiliary array of a
call, and the C-ABI takes plain pointers, so the binding must refuse a tensor
that is too short, strided the wrong way, of the wrong type or on another
device before anything is launched.  These tests drive the checks with
stand-ins that report CUDA placement, so nothing reaches a device."""
import sys
from pathlib import Path

import pytest
import torch

sys.path.insert(0, str(Path(__file__).resolve().parents[1]))

import paper_0907_3768_amd as dust  # noqa: E402


class _Dev:
    def __init__(self, index):
        self.index = index


class FakeCuda:
    """Shape, strides and dtype of a CUDA tensor, without memory."""

    def __init__(self, shape, dtype=torch.float32, strides=None, device=0, cuda=True):
        self.shape = tuple(shape)
        self.dtype = dtype
        if strides is None:
            strides, acc = [], 1
            for d in reversed(self.shape):
                strides.insert(0, acc)
                acc *= max(d, 1)
        self._strides = tuple(strides)
        self.is_cuda = cuda
        self.device = _Dev(device)

    def dim(self):
        return len(self.shape)

    def stride(self, i):
        return self._strides[i]

    def numel(self):
        n = 1
        for d in self.shape:
            n *= d
        return n

    def is_contiguous(self):
        return self._strides == FakeCuda(self.shape)._strides

    def data_ptr(self):
        return 0x1000


def test_rows_accepts_a_view_with_a_wider_leading_dimension():
    p, ld = dust._rows(FakeCuda((10, 8), strides=(12, 1)), 8, "T", rows=10, device=0)
    assert p.value == 0x1000 and ld == 12


@pytest.mark.parametrize("t,err", [
    (FakeCuda((9, 8)), ValueError),                       # fewer rows than the call covers
    (FakeCuda((10, 7)), ValueError),                      # fewer columns than the row width
    (FakeCuda((10, 8), strides=(1, 10)), ValueError),     # column-major
    (FakeCuda((80,)), ValueError),                        # not 2-D
    (FakeCuda((10, 8), dtype=torch.float64), TypeError),  # wrong type
    (FakeCuda((10, 8), cuda=False), TypeError),           # host memory
    (FakeCuda((10, 8), device=1), ValueError),            # another device than the plan's
])
def test_rows_refuses(t, err):
    with pytest.raises(err):
        dust._rows(t, 8, "T", rows=10, device=0)


def test_masses_and_counters():
    assert dust._masses(None, 10).value in (None, 0)
    assert dust._masses(FakeCuda((10,)), 10, 0).value == 0x1000
    with pytest.raises(ValueError):
        dust._masses(FakeCuda((9,)), 10, 0)                      # too short
    with pytest.raises(ValueError):
        dust._masses(FakeCuda((10,), strides=(2,)), 10, 0)       # strided
    with pytest.raises(TypeError):
        dust._masses(FakeCuda((10,), dtype=torch.float64), 10, 0)
    assert dust._counters(FakeCuda((dust.N_COUNTERS,), dtype=torch.int64), 0).value == 0x1000
    with pytest.raises(ValueError):
        dust._counters(FakeCuda((dust.N_COUNTERS - 1,), dtype=torch.int64), 0)
    with pytest.raises(TypeError):
        dust._counters(FakeCuda((dust.N_COUNTERS,), dtype=torch.int32), 0)


def test_extra_heating_rows_checked():
    assert dust._ext(None, False, 8, 10) is None
    x = dust._ext(FakeCuda((10, 8)), False, 8, 10, 0)
    assert x.ldq == 8 and x.warm_start == 0
    with pytest.raises(ValueError):
        dust._ext(FakeCuda((9, 8)), False, 8, 10, 0)


def test_probe_output_must_be_device_memory():
    import bench
    with pytest.raises(TypeError):
        bench.probe_launch(None, 2, 4, 16, FakeCuda((1024,), cuda=False))
    with pytest.raises(ValueError):
        bench.probe_launch(None, 2, 4, 16, FakeCuda((1023,)))


def test_batched_calls_need_one_entry_per_grid():
    with pytest.raises(ValueError):
        dust.batch_run([], [FakeCuda((4, 8))], [None], [], [])
    with pytest.raises(ValueError):
        dust.Batch([], [FakeCuda((4, 8))], [None], [], [])
