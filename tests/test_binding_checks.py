"""CPU tests of the binding's argument checks: a tensor of the wrong dtype,
shape or device, or a host tensor where a device address is expected, is
refused with ValueError before any library call (the C ABI takes raw device
pointers and cannot size-check them)."""

import numpy as np
import pytest
import torch

from paper_1806_04593_amd import yyg


class _NoLib:
    """Stand-in handle: any library call through it would fail the test."""

    @property
    def value(self):
        raise AssertionError("library reached")


def _fake_grid(shape=(2, 3, 4, 5)):
    g = yyg.Grid.__new__(yyg.Grid)
    g._h = _NoLib()
    g.device = 0
    g.shape = shape
    return g


def _fake_batch(grids):
    b = yyg.Batch.__new__(yyg.Batch)
    b.grids = grids
    b._h = _NoLib()
    return b


def _bad_tensors(shape):
    return [
        torch.zeros(shape, dtype=torch.float32),          # host, wrong dtype
        torch.zeros(shape, dtype=torch.float64),          # host tensor where a device one is needed
        np.zeros(shape, dtype=np.float64),                # not a tensor at all (batch, sep_phase)
    ]


def test_device_array_refuses_before_any_library_call():
    shape = (2, 3, 4, 5)
    with pytest.raises(ValueError, match="dtype"):
        yyg.device_array(torch.zeros(shape, dtype=torch.float32), shape, "x")
    with pytest.raises(ValueError, match="CUDA"):
        yyg.device_array(torch.zeros(shape, dtype=torch.float64), shape, "x")
    with pytest.raises(ValueError, match="torch"):
        yyg.device_array(np.zeros(shape), shape, "x")


def test_host_array_checks():
    shape = (2, 3, 4, 5)
    with pytest.raises(ValueError):
        yyg.host_array(np.zeros(shape, dtype=np.float32), shape, "x")
    with pytest.raises(ValueError):
        yyg.host_array(np.zeros((2, 3, 4, 6)), shape, "x")
    with pytest.raises(ValueError):
        yyg.host_array(np.zeros((2, 3, 5, 4)).transpose(0, 1, 3, 2), shape, "x")
    assert yyg.host_array(np.zeros(shape), shape, "x") != 0


@pytest.mark.parametrize("i", range(2))
def test_grid_methods_refuse_bad_tensors(i):
    g = _fake_grid()
    t = _bad_tensors(g.shape)[i]
    with pytest.raises(ValueError):
        g.solve(t)
    with pytest.raises(ValueError):
        g.upload_rho(t)
    with pytest.raises(ValueError):
        g.sep_phase(4, t)


def test_grid_numpy_paths_check_shape_and_dtype():
    g = _fake_grid()
    with pytest.raises(ValueError):
        g.solve(np.zeros((2, 3, 4, 6)))
    with pytest.raises(ValueError):
        g.solve(np.zeros(g.shape, dtype=np.float32))
    with pytest.raises(ValueError):
        g.upload_rho(np.zeros((1, 3, 4, 5)))


@pytest.mark.parametrize("i", range(3))
def test_batch_solve_refuses_bad_tensors(i):
    grids = [_fake_grid((2, 3, 4, 5)), _fake_grid((2, 2, 4, 5))]
    b = _fake_batch(grids)
    bad = _bad_tensors(grids[1].shape)[i]
    good0 = _bad_tensors(grids[0].shape)[1]   # also refused: host tensor
    with pytest.raises(ValueError):
        b.solve([good0, bad], [good0, bad])
    with pytest.raises(ValueError):
        b.solve([good0], [good0, bad])        # wrong count


def test_safety_entry_points_without_a_device():
    """The host-side halves of the safety entry points: the device-memory
    figure is readable without a GPU (nothing held), and the input check
    refuses a null plan."""
    L = yyg.lib()
    assert yyg.device_bytes() >= 0
    assert L.yyg_device_bytes(None) == yyg.ERR_INVALID_ARG
    assert L.yyg_set_check_finite(None, 1) == yyg.ERR_INVALID_ARG
