"""The homogeneous-ellipsoid test of Sect. 5 at reduced size, through the C
library: the trends of the paper's lmax sweep must hold.  The error against
the semi-analytic potential falls with lmax on both grids, the finer grid is
more accurate once the multipole truncation no longer dominates, and the
error concentrates at the ellipsoid's surface."""

import sys

import pytest

pytestmark = pytest.mark.gpu

LMAX = [0, 4, 8, 16, 32]
SETUPS = {"low": (100, 4.0), "high": (200, 2.0)}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rows():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04593_amd import validation as V
    return V.sweep(["yinyang", "polar"], SETUPS, LMAX, "separable", log=_say)


def _errs(rows, grid, setup, key="max_rel_err"):
    return [r[key] for r in rows if r["grid"] == grid and r["setup"] == setup]


@pytest.mark.parametrize("grid", ["yinyang", "polar"])
@pytest.mark.parametrize("setup", ["low", "high"])
def test_error_falls_with_lmax(rows, grid, setup):
    e = _errs(rows, grid, setup)
    assert all(e[i + 1] < e[i] for i in range(3)), e          # up to lmax 16
    assert e[4] <= e[3] * 1.02, e                              # and no growth after


@pytest.mark.parametrize("grid", ["yinyang", "polar"])
def test_finer_grid_is_more_accurate(rows, grid):
    lo, hi = _errs(rows, grid, "low"), _errs(rows, grid, "high")
    assert hi[3] < lo[3] and hi[4] < lo[4], (lo, hi)


def test_grids_agree_and_error_sits_at_the_surface(rows):
    yy, po = _errs(rows, "yinyang", "high"), _errs(rows, "polar", "high")
    assert abs(yy[4] - po[4]) < 0.5 * po[4], (yy, po)
    for grid in ("yinyang", "polar"):
        near = _errs(rows, grid, "high", "max_rel_err_near_surface")[4]
        core = _errs(rows, grid, "high", "max_rel_err_core")[4]
        assert near > 3.0 * core, (grid, near, core)
