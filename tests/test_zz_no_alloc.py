"""yyg_solve_noalloc (the allocation-free separable solve) through the C ABI
against yyg_solve on the same plan: bit-identical potentials, on two calls
in a row, the second on a smaller grid; over-size plans refused."""

import ctypes

import numpy as np
import pytest

import oracle as O
from paper_1806_04593_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _case(name):
    torch = _torch()
    from paper_1806_04593_amd import yyg
    desc = W.describe(name)
    rho = W.density(desc)
    g = yyg.Grid(desc, 0)
    g.set_method("separable")
    d_rho = torch.from_numpy(rho).to("cuda")
    g.upload_rho(d_rho)
    ref = torch.empty(g.shape, dtype=torch.float64, device="cuda")
    g.solve(ref)
    torch.cuda.synchronize()
    return desc, rho, g, d_rho, ref


def _noalloc(g, d_rho, d_phi, stream):
    from paper_1806_04593_amd import yyg
    st = yyg.lib().yyg_solve_noalloc(g.handle, ctypes.c_void_p(d_rho.data_ptr()), ctypes.c_void_p(d_phi.data_ptr()),
                                     ctypes.c_void_p(stream.cuda_stream))
    return st


def test_noalloc_matches_solve_twice_then_smaller():
    torch = _torch()
    stream = torch.cuda.current_stream()
    for name in ("sn_core", "small"):        # the second call on a smaller grid
        desc, rho, g, d_rho, ref = _case(name)
        out = torch.full(g.shape, float("nan"), dtype=torch.float64, device="cuda")
        assert _noalloc(g, d_rho, out, stream) == 0
        torch.cuda.synchronize()
        assert torch.equal(out, ref), name
        if name == "small":
            phi = out.cpu().numpy()
            full = O.solve(desc["r_edges"], desc["n_theta"], desc["n_phi"], desc["delta_theta"], desc["delta_phi"],
                           desc["lmax"], desc["G"], rho)
            assert float(np.max(np.abs(phi - full) / np.abs(full))) <= 1e-12
        g.close()


def test_noalloc_streaming_phi_kernels():
    """The allocation-free solve with the streaming phi synthesis and analysis
    and an extra-column analysis tile selected (their own argument blocks,
    pointed at the scratch regions) equals yyg_solve with the same kernels,
    bit for bit."""
    torch = _torch()
    stream = torch.cuda.current_stream()
    desc, rho, g, d_rho, _ = _case("sn_core")
    n0, n4 = g.sep_variant_count(0), g.sep_variant_count(4)
    # first streaming analysis + first streaming synthesis; last extra-column
    # tile + last streaming synthesis (8 streaming analysis kernels and 8
    # extra-column tiles end the analysis range, 16 streaming kernels the
    # synthesis range)
    for v0, v4 in ((n0 - 16, n4 - 16), (n0 - 1, n4 - 1)):
        g.sep_config(0, v0)
        g.sep_config(4, v4)
        ref = torch.empty(g.shape, dtype=torch.float64, device="cuda")
        g.upload_rho(d_rho)
        g.solve(ref)
        out = torch.full(g.shape, float("nan"), dtype=torch.float64, device="cuda")
        assert _noalloc(g, d_rho, out, stream) == 0
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (g.sep_kernel(0), g.sep_kernel(4))
    g.close()


def test_noalloc_refusals():
    torch = _torch()
    from paper_1806_04593_amd import yyg
    stream = torch.cuda.current_stream()
    desc = W.describe("small")
    g = yyg.Grid(desc, 0)
    d = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    assert _noalloc(g, d, d, stream) == -4          # dense plan: YYG_ERR_NOT_READY
    g.close()
    # spheroid (n_r 550, 1 deg, lmax 40): its intermediates exceed 64 MiB
    desc = W.describe("spheroid")
    g = yyg.Grid(desc, 0)
    g.set_method("separable")
    d = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    assert _noalloc(g, d, d, stream) == -5          # YYG_ERR_UNSUPPORTED
    g.close()
