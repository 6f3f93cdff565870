"""Failure detection through the C ABI on the GPU: the opt-in non-finite
density check (YYG_ERR_NONFINITE from yyg_solve, yyg_solve_noalloc and
yyg_batch_solve, with phi untouched) and the device-memory cap of the
environment variable YYG_MAX_DEVICE_BYTES (YYG_ERR_OUT_OF_MEMORY, nothing
left allocated by the failed call).  Every kernel runs on valid inputs and
exits normally; the conditions are forced from the host."""

import gc
import sys

import pytest

from paper_1806_04593_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04593_amd import yyg
    return torch, yyg


@pytest.mark.parametrize("method", ["dense", "separable"])
@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
def test_nonfinite_density_is_refused(method, bad):
    torch, yyg = _env()
    desc = W.describe("small")
    rho = W.density(desc)
    g = yyg.Grid(desc, 0)
    g.set_method(method)
    d_rho = torch.from_numpy(rho).to("cuda")
    g.upload_rho(d_rho)
    ref = torch.empty(g.shape, dtype=torch.float64, device="cuda")
    g.solve(ref)
    torch.cuda.synchronize()
    # the check on, finite density: the same result bit for bit
    g.set_check_finite(True)
    out = torch.empty_like(ref)
    g.solve(out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    # one bad cell (the last one: the scan's tail) -> refused, phi untouched
    bad_rho = rho.copy()
    bad_rho.reshape(-1)[-1] = bad
    d_bad = torch.from_numpy(bad_rho).to("cuda")
    g.upload_rho(d_bad)
    out.fill_(7.0)
    with pytest.raises(yyg.YygError) as e:
        g.solve(out)
    assert e.value.status == yyg.ERR_NONFINITE
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    if method == "separable":
        with pytest.raises(yyg.YygError) as e:
            g.solve_noalloc(d_bad, out)
        assert e.value.status == yyg.ERR_NONFINITE
        torch.cuda.synchronize()
        assert bool((out == 7.0).all())
    # the check off again: the solve runs (and propagates the bad value)
    g.set_check_finite(False)
    g.solve(out)
    torch.cuda.synchronize()
    assert not bool(torch.isfinite(out).all())
    g.close()
    _say(f"non-finite check ({method}, {bad}): refused with the check on, solved with it off")


def test_nonfinite_density_is_refused_in_a_batch():
    torch, yyg = _env()
    descs = W.batch_descs(3)
    grids = [yyg.Grid(d, 0) for d in descs]
    rhos = [W.density(d) for d in descs]
    rhos[1].reshape(-1)[17] = float("nan")
    d_rho = [torch.from_numpy(r).to("cuda") for r in rhos]
    d_phi = [torch.full(g.shape, 7.0, dtype=torch.float64, device="cuda") for g in grids]
    b = yyg.Batch(grids, "fp64")
    grids[1].set_check_finite(True)
    with pytest.raises(yyg.YygError) as e:
        b.solve(d_rho, d_phi)
    assert e.value.status == yyg.ERR_NONFINITE
    torch.cuda.synchronize()
    assert all(bool((p == 7.0).all()) for p in d_phi)
    # the field repaired: the batch solves
    d_rho[1] = torch.from_numpy(W.density(descs[1])).to("cuda")
    b.solve(d_rho, d_phi)
    torch.cuda.synchronize()
    assert all(bool(torch.isfinite(p).all()) for p in d_phi)
    b.close()
    for g in grids:
        g.close()


def test_device_memory_cap(monkeypatch):
    torch, yyg = _env()
    desc = W.describe("sn_core")
    gc.collect()   # plans of earlier tests that only a collection would release
    base = yyg.device_bytes()
    # far below one plan: creation fails, and nothing stays allocated
    monkeypatch.setenv("YYG_MAX_DEVICE_BYTES", str(base + (1 << 20)))
    with pytest.raises(yyg.YygError) as e:
        yyg.Grid(desc, 0)
    assert e.value.status == yyg.ERR_OUT_OF_MEMORY
    assert yyg.device_bytes() == base
    monkeypatch.delenv("YYG_MAX_DEVICE_BYTES")
    g = yyg.Grid(desc, 0)
    held = yyg.device_bytes()
    assert held > base
    # at the current figure: the separable form's buffers do not fit; its
    # partial allocations are released, and a retry without the cap works
    monkeypatch.setenv("YYG_MAX_DEVICE_BYTES", str(held))
    with pytest.raises(yyg.YygError) as e:
        g.set_method("separable")
    assert e.value.status == yyg.ERR_OUT_OF_MEMORY
    assert yyg.device_bytes() == held
    with pytest.raises(yyg.YygError) as e:
        g.prepare("fp32")
    assert e.value.status == yyg.ERR_OUT_OF_MEMORY
    assert yyg.device_bytes() == held
    # not a plain number: no cap
    monkeypatch.setenv("YYG_MAX_DEVICE_BYTES", "lots")
    g.set_method("separable")
    monkeypatch.delenv("YYG_MAX_DEVICE_BYTES")
    rho = W.density(desc)
    d_rho = torch.from_numpy(rho).to("cuda")
    g.upload_rho(d_rho)
    out = torch.empty(g.shape, dtype=torch.float64, device="cuda")
    g.solve(out)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
    g.close()
    assert yyg.device_bytes() == base
    _say(f"device memory cap: plan held {held - base} bytes; failures left nothing behind")
