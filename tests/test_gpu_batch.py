"""Batched solves of uneven fields (grouped persistent launches replayed from
a HIP graph) against the oracle and against single-plan solves."""

import sys

import numpy as np
import pytest

import oracle as O
from paper_1806_04593_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-4, "bf16x3": 1e-6, "fp16x2": 1e-6}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _fields(n=6):
    """Uneven fields drawn like the 64-field batch, with smaller radial counts
    so the oracle stays quick."""
    rng = np.random.default_rng(44)
    out = []
    for f in range(n):
        n_r = int(rng.integers(20, 90))
        res = float(rng.choice([2.0, 3.0, 4.0]))
        lmax = int(rng.integers(10, 31))
        out.append(W.make_desc(f"batch{f}", np.linspace(0.0, 1.0, n_r + 1), res, lmax, 1.0, 1000 + f))
    return out


def _samples(desc, k, seed):
    rng = np.random.default_rng(seed)
    nR = len(desc["r_edges"]) - 1
    return np.stack([rng.integers(0, 2, k), rng.integers(0, nR, k),
                     rng.integers(0, desc["n_theta"], k), rng.integers(0, desc["n_phi"], k)], 1)


def _oracle(desc, rho, s):
    return O.solve_sampled(desc["r_edges"], desc["n_theta"], desc["n_phi"], desc["delta_theta"],
                           desc["delta_phi"], desc["lmax"], desc["G"], rho, s)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "fp16x2"])
def test_batch_against_oracle_and_replays(precision):
    torch = _torch()
    from paper_1806_04593_amd import yyg
    descs = _fields()
    rhos = [W.density(d) for d in descs]
    grids = [yyg.Grid(d, 0) for d in descs]
    if precision != "fp64":
        for g in grids:
            g.prepare(precision)
    b = yyg.Batch(grids, precision)
    d_rho = [torch.from_numpy(r).to("cuda") for r in rhos]
    d_phi = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for g in grids]
    samples = [_samples(d, 120, 7 + i) for i, d in enumerate(descs)]
    refs = [_oracle(d, r, s) for d, r, s in zip(descs, rhos, samples)]

    def check(tag):
        worst = 0.0
        for p, s, ref in zip(d_phi, samples, refs):
            got = p.cpu().numpy()[s[:, 0], s[:, 1], s[:, 2], s[:, 3]]
            worst = max(worst, float(np.max(np.abs(got - ref) / np.abs(ref))))
        _say(f"batch {precision} {tag}: max rel err {worst:.3e} ({b.info()})")
        assert worst <= TOL[precision], (tag, worst)

    b.solve(d_rho, d_phi)
    torch.cuda.synchronize()
    check("first launch (records the graph)")
    # replays, with eager work and a clobbered output between them
    for rep in range(3):
        for p in d_phi:
            p.zero_()
        torch.cuda.synchronize()
        b.solve(d_rho, d_phi)
        torch.cuda.synchronize()
        check(f"replay {rep}")
    # new output buffers: the argument arrays are rewritten, graph reused
    d_phi = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for g in grids]
    b.solve(d_rho, d_phi)
    torch.cuda.synchronize()
    check("new pointers")
    b.autotune()
    for p in d_phi:
        p.zero_()
    b.solve(d_rho, d_phi)
    torch.cuda.synchronize()
    check("after autotune")


def test_batch_matches_single_solves_fp64():
    torch = _torch()
    from paper_1806_04593_amd import yyg
    descs = _fields(5)
    rhos = [W.density(d) for d in descs]
    grids = [yyg.Grid(d, 0) for d in descs]
    single = []
    for g, r in zip(grids, rhos):
        d_r = torch.from_numpy(r).to("cuda")
        d_p = torch.empty(g.shape, dtype=torch.float64, device="cuda")
        g.upload_rho(d_r)
        g.solve(d_p)
        torch.cuda.synchronize()
        single.append(d_p.cpu().numpy())
    b = yyg.Batch(grids, "fp64")
    stream = torch.cuda.Stream()
    d_rho = [torch.from_numpy(r).to("cuda") for r in rhos]
    d_phi = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for g in grids]
    torch.cuda.synchronize()
    b.solve(d_rho, d_phi, stream=stream)
    stream.synchronize()
    for p, ref in zip(d_phi, single):
        got = p.cpu().numpy()
        assert float(np.max(np.abs(got - ref) / np.abs(ref))) < 1e-13


def test_batch_rejects_bad_arguments():
    _torch()
    from paper_1806_04593_amd import yyg
    descs = _fields(2)
    grids = [yyg.Grid(d, 0) for d in descs]
    with pytest.raises(yyg.YygError) as ei:
        yyg.Batch(grids, "bf16x3")     # not prepared
    assert ei.value.status == -4
    b = yyg.Batch(grids, "fp64")
    with pytest.raises(yyg.YygError) as ei:
        b.autotune()                   # needs one solve first
    assert ei.value.status == -4


def test_separable_batch_against_oracle_replays_and_mixed_grids():
    """Every plan in the separable form: the batch runs the separable phases
    as grouped launches over all fields (here with a polar plan among the
    Yin-Yang ones): against the oracle on first launch, on graph replays,
    with new pointers and after the batch autotuner; against per-plan
    separable solves of the same fields."""
    torch = _torch()
    from paper_1806_04593_amd import yyg
    descs = _fields(5)
    descs.append(W.make_polar_desc("polar_f", np.linspace(0.0, 1.0, 41), 6.0, 12, 1.0, 1099, recipe="small"))
    rhos = [W.density(d) for d in descs]
    grids = [yyg.Grid(d, 0) for d in descs]
    single = []
    for g, r in zip(grids, rhos):
        g.set_method("separable")
        d_r = torch.from_numpy(r).to("cuda")
        d_p = torch.empty(g.shape, dtype=torch.float64, device="cuda")
        g.upload_rho(d_r)
        g.solve(d_p)
        torch.cuda.synchronize()
        single.append(d_p.cpu().numpy())
    samples = [_samples(d, 120, 70 + i) for i, d in enumerate(descs)]
    refs = []
    for d, r, s in zip(descs, rhos, samples):
        if d.get("kind") == "polar":
            refs.append(O.solve_polar_sampled(d["r_edges"], d["n_theta"], d["n_phi"], d["lmax"], d["G"], r,
                                              np.stack([np.zeros(len(s), int), s[:, 1], s[:, 2], s[:, 3]], 1)))
            s[:, 0] = 0
        else:
            refs.append(_oracle(d, r, s))
    b = yyg.Batch(grids, "fp64")
    info = b.info()
    assert info["var_theta_ana"] >= 0, info           # the separable batch
    d_rho = [torch.from_numpy(r).to("cuda") for r in rhos]
    d_phi = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for g in grids]

    def check(tag):
        worst = worst_single = 0.0
        for p, s, ref, one in zip(d_phi, samples, refs, single):
            got = p.cpu().numpy()
            worst = max(worst, float(np.max(np.abs(got[s[:, 0], s[:, 1], s[:, 2], s[:, 3]] - ref) / np.abs(ref))))
            worst_single = max(worst_single, float(np.max(np.abs(got - one) / np.abs(one))))
        _say(f"separable batch {tag}: max rel err {worst:.3e} vs oracle, {worst_single:.3e} vs single ({b.info()})")
        assert worst <= TOL["fp64"], (tag, worst)
        assert worst_single <= 1e-13, (tag, worst_single)

    b.solve(d_rho, d_phi)
    torch.cuda.synchronize()
    check("first launch")
    for rep in range(2):
        for p in d_phi:
            p.zero_()
        _ = (torch.arange(4096, device="cuda", dtype=torch.float64) * rep).sum().item()
        torch.cuda.synchronize()
        b.solve(d_rho, d_phi)
        torch.cuda.synchronize()
        check(f"replay {rep}")
    d_phi = [torch.zeros(g.shape, dtype=torch.float64, device="cuda") for g in grids]
    b.solve(d_rho, d_phi)
    torch.cuda.synchronize()
    check("new pointers")
    b.autotune()
    for p in d_phi:
        p.zero_()
    b.solve(d_rho, d_phi)
    torch.cuda.synchronize()
    check("after autotune")
    ms = b.profile()
    assert ms[0] > 0 and ms[1] > 0 and ms[2] > 0
    b.close()
