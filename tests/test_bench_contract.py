"""CPU checks of the benchmark's bookkeeping: the roofline counts the
folded kernels' work once, and the counter figures are tied to every
source a timed kernel is compiled from."""

import importlib.util
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1806_04593_amd", "csrc")


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


BINARY = dict(lmax=64, n_theta=182)
M, NANG = 2000, 182 * 542


def _head(name, phase="phi_synthesis", ms=0.7):
    other = "phi_analysis" if phase == "phi_synthesis" else "phi_synthesis"
    return {
        "kernels_ms": {phase: ms, other: ms / 2},
        "phase_alone_ms": {phase: ms, other: ms / 2},
        "kernel_names": {phase: name, other: "yyg::gemm_nt_f64_batched<0, 64, 64, 2, 2, 66180>"},
    }


@pytest.mark.parametrize("name, folded", [
    ("yyg::phi_syn_stream<1, 9, 8, 4, 138>", True),
    ("yyg::phi_syn_stream_cf<1, 9, 8, 4, 138>", True),
    ("yyg::phi_ana_stream<2, 3, 4, 2, 276>", True),
    ("yyg::phi_syn_lean_kernel<2, 4>", True),
    ("yyg::phi_direct_kernel<false, 8, 4, 2, true>", True),
    ("yyg::phi_direct_kernel<false, 8, 4, 2, false>", False),
    ("yyg::gemm_nt_f64_batched<1, 64, 80, 4, 1, 258>", True),     # FoldC synthesis tile
    ("yyg::gemm_nt_f64_batched<0, 64, 64, 2, 2, 66180>", True),   # FoldA + extra column
    ("yyg::gemm_nt_f64_batched<1, 128, 48, 4, 1, 2>", False),     # unfolded synthesis tile
])
def test_roofline_counts_folded_work_once(name, folded):
    """A folded phi transform does half the multiply-adds of the unfolded
    count 2 M n_ang (2L + 1): its achieved TFLOP/s must be halved."""
    b = _bench()
    phase = "phi_analysis" if "<0," in name or "ana" in name else "phi_synthesis"
    roof, got_phase, kname = b.phi_roofline(_head(name, phase), BINARY, M, NANG)
    assert got_phase == phase and kname == name
    full = 2.0 * M * NANG * (2 * BINARY["lmax"] + 1)
    assert roof["algorithmic_flops"] == pytest.approx(full / 2 if folded else full)


def test_counter_figures_cover_every_timed_kernel_source():
    """Every source that defines kernels the solves time is hashed into the
    sha that validates the committed counter figures (the finiteness check
    is not timed)."""
    b = _bench()
    hashed = {os.path.basename(p) for p in b.KERNEL_SRCS}
    for f in sorted(os.listdir(CSRC)):
        if not f.endswith((".hip", ".h")):
            continue
        text = open(os.path.join(CSRC, f)).read()
        if re.search(r"__global__", text) and f != "yyg_checks.hip":
            assert f in hashed, f
    # headers with the argument layouts the kernels read
    assert "yyg_internal.h" in hashed
    for p in b.KERNEL_SRCS:
        assert os.path.exists(p), p
