"""Writes small_phi_samples.json and polar_small_phi_samples.json: oracle
potentials at seeded sample cells of the small workload (32 uniform shells,
5 deg, lmax 8) on the Yin-Yang grid and on the full-sphere polar grid.  Calls
only the oracle and the seeded workload generator."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1806_04593_amd import workloads as W  # noqa: E402


def main():
    desc = W.describe("small")
    rho = W.density(desc)
    rng = np.random.default_rng(2024)
    samples = np.stack([rng.integers(0, 2, 64), rng.integers(0, 32, 64),
                        rng.integers(0, desc["n_theta"], 64), rng.integers(0, desc["n_phi"], 64)], 1)
    vals = O.solve_sampled(desc["r_edges"], desc["n_theta"], desc["n_phi"], desc["delta_theta"],
                           desc["delta_phi"], desc["lmax"], desc["G"], rho, samples)
    out = {"workload": "small", "written_by": "tests/golden/make_golden.py (oracle only)",
           "samples": samples.tolist(), "phi": [float(v) for v in vals]}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "small_phi_samples.json"), "w") as fh:
        json.dump(out, fh, indent=1)

    desc = W.describe("polar_small")
    rho = W.density(desc)
    rng = np.random.default_rng(2025)
    samples = np.stack([np.zeros(64, dtype=np.int64), rng.integers(0, 32, 64),
                        rng.integers(0, desc["n_theta"], 64), rng.integers(0, desc["n_phi"], 64)], 1)
    vals = O.solve_polar_sampled(desc["r_edges"], desc["n_theta"], desc["n_phi"], desc["lmax"], desc["G"], rho,
                                 samples)
    out = {"workload": "polar_small", "written_by": "tests/golden/make_golden.py (oracle only)",
           "samples": samples.tolist(), "phi": [float(v) for v in vals]}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "polar_small_phi_samples.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
