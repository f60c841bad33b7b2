"""Write oracle reference values for sampled targets of the large standard
cases, which the oracle cannot evaluate in full within a test's time.

Calls only the oracle (direct Ewald1P sums at xi_o = 0.45/L3) and the seeded
input generators.  Usage:  python tests/golden/make_oracle_samples.py [case ...]
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1611_09538_amd import workloads  # noqa: E402

# case -> (number of sampled targets, sampling seed)
SAMPLES = {"fp32_1e6": (2000, 2024)}


def path(case):
    return os.path.join(HERE, f"oracle_{case}.npz")


def inputs(case):
    """The case's positions and charges as the evaluation receives them:
    FP32 cases take positions rounded to float32 (the FP32 entry points
    receive float32 coordinates); charges stay exactly neutral."""
    x, q, box, c = workloads.make_case(case)
    if c["precision"] == "fp32":
        x = x.astype(np.float32).astype(np.float64)
    return x, q, box


def make(case):
    nt, seed = SAMPLES[case]
    x, q, box = inputs(case)
    tg = np.sort(np.random.default_rng(seed).choice(x.shape[0], nt, replace=False))
    phi, E = oracle.ewald_total(x, q, box, targets=tg)
    np.savez_compressed(path(case), targets=tg, phi=phi, E=E)
    print("wrote", path(case), flush=True)


if __name__ == "__main__":
    for c in (sys.argv[1:] or list(SAMPLES)):
        make(c)
