"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic, so both the GPU path and the CPU oracle can take inputs
from it without sharing any computation.  The systems follow the workloads the
paper uses for timing and accuracy (uniformly distributed random charges in a
box, neutral, section 6), at the sizes the five standard cases name.
"""
from __future__ import annotations

import numpy as np


def neutral_pm1(rng, n):
    """+-1 charges, n/2 of each sign, shuffled (n even)."""
    if n % 2:
        raise ValueError("n must be even for exact +-1 neutrality")
    q = np.concatenate([np.ones(n // 2), -np.ones(n // 2)])
    rng.shuffle(q)
    return q


def neutral_uniform(rng, n):
    """Charges uniform in [-1, 1] shifted to zero sum."""
    q = rng.uniform(-1.0, 1.0, n)
    return q - q.mean()


def density_system(n, density, seed):
    """n particles uniform in a cube of side (n / density)^(1/3), charges
    uniform in [-1, 1] shifted to zero sum.  Returns (x, q, box)."""
    rng = np.random.default_rng(seed)
    L = (n / float(density)) ** (1.0 / 3.0)
    box = np.array([L, L, L])
    return uniform_positions(rng, n, box), neutral_uniform(rng, n), box


def density125_system(n, seed):
    """The timing systems of the paper's per-particle timing and SE1P / SE3P
    comparison examples: n particles uniform in a cube of side
    L = (n / 125)^(1/3) (number density 125), charges uniform in [-1, 1]
    shifted to zero sum.  Returns (x, q, box)."""
    rng = np.random.default_rng(seed)
    L = (n / 125.0) ** (1.0 / 3.0)
    box = np.array([L, L, L])
    return uniform_positions(rng, n, box), neutral_uniform(rng, n), box


def uniform_positions(rng, n, box):
    """Positions uniform in [0, L1) x [0, L2) x [0, L3)."""
    box = np.asarray(box, dtype=np.float64)
    x = rng.random((n, 3)) * box
    # keep strictly inside the half-open box after the multiply
    for d in range(3):
        x[:, d] = np.minimum(x[:, d], np.nextafter(box[d], 0.0))
    return x


# Standard cases.  Each returns (x, q, box, info) with x (n,3) float64.
# The method parameters (xi, n_l, s_l, rc, pad_free) next to each case were
# chosen by measured error sweeps against the oracle at the stated tolerance.
CASES = {
    # Plain FP64, N=500, unit box, +-1 charges, M3=32, P=16, rel-RMS 1e-8.
    "small": dict(n=500, box=(1.0, 1.0, 1.0), charges="pm1", seed=1,
                  M3=32, P=16, tol=1e-8, precision="fp64",
                  xi=11.0, nl=4, sl=3.0, rc=0.45, pad_free=0),
    # Plain FP64, N=1e5, unit box, uniform charges, M3=64, P=24, n_l=4.
    "fp64_1e5": dict(n=100_000, box=(1.0, 1.0, 1.0), charges="uniform",
                     seed=2, M3=64, P=24, nl=4, tol=1e-8, precision="fp64",
                     xi=25.0, sl=3.0, rc=0.16, pad_free=8),
    # Differentiation: N=2e5, 1x1x2 box (z long and periodic), +-1 charges.
    # Same grid spacing and xi as fp64_1e5; the k3 spacing halves with the
    # longer period, so twice the upsampled slabs and twice the padding.
    "grad_2e5": dict(n=200_000, box=(1.0, 1.0, 2.0), charges="pm1", seed=3,
                     M3=128, P=24, tol=1e-8, precision="fp64",
                     xi=25.0, nl=8, sl=6.0, rc=0.17, pad_free=8),
    # Precision: N=1e6, 2x2x1 box, uniform charges, FP32, P=12, rel-RMS 1e-5.
    # xi large enough that the real-space pairs stay few at this density
    # (2.5e5 per unit volume); M3 follows xi at the 1e-5 Fourier bar.
    "fp32_1e6": dict(n=1_000_000, box=(2.0, 2.0, 1.0), charges="uniform",
                     seed=4, M3=120, P=12, tol=1e-5, precision="fp32",
                     xi=60.0, nl=10, sl=2.0, rc=0.055, pad_free=4),
}


def make_case(name, n=None, seed=None):
    c = CASES[name]
    n = c["n"] if n is None else n
    rng = np.random.default_rng(c["seed"] if seed is None else seed)
    x = uniform_positions(rng, n, c["box"])
    if c["charges"] == "pm1":
        q = neutral_pm1(rng, n)
    else:
        q = neutral_uniform(rng, n)
    return x, q, np.asarray(c["box"], dtype=np.float64), dict(c, n=n)


def batched_systems(seed=5, nsys=64, nmin=1e3, nmax=5e4):
    """Batch of independent neutral +-1 systems: N log-uniform in
    [nmin, nmax] (made even), period L3 uniform in [0.5, 2], cross-section
    1 x 1.  Returns a list of (x, q, box)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nsys):
        n = int(round(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        n += n % 2
        L3 = rng.uniform(0.5, 2.0)
        box = np.array([1.0, 1.0, L3])
        x = uniform_positions(rng, n, box)
        q = neutral_pm1(rng, n)
        out.append((x, q, box))
    return out
