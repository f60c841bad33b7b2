"""Pins for the triply periodic Ewald oracle (no GPU).

The oracle is tied to facts outside its own formula: the published Madelung
constants of the rock-salt and caesium-chloride lattices (a rock-salt cell in
a non-cubic supercell too), the xi-independence of the Ewald total, the
vanishing field at a lattice site, and finite differences of the energy.
"""
import numpy as np
import pytest

import oracle
from paper_1611_09538_amd import workloads

# Madelung constants referred to the nearest-neighbour distance
# (rock salt: Sakamoto 1958 and later refinements; caesium chloride: same
# sources), to the digits quoted in the literature.
M_NACL = 1.747564594633182
M_CSCL = 1.762674773070988


def _rocksalt(nx, ny, nz, shift):
    pts, q = [], []
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                pts.append([i, j, k])
                q.append((-1.0) ** (i + j + k))
    return np.asarray(pts, float) + np.asarray(shift), np.asarray(q)


@pytest.mark.parametrize("xi", [0.9, 2.5])
def test_rocksalt_madelung_constant(xi):
    x, q = _rocksalt(2, 2, 2, [0.31, 0.17, 0.43])
    phi, E = oracle.ewald3p_total(x, q, [2.0, 2.0, 2.0], xi)
    assert np.allclose(q * phi, -M_NACL, rtol=0, atol=2e-14)
    assert np.abs(E).max() < 1e-13          # every site is a centre of symmetry


def test_rocksalt_in_noncubic_supercell():
    x, q = _rocksalt(2, 4, 2, [0.05, 0.6, 0.9])
    phi, _ = oracle.ewald3p_total(x, q, [2.0, 4.0, 2.0], 1.7)
    assert np.allclose(q * phi, -M_NACL, rtol=0, atol=2e-14)


def test_caesium_chloride_madelung_constant():
    x = np.array([[0.1, 0.2, 0.3], [0.6, 0.7, 0.8]])
    q = np.array([1.0, -1.0])
    phi, E = oracle.ewald3p_total(x, q, [1.0, 1.0, 1.0], 3.0)
    d = np.sqrt(3.0) / 2.0
    assert np.allclose(q * phi * d, -M_CSCL, rtol=0, atol=1e-13)
    assert np.abs(E).max() < 1e-13


def test_total_is_xi_independent():
    rng = np.random.default_rng(11)
    box = np.array([1.0, 1.3, 0.8])
    x = workloads.uniform_positions(rng, 40, box)
    q = workloads.neutral_uniform(rng, 40)
    pa, Ea = oracle.ewald3p_total(x, q, box, 4.0)
    pb, Eb = oracle.ewald3p_total(x, q, box, 7.5)
    assert np.linalg.norm(pa - pb) / np.linalg.norm(pa) < 1e-13
    assert np.linalg.norm(Ea - Eb) / np.linalg.norm(Ea) < 1e-13


def test_energy_gradient_is_minus_force():
    rng = np.random.default_rng(12)
    box = np.array([1.1, 0.9, 1.0])
    x = workloads.uniform_positions(rng, 16, box)
    q = workloads.neutral_uniform(rng, 16)
    xi = 5.0

    def energy(xx):
        phi, _ = oracle.ewald3p_total(xx, q, box, xi)
        return 0.5 * float(np.dot(q, phi))

    _, E = oracle.ewald3p_total(x, q, box, xi)
    h = 1e-5
    for m in (0, 7):
        for d in range(3):
            xp = x.copy(); xp[m, d] += h
            xm = x.copy(); xm[m, d] -= h
            dU = (energy(xp) - energy(xm)) / (2 * h)
            assert dU == pytest.approx(-q[m] * E[m, d], rel=1e-7, abs=1e-9)
