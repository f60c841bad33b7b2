"""Step-by-step numpy model of the SE1P k-space algorithm (test infrastructure).

Follows Algorithm 1 of the paper in its order and notation, with the adaptive
transforms of Algorithms 2-3, using numpy's FFT as a library step and plain
loops over particles.  It exists to check intermediate arrays of the GPU path
(the gridded charge H after step 2, the potentials after step 6) far more
tightly than the approximation error allows against the direct Ewald sums.
It shares no code with the GPU path; the grid geometry (sizes, padded FFT
lengths) is passed in explicitly so both sides discretise the same way.

Pins (tests/test_discrete.py, CPU): G_R against a numerical Hankel
transform of the truncated logarithm and its kappa -> 0 limit; the gridded
Gaussian of one charge against the mass, mean and variance of a normalised
Gaussian; the AFT against the discrete Fourier sum written out on a tiny
grid with per-slab padded sizes; AIFT o AFT against the identity; the gather
against the transpose of the gridding and its gradient against finite
differences; the whole k-space potential and field against the direct
Ewald1P sums in three boxes; the dropped (0, 0) coefficient against keeping
it.

Readings taken where the paper is silent or garbled (each also listed in the
design notes):

* Grid placement (step 2): along the free directions x, y, array index i sits
  at position (i - P/2) h, so the extended grid starts P/2 points before the
  charge box; along z, index l sits at l h.  The support of a particle at x
  (even P) is the P points with unshifted index floor(x/h) - P/2 + 1 ...
  floor(x/h) + P/2 in every direction (z taken modulo M3).
* Gather prefactor (step 6): derived from eqs. ewald1p_allk, mft and imft
  instead of the printed constant: phi^F = 4 pi h^3 sum_grid Htilde g, with g
  the same normalised truncated Gaussian as in step 2, and Htilde the
  normalised inverse transform of the scaled unnormalised forward transform
  (the h^2 and Delta kappa^2 factors cancel as noted in section 3.4).
* Field: the analytic gradient of the gather, E^F = -grad phi^F
  = 4 pi h^3 (4 xi^2/eta) sum Htilde (x_m - x_grid) g.
* The (kappa = 0, k3 = 0) coefficient is set to zero: for a neutral system it
  is the total charge times the discrete Gaussian mass, zero up to the
  approximation error, and leaving it in turns rounding into a constant
  potential offset.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp

C_SHAPE = 0.95  # c in eq. comp_eta


def eta_of(P, xi, h):
    """Gaussian width parameter, eq. comp_eta."""
    return P * xi * xi * h * h / (C_SHAPE ** 2 * np.pi)


def G_R(kappa, R):
    """Fourier transform of the truncated 2D Green's function,
    eqs. g_zeromod and g_zeromod0."""
    kappa = np.asarray(kappa, dtype=np.float64)
    out = np.empty_like(kappa)
    z = kappa == 0
    k = kappa[~z]
    out[~z] = (1.0 - sp.j0(R * k)) / (k * k) - R * np.log(R) * sp.j1(R * k) / k
    out[z] = R * R / 4.0 * (1.0 - 2.0 * np.log(R))
    return out


def windows(xc, h, P, M3):
    """Support index windows of one particle: (ix, iy, iz, dx, dy, dz) with
    array indices and the signed distances particle - grid point."""
    c = np.floor(xc / h).astype(np.int64)
    off = np.arange(P) - P // 2 + 1
    u = c[:, None] + off[None, :]          # unshifted indices, 3 x P
    ix = u[0] + P // 2
    iy = u[1] + P // 2
    iz = np.mod(u[2], M3)
    dx = xc[0] - u[0] * h
    dy = xc[1] - u[1] * h
    dz = xc[2] - u[2] * h
    return ix, iy, iz, dx, dy, dz


class Geometry:
    """Grid geometry of one SE1P evaluation (all sizes explicit)."""

    def __init__(self, box, M3, P, xi, Mt, n0, nl_size, n_l):
        self.box = np.asarray(box, dtype=np.float64)
        self.M3 = int(M3)
        self.P = int(P)
        self.xi = float(xi)
        self.h = self.box[2] / self.M3
        self.Mt = tuple(int(v) for v in Mt)          # (Mt1, Mt2) extended grid
        self.n0 = tuple(int(v) for v in n0)          # padded sizes, k3 = 0
        self.nl_size = tuple(int(v) for v in nl_size)  # padded sizes, set I
        self.n_l = int(n_l)
        self.eta = eta_of(P, xi, self.h)
        self.alpha = 2.0 * xi * xi / self.eta      # Gaussian exponent
        self.cg = (2.0 * xi * xi / (np.pi * self.eta)) ** 1.5
        # R: largest distance between two points of the support region
        M = np.ceil(self.box[:2] / self.h - 1e-9).astype(int)
        ext = (M + self.P) * self.h
        self.R = float(np.hypot(ext[0], ext[1]))

    def slab_size(self, n3):
        """Upsampling of eq. upsamplings as padded 2D FFT sizes."""
        a = abs(n3)
        if a == 0:
            return self.n0
        if a <= self.n_l:
            return self.nl_size
        return self.Mt


def spread(geo, x, q):
    """Step 2: H on the M~1 x M~2 x M3 grid (eq. spread_1p)."""
    P, h, M3 = geo.P, geo.h, geo.M3
    H = np.zeros((geo.Mt[0], geo.Mt[1], M3))
    for n in range(x.shape[0]):
        xc = np.array([x[n, 0], x[n, 1], np.mod(x[n, 2], geo.box[2])])
        ix, iy, iz, dx, dy, dz = windows(xc, h, P, M3)
        wx = np.exp(-geo.alpha * dx * dx)
        wy = np.exp(-geo.alpha * dy * dy)
        wz = np.exp(-geo.alpha * dz * dz)
        H[np.ix_(ix, iy, iz)] += q[n] * geo.cg * np.einsum(
            "i,j,k->ijk", wx, wy, wz)
    return H


def scaling(geo, n3, shape, zero_dc=True):
    """Scaling factor of eq. scale_1p with G of eq. G_kappa_k on one slab.

    ``zero_dc`` sets the (kappa, k3) = (0, 0) coefficient to zero (see the
    module docstring); with it False the coefficient keeps the value
    G_R(0) = R^2/4 (1 - 2 log R) of eq. g_zeromod0."""
    n1, n2 = shape
    h, xi, eta = geo.h, geo.xi, geo.eta
    k1 = 2 * np.pi * np.fft.fftfreq(n1, d=h)
    k2 = 2 * np.pi * np.fft.fftfreq(n2, d=h)
    kap2 = k1[:, None] ** 2 + k2[None, :] ** 2
    k3 = 2 * np.pi * n3 / geo.box[2]
    damp = np.exp(-(1.0 - eta) * (kap2 + k3 * k3) / (4 * xi * xi))
    if n3 != 0:
        G = 1.0 / (kap2 + k3 * k3)
    else:
        G = G_R(np.sqrt(kap2), geo.R)
    S = damp * G
    if n3 == 0 and zero_dc:
        S[0, 0] = 0.0
    return S


def aft(geo, H):
    """Adaptive Fourier transform (Algorithm 2): the 1D FFT along z, then
    per k3 slab a 2D FFT zero-padded to the slab's size (eq. upsamplings).
    Returns the list of slab spectra, index k = n3 mod M3."""
    Hz = np.fft.fft(H, axis=2)                 # step 1
    slabs = []
    for k in range(geo.M3):
        n3 = k if k < geo.M3 // 2 else k - geo.M3
        slabs.append(np.fft.fft2(Hz[:, :, k], s=geo.slab_size(n3)))
    return slabs


def aift(geo, slabs):
    """Adaptive inverse transform (Algorithm 3): per slab the normalised 2D
    IFFT, restricted to the first M~1 x M~2 points, then the normalised
    inverse 1D FFT along z.  Returns the real grid."""
    out = np.zeros((geo.Mt[0], geo.Mt[1], geo.M3), dtype=np.complex128)
    for k, F in enumerate(slabs):
        out[:, :, k] = np.fft.ifft2(F)[:geo.Mt[0], :geo.Mt[1]]
    return np.real(np.fft.ifft(out, axis=2))


def kspace_solve(geo, H, scale=None):
    """Steps 3-5: AFT (Algorithm 2), scaling, AIFT (Algorithm 3).
    Returns Htilde on the same grid, normalised so that phi^F is
    4 pi h^3 sum Htilde g.  ``scale(geo, n3, shape)`` replaces the scaling
    of eq. scale_1p when given."""
    scale = scaling if scale is None else scale
    slabs = aft(geo, H)
    for k, F in enumerate(slabs):
        n3 = k if k < geo.M3 // 2 else k - geo.M3
        F *= scale(geo, n3, F.shape)
    return aift(geo, slabs)


def gather(geo, Ht, x, field=True):
    """Step 6 and its analytic gradient: phi^F and E^F at the particles."""
    P, h, M3 = geo.P, geo.h, geo.M3
    pref = 4.0 * np.pi * h ** 3 * geo.cg
    phi = np.zeros(x.shape[0])
    E = np.zeros((x.shape[0], 3))
    for n in range(x.shape[0]):
        xc = np.array([x[n, 0], x[n, 1], np.mod(x[n, 2], geo.box[2])])
        ix, iy, iz, dx, dy, dz = windows(xc, h, P, M3)
        wx = np.exp(-geo.alpha * dx * dx)
        wy = np.exp(-geo.alpha * dy * dy)
        wz = np.exp(-geo.alpha * dz * dz)
        B = Ht[np.ix_(ix, iy, iz)]
        phi[n] = pref * np.einsum("ijk,i,j,k->", B, wx, wy, wz)
        if field:
            c = 2.0 * geo.alpha * pref
            E[n, 0] = c * np.einsum("ijk,i,j,k->", B, wx * dx, wy, wz)
            E[n, 1] = c * np.einsum("ijk,i,j,k->", B, wx, wy * dy, wz)
            E[n, 2] = c * np.einsum("ijk,i,j,k->", B, wx, wy, wz * dz)
    return phi, E


def se1p_kspace(geo, x, q, field=True, scale=None):
    """phi^F (and E^F) by Algorithm 1 (``scale`` as in kspace_solve)."""
    H = spread(geo, x, q)
    Ht = kspace_solve(geo, H, scale=scale)
    return gather(geo, Ht, x, field=field)
