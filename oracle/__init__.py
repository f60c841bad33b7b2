"""FP64 CPU oracle for the singly periodic Ewald sum (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The product path (the HIP library
and its Python binding under ``paper_1611_09538_amd``) never imports, links or
calls anything here, and nothing here imports the product path.

Two independent references live here:

* ``ewald`` -- the direct Ewald1P sums of section 2.1 (eqs. ewald1p_real,
  ewald1p_fourier_complete, ewald1p_zero, ewald1p_self) and their gradients,
  in plain C (``se1p_oracle.c``), with the special functions of appendix A.
* ``ewald3p`` -- the direct triply periodic Ewald sums (real space, k-space
  over the full reciprocal lattice, self term) in plain C
  (``se3p_oracle.c``), the reference for the SE3P comparison path.
* ``discrete`` -- a step-by-step numpy transcription of the SE1P k-space
  algorithm (Algorithm 1 with the AFT/AIFT of Algorithms 2-3) in the paper's
  order, used to check intermediate arrays (grid after gridding, potentials
  after gathering) of the GPU path.

Pins (tests marked ``not gpu``) tie both to facts outside themselves: closed
forms and library special functions, the xi-independence of the total,
brute-force image sums, Lekner's Bessel-series form of the periodic line
potential, finite differences, and the published Madelung constants of
the rock-salt and caesium-chloride lattices for the triply periodic sum.
"""
from .ewald import (  # noqa: F401
    E1, Ein, K0inc, K0inc_m1, ewald, ewald_total, image_sum, kmodes,
    num_threads, lib_path, build, PARTS_REAL, PARTS_FK, PARTS_F0,
    PARTS_SELF, PARTS_FIELD, PARTS_ALL, ewald3p, ewald3p_total,
)
