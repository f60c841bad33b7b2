"""ctypes wrapper around the C oracle (``se1p_oracle.c``).

Test infrastructure: see the package docstring for who may use it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "se1p_oracle.c")
_SRC3 = os.path.join(_HERE, "se3p_oracle.c")
_LIB = os.path.join(_HERE, "libse1p_oracle.so")

PARTS_REAL = 1
PARTS_FK = 2
PARTS_F0 = 4
PARTS_SELF = 8
PARTS_FIELD = 16
PARTS_ALL = 31

_lock = threading.Lock()
_lib = None


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no -march so the object runs
    on any x86-64 host)."""
    if force or _stale():
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", _SRC, _SRC3, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _stale() -> bool:
    if not os.path.exists(_LIB):
        return True
    t = os.path.getmtime(_LIB)
    return t < os.path.getmtime(_SRC) or t < os.path.getmtime(_SRC3)


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if _stale():
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        d = ctypes.c_double
        lib.se1p_oracle_E1.restype = d
        lib.se1p_oracle_E1.argtypes = [d]
        lib.se1p_oracle_Ein.restype = d
        lib.se1p_oracle_Ein.argtypes = [d]
        lib.se1p_oracle_K0inc.restype = d
        lib.se1p_oracle_K0inc.argtypes = [d, d]
        lib.se1p_oracle_K0inc_m1.restype = d
        lib.se1p_oracle_K0inc_m1.argtypes = [d, d]
        lib.se1p_oracle_kmodes.restype = ctypes.c_int
        lib.se1p_oracle_kmodes.argtypes = [d, d]
        lib.se1p_oracle_num_threads.restype = ctypes.c_int
        lib.se1p_oracle_num_threads.argtypes = []
        p = ctypes.c_void_p
        lib.se1p_oracle_ewald.restype = ctypes.c_int
        lib.se1p_oracle_ewald.argtypes = [ctypes.c_long, p, p, p, d, d,
                                          ctypes.c_long, p, ctypes.c_uint, p]
        lib.se1p_oracle_image_sum.restype = ctypes.c_int
        lib.se1p_oracle_image_sum.argtypes = [ctypes.c_long, p, p, d,
                                              ctypes.c_long, p]
        lib.se3p_oracle_ewald.restype = ctypes.c_int
        lib.se3p_oracle_ewald.argtypes = [ctypes.c_long, p, p, p, d, d,
                                          ctypes.c_long, p, p]
        lib.se1p_oracle_init()
        _lib = lib
        return lib


def E1(x: float) -> float:
    """Exponential integral E1(x), x > 0 (appendix A)."""
    return _load().se1p_oracle_E1(float(x))


def Ein(x: float) -> float:
    """gamma + log(x) + E1(x), continuous at 0 where it vanishes."""
    return _load().se1p_oracle_Ein(float(x))


def K0inc(a: float, b: float) -> float:
    """Incomplete Bessel K0(a,b) = int_1^inf exp(-a t - b/t) dt / t."""
    return _load().se1p_oracle_K0inc(float(a), float(b))


def K0inc_m1(a: float, b: float) -> float:
    """int_1^inf exp(-a t - b/t) dt / t^2 = -dK0(a,b)/db."""
    return _load().se1p_oracle_K0inc_m1(float(a), float(b))


def kmodes(xi: float, L3: float) -> int:
    """Number of positive k3 modes the oracle keeps."""
    return _load().se1p_oracle_kmodes(float(xi), float(L3))


def num_threads() -> int:
    return _load().se1p_oracle_num_threads()


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def ewald(x, q, box, xi, rc=None, targets=None, parts=PARTS_ALL):
    """Direct Ewald1P sums at the targets.

    Returns a dict of arrays over the targets:
      phi_R, phi_Fk, phi_F0, phi_self  (ntarget,)
      E_R, E_Fk, E_F0                  (ntarget, 3)
    ``rc`` defaults to 6.5/xi, where erfc(xi rc) < 4e-20.
    """
    lib = _load()
    x = _c(x, np.float64).reshape(-1, 3)
    q = _c(q, np.float64).reshape(-1)
    box = _c(box, np.float64).reshape(3)
    N = x.shape[0]
    if q.shape[0] != N:
        raise ValueError("x and q sizes differ")
    if rc is None:
        rc = 6.5 / xi
    if targets is None:
        tg = None
        nt = N
    else:
        tg = _c(targets, np.int64).reshape(-1)
        nt = tg.shape[0]
    out = np.zeros((nt, 13), dtype=np.float64)
    rcode = lib.se1p_oracle_ewald(
        N, x.ctypes.data, q.ctypes.data, box.ctypes.data, float(xi),
        float(rc), nt, None if tg is None else tg.ctypes.data, int(parts),
        out.ctypes.data)
    if rcode != 0:
        raise RuntimeError(f"oracle error {rcode}")
    return {
        "phi_R": out[:, 0].copy(), "phi_Fk": out[:, 1].copy(),
        "phi_F0": out[:, 2].copy(), "phi_self": out[:, 3].copy(),
        "E_R": out[:, 4:7].copy(), "E_Fk": out[:, 7:10].copy(),
        "E_F0": out[:, 10:13].copy(),
    }


def ewald_total(x, q, box, targets=None, field=True, xi=None):
    """Total potential (and field) of a neutral system.

    The total does not depend on xi (section 1), so it is evaluated at a
    small xi_o = 0.45/L3 where the k3 != 0 sum is below 1e-22 and the
    real-space sum runs over roughly 30 z-images with erfc.  Returns
    (phi, E) over the targets.
    """
    box = np.asarray(box, dtype=np.float64)
    if xi is None:
        xi = 0.45 / box[2]
    parts = PARTS_ALL if field else (PARTS_ALL & ~PARTS_FIELD)
    r = ewald(x, q, box, xi, rc=6.5 / xi, targets=targets, parts=parts)
    phi = r["phi_R"] + r["phi_Fk"] + r["phi_F0"] + r["phi_self"]
    E = r["E_R"] + r["E_Fk"] + r["E_F0"]
    return phi, E


def image_sum(x, q, L3, J):
    """Symmetric partial image sum of eq. coulomb over |j| <= J."""
    lib = _load()
    x = _c(x, np.float64).reshape(-1, 3)
    q = _c(q, np.float64).reshape(-1)
    out = np.zeros(x.shape[0], dtype=np.float64)
    rc = lib.se1p_oracle_image_sum(x.shape[0], x.ctypes.data, q.ctypes.data,
                                   float(L3), int(J), out.ctypes.data)
    if rc != 0:
        raise RuntimeError("image_sum failed")
    return out


def ewald3p(x, q, box, xi, rc=None, targets=None):
    """Direct triply periodic Ewald sums at the targets (se3p_oracle.c).

    Returns a dict of arrays over the targets:
      phi_R, phi_F, phi_self  (ntarget,)
      E_R, E_F                (ntarget, 3)
    ``rc`` defaults to 6.5/xi, where erfc(xi rc) < 4e-20.
    """
    lib = _load()
    x = _c(x, np.float64).reshape(-1, 3)
    q = _c(q, np.float64).reshape(-1)
    box = _c(box, np.float64).reshape(3)
    N = x.shape[0]
    if q.shape[0] != N:
        raise ValueError("x and q sizes differ")
    if rc is None:
        rc = 6.5 / xi
    if targets is None:
        tg = None
        nt = N
    else:
        tg = _c(targets, np.int64).reshape(-1)
        nt = tg.shape[0]
    out = np.zeros((nt, 9), dtype=np.float64)
    rcode = lib.se3p_oracle_ewald(
        N, x.ctypes.data, q.ctypes.data, box.ctypes.data, float(xi),
        float(rc), nt, None if tg is None else tg.ctypes.data, out.ctypes.data)
    if rcode != 0:
        raise RuntimeError(f"oracle error {rcode}")
    return {
        "phi_R": out[:, 0].copy(), "phi_F": out[:, 1].copy(),
        "phi_self": out[:, 2].copy(),
        "E_R": out[:, 3:6].copy(), "E_F": out[:, 6:9].copy(),
    }


def ewald3p_total(x, q, box, xi, rc=None, targets=None):
    """Total triply periodic potential and field at the targets."""
    r = ewald3p(x, q, box, xi, rc=rc, targets=targets)
    return r["phi_R"] + r["phi_F"] + r["phi_self"], r["E_R"] + r["E_F"]
