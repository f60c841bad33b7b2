"""Host-only checks of the C ABI library: it loads without a GPU, exports
every symbol include/se1p.h declares, and its host logic (parameter
selection, argument checks) behaves."""
import ctypes
import math
import os
import re

import pytest

from paper_1611_09538_amd import se1p

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "se1p.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(se[13]p_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(se1p.LIB_PATH)
    decl = _declared()
    assert len(decl) >= 10
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(se1p.EXPORTS) == decl


def test_version_and_error_strings():
    assert "gfx950" in se1p.version()
    lib = se1p._lib()
    for code in range(0, -9, -1):
        s = lib.se1p_error_string(code).decode()
        assert s and s != "unknown error"
    assert lib.se1p_error_string(-99).decode() == "unknown error"


def test_suggest_params_follows_recipe():
    # cube, tolerance 1e-8 with M3 fixed: xi from the Fourier estimate,
    # P from the approximation estimate, s_l from
    # exp(-2 pi (s_l - 1) Lt / L3) < tol
    p = se1p.suggest_params(1e-8, (1.0, 1.0, 1.0), 100000, 100000 / 3.0, M3=64)
    assert p.M3 == 64
    kinf = 32.0
    Q = 100000 / 3.0
    errF = p.xi / math.pi ** 2 * kinf ** -1.5 * math.sqrt(Q) * math.exp(-(math.pi * kinf / p.xi) ** 2)
    assert errF == pytest.approx(1e-8, rel=1e-6)
    assert p.P % 2 == 0 and 4 <= p.P <= 32
    A = math.sqrt(Q * p.xi) / 1.0
    assert A * math.exp(-0.95 ** 2 * math.pi * p.P / 2) < 1e-8
    h = 1.0 / 64
    Lt = 1.0 + p.P * h
    assert math.exp(-2 * math.pi * (p.s_l - 1) * Lt) == pytest.approx(1e-8, rel=1e-9)
    assert p.n_l == round(64 / 10)
    assert p.s0 == pytest.approx(1 + math.sqrt(2))
    # real-space estimate (eq. trunc_error_estimate_real) at the chosen rc
    errR = math.sqrt(Q * p.rc / 2) * (p.xi * p.rc) ** -2 * math.exp(-(p.xi * p.rc) ** 2)
    assert errR == pytest.approx(1e-8, rel=1e-6)


def test_suggest_params_from_xi_picks_grid():
    p = se1p.suggest_params(1e-6, (1.0, 1.0, 1.0), 1000, 1000.0, xi=10.0)
    assert p.M3 % 2 == 0 and p.M3 >= 8
    r = p.M3
    for f in (2, 3, 5):
        while r % f == 0:
            r //= f
    assert r == 1          # a size the radix-2/3/4/5 transforms take
    kinf = p.M3 / 2
    errF = 10.0 / math.pi ** 2 * kinf ** -1.5 * math.sqrt(1000.0) * math.exp(-(math.pi * kinf / 10.0) ** 2)
    assert errF <= 1e-6


@pytest.mark.parametrize("field,val", [("M3", 7), ("P", 5), ("P", 34), ("P", 2),
                                       ("xi", -1.0), ("s_l", 0.5), ("precision", 3),
                                       ("pad_free", -1)])
def test_plan_create_rejects_bad_params_before_touching_gpu(field, val):
    p = se1p.make_params((1, 1, 1), 10.0, 32, 16, 4, 3.0, rc=0.3)
    setattr(p, field, val)
    h = ctypes.c_void_p()
    rc = se1p._lib().se1p_plan_create(ctypes.byref(p), 100, None, ctypes.byref(h))
    assert rc == se1p.ERR_PARAM
    assert not h.value


def test_plan_create_rejects_bad_sizes():
    p = se1p.make_params((1, 1, 1), 10.0, 32, 16, 4, 3.0, rc=0.3)
    h = ctypes.c_void_p()
    assert se1p._lib().se1p_plan_create(ctypes.byref(p), 0, None, ctypes.byref(h)) == se1p.ERR_ARG
    assert se1p._lib().se1p_plan_create(None, 10, None, ctypes.byref(h)) == se1p.ERR_ARG


def test_eval_rejects_null_plan():
    assert se1p._lib().se1p_eval(None, 10, None, None, None, None, None, 7) == se1p.ERR_ARG


def test_flag_values_match_the_header():
    # the binding's flag constants are the header's #defines
    txt = open(os.path.join(ROOT, "include", "se1p.h")).read()
    defs = dict(re.findall(r"#define SE1P_([A-Z_0-9]+)\s+(\d+)u", txt))
    for name in ("KSPACE", "REAL", "SELF", "ALL", "CHECK_INPUT", "NO_NEUTRAL",
                 "FIELD_IK", "FORCE", "BATCH_EAGER"):
        assert int(defs[name]) == getattr(se1p, name), name
    # component and option bits do not overlap
    opts = [se1p.CHECK_INPUT, se1p.NO_NEUTRAL, se1p.FIELD_IK, se1p.FORCE, se1p.BATCH_EAGER]
    for o in opts:
        assert o & se1p.ALL == 0 and bin(o).count("1") == 1
    assert len(set(opts)) == len(opts)
