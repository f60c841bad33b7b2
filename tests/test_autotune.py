"""Host-only checks of the autotuner and of the batch ABI's argument
checks (no GPU needed)."""
import ctypes
import math

import pytest

from paper_1611_09538_amd import se1p


def _lib():
    try:
        return se1p._lib()
    except ImportError:
        pytest.skip("HIP library not built")


def _fft_friendly(n):
    for f in (2, 3, 5):
        while n % f == 0:
            n //= f
    return n == 1


BOXES = [(1.0, 1.0, 0.7), (1.0, 1.0, 1.5), (1.0, 1.0, 1.0)]
COUNTS = [3000, 20000, 50000]


def test_autotune_meets_recipe():
    _lib()
    ps = se1p.autotune(1e-5, BOXES, COUNTS, precision=se1p.FP32, P=12)
    for p, box, n in zip(ps, BOXES, COUNTS):
        assert p.P == 12 and p.precision == se1p.FP32
        assert p.M3 % 2 == 0 and p.M3 >= 12 and _fft_friendly(p.M3)
        # xi, rc, s_l, n_l are the recipe's at the chosen M3
        q = se1p.suggest_params(1e-5, box, n, float(n), M3=p.M3, P=12, precision=se1p.FP32)
        assert p.xi == pytest.approx(q.xi, rel=1e-12)
        assert p.rc == pytest.approx(q.rc, rel=1e-12)
        assert p.s_l == pytest.approx(q.s_l, rel=1e-12) and p.n_l == q.n_l


def _model(pair, grid, fft):
    m = se1p.CostModel()
    m.pair_ns, m.grid_ns, m.fft_ns, m.particle_ns, m.system_ns = pair, grid, fft, 0.5, 1000.0
    return m


def test_autotune_follows_the_cost_model():
    # dear pairs push the grid finer (larger xi, shorter rc); a dear FFT
    # pushes it coarser
    _lib()
    base = _model(0.01, 0.001, 0.004)
    pairs = _model(1.0, 0.001, 0.004)
    fft = _model(0.01, 0.001, 10.0)
    for box, n in zip(BOXES, COUNTS):
        m0 = se1p.autotune(1e-5, [box], [n], P=12, model=base)[0].M3
        m1 = se1p.autotune(1e-5, [box], [n], P=12, model=pairs)[0].M3
        m2 = se1p.autotune(1e-5, [box], [n], P=12, model=fft)[0].M3
        assert m1 >= m0 >= m2, (m1, m0, m2)
        assert m1 > m2


def test_autotune_rejects_bad_arguments():
    lib = _lib()
    out = (se1p.Params * 1)()
    box = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    n = (ctypes.c_longlong * 1)(100)
    assert lib.se1p_autotune(1e-5, 0, box, n, None, 1, 12, None, out) == se1p.ERR_ARG
    assert lib.se1p_autotune(1e-5, 1, box, n, None, 1, 13, None, out) == se1p.ERR_ARG
    assert lib.se1p_autotune(0.0, 1, box, n, None, 1, 12, None, out) == se1p.ERR_ARG
    n0 = (ctypes.c_longlong * 1)(0)
    assert lib.se1p_autotune(1e-5, 1, box, n0, None, 1, 12, None, out) == se1p.ERR_ARG


def test_batch_create_checks_arguments_before_the_device():
    lib = _lib()
    h = ctypes.c_void_p()
    p = se1p.make_params((1, 1, 1), 10.0, 16, 8, 2, 2.0, rc=0.3, precision=se1p.FP32)
    q = se1p.make_params((1, 1, 1), 10.0, 16, 10, 2, 2.0, rc=0.3, precision=se1p.FP32)
    arr = (se1p.Params * 2)(p, q)
    cnt = (ctypes.c_longlong * 2)(100, 100)
    # mixed support P in one batch
    assert lib.se1p_batch_create(2, arr, cnt, None, ctypes.byref(h)) == se1p.ERR_PARAM
    bad = (ctypes.c_longlong * 2)(100, 0)
    arr2 = (se1p.Params * 2)(p, p)
    assert lib.se1p_batch_create(2, arr2, bad, None, ctypes.byref(h)) == se1p.ERR_ARG
    assert lib.se1p_batch_create(0, arr2, cnt, None, ctypes.byref(h)) == se1p.ERR_ARG
    r = se1p.make_params((1, 1, 1), 10.0, 15, 8, 2, 2.0, rc=0.3)   # odd M3
    arr3 = (se1p.Params * 1)(r)
    assert lib.se1p_batch_create(1, arr3, cnt, None, ctypes.byref(h)) == se1p.ERR_PARAM
    assert lib.se1p_batch_eval(None, None, None, None, None, None, 7) == se1p.ERR_ARG
    assert lib.se1p_batch_destroy(None) == se1p.ERR_ARG
