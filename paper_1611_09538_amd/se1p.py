"""Thin Python binding of the SE1P C ABI (include/se1p.h).

Argument marshalling only: every step of the computation runs in the HIP
library ``libse1p.so`` built next to this file.  PyTorch supplies device
memory and the current HIP stream.  There is no CPU fallback: if the library
is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
# SE1P_LIB may name another build of the same library (profiling variants)
LIB_PATH = os.environ.get("SE1P_LIB") or os.path.join(_HERE, "libse1p.so")

# error codes / flags (include/se1p.h)
OK = 0
ERR_ARG = -1
ERR_PARAM = -2
ERR_NONNEUTRAL = -3
ERR_OUT_OF_BOX = -4
ERR_HIP = -5
ERR_NOMEM = -6
ERR_TOO_MANY = -7
ERR_UNSUPPORTED = -8
ERR_SCRATCH = -9
NOALLOC_SCRATCH_BYTES = 256 << 20

FP64 = 0
FP32 = 1

KSPACE = 1
REAL = 2
SELF = 4
ALL = 7
CHECK_INPUT = 16
NO_NEUTRAL = 32
FIELD_IK = 128
FORCE = 256
BATCH_EAGER = 64


class SE1PError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = _lib().se1p_error_string(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{what}: {msg} (code {code})" if what else f"{msg} (code {code})")


class Params(ctypes.Structure):
    _fields_ = [
        ("box", ctypes.c_double * 3),
        ("xi", ctypes.c_double),
        ("M3", ctypes.c_int),
        ("P", ctypes.c_int),
        ("n_l", ctypes.c_int),
        ("s_l", ctypes.c_double),
        ("s0", ctypes.c_double),
        ("rc", ctypes.c_double),
        ("pad_free", ctypes.c_int),
        ("precision", ctypes.c_int),
    ]

    def as_dict(self):
        return {"box": tuple(self.box), "xi": self.xi, "M3": self.M3, "P": self.P,
                "n_l": self.n_l, "s_l": self.s_l, "s0": self.s0, "rc": self.rc,
                "pad_free": self.pad_free, "precision": self.precision}


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("h", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("R", ctypes.c_double),
        ("M", ctypes.c_int * 2),
        ("Mt", ctypes.c_int * 2),
        ("M3", ctypes.c_int),
        ("P", ctypes.c_int),
        ("n0", ctypes.c_int * 2),
        ("nl", ctypes.c_int * 2),
        ("n_l", ctypes.c_int),
        ("nslab", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("n_max", ctypes.c_longlong),
        ("workspace_bytes", ctypes.c_size_t),
        ("gather_block", ctypes.c_int * 3),
        ("gather_chunks", ctypes.c_int),
        ("spread_cz", ctypes.c_int),
        ("spread_kp", ctypes.c_int),
        ("bin_cells", ctypes.c_longlong * 2),
        ("gather_pair", ctypes.c_int),
    ]

    def as_dict(self):
        return {"h": self.h, "eta": self.eta, "R": self.R, "M": tuple(self.M),
                "Mt": tuple(self.Mt), "M3": self.M3, "P": self.P,
                "n0": tuple(self.n0), "nl": tuple(self.nl), "n_l": self.n_l,
                "nslab": self.nslab, "precision": self.precision,
                "n_max": self.n_max, "workspace_bytes": self.workspace_bytes,
                "gather_block": tuple(self.gather_block),
                "gather_chunks": self.gather_chunks, "spread_cz": self.spread_cz,
                "spread_kp": self.spread_kp, "bin_cells": tuple(self.bin_cells),
                "gather_pair": self.gather_pair}


class CostModel(ctypes.Structure):
    _fields_ = [
        ("pair_ns", ctypes.c_double),
        ("grid_ns", ctypes.c_double),
        ("fft_ns", ctypes.c_double),
        ("particle_ns", ctypes.c_double),
        ("system_ns", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("nsys", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("P", ctypes.c_int),
        ("n_total", ctypes.c_longlong),
        ("workspace_bytes", ctypes.c_size_t),
        ("items", ctypes.c_int * 10),
        ("grid", ctypes.c_int * 10),
        ("graph_captures", ctypes.c_int),
    ]


QUEUES = ["spread", "zfft", "rowfwd", "cols", "rowinv", "zifft", "gather",
          "realspace", "combine"]

# every symbol include/se1p.h declares
EXPORTS = [
    "se1p_suggest_params", "se1p_plan_create", "se1p_plan_destroy",
    "se1p_plan_get_info", "se1p_set_stream", "se1p_eval", "se1p_eval_noalloc",
    "se1p_bin", "se1p_spread",
    "se1p_kspace_solve", "se1p_gather", "se1p_error_string", "se1p_version",
    "se1p_timing_enable", "se1p_timing_select", "se1p_timing_read", "se1p_calibrate",
    "se1p_autotune", "se1p_batch_create", "se1p_batch_destroy",
    "se1p_batch_eval", "se1p_batch_get_info", "se1p_batch_system_info",
    "se3p_plan_create",
]

NSTAGE = 6
STAGES = ["bin", "spread", "kspace", "gather", "realspace", "combine"]

_LIB = None


def _lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"SE1P HIP library not built: {LIB_PATH} is missing "
            "(run __graft_entry__.build() or python paper_1611_09538_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ll, i, d, u = ctypes.c_void_p, ctypes.c_longlong, ctypes.c_int, ctypes.c_double, ctypes.c_uint
    lib.se1p_error_string.restype = ctypes.c_char_p
    lib.se1p_error_string.argtypes = [i]
    lib.se1p_version.restype = ctypes.c_char_p
    lib.se1p_version.argtypes = []
    lib.se1p_suggest_params.restype = i
    lib.se1p_suggest_params.argtypes = [d, ctypes.POINTER(d), ll, d, d, i, i, i, i,
                                        ctypes.POINTER(Params)]
    lib.se1p_plan_create.restype = i
    lib.se1p_plan_create.argtypes = [ctypes.POINTER(Params), ll, vp, ctypes.POINTER(vp)]
    lib.se3p_plan_create.restype = i
    lib.se3p_plan_create.argtypes = [ctypes.POINTER(Params), ll, vp, ctypes.POINTER(vp)]
    lib.se1p_plan_destroy.restype = i
    lib.se1p_plan_destroy.argtypes = [vp]
    lib.se1p_plan_get_info.restype = i
    lib.se1p_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.se1p_set_stream.restype = i
    lib.se1p_set_stream.argtypes = [vp, vp]
    lib.se1p_eval.restype = i
    lib.se1p_eval.argtypes = [vp, ll, vp, vp, vp, vp, vp, u]
    lib.se1p_eval_noalloc.restype = i
    lib.se1p_eval_noalloc.argtypes = [vp, ll, vp, vp, vp, vp, vp, u]
    lib.se1p_bin.restype = i
    lib.se1p_bin.argtypes = [vp, ll, vp, vp, vp, vp, vp, vp]
    lib.se1p_spread.restype = i
    lib.se1p_spread.argtypes = [vp, ll, vp, vp, vp]
    lib.se1p_kspace_solve.restype = i
    lib.se1p_kspace_solve.argtypes = [vp, vp, vp]
    lib.se1p_gather.restype = i
    lib.se1p_gather.argtypes = [vp, ll, vp, vp, vp, vp]
    lib.se1p_timing_enable.restype = i
    lib.se1p_timing_enable.argtypes = [vp, i]
    lib.se1p_timing_select.restype = i
    lib.se1p_timing_select.argtypes = [vp, ctypes.c_uint]
    lib.se1p_timing_read.restype = i
    lib.se1p_timing_read.argtypes = [vp, ctypes.POINTER(d), ctypes.POINTER(i)]
    lib.se1p_calibrate.restype = i
    lib.se1p_calibrate.argtypes = [d, i, i, vp, ctypes.POINTER(CostModel)]
    lib.se1p_autotune.restype = i
    lib.se1p_autotune.argtypes = [d, i, ctypes.POINTER(d), ctypes.POINTER(ll),
                                  ctypes.POINTER(d), i, i, ctypes.POINTER(CostModel),
                                  ctypes.POINTER(Params)]
    lib.se1p_batch_create.restype = i
    lib.se1p_batch_create.argtypes = [i, ctypes.POINTER(Params), ctypes.POINTER(ll), vp,
                                      ctypes.POINTER(vp)]
    lib.se1p_batch_destroy.restype = i
    lib.se1p_batch_destroy.argtypes = [vp]
    lib.se1p_batch_eval.restype = i
    lib.se1p_batch_eval.argtypes = [vp, vp, vp, vp, vp, vp, u]
    lib.se1p_batch_get_info.restype = i
    lib.se1p_batch_get_info.argtypes = [vp, ctypes.POINTER(BatchInfo)]
    lib.se1p_batch_system_info.restype = i
    lib.se1p_batch_system_info.argtypes = [vp, i, ctypes.POINTER(Params),
                                           ctypes.POINTER(PlanInfo)]
    _LIB = lib
    return lib


def version() -> str:
    return _lib().se1p_version().decode()


def _check(code: int, what: str):
    if code != OK:
        raise SE1PError(code, what)


def suggest_params(tol, box, N, Q, xi=0.0, M3=0, P=0, n_l=-1, precision=FP64) -> Params:
    """Parameter selection of section 4.3 (host only, no GPU needed)."""
    out = Params()
    b = (ctypes.c_double * 3)(*[float(v) for v in box])
    _check(_lib().se1p_suggest_params(float(tol), b, int(N), float(Q), float(xi),
                                      int(M3), int(P), int(n_l), int(precision),
                                      ctypes.byref(out)), "se1p_suggest_params")
    return out


def make_params(box, xi, M3, P, n_l, s_l, s0=0.0, rc=0.0, precision=FP64,
                pad_free=0) -> Params:
    p = Params()
    for k in range(3):
        p.box[k] = float(box[k])
    p.xi = float(xi)
    p.M3 = int(M3)
    p.P = int(P)
    p.n_l = int(n_l)
    p.s_l = float(s_l)
    p.s0 = float(s0)
    p.rc = float(rc)
    p.pad_free = int(pad_free)
    p.precision = int(precision)
    return p


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Plan:
    """An SE1P plan: geometry, tables and device workspace for up to n_max
    particles.  Calls enqueue on the current torch stream of the plan's
    device unless a stream is given.  periodic=True plans the triply
    periodic comparison method (SE3P, se3p_plan_create)."""

    def __init__(self, params: Params, n_max: int, stream=None, periodic: bool = False):
        torch = _torch()
        self.params = params
        self.periodic = bool(periodic)
        self.dtype = torch.float64 if params.precision == FP64 else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._stream = s
        h = ctypes.c_void_p()
        create = _lib().se3p_plan_create if self.periodic else _lib().se1p_plan_create
        _check(create(ctypes.byref(params), int(n_max), ctypes.c_void_p(s.cuda_stream),
                      ctypes.byref(h)),
               "se3p_plan_create" if self.periodic else "se1p_plan_create")
        self._h = h
        info = PlanInfo()
        _check(_lib().se1p_plan_get_info(self._h, ctypes.byref(info)), "se1p_plan_get_info")
        self.info = info.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib().se1p_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        torch = _torch()
        s = torch.cuda.current_stream(self.device)
        if s.cuda_stream != self._stream.cuda_stream:
            _check(_lib().se1p_set_stream(self._h, ctypes.c_void_p(s.cuda_stream)),
                   "se1p_set_stream")
            self._stream = s

    def _prep(self, x, q=None):
        torch = _torch()
        if x.device.type != "cuda":
            raise ValueError("x must be a device tensor")
        x = x.to(self.dtype).contiguous()
        if x.dim() != 2 or x.shape[1] != 3:
            raise ValueError("x must be N x 3")
        if q is not None:
            q = q.to(device=x.device, dtype=self.dtype).contiguous().reshape(-1)
            if q.shape[0] != x.shape[0]:
                raise ValueError("x and q sizes differ")
        return x, q

    def eval(self, x, q, flags=ALL, want_phi=True, want_field=True,
             want_energy=True):
        """Returns (phi, E, U) as device tensors (None where not requested)."""
        torch = _torch()
        self._sync_stream()
        x, q = self._prep(x, q)
        N = x.shape[0]
        phi = torch.empty(N, dtype=self.dtype, device=x.device) if want_phi else None
        E = torch.empty((N, 3), dtype=self.dtype, device=x.device) if want_field else None
        U = torch.empty(1, dtype=torch.float64, device=x.device) if want_energy else None
        _check(_lib().se1p_eval(self._h, N, _ptr(x), _ptr(q), _ptr(phi), _ptr(E),
                                _ptr(U), int(flags)), "se1p_eval")
        return phi, E, U

    def eval_into(self, x, q, phi, E, U, flags=ALL):
        """Enqueue an evaluation into preallocated outputs (no allocation)."""
        self._sync_stream()
        _check(_lib().se1p_eval(self._h, x.shape[0], _ptr(x), _ptr(q), _ptr(phi),
                                _ptr(E), _ptr(U), int(flags)), "se1p_eval")

    def eval_noalloc_into(self, x, q, phi, E, U, flags=ALL):
        """se1p_eval_noalloc into preallocated outputs: the library's static
        device scratch instead of the plan's (no allocation anywhere)."""
        self._sync_stream()
        _check(_lib().se1p_eval_noalloc(self._h, x.shape[0], _ptr(x), _ptr(q), _ptr(phi),
                                        _ptr(E), _ptr(U), int(flags)), "se1p_eval_noalloc")

    def timing_enable(self, on=True):
        _check(_lib().se1p_timing_enable(self._h, 1 if on else 0), "se1p_timing_enable")

    def timing_select(self, stages=None):
        """Record events only around the named stages (None: every stage)."""
        bits = (1 << NSTAGE) - 1 if stages is None else sum(1 << STAGES.index(s) for s in stages)
        _check(_lib().se1p_timing_select(self._h, bits), "se1p_timing_select")

    def timing_read(self):
        """(dict stage -> summed ms, number of calls); synchronises."""
        arr = (ctypes.c_double * NSTAGE)()
        n = ctypes.c_int()
        _check(_lib().se1p_timing_read(self._h, arr, ctypes.byref(n)), "se1p_timing_read")
        return {STAGES[k]: arr[k] for k in range(NSTAGE)}, n.value

    def grid_shape(self):
        i = self.info
        return (i["M3"], i["Mt"][0], i["Mt"][1])

    def bin(self, x, q):
        """Binning stage: (lex_perm, lex_start, blk_perm, blk_start) as
        int32 device tensors (se1p_bin)."""
        torch = _torch()
        self._sync_stream()
        x, q = self._prep(x, q)
        N = x.shape[0]
        nl, nb = self.info["bin_cells"]
        kw = dict(dtype=torch.int32, device=x.device)
        out = (torch.empty(N, **kw), torch.empty(nl + 1, **kw),
               torch.empty(N, **kw), torch.empty(nb + 1, **kw))
        _check(_lib().se1p_bin(self._h, N, _ptr(x), _ptr(q), *[_ptr(t) for t in out]),
               "se1p_bin")
        return out

    def spread(self, x, q):
        torch = _torch()
        self._sync_stream()
        x, q = self._prep(x, q)
        g = torch.empty(self.grid_shape(), dtype=self.dtype, device=x.device)
        _check(_lib().se1p_spread(self._h, x.shape[0], _ptr(x), _ptr(q), _ptr(g)),
               "se1p_spread")
        return g

    def kspace_solve(self, grid):
        torch = _torch()
        self._sync_stream()
        grid = grid.to(self.dtype).contiguous()
        out = torch.empty_like(grid)
        _check(_lib().se1p_kspace_solve(self._h, _ptr(grid), _ptr(out)),
               "se1p_kspace_solve")
        return out

    def gather(self, x, grid, want_field=True):
        torch = _torch()
        self._sync_stream()
        x, _ = self._prep(x)
        grid = grid.to(self.dtype).contiguous()
        N = x.shape[0]
        phi = torch.empty(N, dtype=self.dtype, device=x.device)
        E = torch.empty((N, 3), dtype=self.dtype, device=x.device) if want_field else None
        _check(_lib().se1p_gather(self._h, N, _ptr(x), _ptr(grid), _ptr(phi), _ptr(E)),
               "se1p_gather")
        return phi, E


def autotune(tol, boxes, counts, Q=None, precision=FP32, P=12, model=None):
    """Per-system parameters with the least predicted cost at tolerance tol
    (host only).  boxes: (nsys, 3); counts: nsys; Q: nsys sums of q^2 or
    None for unit charges; model: CostModel or None for the built-in one."""
    n = len(counts)
    bx = (ctypes.c_double * (3 * n))(*[float(v) for b in boxes for v in b])
    ct = (ctypes.c_longlong * n)(*[int(c) for c in counts])
    qq = None if Q is None else (ctypes.c_double * n)(*[float(v) for v in Q])
    out = (Params * n)()
    _check(_lib().se1p_autotune(float(tol), n, bx, ct, qq, int(precision), int(P),
                                None if model is None else ctypes.byref(model), out),
           "se1p_autotune")
    return [out[k] for k in range(n)]


def calibrate(tol, precision=FP32, P=12, stream=None) -> CostModel:
    """Cost model measured on the current device (synchronises)."""
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    m = CostModel()
    _check(_lib().se1p_calibrate(float(tol), int(precision), int(P),
                                 ctypes.c_void_p(s.cuda_stream), ctypes.byref(m)),
           "se1p_calibrate")
    return m


class Batch:
    """Many independent systems evaluated together (one launch per stage,
    persistent work queues, replayed as one HIP graph)."""

    def __init__(self, params, counts, stream=None):
        torch = _torch()
        n = len(params)
        if n != len(counts) or n == 0:
            raise ValueError("params and counts must be non-empty and of equal length")
        self.params = list(params)
        self.counts = [int(c) for c in counts]
        self.offsets = [0]
        for c in self.counts:
            self.offsets.append(self.offsets[-1] + c)
        self.dtype = torch.float64 if params[0].precision == FP64 else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._stream = s
        arr = (Params * n)(*self.params)
        ct = (ctypes.c_longlong * n)(*self.counts)
        h = ctypes.c_void_p()
        _check(_lib().se1p_batch_create(n, arr, ct, ctypes.c_void_p(s.cuda_stream),
                                        ctypes.byref(h)), "se1p_batch_create")
        self._h = h

    @property
    def n_total(self):
        return self.offsets[-1]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib().se1p_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        bi = BatchInfo()
        _check(_lib().se1p_batch_get_info(self._h, ctypes.byref(bi)), "se1p_batch_get_info")
        return {"nsys": bi.nsys, "precision": bi.precision, "P": bi.P,
                "n_total": bi.n_total, "workspace_bytes": bi.workspace_bytes,
                "items": {QUEUES[k]: bi.items[k] for k in range(len(QUEUES))},
                "grid": {QUEUES[k]: bi.grid[k] for k in range(len(QUEUES))},
                "graph_captures": bi.graph_captures}

    def system_info(self, s):
        p = Params()
        pi = PlanInfo()
        _check(_lib().se1p_batch_system_info(self._h, int(s), ctypes.byref(p),
                                             ctypes.byref(pi)), "se1p_batch_system_info")
        return p, pi.as_dict()

    def eval_into(self, x, q, phi, E, U, flags=ALL, eager=False):
        """Enqueue on the batch's stream into preallocated packed outputs."""
        torch = _torch()
        if torch.cuda.current_stream(self.device).cuda_stream != self._stream.cuda_stream:
            raise RuntimeError("Batch calls must run on the stream it was created with")
        if x.shape[0] != self.n_total or q.shape[0] != self.n_total:
            raise ValueError("x and q must hold the packed particles of every system")
        f = int(flags) | (BATCH_EAGER if eager else 0)
        _check(_lib().se1p_batch_eval(self._h, _ptr(x), _ptr(q), _ptr(phi), _ptr(E),
                                      _ptr(U), f), "se1p_batch_eval")

    def eval(self, x, q, flags=ALL, eager=False):
        """Returns packed (phi, E) and the per-system energies."""
        torch = _torch()
        x = x.to(self.dtype).contiguous()
        q = q.to(device=x.device, dtype=self.dtype).contiguous().reshape(-1)
        N = self.n_total
        phi = torch.empty(N, dtype=self.dtype, device=x.device)
        E = torch.empty((N, 3), dtype=self.dtype, device=x.device)
        U = torch.empty(len(self.counts), dtype=torch.float64, device=x.device)
        self.eval_into(x, q, phi, E, U, flags, eager)
        return phi, E, U
