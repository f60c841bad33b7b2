"""Binning (the cell lists of section 2.2 that gridding, gathering and the
real-space sum run on) against a stable sort on the host: bit-exact.

The reference is numpy: each particle's cell from floor(x / h) in the plan's
precision (z wrapped into [0, L3), indices clamped to the grid), the lex key
(cz, cx, cy) and the block key of the documented serpentine block order, and
a stable argsort of each key (equal keys keep input order).  The cell starts
are the first sorted position of each cell.  No HIP code is involved in the
reference.
"""
import numpy as np
import pytest

from paper_1611_09538_amd import workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _say(*a):
    print(*a, flush=True)


def _keys(x, box, info, dtype):
    """Lex and block cell keys of every particle, in the plan's precision."""
    h = dtype(box[2] / info["M3"])
    L3 = dtype(box[2])
    M1, M2 = info["M"]
    M3 = info["M3"]
    xs = x.astype(dtype)
    z = xs[:, 2]
    zw = (z - L3 * np.floor(z / L3)).astype(dtype)
    zw = np.where(zw < L3, zw, dtype(0))
    zw = np.where(zw < 0, dtype(0), zw)
    cx = np.clip(np.floor(xs[:, 0] / h).astype(np.int64), 0, M1 - 1)
    cy = np.clip(np.floor(xs[:, 1] / h).astype(np.int64), 0, M2 - 1)
    cz = np.clip(np.floor(zw / h).astype(np.int64), 0, M3 - 1)
    kl = (cz * M1 + cx) * M2 + cy
    BX, BY, BZ = info["gather_block"]
    nbx, nby, nbz = -(-M1 // BX), -(-M2 // BY), -(-M3 // BZ)
    bz, iz = cz // BZ, cz % BZ
    bx, ix = cx // BX, cx % BX
    by, iy = cy // BY, cy % BY
    # blocks along a serpentine path: x reversed on odd z layers, y on odd rows
    bxs = np.where(bz & 1, nbx - 1 - bx, bx)
    row = bz * nbx + bxs
    bys = np.where(row & 1, nby - 1 - by, by)
    b = row * nby + bys
    # cells z-major inside a block, z reversed in odd blocks
    izs = np.where(b & 1, BZ - 1 - iz, iz)
    cpb = BX * BY * BZ
    kb = b * cpb + (izs * BX + ix) * BY + iy
    ncl = M1 * M2 * M3
    ncb = nbx * nby * nbz * cpb
    return kl, kb, ncl, ncb


def _reference(keys, ncell):
    perm = np.argsort(keys, kind="stable")
    start = np.searchsorted(keys[perm], np.arange(ncell + 1), side="left")
    return perm, start


def _case_positions(kind, box, h, rng, n):
    if kind == "uniform":
        return workloads.uniform_positions(rng, n, box)
    if kind == "edges":
        # cell boundaries, the box faces, z outside [0, L3), one crowded cell
        x = workloads.uniform_positions(rng, n, box)
        k = n // 4
        x[:k, 0] = rng.integers(0, int(box[0] / h), k) * h
        x[:k, 1] = rng.integers(0, int(box[1] / h), k) * h
        x[k:2 * k, 2] = rng.integers(-3, 4, k) * box[2] + x[k:2 * k, 2]
        x[2 * k:2 * k + 5, 0] = np.nextafter(box[0], 0.0)
        x[2 * k + 5:2 * k + 10, 2] = np.nextafter(box[2], 0.0)
        x[3 * k:, :] = (np.array([3.5, 2.5, 7.5]) * h
                        + rng.random((n - 3 * k, 3)) * 0.5 * h)
        return x
    raise ValueError(kind)


CASES = [
    # (case, n, precision, positions)
    ("small", 1, "fp64", "uniform"),
    ("small", 500, "fp64", "uniform"),
    ("small", 777, "fp32", "edges"),
    ("fp64_1e5", 100_000, "fp64", "uniform"),
    ("fp64_1e5", 4099, "fp64", "edges"),
    ("fp32_1e6", 1_000_000, "fp32", "uniform"),
]


@pytest.mark.parametrize("case,n,prec,kind", CASES)
def test_bin_orders_match_stable_sort(case, n, prec, kind):
    from paper_1611_09538_amd import se1p
    dev = _dev()
    c = dict(workloads.CASES[case])
    precision = se1p.FP64 if prec == "fp64" else se1p.FP32
    dtype = np.float64 if prec == "fp64" else np.float32
    box = np.asarray(c["box"], dtype=np.float64)
    h = box[2] / c["M3"]
    rng = np.random.default_rng(11 + n)
    x = _case_positions(kind, box, h, rng, n)
    q = rng.uniform(-1.0, 1.0, n)
    _say(f"binning {case} n={n} {prec} {kind}")
    prm = se1p.make_params(c["box"], c["xi"], c["M3"], c["P"], c["nl"], c["sl"],
                           rc=c["rc"], pad_free=c["pad_free"], precision=precision)
    plan = se1p.Plan(prm, n_max=n)
    tdt = torch.float64 if prec == "fp64" else torch.float32
    xt = torch.tensor(x, dtype=tdt, device=dev)
    qt = torch.tensor(q, dtype=tdt, device=dev)
    got = [t.cpu().numpy() for t in plan.bin(xt, qt)]
    # twice: the counts are cleared and the order does not depend on the run
    again = [t.cpu().numpy() for t in plan.bin(xt, qt)]
    torch.cuda.synchronize()
    kl, kb, ncl, ncb = _keys(x, box, plan.info, dtype)
    assert tuple(plan.info["bin_cells"]) == (ncl, ncb)
    lp, ls = _reference(kl, ncl)
    bp, bs = _reference(kb, ncb)
    for name, g, r in (("lex_perm", got[0], lp), ("lex_start", got[1], ls),
                       ("blk_perm", got[2], bp), ("blk_start", got[3], bs)):
        assert g.shape == r.shape, name
        bad = np.flatnonzero(g != r)
        assert bad.size == 0, f"{name}: {bad.size} differ, first at {bad[:5]}"
    for g, a in zip(got, again):
        assert np.array_equal(g, a)
    plan.close()
