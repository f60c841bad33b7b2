"""Benchmark: SE1P potential + field throughput on one MI355X.

One step = one full SE1P evaluation (binning, gridding, adaptive FFT with
scaling, inverse transform, gathering of phi and E, real-space sum, self
term, FP64 energy) of the N = 1e5 FP64 system in a unit box periodic in z
(M3 = 64, P = 24, n_l = 4, rel-RMS 1e-8), inputs already resident in device
memory.  Prints one JSON line.

Extra fields:
  stages_ms       per-stage times from HIP events on the plan's stream, from
                  a run of their own after the timed region (the timed region
                  records events only around the real-space sum: every event
                  between two kernels costs time of its own)
  roofline        the dominant kernel (the real-space sum): algorithmic flops
                  (exact in-range pair count x flops per pair) over its
                  event-timed duration, against the MI355X vector peak;
                  traffic from the committed FETCH_SIZE / WRITE_SIZE counter
                  summary when it was taken on the current kernel source
  kernels         the gathering kernel against the nominal LDS bandwidth
                  (algorithmic LDS bytes w P^3 per particle) and the vector
                  ALU peak; the gridding stage against the vector FMA peak
                  (it keeps its sums in registers), with its HBM traffic
                  over its algorithmic bytes (particles in, grid out)
  fp32            the N = 1e6 FP32 system (2 x 2 x 1, P = 12, rel-RMS 1e-5):
                  FP32 path and the FP64 path at the same parameters
  adaptive_fft    the transform stage against the plain upsampled transform
                  (every k3 slab upsampled) on the same system
  aft_sweep       the same ratio on the grids of the paper's FFT ratio table
                  (M = 16 .. 128, s_l = 2 and 4, n_l = 8), beside its values
  se3p_comparison k-space time of SE1P against the triply periodic SE3P on
                  the paper's density-125, xi = 4 timing systems (N = 1e5) at
                  its 1e-5 and 1e-9 parameters, and per particle over its
                  N = 2e4 .. 1e5 sweep at 1e-5
  ik_field        the field by ik-differentiation (SE1P_FIELD_IK) on the
                  headline system: time and accuracy on the oracle sample
  total_runtime   total time (real space included) over the paper's
                  density-100 total-runtime systems, N = 21600 .. 274400
  batched         64 systems (N log-uniform in [1e3, 5e4]) in one graph
                  launch, FP32 at 1e-5, against one plan per system (FP32 and
                  FP64) at the same parameters
  cpu_baseline    the oracle on the host cores on a bounded target sample
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SE1P potential+force particles/s at rel-RMS 1e-8 (FP64) and 1e-5 (FP32)"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}   # MI355X vector, dense
HBM_PEAK_GBS = 8000.0
# LDS: 256 CUs x 128 bytes per clock x 2.4 GHz (nominal)
LDS_PEAK_TBS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1611_09538_amd", "csrc", "se1p_kernels.hip")

# Flops per in-range pair of the real-space sum (phi and E) as the kernel
# formulates it, counting each add and multiply (an FMA as two) and rsqrt /
# exp / reciprocal as one each:
#   FP64: distance and r^2 8, rsqrt and r 2, exponent and exp 3,
#         reciprocal with two Newton steps 9, Chebyshev variable 2,
#         degree-12 Horner 24, erfc / r 2, phi update 2, radial factor 5,
#         field update 6                                          = 63
#   FP32: the same with one reciprocal and a degree-8 Horner      = 47
PAIR_FLOPS = {"f64": 63.0, "f32": 47.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--case", default="fp64_1e5")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the adaptive-transform, FP32 and batched measurements")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 512 MiB device copy (counter calibration)")
    ap.add_argument("--leg", choices=["batched"], default=None,
                    help="run only this extra measurement and print its JSON "
                         "(for profiling one workload)")
    return ap.parse_args()


def gather_flops(N, P):
    # per particle and support point: phi and the x, y, z gradient sums,
    # 4 FMA with the row sums shared (2 flops each)
    return 4.0 * N * P ** 3


def spread_flops(N, P):
    return 2.0 * N * P ** 3


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def pair_count(x, box, rc):
    """Ordered pairs (i != j) closer than rc, periodic images along z only."""
    import numpy as np
    from scipy.spatial import cKDTree
    L3 = box[2]
    img = [x]
    k = 1
    while (k - 1) * L3 < rc:
        for s in (k, -k):
            y = x.copy()
            y[:, 2] += s * L3
            img.append(y)
        k += 1
    a = cKDTree(x)
    b = cKDTree(np.concatenate(img))
    return int(a.count_neighbors(b, rc)) - x.shape[0]


def src_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(kernel, case):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(case, {}).get(kernel)
    if not e or t.get("kernel_source_sha256_16") != src_hash():
        return None
    return e["bytes_per_launch"]


def timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def timed_and_staged(plan, fn, steps, warmup, torch):
    """Seconds per call with no events recorded, then the per-stage times in
    ms from a second run with events around every stage (each event between
    two kernels costs time of its own, so the two are not taken together)."""
    t = timed(fn, steps, warmup, torch)
    plan.timing_select(None)
    plan.timing_enable(True)
    timed(fn, steps, 0, torch)
    st, nc = plan.timing_read()
    plan.timing_enable(False)
    return t, {k: v / max(nc, 1) for k, v in st.items()}


def plan_for(se1p, c, box, n, precision):
    prm = se1p.make_params(box, c["xi"], c["M3"], c["P"], c["nl"], c["sl"],
                           rc=c["rc"], pad_free=c["pad_free"], precision=precision)
    return se1p.Plan(prm, n_max=n)


def fp32_extra(se1p, workloads, torch, dev, steps, warmup):
    import numpy as np
    x, q, box, c = workloads.make_case("fp32_1e6")
    N = x.shape[0]
    out = {"workload": f"fp32_1e6: N={N}, box {tuple(box)}, M3={c['M3']}, P={c['P']}, "
                       f"xi={c['xi']}, n_l={c['nl']}, s_l={c['sl']}, rc={c['rc']}"}
    for prec, name in ((se1p.FP32, "f32"), (se1p.FP64, "f64")):
        dt = torch.float32 if prec == se1p.FP32 else torch.float64
        plan = plan_for(se1p, c, box, N, prec)
        xt = torch.tensor(x.astype(np.float32), device=dev).to(dt)
        qt = torch.tensor(q, device=dev, dtype=dt)
        phi = torch.empty(N, device=dev, dtype=dt)
        E = torch.empty((N, 3), device=dev, dtype=dt)
        U = torch.empty(1, device=dev, dtype=torch.float64)
        s, st = timed_and_staged(plan, lambda: plan.eval_into(xt, qt, phi, E, U),
                                 steps, warmup, torch)
        out[name] = {"ms_per_step": s * 1e3, "particles_per_s": N / s, "stages_ms": st}
        plan.close()
        del xt, qt, phi, E, U
    out["speedup_fp32_over_fp64"] = out["f64"]["ms_per_step"] / out["f32"]["ms_per_step"]
    return out


def adaptive_extra(se1p, workloads, torch, dev, steps, warmup, case, kspace_ms, phi_ad):
    """The adaptive transform against the plain upsampled one (every k3 slab
    upsampled by s_l, the k3 = 0 slab as before) on the same system."""
    x, q, box, c = workloads.make_case(case)
    N = x.shape[0]
    prm = se1p.make_params(box, c["xi"], c["M3"], c["P"], c["M3"] // 2, c["sl"],
                           rc=c["rc"], pad_free=c["pad_free"])
    plan = se1p.Plan(prm, n_max=N)
    xt = torch.tensor(x, device=dev)
    qt = torch.tensor(q, device=dev)
    phi = torch.empty(N, device=dev, dtype=torch.float64)
    E = torch.empty((N, 3), device=dev, dtype=torch.float64)
    U = torch.empty(1, device=dev, dtype=torch.float64)
    plan.timing_enable(True)
    timed(lambda: plan.eval_into(xt, qt, phi, E, U), steps, warmup, torch)
    st, nc = plan.timing_read()
    plan.close()
    plain = st["kspace"] / max(nc, 1)
    d = (phi - phi_ad).norm() / phi_ad.norm()
    return {"adaptive_kspace_ms": kspace_ms, "plain_kspace_ms": plain,
            "speedup": plain / kspace_ms, "n_l_plain": c["M3"] // 2,
            "rel_rms_phi_adaptive_vs_plain": float(d.item())}


# The paper's FFT ratio table (plain upsampled over adaptive transform,
# n_l = 8) for M = 16 .. 128 and s_l = 2, 4, as printed there.
AFT_TABLE_M = (16, 32, 48, 64, 80, 96, 112, 128)
AFT_TABLE = {2.0: (0.78, 1.43, 1.77, 2.23, 2.28, 2.51, 2.64, 2.51),
             4.0: (1.23, 2.43, 3.36, 4.65, 5.06, 5.99, 6.85, 6.30)}


def aft_sweep_extra(se1p, workloads, torch, dev, steps, warmup):
    """Transform-stage time (forward transforms, scaling, inverse transforms)
    of the plain upsampled FFT over the adaptive one, on the grids of the
    paper's FFT ratio table: unit box, P = 8, xi = 0.3 M, n_l = 8, s_l = 2
    and 4.  The plain transform upsamples every k3 slab by s_l; both take
    the k3 = 0 slab at s0 = max(s_l, 1 + sqrt 2).  M = 112 becomes 108 (the
    transforms take radices 2, 3, 4, 5).  The stage time does not depend on
    the particles: 2000 charges, k-space only."""
    import numpy as np
    rng = np.random.default_rng(5)
    box = np.array([1.0, 1.0, 1.0])
    n = 2000
    xt = torch.tensor(workloads.uniform_positions(rng, n, box), device=dev)
    qt = torch.tensor(workloads.neutral_uniform(rng, n), device=dev)
    phi = torch.empty(n, device=dev, dtype=torch.float64)
    E = torch.empty((n, 3), device=dev, dtype=torch.float64)
    U = torch.empty(1, device=dev, dtype=torch.float64)
    rows = []
    for s in (2.0, 4.0):
        for k, Mp in enumerate(AFT_TABLE_M):
            M = 108 if Mp == 112 else Mp
            ms = {}
            for name, nl in (("adaptive", min(8, M // 2)), ("plain", M // 2)):
                prm = se1p.make_params(box, 0.3 * M, M, 8, nl, s, s0=s, rc=0.0)
                plan = se1p.Plan(prm, n_max=n)
                plan.timing_select(["kspace"])
                plan.timing_enable(True)
                timed(lambda: plan.eval_into(xt, qt, phi, E, U, flags=se1p.KSPACE),
                      steps, warmup, torch)
                st, nc = plan.timing_read()
                plan.close()
                ms[name] = st["kspace"] / max(nc, 1)
            rows.append({"M": M, "s_l": s, "plain_ms": ms["plain"], "adaptive_ms": ms["adaptive"],
                         "ratio": ms["plain"] / ms["adaptive"], "paper_ratio": AFT_TABLE[s][k]})
    return {"workload": "unit box, P 8, xi 0.3 M, n_l 8, FP64, transform stage only",
            "rows": rows}


def se3p_extra(se1p, workloads, torch, dev, steps, warmup):
    """k-space time of SE1P against the triply periodic SE3P on the paper's
    timing systems (density 125, xi = 4), N = 1e5, FP64: gridding, transforms
    with scaling, and gathering of phi and E, no real-space sum."""
    N = 100_000
    x, q, box = workloads.density125_system(N, seed=5)
    xt = torch.tensor(x, device=dev)
    qt = torch.tensor(q, device=dev)
    phi = torch.empty(N, device=dev, dtype=torch.float64)
    E = torch.empty((N, 3), device=dev, dtype=torch.float64)
    U = torch.empty(1, device=dev, dtype=torch.float64)
    out = {"workload": f"N = {N}, uniform in a cube of side {box[0]:.3f} (density 125), "
                       "charges uniform in [-1, 1] minus the mean, xi = 4, FP64"}
    # the paper's parameter table at tolerances 1e-5 and 1e-9; M = 120 stands
    # for its 114 (a prime factor 19 the radix-2/3/4/5 transforms do not take)
    for tol, M, P, sl, nl in ((1e-5, 96, 12, 2.0, 12), (1e-9, 120, 24, 3.0, 15)):
        r = {"M": M, "P": P, "s_l": sl, "n_l": nl}
        for periodic, name in ((False, "se1p"), (True, "se3p")):
            prm = se1p.make_params(box, 4.0, M, P, nl, sl, rc=0.0, pad_free=8)
            plan = se1p.Plan(prm, n_max=N, periodic=periodic)
            plan.timing_enable(True)
            t = timed(lambda: plan.eval_into(xt, qt, phi, E, U, flags=se1p.KSPACE),
                      steps, warmup, torch)
            st, nc = plan.timing_read()
            plan.close()
            st = {k: v / max(nc, 1) for k, v in st.items()}
            r[name] = {"ms": t * 1e3,
                       "stages_ms": {k: st[k] for k in ("bin", "spread", "kspace", "gather")}}
        r["ratio_se1p_over_se3p"] = r["se1p"]["ms"] / r["se3p"]["ms"]
        r["transform_ratio"] = (r["se1p"]["stages_ms"]["kspace"] /
                                r["se3p"]["stages_ms"]["kspace"])
        out[f"tol_{tol:.0e}"] = r
    # per-particle k-space time over the paper's N sweep at 1e-5 (M of its
    # table rounded up to 2/3/5-smooth sizes: 52 -> 54, 76 -> 80, 88 -> 90)
    sweep = []
    for n, M, nl in ((20000, 54, 7), (40000, 64, 9), (60000, 80, 10), (80000, 90, 10),
                     (100000, 96, 12)):
        xs, qs, bs = workloads.density125_system(n, seed=5)
        xt2 = torch.tensor(xs, device=dev)
        qt2 = torch.tensor(qs, device=dev)
        p2 = torch.empty(n, device=dev, dtype=torch.float64)
        E2 = torch.empty((n, 3), device=dev, dtype=torch.float64)
        row = {"N": n, "M": M, "n_l": nl}
        for periodic, name in ((False, "se1p"), (True, "se3p")):
            prm = se1p.make_params(bs, 4.0, M, 12, nl, 2.0, rc=0.0, pad_free=8)
            plan = se1p.Plan(prm, n_max=n, periodic=periodic)
            t = timed(lambda: plan.eval_into(xt2, qt2, p2, E2, U, flags=se1p.KSPACE),
                      steps, warmup, torch)
            plan.close()
            row[name + "_us_per_particle"] = t * 1e6 / n
        row["ratio"] = row["se1p_us_per_particle"] / row["se3p_us_per_particle"]
        sweep.append(row)
    out["sweep_1e-05"] = sweep
    out["paper_ratio"] = "about 1.5 at both tolerances (k-space runtime, one CPU core)"
    return out


def total_runtime_extra(se1p, workloads, oracle_mod, torch, dev, steps, warmup):
    """Total runtime (real space included) on the scaled systems of the
    paper's total-runtime example: density 100, xi = 3.5, P = 16, rc = 0.9,
    s_l = 3, M and n_l from its table (M rounded up to 2/3/5-smooth even
    sizes: 46 -> 48, 62 -> 64, 84 -> 90, 92 -> 96), FP64."""
    import numpy as np
    rows = []
    for N, M, nl in ((21600, 48, 4), (51200, 64, 6), (100000, 80, 6),
                     (172800, 96, 8), (274400, 108, 10)):
        x, q, box = workloads.density_system(N, 100.0, seed=7)
        prm = se1p.make_params(box, 3.5, M, 16, nl, 3.0, rc=0.9, pad_free=8)
        plan = se1p.Plan(prm, n_max=N)
        xt = torch.tensor(x, device=dev)
        qt = torch.tensor(q, device=dev)
        phi = torch.empty(N, device=dev, dtype=torch.float64)
        E = torch.empty((N, 3), device=dev, dtype=torch.float64)
        U = torch.empty(1, device=dev, dtype=torch.float64)
        t, st = timed_and_staged(plan, lambda: plan.eval_into(xt, qt, phi, E, U),
                                 steps, warmup, torch)
        plan.close()
        r = {"N": N, "L": float(box[0]), "M": M, "n_l": nl, "ms": t * 1e3,
             "us_per_particle": t * 1e6 / N, "stages_ms": st}
        if N == 21600 and oracle_mod is not None:
            tg = np.arange(0, N, 108)
            po, _ = oracle_mod.ewald_total(x, q, box, targets=tg, field=False)
            pg = phi.cpu().numpy()[tg]
            r["rel_rms_phi_sample"] = float(np.linalg.norm(pg - po) / np.linalg.norm(po))
            r["sample_targets"] = int(tg.size)
        rows.append(r)
    return {"workload": "density 100, xi 3.5, P 16, rc 0.9, s_l 3, FP64, "
                        "charges uniform in [-1, 1] minus the mean",
            "paper_target_rel_rms": 2e-6, "rows": rows}


def batched_extra(se1p, workloads, torch, dev, steps, warmup):
    import numpy as np
    sysl = workloads.batched_systems()
    boxes = [s[2] for s in sysl]
    counts = [s[0].shape[0] for s in sysl]
    Ntot = sum(counts)
    params = se1p.autotune(1e-5, boxes, counts, precision=se1p.FP32, P=12)
    batch = se1p.Batch(params, counts)
    x = torch.tensor(np.concatenate([s[0] for s in sysl]), device=dev, dtype=torch.float32)
    q = torch.tensor(np.concatenate([s[1] for s in sysl]), device=dev, dtype=torch.float32)
    phi = torch.empty(Ntot, device=dev, dtype=torch.float32)
    E = torch.empty((Ntot, 3), device=dev, dtype=torch.float32)
    U = torch.empty(len(counts), device=dev, dtype=torch.float64)
    t_graph = timed(lambda: batch.eval_into(x, q, phi, E, U), steps, warmup, torch)
    t_eager = timed(lambda: batch.eval_into(x, q, phi, E, U, eager=True), steps, warmup, torch)
    info = batch.info()
    batch.close()
    out = {"workload": f"64 systems, N log-uniform in [1e3, 5e4] (sum {Ntot}), "
                       "L3 uniform in [0.5, 2], 1 x 1 cross-section, +-1 charges, "
                       "FP32, P=12, autotuned for 1e-5",
           "n_total": Ntot,
           "graph_ms": t_graph * 1e3, "eager_ms": t_eager * 1e3,
           "particles_per_s": Ntot / t_graph,
           "queue_items": info["items"], "persistent_grid": info["grid"]}
    # one plan per system, launched back to back on one stream
    for prec, name in ((se1p.FP32, "loop_f32"), (se1p.FP64, "loop_f64")):
        dt = torch.float32 if prec == se1p.FP32 else torch.float64
        plans, bufs = [], []
        off = 0
        for s, p in enumerate(params):
            p2 = se1p.Params.from_buffer_copy(p)
            p2.precision = prec
            plans.append(se1p.Plan(p2, n_max=counts[s]))
            n = counts[s]
            bufs.append((x[off:off + n].to(dt), q[off:off + n].to(dt),
                         torch.empty(n, device=dev, dtype=dt),
                         torch.empty((n, 3), device=dev, dtype=dt),
                         torch.empty(1, device=dev, dtype=torch.float64)))
            off += n

        def loop():
            for pl, b in zip(plans, bufs):
                pl.eval_into(*b)
        t = timed(loop, max(2, steps // 4), 1, torch)
        out[name + "_ms"] = t * 1e3
        for pl in plans:
            pl.close()
    out["speedup_over_loop_f32"] = out["loop_f32_ms"] / out["graph_ms"]
    out["speedup_over_plain_f64"] = out["loop_f64_ms"] / out["graph_ms"]
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1611_09538_amd import se1p, workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if a.leg == "batched":
        print(json.dumps({"batched": batched_extra(se1p, workloads, torch, dev,
                                                   a.steps, a.warmup)}))
        return
    x, q, box, c = workloads.make_case(a.case)
    N = x.shape[0]
    prec = se1p.FP64 if c["precision"] == "fp64" else se1p.FP32
    dname = "f64" if prec == se1p.FP64 else "f32"
    plan = plan_for(se1p, c, box, N, prec)
    dt = plan.dtype
    xt = torch.tensor(x, device=dev, dtype=dt)
    qt = torch.tensor(q, device=dev, dtype=dt)
    phi = torch.empty(N, device=dev, dtype=dt)
    E = torch.empty((N, 3), device=dev, dtype=dt)
    U = torch.empty(1, device=dev, dtype=torch.float64)

    for _ in range(a.warmup):
        plan.eval_into(xt, qt, phi, E, U)
    torch.cuda.synchronize()

    # the timed region records two events per step, around the real-space
    # sum (the kernel the roofline prices), on the plan's stream
    plan.timing_select(["realspace"])
    plan.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        plan.eval_into(xt, qt, phi, E, U)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages, ncalls = plan.timing_read()
    plan.timing_enable(False)
    rs_ms = stages["realspace"] / max(ncalls, 1)
    print(f"timed {a.steps} steps", file=sys.stderr, flush=True)

    ms_step = (t1 - t0) * 1e3 / a.steps
    value = N / (ms_step * 1e-3)
    # per-stage times from a run of their own with events around every stage
    plan.timing_select(None)
    plan.timing_enable(True)
    timed(lambda: plan.eval_into(xt, qt, phi, E, U), max(5, a.steps // 2), 0, torch)
    stages, ncalls = plan.timing_read()
    plan.timing_enable(False)
    st_ms = {k: v / max(ncalls, 1) for k, v in stages.items()}
    kspace_ms = st_ms["bin"] + st_ms["spread"] + st_ms["kspace"] + st_ms["gather"]

    P = c["P"]
    peak = PEAK_TFLOPS[dname]
    npairs = pair_count(x, box, c["rc"])
    rs_flops = PAIR_FLOPS[dname] * npairs
    rs_ach = rs_flops / (rs_ms * 1e-3) / 1e12
    roof = {"kernel": "realspace_kernel", "bound": "alu", "achieved": rs_ach,
            "peak": peak, "unit": "TFLOP/s", "frac": rs_ach / peak,
            "traffic": traffic_for("realspace_kernel", a.case),
            "pairs_per_launch": npairs, "flops_per_pair": PAIR_FLOPS[dname],
            "algorithmic_flops_per_launch": rs_flops, "avg_ms": rs_ms}
    g_fl = gather_flops(N, P)
    g_ach = g_fl / (st_ms["gather"] * 1e-3) / 1e12
    w = 8 if dname == "f64" else 4
    # the gather reads w P^3 bytes of window values from LDS per particle
    g_lds = float(N) * w * P ** 3
    g_tbs = g_lds / (st_ms["gather"] * 1e-3) / 1e12
    # gridding keeps its sums in registers: bound by vector FMA issue, one
    # FMA (2 flops) per particle and support point; its algorithmic HBM
    # bytes are the particles in (x, y, z, q) and the grid out
    s_ach = spread_flops(N, P) / (st_ms["spread"] * 1e-3) / 1e12
    grid_bytes = float(c["M3"]) * plan.info["Mt"][0] * plan.info["Mt"][1] * w
    s_alg_bytes = 4.0 * w * N + grid_bytes
    s_tr = [traffic_for(k, a.case) for k in ("spread_kernel", "spread_weights_kernel")]
    s_traffic = None if None in s_tr else float(sum(s_tr))
    kern = {
        "gather_kernel": {"bound": "lds", "achieved": g_tbs, "peak": LDS_PEAK_TBS,
                          "unit": "TB/s", "frac": g_tbs / LDS_PEAK_TBS,
                          "algorithmic_lds_bytes_per_launch": g_lds,
                          "alu_tflops": g_ach, "alu_frac": g_ach / peak,
                          "algorithmic_flops_per_launch": g_fl,
                          "avg_ms": st_ms["gather"],
                          "traffic": traffic_for("gather_kernel", a.case)},
        "spread_stage": {"bound": "alu", "achieved": s_ach, "peak": peak,
                         "unit": "TFLOP/s", "frac": s_ach / peak,
                         "algorithmic_flops_per_launch": spread_flops(N, P),
                         "avg_ms": st_ms["spread"],
                         "algorithmic_hbm_bytes": s_alg_bytes,
                         "traffic": s_traffic,
                         "traffic_over_algorithmic":
                             None if s_traffic is None else s_traffic / s_alg_bytes},
    }

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dname,
        "data": "synthetic",
        "config": {"workload": f"{a.case}: N={N} neutral charges, box {tuple(box)} periodic in z",
                   "N": N, "M3": c["M3"], "P": P, "xi": c["xi"], "n_l": c["nl"],
                   "s_l": c["sl"], "rc": c["rc"], "pad_free": c["pad_free"],
                   "grid": [c["M3"], plan.info["Mt"][0], plan.info["Mt"][1]],
                   "n0": list(plan.info["n0"]), "nl": list(plan.info["nl"]),
                   "parallelism": "single GPU"},
        "stages_ms": st_ms,
        "kspace_particles_per_s": N / (kspace_ms * 1e-3),
        "roofline": roof,
        "kernels": kern,
    }
    plan.close()

    if a.copy_calib:
        src = torch.empty(1 << 27, device=dev, dtype=torch.float32)   # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calib_bytes_each_way"] = src.numel() * 4
        del src, dst

    if not a.no_extras:
        if prec == se1p.FP64:
            out["adaptive_fft"] = adaptive_extra(se1p, workloads, torch, dev,
                                                 max(5, a.steps // 2), 2, a.case,
                                                 st_ms["kspace"], phi)
            out["aft_sweep"] = aft_sweep_extra(se1p, workloads, torch, dev,
                                               max(5, a.steps // 2), 2)
            print("transform sweep done", file=sys.stderr, flush=True)
        out["fp32"] = fp32_extra(se1p, workloads, torch, dev, max(5, a.steps // 2), 2)
        print("fp32 done", file=sys.stderr, flush=True)
        out["batched"] = batched_extra(se1p, workloads, torch, dev, max(5, a.steps // 2), 2)
        print("batched done", file=sys.stderr, flush=True)
        out["se3p_comparison"] = se3p_extra(se1p, workloads, torch, dev, max(5, a.steps // 2), 2)
        print("se3p comparison done", file=sys.stderr, flush=True)
        orc = None
        if not a.no_cpu_baseline:
            import oracle as orc
        out["total_runtime"] = total_runtime_extra(se1p, workloads, orc, torch, dev,
                                                   max(5, a.steps // 2), 2)
        print("total runtime sweep done", file=sys.stderr, flush=True)

    if not a.no_cpu_baseline:
        import oracle
        # bounded sample: time a few targets first, then scale the sample to
        # the requested CPU seconds (the direct sum is O(N) per target)
        rng = np.random.default_rng(99)
        probe = np.sort(rng.choice(N, 16, replace=False))
        s0 = time.perf_counter()
        oracle.ewald_total(x, q, box, targets=probe)
        per = (time.perf_counter() - s0) / len(probe)
        nt = int(max(16, min(N, a.cpu_seconds / max(per, 1e-6))))
        tg = np.sort(rng.choice(N, nt, replace=False))
        s0 = time.perf_counter()
        phi_ref, E_ref = oracle.ewald_total(x, q, box, targets=tg)
        cpu_t = time.perf_counter() - s0
        pg, Eg = phi.cpu().numpy(), E.cpu().numpy()
        out["cpu_baseline"] = {
            "value": nt / cpu_t, "unit": "particles/s", "cores": oracle.num_threads(),
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"{nt} of {N} targets, direct Ewald1P sums at xi_o = 0.45/L3 "
                      f"(potential and field), {cpu_t:.1f} s"}
        out["rel_rms_sample"] = {
            "phi": float(np.linalg.norm(pg[tg] - phi_ref) / np.linalg.norm(phi_ref)),
            "E": float(np.linalg.norm(Eg[tg] - E_ref) / np.linalg.norm(E_ref)),
            "targets": nt}

    if not a.no_extras and prec == se1p.FP64:
        # the field by ik-differentiation (three more inverse transforms and
        # potential-only gathers) against the analytic gradient of the gather
        Eik = torch.empty_like(E)
        pik = plan_for(se1p, c, box, N, prec)
        t_ik, st_ik = timed_and_staged(
            pik, lambda: pik.eval_into(xt, qt, phi, Eik, U, flags=se1p.ALL | se1p.FIELD_IK),
            max(5, a.steps // 2), 2, torch)
        pik.close()
        ik = {"ms_per_step": t_ik * 1e3, "analytic_ms_per_step": ms_step,
              "kspace_ms": st_ik["kspace"], "gather_ms": st_ik["gather"],
              "analytic_kspace_ms": st_ms["kspace"], "analytic_gather_ms": st_ms["gather"]}
        if not a.no_cpu_baseline:
            Ek = Eik.cpu().numpy()
            ik["rel_rms_E_sample"] = float(np.linalg.norm(Ek[tg] - E_ref) / np.linalg.norm(E_ref))
        out["ik_field"] = ik
        print("ik field done", file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
