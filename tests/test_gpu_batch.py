"""Batched evaluation: many independent systems per launch (persistent work
queues), the autotuner's parameters, and the HIP-graph replay.

* Every system of a batch must give what a plan of its own gives (the two
  share kernels; the packed binning keeps each system's particle order).
  A single plan splits each chunk's real-space candidates into parts summed
  afterwards, while the batch's persistent queue runs whole chunks, so the
  two agree to rounding, not bitwise.
* Graph replays must equal the eager sequence, replay after replay, with
  other device work and synchronisations between them.
* The batched workload (64 systems, N log-uniform in [1e3, 5e4], L3 uniform
  in [0.5, 2], unit cross-section, +-1 charges, FP32, P = 12, autotuned for
  1e-5) must meet rel-RMS 1e-5 per system against the oracle on 64 targets
  of every system.
"""
import numpy as np
import pytest

import oracle
from paper_1611_09538_amd import workloads

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _se1p():
    from paper_1611_09538_amd import se1p
    return se1p


def _say(*a):
    print(*a, flush=True)


def _pack(systems, dt):
    dev = _dev()
    x = torch.tensor(np.concatenate([s[0] for s in systems]), device=dev, dtype=dt)
    q = torch.tensor(np.concatenate([s[1] for s in systems]), device=dev, dtype=dt)
    return x, q


def _systems(k):
    return workloads.batched_systems()[:k]


@pytest.mark.parametrize("prec,tol,P", [("fp64", 1e-8, 16), ("fp32", 1e-5, 12)])
def test_batch_equals_single_plans(prec, tol, P):
    se1p = _se1p()
    _say(f"batch vs single plans, {prec}")
    sysl = _systems(6)
    boxes = [s[2] for s in sysl]
    counts = [s[0].shape[0] for s in sysl]
    pr = se1p.FP64 if prec == "fp64" else se1p.FP32
    dt = torch.float64 if prec == "fp64" else torch.float32
    params = se1p.autotune(tol, boxes, counts, precision=pr, P=P)
    batch = se1p.Batch(params, counts)
    x, q = _pack(sysl, dt)
    phi, E, U = batch.eval(x, q, eager=True)
    torch.cuda.synchronize()
    for s in range(len(sysl)):
        o0, o1 = batch.offsets[s], batch.offsets[s + 1]
        plan = se1p.Plan(params[s], n_max=counts[s])
        ps, Es, Us = plan.eval(x[o0:o1], q[o0:o1])
        dphi = ((phi[o0:o1] - ps).norm() / ps.norm()).item()
        dE = ((E[o0:o1] - Es).norm() / Es.norm()).item()
        # U = 1/2 sum q phi cancels; its rounding error scales with the sum
        # of the magnitudes of its terms
        uscale = 0.5 * (q[o0:o1].double() * ps.double()).abs().sum().item()
        dU = abs(U[s].item() - Us.item()) / uscale
        _say(f"system {s}: N={counts[s]} M3={params[s].M3} rel-rms dphi={dphi:.3e} "
             f"dE={dE:.3e} |dU|/(sum|q phi|/2)={dU:.3e}")
        bar = 1e-13 if prec == "fp64" else 1e-6
        assert dphi < bar and dE < bar and dU < 10 * bar
        plan.close()
    batch.close()


def test_batch_graph_replays_match_eager():
    se1p = _se1p()
    _say("batch graph replays vs eager")
    sysl = _systems(12)
    boxes = [s[2] for s in sysl]
    counts = [s[0].shape[0] for s in sysl]
    params = se1p.autotune(1e-5, boxes, counts, precision=se1p.FP32, P=12)
    batch = se1p.Batch(params, counts)
    x, q = _pack(sysl, torch.float32)
    ref = batch.eval(x, q, eager=True)
    torch.cuda.synchronize()
    N = batch.n_total
    phi = torch.empty(N, device=x.device, dtype=torch.float32)
    E = torch.empty((N, 3), device=x.device, dtype=torch.float32)
    U = torch.empty(len(counts), device=x.device, dtype=torch.float64)
    for rep in range(4):
        phi.fill_(float("nan"))
        E.fill_(float("nan"))
        U.fill_(float("nan"))
        batch.eval_into(x, q, phi, E, U)
        # unrelated eager work and a synchronisation between replays
        junk = torch.randn(1 << 20, device=x.device).sum()
        torch.cuda.synchronize()
        assert torch.equal(phi, ref[0]) and torch.equal(E, ref[1]) and torch.equal(U, ref[2]), rep
        _say(f"replay {rep}: equal to eager ({junk.item():.1f})")
    info = batch.info()
    assert info["graph_captures"] == 1
    # new output buffers -> captured again, same values
    out = batch.eval(x, q)
    torch.cuda.synchronize()
    assert batch.info()["graph_captures"] == 2
    assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])
    batch.close()


def test_batch_workload_vs_oracle():
    se1p = _se1p()
    _say("batched workload (64 systems, FP32, autotuned for 1e-5) vs the oracle")
    sysl = workloads.batched_systems()
    boxes = [s[2] for s in sysl]
    counts = [s[0].shape[0] for s in sysl]
    params = se1p.autotune(1e-5, boxes, counts, precision=se1p.FP32, P=12)
    batch = se1p.Batch(params, counts)
    x, q = _pack(sysl, torch.float32)
    phi, E, U = batch.eval(x, q)
    torch.cuda.synchronize()
    phi, E, U = phi.double().cpu().numpy(), E.double().cpu().numpy(), U.cpu().numpy()
    info = batch.info()
    _say("items", info["items"], "grid", info["grid"])
    rng = np.random.default_rng(77)
    errs = []
    for s, (xs, qs, box) in enumerate(sysl):
        o0, o1 = batch.offsets[s], batch.offsets[s + 1]
        tg = np.sort(rng.choice(xs.shape[0], 64, replace=False))
        # the FP32 batch received float32 positions: the oracle takes the same
        x32 = xs.astype(np.float32).astype(np.float64)
        pr, Er = oracle.ewald_total(x32, qs, box, targets=tg)
        ep = np.linalg.norm(phi[o0:o1][tg] - pr) / np.linalg.norm(pr)
        eE = np.linalg.norm(E[o0:o1][tg] - Er) / np.linalg.norm(Er)
        errs.append((ep, eE))
        Uc = 0.5 * np.dot(qs, phi[o0:o1])
        assert abs(U[s] - Uc) <= 1e-6 * abs(Uc)
        _say(f"system {s}: N={xs.shape[0]} L3={box[2]:.3f} M3={params[s].M3} "
             f"xi={params[s].xi:.2f} rc={params[s].rc:.4f} phi {ep:.2e} E {eE:.2e}")
    errs = np.array(errs)
    _say("worst rel-rms over systems: phi %.2e E %.2e" % tuple(errs.max(axis=0)))
    assert errs.max() < 1e-5
    batch.close()
