"""The force output (SE1P_FORCE): the totals kernel writes q_m E_m in place
of E_m.  It must equal the product of the charge and the field of an
evaluation without the flag, bit for bit (the same rounded E times the same
q), for one plan in FP64 and FP32, with the ik-differentiated field, and for
a batch; and the energy gradient of autograd.energy, which now takes the
force from the library, must still match the field path."""
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


@pytest.mark.parametrize("prec,extra", [("fp64", 0), ("fp32", 0), ("fp64", "ik")])
def test_force_is_charge_times_field(prec, extra):
    from paper_1611_09538_amd import se1p
    dev = _dev()
    _say(f"force output {prec} {extra or ''}")
    c = dict(workloads.CASES["small"])
    n = 300
    x, q, box, _ = workloads.make_case("small", n=n, seed=7)
    precision = se1p.FP64 if prec == "fp64" else se1p.FP32
    dt = torch.float64 if prec == "fp64" else torch.float32
    prm = se1p.make_params(c["box"], c["xi"], c["M3"], c["P"], c["nl"], c["sl"],
                           rc=c["rc"], pad_free=c["pad_free"], precision=precision)
    plan = se1p.Plan(prm, n_max=n)
    xt = torch.tensor(x, dtype=dt, device=dev)
    qt = torch.tensor(q, dtype=dt, device=dev)
    base = se1p.ALL | (se1p.FIELD_IK if extra == "ik" else 0)
    phi, E, U = plan.eval(xt, qt, flags=base)
    phi2, F, U2 = plan.eval(xt, qt, flags=base | se1p.FORCE)
    torch.cuda.synchronize()
    assert torch.equal(phi, phi2) and torch.equal(U, U2)
    assert torch.equal(F, qt[:, None] * E)
    plan.close()


def test_force_in_a_batch():
    from paper_1611_09538_amd import se1p
    dev = _dev()
    _say("force output, batch of 6 systems (FP32)")
    sysl = workloads.batched_systems()[:6]
    boxes = [s[2] for s in sysl]
    counts = [s[0].shape[0] for s in sysl]
    params = se1p.autotune(1e-5, boxes, counts, precision=se1p.FP32, P=12)
    batch = se1p.Batch(params, counts)
    x = torch.tensor(np.concatenate([s[0] for s in sysl]), device=dev, dtype=torch.float32)
    q = torch.tensor(np.concatenate([s[1] for s in sysl]), device=dev, dtype=torch.float32)
    phi, E, U = batch.eval(x, q, eager=True)
    phi2, F, U2 = batch.eval(x, q, flags=se1p.ALL | se1p.FORCE, eager=True)
    torch.cuda.synchronize()
    assert torch.equal(phi, phi2) and torch.equal(U, U2)
    assert torch.equal(F, q[:, None] * E)
    batch.close()


def test_energy_gradient_uses_the_force():
    from paper_1611_09538_amd import se1p, autograd
    dev = _dev()
    _say("autograd.energy gradient from the force output")
    c = dict(workloads.CASES["small"])
    n = 200
    x, q, box, _ = workloads.make_case("small", n=n, seed=9)
    prm = se1p.make_params(c["box"], c["xi"], c["M3"], c["P"], c["nl"], c["sl"],
                           rc=c["rc"], pad_free=c["pad_free"])
    plan = se1p.Plan(prm, n_max=n)
    xt = torch.tensor(x, dtype=torch.float64, device=dev, requires_grad=True)
    qt = torch.tensor(q, dtype=torch.float64, device=dev, requires_grad=True)
    U = autograd.energy(xt, qt, plan)
    U.backward()
    phi, E, _ = plan.eval(xt.detach(), qt.detach())
    torch.cuda.synchronize()
    assert torch.equal(xt.grad, -(qt.detach()[:, None] * E))
    assert torch.equal(qt.grad, phi)
    plan.close()
