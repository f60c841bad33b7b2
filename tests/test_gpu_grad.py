"""Adjoint / autograd checks of the HIP path (through the C ABI).

* U = 1/2 q^T A q: central finite differences of U (h = 1e-6) on random
  particles against the hand-written backward (-q E), and the forces
  against the oracle's analytic fields; dU/dq against the oracle potential.
  The finite-difference plan uses a real-space cut-off where erfc(xi rc) is
  below 1e-18, so no pair crossing the cut-off makes U jump.
* phi = A q with an upstream gradient g: dL/dq = A g is checked by the
  symmetry <A g, q> = <g, A q>, and dL/dx by finite differences of g . phi.
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


def _mods():
    from paper_1611_09538_amd import autograd, se1p
    return se1p, autograd


def _plan(case, n_max, **over):
    se1p, _ = _mods()
    c = dict(workloads.CASES[case])
    c.update(over)
    prm = se1p.make_params(c["box"], c["xi"], c["M3"], c["P"], c["nl"], c["sl"],
                           rc=c["rc"], pad_free=c["pad_free"])
    return se1p.Plan(prm, n_max=n_max), c


def _say(*a):
    print(*a, flush=True)


def test_energy_gradient_fd_and_oracle():
    dev = _dev()
    se1p, ag = _mods()
    _say("grad_2e5: finite differences of U and oracle forces")
    x, q, box, c = workloads.make_case("grad_2e5")
    N = x.shape[0]
    rc_fd = 6.5 / c["xi"]
    plan, c = _plan("grad_2e5", N, rc=rc_fd)
    xt = torch.tensor(x, device=dev, requires_grad=True)
    qt = torch.tensor(q, device=dev, requires_grad=True)
    U = ag.energy(xt, qt, plan)
    U.backward()
    gx = xt.grad.cpu().numpy()
    gq = qt.grad.cpu().numpy()
    rng = np.random.default_rng(31)
    fd_idx = rng.choice(N, 32, replace=False)
    h = 1e-6
    xb = torch.tensor(x, device=dev)
    qb = torch.tensor(q, device=dev)
    errs = []
    scale = np.abs(gx[fd_idx]).max()
    for m in fd_idx:
        for d in range(3):
            xp = xb.clone()
            xp[m, d] += h
            Up = plan.eval(xp, qb)[2].item()
            xp[m, d] -= 2 * h
            Um = plan.eval(xp, qb)[2].item()
            fd = (Up - Um) / (2 * h)
            errs.append(abs(fd - gx[m, d]) / scale)
    _say("max FD error / max |dU/dx|:", max(errs))
    assert max(errs) < 1e-5
    # forces and dU/dq against the oracle on the FD particles plus 224 more
    tg = np.unique(np.concatenate([fd_idx, rng.choice(N, 224, replace=False)]))
    phi_ref, E_ref = oracle.ewald_total(x, q, box, targets=tg)
    F_ref = -q[tg, None] * E_ref           # dU/dx = -q E
    eF = np.linalg.norm(gx[tg] - F_ref) / np.linalg.norm(F_ref)
    eq = np.linalg.norm(gq[tg] - phi_ref) / np.linalg.norm(phi_ref)
    _say("rel-rms dU/dx vs oracle", eF, "dU/dq vs oracle", eq)
    assert eF < 1e-8 and eq < 1e-8


def test_potential_adjoint_symmetry_and_fd():
    dev = _dev()
    se1p, ag = _mods()
    _say("potential adjoint on the small case")
    x, q, box, c = workloads.make_case("small")
    N = x.shape[0]
    plan, c = _plan("small", N)
    rng = np.random.default_rng(8)
    g = rng.standard_normal(N)
    xt = torch.tensor(x, device=dev, requires_grad=True)
    qt = torch.tensor(q, device=dev, requires_grad=True)
    gt = torch.tensor(g, device=dev)
    phi = ag.potential(xt, qt, plan)
    L = torch.dot(gt, phi)
    L.backward()
    gq = qt.grad.cpu().numpy()
    gx = xt.grad.cpu().numpy()
    # symmetry of the operator: <A g, q> = <g, A q>, to rounding of the
    # terms (the sums cancel, so the bar is on the size of the terms)
    lhs = np.dot(gq, q)
    rhs = L.item()
    scale_t = np.linalg.norm(g) * np.linalg.norm(phi.detach().cpu().numpy())
    _say("symmetry", lhs, rhs, "term scale", scale_t)
    assert abs(lhs - rhs) <= 1e-12 * scale_t
    # finite differences of L in the positions (operator at fixed charges)
    xb = torch.tensor(x, device=dev)
    qb = torch.tensor(q, device=dev)
    h = 1e-6
    worst = 0.0
    scale = np.abs(gx).max()
    for m in rng.choice(N, 8, replace=False):
        for d in range(3):
            xp = xb.clone()
            xp[m, d] += h
            Lp = torch.dot(gt, plan.eval(xp, qb, flags=se1p.ALL)[0]).item()
            xp[m, d] -= 2 * h
            Lm = torch.dot(gt, plan.eval(xp, qb, flags=se1p.ALL)[0]).item()
            worst = max(worst, abs((Lp - Lm) / (2 * h) - gx[m, d]) / scale)
    _say("max FD error / max |dL/dx|:", worst)
    assert worst < 1e-5
