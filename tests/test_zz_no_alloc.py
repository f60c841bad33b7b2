"""se1p_eval_noalloc (static device scratch, no allocation) against se1p_eval
through the C ABI, on the same plan and inputs.

Both entry points run the same kernels; only the scratch differs (the
library's static array instead of the plan's workspace), so the results
agree to rounding: identical when the call's N equals the plan's n_max (same
buffer layout), and within 1e-12 relative RMS (FP64) otherwise, where the
real-space sum may be split into a different number of parts.  Two calls in
a row, the second with fewer particles, then a call on an FP32 plan and one
with the ik-differentiated field, each against se1p_eval.
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


def _rel(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _plan(case, n_max, precision=None):
    from paper_1611_09538_amd import se1p
    c = dict(workloads.CASES[case])
    prec = se1p.FP64 if (precision or c["precision"]) == "fp64" else se1p.FP32
    prm = se1p.make_params(c["box"], c["xi"], c["M3"], c["P"], c["nl"], c["sl"],
                           rc=c["rc"], pad_free=c["pad_free"], precision=prec)
    return se1p.Plan(prm, n_max=n_max), c


def _both(plan, x, q, flags):
    dev = x.device
    N = x.shape[0]
    out = []
    for fn in (plan.eval_into, plan.eval_noalloc_into):
        phi = torch.full((N,), float("nan"), dtype=plan.dtype, device=dev)
        E = torch.full((N, 3), float("nan"), dtype=plan.dtype, device=dev)
        U = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
        fn(x, q, phi, E, U, flags=flags)
        out.append((phi, E, U))
    torch.cuda.synchronize()
    return out


def test_noalloc_matches_eval_twice_then_smaller():
    from paper_1611_09538_amd import se1p
    dev = _dev()
    n1, n2 = 500, 338
    plan, c = _plan("small", n1)
    for n in (n1, n2):
        _say(f"noalloc vs eval: small FP64 n={n} (plan n_max={n1})")
        x, q, box, _ = workloads.make_case("small", n=n, seed=70 + n)
        xt = torch.tensor(x, device=dev)
        qt = torch.tensor(q, device=dev)
        (p0, E0, U0), (p1, E1, U1) = _both(plan, xt, qt, se1p.ALL)
        assert torch.isfinite(p1).all() and torch.isfinite(E1).all()
        ep, eE = _rel(p1, p0), _rel(E1, E0)
        eU = abs(U1.item() - U0.item()) / abs(U0.item())
        _say(f"  rel-rms phi {ep:.2e}  E {eE:.2e}  |dU|/|U| {eU:.2e}")
        if n == n1:
            assert torch.equal(p0, p1) and torch.equal(E0, E1) and torch.equal(U0, U1)
        else:
            assert ep < 1e-12 and eE < 1e-12 and eU < 1e-12
    plan.close()


def test_noalloc_fp32_and_ik_field():
    from paper_1611_09538_amd import se1p
    dev = _dev()
    n = 4096
    x, q, box, _ = workloads.make_case("fp64_1e5", n=n, seed=77)
    for prec, flags, bar in (("fp32", se1p.ALL, 1e-6),
                             ("fp64", se1p.ALL | se1p.FIELD_IK, 1e-12)):
        _say(f"noalloc vs eval: fp64_1e5 geometry n={n} {prec} flags={flags}")
        plan, c = _plan("fp64_1e5", 2 * n, precision=prec)
        dt = plan.dtype
        xt = torch.tensor(x, device=dev, dtype=dt)
        qt = torch.tensor(q, device=dev, dtype=dt)
        (p0, E0, U0), (p1, E1, U1) = _both(plan, xt, qt, flags)
        ep, eE = _rel(p1, p0), _rel(E1, E0)
        eU = abs(U1.item() - U0.item()) / abs(U0.item())
        _say(f"  rel-rms phi {ep:.2e}  E {eE:.2e}  |dU|/|U| {eU:.2e}")
        assert ep < bar and eE < bar and eU < bar
        plan.close()


def test_noalloc_rejects_oversize_on_the_host():
    from paper_1611_09538_amd import se1p
    dev = _dev()
    _say("noalloc: N = 1e6 on the N = 1e6 FP32 geometry exceeds the static scratch")
    plan, c = _plan("fp32_1e6", 1)
    n = 1_000_000
    x = torch.zeros((n, 3), device=dev, dtype=torch.float32)
    q = torch.zeros(n, device=dev, dtype=torch.float32)
    phi = torch.empty(n, device=dev, dtype=torch.float32)
    rc = se1p._lib().se1p_eval_noalloc(plan._h, n, se1p._ptr(x), se1p._ptr(q),
                                       se1p._ptr(phi), None, None, se1p.ALL)
    assert rc == se1p.ERR_SCRATCH
    assert b"static" in se1p._lib().se1p_error_string(rc)
    plan.close()


def test_noalloc_replays_in_a_hip_graph():
    """The reason for the entry point: a caller that captures the evaluation
    in a HIP graph (no allocation may happen while capturing).  The graph is
    replayed several times with other device work and synchronisations in
    between, each replay checked bit for bit against the eager call (the
    same kernels on the same inputs)."""
    from paper_1611_09538_amd import se1p
    dev = _dev()
    n = 500
    plan, c = _plan("small", n)
    x, q, box, _ = workloads.make_case("small", n=n, seed=91)
    xt = torch.tensor(x, device=dev)
    qt = torch.tensor(q, device=dev)
    phi = torch.empty(n, dtype=torch.float64, device=dev)
    E = torch.empty((n, 3), dtype=torch.float64, device=dev)
    U = torch.empty(1, dtype=torch.float64, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.eval_noalloc_into(xt, qt, phi, E, U)        # first call: symbol lookup
        torch.cuda.synchronize()
        ref = (phi.clone(), E.clone(), U.clone())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            plan.eval_noalloc_into(xt, qt, phi, E, U)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for k in range(4):
        phi.fill_(float("nan"))
        E.fill_(float("nan"))
        U.fill_(float("nan"))
        junk = torch.randn(1 << 16, device=dev).sum()      # other device work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _say(f"replay {k}: max |dphi| {float((phi - ref[0]).abs().max()):.1e}")
        assert torch.equal(phi, ref[0]) and torch.equal(E, ref[1]) and torch.equal(U, ref[2])
        del junk
    plan.close()
