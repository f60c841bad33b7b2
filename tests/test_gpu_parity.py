"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Two references, both CPU-only and independent of the HIP code:
  * oracle.ewald / oracle.ewald_total -- the direct Ewald1P sums;
  * oracle.discrete -- the numpy transcription of Algorithm 1, used to check
    intermediate arrays (gridded H, solved Htilde, gathered phi^F) to near
    rounding level, with the grid geometry read from the plan.
Tolerances: rel-RMS 1e-8 against the direct sums in FP64 (the target of the
method at these parameters); 1e-12 against the step-by-step model (rounding
of FFTs of a few hundred points and sums of P^3 terms).
"""
import numpy as np
import pytest

import oracle
from oracle import discrete as D
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


def _plan(case, n_max, **over):
    se1p = _se1p()
    c = dict(workloads.CASES[case])
    c.update(over)
    prec = se1p.FP64 if c["precision"] == "fp64" else se1p.FP32
    prm = se1p.make_params(c["box"], c["xi"], c["M3"], c["P"], c["nl"], c["sl"],
                           rc=c["rc"], pad_free=c["pad_free"], precision=prec)
    return se1p.Plan(prm, n_max=n_max), c


def _geo(plan, c):
    i = plan.info
    return D.Geometry(c["box"], i["M3"], i["P"], c["xi"], i["Mt"], i["n0"], i["nl"], i["n_l"])


def _relrms(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def _say(*a):
    print(*a, flush=True)


# --------------------------------------------------------------------------
# stage parity against the step-by-step model
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 38, 130])
def test_spread_matches_model(n):
    dev = _dev()
    _say("spread parity n=", n)
    x, q, box, _ = workloads.make_case("small", n=n, seed=100 + n)
    plan, c = _plan("small", n)
    H = plan.spread(torch.tensor(x, device=dev), torch.tensor(q, device=dev))
    torch.cuda.synchronize()
    Hg = H.cpu().numpy().transpose(1, 2, 0)
    Hr = D.spread(_geo(plan, c), x, q)
    assert Hg.shape == Hr.shape
    err = np.abs(Hg - Hr).max() / np.abs(Hr).max()
    _say("spread max rel err", err)
    assert err < 1e-13


@pytest.mark.parametrize("M3,cz,kp", [(30, 2, 15), (50, 5, 5), (90, 10, 3)])
def test_spread_chunks_of_odd_factors_match_model(M3, cz, kp):
    # grids whose M3 has odd factors: gridding chunks of 2, 5 and 10 z cells
    # with 15, 5 and 3 partial grids (the plan's choice is asserted), against
    # the step-by-step model
    dev = _dev()
    n = 130
    _say("spread parity M3=", M3)
    x, q, box, _ = workloads.make_case("small", n=n, seed=200 + M3)
    plan, c = _plan("small", n, M3=M3)
    assert (plan.info["spread_cz"], plan.info["spread_kp"]) == (cz, kp)
    H = plan.spread(torch.tensor(x, device=dev), torch.tensor(q, device=dev))
    torch.cuda.synchronize()
    Hg = H.cpu().numpy().transpose(1, 2, 0)
    Hr = D.spread(_geo(plan, c), x, q)
    assert Hg.shape == Hr.shape
    err = np.abs(Hg - Hr).max() / np.abs(Hr).max()
    _say("spread max rel err", err)
    assert err < 1e-13
    plan.close()


def test_kspace_solve_and_gather_match_model():
    dev = _dev()
    n = 200
    _say("kspace/gather parity n=", n)
    x, q, box, _ = workloads.make_case("small", n=n, seed=7)
    plan, c = _plan("small", n)
    geo = _geo(plan, c)
    Hr = D.spread(geo, x, q)
    Htr = D.kspace_solve(geo, Hr)
    Hin = torch.tensor(np.ascontiguousarray(Hr.transpose(2, 0, 1)), device=dev)
    Ht = plan.kspace_solve(Hin)
    torch.cuda.synchronize()
    Htg = Ht.cpu().numpy().transpose(1, 2, 0)
    err = np.abs(Htg - Htr).max() / np.abs(Htr).max()
    _say("kspace_solve max rel err", err)
    assert err < 1e-12
    phi_r, E_r = D.gather(geo, Htr, x)
    Htr_t = torch.tensor(np.ascontiguousarray(Htr.transpose(2, 0, 1)), device=dev)
    phi, E = plan.gather(torch.tensor(x, device=dev), Htr_t)
    torch.cuda.synchronize()
    ep = _relrms(phi.cpu().numpy(), phi_r)
    ee = _relrms(E.cpu().numpy(), E_r)
    _say("gather rel-rms phi", ep, "E", ee)
    assert ep < 1e-12 and ee < 1e-12


# --------------------------------------------------------------------------
# end to end against the direct Ewald sums
# --------------------------------------------------------------------------
def test_small_fp64_matches_oracle():
    dev = _dev()
    se1p = _se1p()
    _say("small case N=500 FP64 vs oracle")
    x, q, box, _ = workloads.make_case("small")
    plan, c = _plan("small", x.shape[0])
    xt, qt = torch.tensor(x, device=dev), torch.tensor(q, device=dev)
    phi, E, U = plan.eval(xt, qt, flags=se1p.ALL | se1p.CHECK_INPUT)
    torch.cuda.synchronize()
    phi_ref, E_ref = oracle.ewald_total(x, q, box)
    U_ref = 0.5 * np.dot(q, phi_ref)
    ep, ee = _relrms(phi.cpu().numpy(), phi_ref), _relrms(E.cpu().numpy(), E_ref)
    eu = abs(U.item() - U_ref) / abs(U_ref)
    _say("rel-rms phi", ep, "E", ee, "U", eu)
    assert ep < 1e-8 and ee < 1e-8 and eu < 1e-8
    # components: k-space part against the direct k3 != 0 and k3 = 0 sums,
    # error measured against the size of the total (the bar is on totals)
    phiF, EF, _ = plan.eval(xt, qt, flags=se1p.KSPACE)
    r = oracle.ewald(x, q, box, c["xi"], rc=c["rc"])
    torch.cuda.synchronize()
    dphi = phiF.cpu().numpy() - (r["phi_Fk"] + r["phi_F0"])
    dE = EF.cpu().numpy() - (r["E_Fk"] + r["E_F0"])
    assert np.linalg.norm(dphi) / np.linalg.norm(phi_ref) < 1e-8
    assert np.linalg.norm(dE) / np.linalg.norm(E_ref) < 1e-8
    # real space with the same cut-off: the same sum; the kernel's erfc is
    # exp(-x^2) times a fitted erfcx with relative error 6e-12 per pair
    phiR, ER, _ = plan.eval(xt, qt, flags=se1p.REAL)
    torch.cuda.synchronize()
    assert _relrms(phiR.cpu().numpy(), r["phi_R"]) < 6e-12
    assert _relrms(ER.cpu().numpy(), r["E_R"]) < 6e-12
    phiS, _, _ = plan.eval(xt, qt, flags=se1p.SELF)
    torch.cuda.synchronize()
    assert np.allclose(phiS.cpu().numpy(), r["phi_self"], rtol=1e-15, atol=0)


def test_fp64_1e5_sampled_matches_oracle():
    dev = _dev()
    se1p = _se1p()
    _say("fp64_1e5 case vs oracle on sampled targets")
    x, q, box, _ = workloads.make_case("fp64_1e5")
    plan, c = _plan("fp64_1e5", x.shape[0])
    xt, qt = torch.tensor(x, device=dev), torch.tensor(q, device=dev)
    phi, E, U = plan.eval(xt, qt)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1234)
    tg = np.sort(rng.choice(x.shape[0], 300, replace=False))
    phi_ref, E_ref = oracle.ewald_total(x, q, box, targets=tg)
    ep = _relrms(phi.cpu().numpy()[tg], phi_ref)
    ee = _relrms(E.cpu().numpy()[tg], E_ref)
    # the energy is 1/2 sum q phi of the returned potentials (FP64 reduction)
    pg = phi.cpu().numpy()
    eu = abs(U.item() - 0.5 * np.dot(q, pg)) / abs(0.5 * np.dot(q, pg))
    _say("rel-rms phi", ep, "E", ee, "U consistency", eu)
    assert ep < 1e-8 and ee < 1e-8 and eu < 1e-12


# --------------------------------------------------------------------------
# edge cases
# --------------------------------------------------------------------------
def test_two_particles_and_box_edges():
    # Lone pairs at the box corners, across the periodic boundary in z and
    # at z outside [0, L3).  The HIP path must match Algorithm 1 (numpy
    # model) to rounding; against the direct sums a lone dipole at M3 = 32
    # shows the method's truncation error (1.6e-7 of max |phi| measured with
    # the model itself), so that comparison uses 1e-6.
    dev = _dev()
    se1p = _se1p()
    _say("edge: two particles, box edges, z outside [0,L3)")
    box = np.array([1.0, 1.0, 1.0])
    eps = np.nextafter(1.0, 0.0)
    cases = [
        (np.array([[0.0, 0.0, 0.0], [eps, eps, 0.5]]), np.array([1.0, -1.0])),
        (np.array([[0.5, 0.5, -0.25], [0.2, 0.7, 3.6]]), np.array([-1.0, 1.0])),
        (np.array([[0.3, 0.3, 0.999999], [0.3, 0.3, 0.000001]]), np.array([1.0, -1.0])),
    ]
    plan, c = _plan("small", 8)
    geo = _geo(plan, c)
    for x, q in cases:
        xt, qt = torch.tensor(x, device=dev), torch.tensor(q, device=dev)
        phi, E, U = plan.eval(xt, qt, flags=se1p.ALL | se1p.CHECK_INPUT)
        phiF, EF, _ = plan.eval(xt, qt, flags=se1p.KSPACE)
        torch.cuda.synchronize()
        phiF_m, EF_m = D.se1p_kspace(geo, x, q)
        # unit charges: potentials of order one set the absolute floor
        assert np.abs(phiF.cpu().numpy() - phiF_m).max() <= 1e-12 * max(np.abs(phiF_m).max(), 1.0)
        assert np.abs(EF.cpu().numpy() - EF_m).max() <= 1e-12 * max(np.abs(EF_m).max(), 1.0)
        phi_ref, E_ref = oracle.ewald_total(x, q, box)
        ep = np.abs(phi.cpu().numpy() - phi_ref).max() / np.abs(phi_ref).max()
        ee = np.abs(E.cpu().numpy() - E_ref).max() / np.abs(E_ref).max()
        _say("edge case err", ep, ee)
        assert ep < 1e-6 and ee < 1e-6


@pytest.mark.parametrize("n", [1, 63, 64, 65, 257])
def test_ragged_sizes_match_model(n):
    dev = _dev()
    _say("ragged n=", n)
    rng = np.random.default_rng(n)
    box = np.array([1.0, 1.0, 1.0])
    x = workloads.uniform_positions(rng, n, box)
    q = rng.uniform(-1, 1, n)       # operator applied to any vector
    plan, c = _plan("small", 300)
    geo = _geo(plan, c)
    phi_r, E_r = D.se1p_kspace(geo, x, q)
    se1p = _se1p()
    phi, E, _ = plan.eval(torch.tensor(x, device=dev), torch.tensor(q, device=dev),
                          flags=se1p.KSPACE | se1p.NO_NEUTRAL)
    torch.cuda.synchronize()
    # unit charges: norms below sqrt(n) (e.g. the residual self-field of a
    # lone particle) are compared against that floor
    fl = np.sqrt(n)
    assert np.linalg.norm(phi.cpu().numpy() - phi_r) < 1e-12 * max(np.linalg.norm(phi_r), fl)
    assert np.linalg.norm(E.cpu().numpy() - E_r) < 1e-12 * max(np.linalg.norm(E_r), fl)


def test_deterministic_bitwise():
    dev = _dev()
    _say("determinism")
    x, q, box, _ = workloads.make_case("small")
    plan, c = _plan("small", x.shape[0])
    xt, qt = torch.tensor(x, device=dev), torch.tensor(q, device=dev)
    a = plan.eval(xt, qt)
    b = plan.eval(xt, qt)
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        assert torch.equal(u, v)


def test_stage_timing_selection():
    # events around the selected stages only; the others read zero, and the
    # outputs do not depend on what is recorded
    dev = _dev()
    se1p = _se1p()
    _say("stage timing selection")
    x, q, box, _ = workloads.make_case("small")
    plan, c = _plan("small", x.shape[0])
    xt, qt = torch.tensor(x, device=dev), torch.tensor(q, device=dev)
    ref = plan.eval(xt, qt)
    plan.timing_select(["realspace", "bin"])
    plan.timing_enable(True)
    out = [plan.eval(xt, qt) for _ in range(3)]
    st, nc = plan.timing_read()
    assert nc == 3
    assert st["realspace"] > 0 and st["bin"] > 0
    assert all(st[k] == 0 for k in ("spread", "kspace", "gather", "combine"))
    plan.timing_select(None)
    plan.timing_enable(True)
    plan.eval(xt, qt)
    st, nc = plan.timing_read()
    assert nc == 1 and all(v > 0 for v in st.values())
    plan.timing_enable(False)
    for o in out:
        for u, v in zip(o, ref):
            assert torch.equal(u, v)
    for bad in (0, 1 << se1p.NSTAGE):
        assert se1p._lib().se1p_timing_select(plan._h, bad) == se1p.ERR_ARG
    plan.close()


def test_input_errors():
    dev = _dev()
    se1p = _se1p()
    _say("input errors")
    plan, c = _plan("small", 16)
    x = torch.tensor([[0.2, 0.3, 0.4], [0.6, 0.7, 0.8]], device=dev, dtype=torch.float64)
    with pytest.raises(se1p.SE1PError) as e:
        plan.eval(x, torch.tensor([1.0, -0.5], device=dev, dtype=torch.float64),
                  flags=se1p.ALL | se1p.CHECK_INPUT)
    assert e.value.code == se1p.ERR_NONNEUTRAL
    bad = x.clone()
    bad[0, 0] = 1.5
    with pytest.raises(se1p.SE1PError) as e:
        plan.eval(bad, torch.tensor([1.0, -1.0], device=dev, dtype=torch.float64),
                  flags=se1p.ALL | se1p.CHECK_INPUT)
    assert e.value.code == se1p.ERR_OUT_OF_BOX
    big = torch.rand((17, 3), device=dev, dtype=torch.float64)
    with pytest.raises(se1p.SE1PError) as e:
        plan.eval(big, torch.zeros(17, device=dev, dtype=torch.float64))
    assert e.value.code == se1p.ERR_TOO_MANY
    # an empty input is an argument error (N counts from 1), rejected on the
    # host before anything is launched
    qq = torch.tensor([1.0, -1.0], device=dev, dtype=torch.float64)
    phi = torch.empty(2, device=dev, dtype=torch.float64)
    assert se1p._lib().se1p_eval(plan._h, 0, se1p._ptr(x), se1p._ptr(qq), se1p._ptr(phi),
                                 None, None, int(se1p.ALL)) == se1p.ERR_ARG
    torch.cuda.synchronize()


def test_plan_rejects_sizes_the_transforms_do_not_take():
    # M3 = 14 = 2 x 7: the transforms take the radices 2, 3, 4 and 5 only;
    # the plan reports it on creation and allocates nothing
    _dev()
    se1p = _se1p()
    prm = se1p.make_params((1.0, 1.0, 1.0), 5.0, 14, 8, 2, 2.0, rc=0.3)
    with pytest.raises(se1p.SE1PError) as e:
        se1p.Plan(prm, n_max=10)
    assert e.value.code == se1p.ERR_UNSUPPORTED


def test_check_input_accepts_fp32_rounded_neutral_charges():
    """FP32 plans: charges neutral in FP64 and rounded to FP32 (|sum q| up to
    about sqrt(N) 3e-8) pass SE1P_CHECK_INPUT; a charge excess of 1e-3 sum |q|
    is still rejected."""
    dev = _dev()
    se1p = _se1p()
    n = 2000
    plan, c = _plan("small", n, precision="fp32")
    rng = np.random.default_rng(21)
    x = workloads.uniform_positions(rng, n, c["box"])
    q = workloads.neutral_uniform(rng, n)
    xt = torch.tensor(x, device=dev, dtype=torch.float32)
    q32 = torch.tensor(q, device=dev, dtype=torch.float32)
    qs = float(q32.double().sum().abs() / q32.double().abs().sum())
    _say(f"FP32 neutral check: |sum q| / sum |q| = {qs:.2e}")
    assert qs > 1e-10          # the FP64 bar would reject these charges
    phi, _, _ = plan.eval(xt, q32, flags=se1p.ALL | se1p.CHECK_INPUT)
    torch.cuda.synchronize()
    assert torch.isfinite(phi).all()
    qb = q32.clone()
    qb[0] += 1e-3 * float(q32.abs().sum())
    with pytest.raises(se1p.SE1PError) as e:
        plan.eval(xt, qb, flags=se1p.ALL | se1p.CHECK_INPUT)
    assert e.value.code == se1p.ERR_NONNEUTRAL
    plan.close()


def test_adaptive_transform_matches_plain_upsampled():
    """Upsampling only the slabs 0 < |k3| <= 2 pi n_l / L3 (eq. upsamplings)
    must reproduce the plain upsampled transform (every slab upsampled) to
    the method's accuracy; the plain one is the reference of the adaptive
    design (section 3.3)."""
    dev = _dev()
    se1p = _se1p()
    x, q, box, c = workloads.make_case("small")
    out = []
    for nl in (c["nl"], c["M3"] // 2):
        prm = se1p.make_params(box, c["xi"], c["M3"], c["P"], nl, c["sl"], rc=c["rc"],
                               pad_free=c["pad_free"])
        plan = se1p.Plan(prm, n_max=x.shape[0])
        phi, E, _ = plan.eval(torch.tensor(x, device=dev), torch.tensor(q, device=dev),
                              flags=se1p.KSPACE)
        out.append((phi.cpu().numpy(), E.cpu().numpy()))
    p_ref = oracle.ewald_total(x, q, box)[0]
    dphi = np.linalg.norm(out[0][0] - out[1][0]) / np.linalg.norm(p_ref)
    dE = np.linalg.norm(out[0][1] - out[1][1]) / np.linalg.norm(out[1][1])
    print("adaptive vs plain upsampled: phi %.2e E %.2e" % (dphi, dE), flush=True)
    assert dphi < 1e-9 and dE < 1e-8
