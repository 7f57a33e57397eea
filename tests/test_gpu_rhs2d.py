"""GPU parity of the 2D right-hand sides (plain 2D Navier--Stokes and the
Boussinesq system of Sec. 3.2, Eqs. (4a-b)) against the oracle."""
import numpy as np
import pytest

from gpu_util import announce, per_field_rel_l2
from oracle import control, diagnostics, spectral, stepping
from paper_1810_10197_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ns():
    from paper_1810_10197_amd import ns as mod
    return mod


def random2d(n, seed, ncomp):
    """Random real, masked 2D state; the velocity made solenoidal through a
    stream function (test input)."""
    rng = np.random.default_rng(seed)
    m = spectral.mask(n, 2)
    kx, ky = spectral.wavenumbers(n, 2)
    k2 = kx * kx + ky * ky
    psi = spectral.forward(rng.standard_normal((n, n)), 2) * m * np.exp(-k2 / (n / 4) ** 2)
    st = np.zeros((ncomp, n, n // 2 + 1), dtype=complex)
    st[0] = 1j * ky * psi
    st[1] = -1j * kx * psi
    if ncomp == 3:
        st[2] = spectral.forward(rng.standard_normal((n, n)), 2) * m * np.exp(-k2 / (n / 4) ** 2)
    return spectral.forward(spectral.inverse(st, n, 2), 2) * m


@pytest.mark.parametrize("n", [16, 64, 256])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rhs2d_ns(ns, n, prec):
    announce("rhs2d ns n=%d %s" % (n, prec))
    nu = 0.01
    u = random2d(n, n, 2)
    s = ns.Solver(dim=2, n=n, nu=nu, rhs_precision=prec)
    got = s.rhs(u[None]).cpu().numpy()[0]
    s.close()
    ref = spectral.rhs_ns2d(u, nu)
    err = max(per_field_rel_l2(got, ref))
    assert err <= (1e-12 if prec == "fp64" else 2e-6), err


@pytest.mark.parametrize("n", [32, 128, 1024])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rhs2d_boussinesq(ns, n, prec):
    announce("rhs2d boussinesq n=%d %s" % (n, prec))
    nu, kappa, ri = 1e-3, 2e-3, 0.5
    u = random2d(n, 3 * n, 3)
    s = ns.Solver(dim=2, n=n, nu=nu, rhs_precision=prec, scalar=1, ri=ri, kappa=kappa)
    got = s.rhs(u[None]).cpu().numpy()[0]
    s.close()
    ref = spectral.rhs_ns2d(u, nu, kappa, ri)
    err = max(per_field_rel_l2(got, ref))
    assert err <= (1e-12 if prec == "fp64" else 3e-6), err


def test_rayleigh_taylor_1024(ns):
    """The Rayleigh--Taylor workload's initial state at 1024^2, FP32 RHS."""
    n, nu, kappa, ri = 1024, 1e-4, 1e-4, 0.5
    announce("rt 1024 fp32")
    st = inputs.rayleigh_taylor2d(n)
    s = ns.Solver(dim=2, n=n, nu=nu, rhs_precision="fp32", scalar=1, ri=ri, kappa=kappa)
    got = s.rhs(st[None]).cpu().numpy()[0]
    s.close()
    ref = spectral.rhs_ns2d(st, nu, kappa, ri)
    # u = 0 initially: f_u is the projected buoyancy (no FFT involved), f_rho
    # pure diffusion; both agree to rounding
    err = per_field_rel_l2(got, ref)
    assert max(err) <= 1e-6, err


def test_tgv2d_exact_decay_1024(ns):
    n, nu = 1024, 1e-4
    announce("tgv2d exact n=1024")
    u = inputs.tgv2d(n)
    s = ns.Solver(dim=2, n=n, nu=nu, rhs_precision="fp32")
    got = s.rhs(u[None]).cpu().numpy()[0]
    s.close()
    err = np.abs(got + 2 * nu * u).max() / (2 * nu * np.abs(u).max())
    assert err <= 1e-3, err


def test_boussinesq_bs5_steps_and_diagnostics(ns):
    n, nu, kappa, ri = 64, 1e-3, 1e-3, 0.5
    announce("boussinesq bs5 n=%d" % n)
    u0 = random2d(n, 7, 3)
    rhs = lambda u: spectral.rhs_ns2d(u, nu, kappa, ri)
    s = ns.Solver(dim=2, n=n, nu=nu, rhs_precision="fp64", scalar=1, ri=ri, kappa=kappa)
    s.set_state(u0[None])
    ref = u0
    for _ in range(3):
        st, errs = s.step_bs5(0.05, 1e-8, 1e-8, force=True)
        r = stepping.bs5_attempt(rhs, ref, 0.05, 1e-8, 1e-8)
        ref = r["u_new"]
        assert errs[0] == pytest.approx(r["err"], rel=1e-8)
    got = s.get_state().cpu().numpy()[0]
    assert max(per_field_rel_l2(got, ref)) <= 1e-12
    e, eps, sh = s.diagnostics()
    f = rhs(ref)
    assert e[0] == pytest.approx(diagnostics.energy(ref, 2), rel=1e-12)
    assert eps[0] == pytest.approx(diagnostics.dissipation(ref, f, 2), rel=1e-9)
    assert sh[0] == pytest.approx(diagnostics.shells(ref, 2), rel=1e-12, abs=1e-300)
    s.close()


@pytest.mark.parametrize("n,scalar,prec", [(1024, 1, "fp32"), (256, 0, "fp32"), (1024, 1, "fp64")])
def test_rhs2d_every_launch_variant(ns, n, scalar, prec):
    """Each variant of the two column passes (radix plan and tile width; the
    narrow 1024-point plan has four passes; with the scalar, y-forward
    variants 2, 4, 5 and 6 split the fields over two blocks) and of the x-pass
    (both B2 layouts, one wavefront per row or, at 1024, one per transform)
    is a correct right-hand side, and the autotuner keeps one of them."""
    announce("rhs2d variants n=%d scalar=%d %s" % (n, scalar, prec))
    nu, kappa, ri = 1e-3, 2e-3, 0.5
    tol = 3e-6 if prec == "fp32" else 1e-12
    u = random2d(n, 5 * n + scalar, 3 if scalar else 2)
    ref = spectral.rhs_ns2d(u, nu, kappa, ri) if scalar else spectral.rhs_ns2d(u, nu)
    s = ns.Solver(dim=2, n=n, nu=nu, rhs_precision=prec, scalar=scalar, ri=ri if scalar else 0.0,
                  kappa=kappa if scalar else 0.0)
    for v in range(28):                         # x-pass slot: layout bit, row split from 2 on
        s.tune([v % 5, 0, (v // 7) % 4, 0, 6 - v % 7, 0])
        got = s.rhs(u[None]).cpu().numpy()[0]
        err = max(per_field_rel_l2(got, ref))
        assert err <= tol, (v, err)
    s.set_state(u[None])
    variants, ms = s.autotune(reps=2)
    # per slot the fastest variant, or one within 3% of it that won on whole evaluations
    assert ms[0][variants[0]] <= 1.03 * min(x for x in ms[0][:5] if x > 0)
    assert ms[2][variants[2]] <= 1.03 * min(x for x in ms[2][:4] if x > 0)
    assert ms[4][variants[4]] <= 1.03 * min(x for x in ms[4][:7] if x > 0)
    assert ms[4][7] == 0 and ms[0][5] == 0
    with pytest.raises(ns.NsError):
        s.tune([0, 0, 0, 0, 7, 0])               # beyond the y-forward's variants
    with pytest.raises(ns.NsError):
        s.tune([5, 0, 0, 0, 0, 0])               # beyond the y-inverse's
    got = s.rhs(u[None]).cpu().numpy()[0]
    assert max(per_field_rel_l2(got, ref)) <= tol
    s.close()


def unit_speed(u, n):
    """u scaled to a largest physical velocity of one (test input)."""
    return u / np.abs(spectral.inverse(u, n, 2)[:2]).max()


@pytest.mark.parametrize("n,scalar", [(1024, 1), (256, 0)])
def test_bs5_fp32_stage_inputs_every_variant(ns, n, scalar):
    """With an FP32 right-hand side the stages of a BS5 attempt reach the
    first and last passes as FP32 roundings of U_i, formed from the FP32
    copies of u_n and of the k_j (which the last pass writes beside f): one
    attempt per launch variant of the three passes against the oracle's
    attempt (h at a CFL number of 0.5)."""
    announce("bs5 fp32 stage inputs 2d n=%d scalar=%d" % (n, scalar))
    nu, kappa, ri = 1e-3, 2e-3, 0.5
    u = unit_speed(random2d(n, 11 * n + scalar, 3 if scalar else 2), n)
    h = 0.5 * 2 * np.pi / n
    rhs = (lambda x: spectral.rhs_ns2d(x, nu, kappa, ri)) if scalar else (lambda x: spectral.rhs_ns2d(x, nu))
    ref = stepping.bs5_attempt(rhs, u, h, 1e-6, 1e-6)["u_new"]
    s = ns.Solver(dim=2, n=n, nu=nu, rhs_precision="fp32", scalar=scalar, ri=ri if scalar else 0.0,
                  kappa=kappa if scalar else 0.0)
    for v in range(28):
        s.tune([v % 5, 0, (v // 7) % 4, 0, 6 - v % 7, 0])
        s.set_state(u[None])
        s.step_bs5(h, 1e-6, 1e-6, force=True)
        got = s.get_state().cpu().numpy()[0]
        err = max(per_field_rel_l2(got, ref))
        assert err <= 1e-6, (v, err)
    s.close()


def test_fp32_integrate_2d_graph_host_and_oracle(ns):
    """An adaptive FP32 run of the Boussinesq system (FP32 stage inputs and
    k_j copies, kept by the commits), with a rejected first step: the
    graph-captured and the host path agree bitwise, and their decisions equal
    the oracle's (errors of at most 0.34 away from the rejection) with the
    state within the FP32 bound."""
    n, nu, kappa, ri = 64, 1e-3, 1e-3, 0.5
    announce("fp32 integrate 2d n=%d graph vs host vs oracle" % n)
    u0 = unit_speed(random2d(n, 17, 3), n)
    rhs = lambda x: spectral.rhs_ns2d(x, nu, kappa, ri)
    ref = control.integrate(rhs, u0, 0.5, 0.5, 1e-8, 1e-8)
    assert ref["n_reject"] >= 1
    out = []
    for graph in (True, False):
        s = ns.Solver(dim=2, n=n, nu=nu, rhs_precision="fp32", scalar=1, ri=ri, kappa=kappa)
        s.set_state(u0[None])
        st = s.integrate(0.5, 0.5, 1e-8, 1e-8, graph=graph)[0]
        out.append((st, s.get_state().cpu().numpy()[0]))
        s.close()
    (s1, u1), (s2, u2) = out
    assert (s1["n_accept"], s1["n_reject"], s1["n_rhs"]) == (s2["n_accept"], s2["n_reject"], s2["n_rhs"])
    assert np.array_equal(u1.view(np.float64), u2.view(np.float64))
    assert (s1["n_accept"], s1["n_reject"], s1["n_rhs"]) == (ref["n_accept"], ref["n_reject"], ref["n_rhs"])
    assert max(per_field_rel_l2(u1, ref["u"])) <= 1e-5


def test_fp32_2d_partial_acceptance_equals_single_runs(ns):
    """Host BS5 steps of a 2D FP32 batch in which one member accepts and the
    other rejects: the commit keeps each member's FP32 state copy and first
    stage, so every member stays bitwise equal to its own single run."""
    n, kappa, ri = 64, 1e-3, 0.5
    announce("2d fp32 host steps, partial acceptance == single n=%d" % n)
    ua = unit_speed(random2d(n, 21, 3), n)
    ub = 40.0 * unit_speed(random2d(n, 22, 3), n)
    nus = [1e-3, 2e-3]
    kw = dict(dim=2, n=n, rhs_precision="fp32", scalar=1, ri=ri, kappa=kappa)
    sb = ns.Solver(batch=2, nu=nus, **kw)
    sb.set_state(np.stack([ua, ub]))
    singles = []
    for u, nu in ((ua, nus[0]), (ub, nus[1])):
        s1 = ns.Solver(nu=nu, **kw)
        s1.set_state(u[None])
        singles.append(s1)
    mixed = 0
    for h in (0.05, 0.05, 0.02, 0.01, 0.01, 0.005, 0.005, 0.002, 0.002):
        _, eb = sb.step_bs5(h, 1e-6, 1e-6)
        for m, s1 in enumerate(singles):
            _, e1 = s1.step_bs5(h, 1e-6, 1e-6)
            assert eb[m] == e1[0] or (np.isnan(eb[m]) and np.isnan(e1[0]))
        mixed += (eb[0] <= 1.0) != (eb[1] <= 1.0)
    assert mixed >= 1
    ubatch = sb.get_state().cpu().numpy()
    for m, s1 in enumerate(singles):
        u1 = s1.get_state().cpu().numpy()[0]
        assert np.array_equal(u1.view(np.float64), ubatch[m].view(np.float64))
        s1.close()
    sb.close()
