"""GPU parity of the steppers (Sec. 2.2), the embedded error norm and
controller (Sec. 2.2.1) and the diagnostics (Sec. 3.1) against the oracle."""
import math

import numpy as np
import pytest

from gpu_util import announce, per_field_rel_l2
from oracle import control, diagnostics, spectral, stepping, tableaux
from paper_1810_10197_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ns():
    from paper_1810_10197_amd import ns as mod
    return mod


def mk(ns, n, prec, nu, batch=1):
    return ns.Solver(dim=3, n=n, batch=batch, nu=nu, rhs_precision=prec)


@pytest.mark.parametrize("n", [16, 32])
def test_rk4_steps_fp64(ns, n):
    announce("rk4 fp64 n=%d" % n)
    nu, h = 0.01, 0.05
    u0 = inputs.random_isotropic(n, 7)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    s = mk(ns, n, "fp64", nu)
    s.set_state(u0[None])
    ref = u0
    for _ in range(3):
        s.step_rk4(h)
        ref = stepping.rk4_step(rhs, ref, h)
    got = s.get_state().cpu().numpy()[0]
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    assert s.time()[0] == pytest.approx(3 * h)
    s.close()


@pytest.mark.parametrize("n,prec,tol", [(16, "fp64", 1e-13), (32, "fp64", 1e-13),
                                        (32, "fp32", 1e-6)])
def test_bs5_attempt_and_error(ns, n, prec, tol):
    """One BS5 attempt.  h = 0.1 keeps the embedded difference (~h^5) well
    above the FP32 rounding of the stage derivatives (~h), so the FP32 error
    estimate is compared at 1e-3; at h = 0.04 it is noise-dominated (~7%)."""
    announce("bs5 attempt n=%d %s" % (n, prec))
    nu, h, atol, rtol = 0.01, 0.1, 1e-7, 1e-7
    u0 = inputs.random_isotropic(n, 9)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    s = mk(ns, n, prec, nu)
    s.set_state(u0[None])
    st, errs = s.step_bs5(h, atol, rtol, force=True)
    ref = stepping.bs5_attempt(rhs, u0, h, atol, rtol)
    got = s.get_state().cpu().numpy()[0]
    assert max(per_field_rel_l2(got, ref["u_new"])) <= tol
    etol = 1e-9 if prec == "fp64" else 1e-3
    assert abs(errs[0] / ref["err"] - 1) <= etol, (errs[0], ref["err"])
    s.close()


@pytest.mark.parametrize("n,prec,tol", [(16, "fp64", 1e-13), (32, "fp32", 1e-6)])
def test_dp5_attempt_and_error(ns, n, prec, tol):
    """One DP5 attempt against the oracle's (same h as the BS5 test)."""
    announce("dp5 attempt n=%d %s" % (n, prec))
    nu, h, atol, rtol = 0.01, 0.1, 1e-7, 1e-7
    u0 = inputs.random_isotropic(n, 19)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    s = mk(ns, n, prec, nu)
    s.set_state(u0[None])
    st, errs = s.step_dp5(h, atol, rtol, force=True)
    ref = stepping.embedded_attempt(rhs, u0, h, atol, rtol, tableaux.DP5)
    got = s.get_state().cpu().numpy()[0]
    assert max(per_field_rel_l2(got, ref["u_new"])) <= tol
    etol = 1e-9 if prec == "fp64" else 1e-3
    assert abs(errs[0] / ref["err"] - 1) <= etol, (errs[0], ref["err"])
    s.close()


def test_dp5_linear_decay_closed_form(ns):
    """z-independent Taylor-Green field: f = -2 nu u, so three DP5 attempts
    multiply the state by R(-2 nu h)^3, R the pair's stability polynomial
    (Taylor through z^5 plus z^6/600)."""
    n, nu, h = 16, 0.05, 0.7
    announce("dp5 linear decay n=%d" % n)
    u0 = inputs.tgv2d_in3d(n)
    s = mk(ns, n, "fp64", nu)
    s.set_state(u0[None])
    for _ in range(3):
        s.step_dp5(h, 1e-6, 1e-6, force=True)
    got = s.get_state().cpu().numpy()[0]
    s.close()
    z = -2 * nu * h
    R = sum(z ** j / math.factorial(j) for j in range(6)) + z ** 6 / 600
    assert np.abs(got - R ** 3 * u0).max() <= 1e-14 * np.abs(u0).max()


def test_bs5_rejection_keeps_state(ns):
    n, nu = 16, 0.01
    announce("bs5 rejection n=%d" % n)
    u0 = inputs.random_isotropic(n, 4)
    s = mk(ns, n, "fp64", nu)
    s.set_state(u0[None])
    st, errs = s.step_bs5(0.5, 1e-12, 1e-12)
    assert st == ns.NS_STEP_REJECTED and errs[0] > 1
    got = s.get_state().cpu().numpy()[0]
    assert np.array_equal(got.view(np.float64), u0.view(np.float64))
    assert s.time()[0] == 0.0
    s.close()


def test_diagnostics_match_oracle(ns):
    n, nu = 32, 0.02
    announce("diagnostics n=%d" % n)
    u0 = inputs.random_isotropic(n, 12)
    s = mk(ns, n, "fp64", nu)
    s.set_state(u0[None])
    e, eps, sh = s.diagnostics()
    f = spectral.rhs_ns3d(u0, nu)
    assert e[0] == pytest.approx(diagnostics.energy(u0, 3), rel=1e-13)
    assert eps[0] == pytest.approx(diagnostics.dissipation(u0, f, 3), rel=1e-11)
    assert sh[0] == pytest.approx(diagnostics.shells(u0, 3), rel=1e-12, abs=1e-300)
    s.close()
    # Taylor--Green closed forms on the GPU too
    s = mk(ns, n, "fp32", 1.0 / 1600)
    s.set_state(inputs.tgv3d(n)[None])
    e, eps, _ = s.diagnostics()
    assert e[0] == pytest.approx(0.125, rel=1e-15)
    assert eps[0] == pytest.approx(0.75 / 1600, rel=1e-6)
    s.close()


def test_integrate_matches_oracle_controller(ns):
    """Adaptive BS5 with the Sec. 2.2.1 controller: same accepted/rejected
    sequence and the same final state as the oracle (FP64 RHS)."""
    n, nu = 16, 0.01
    announce("integrate n=%d fp64" % n)
    u0 = inputs.random_isotropic(n, 21)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    ref = control.integrate(rhs, u0, t_end=0.6, h0=0.3, atol=1e-8, rtol=1e-8)
    s = mk(ns, n, "fp64", nu)
    s.set_state(u0[None])
    stats = s.integrate(0.6, 0.3, 1e-8, 1e-8)[0]
    got = s.get_state().cpu().numpy()[0]
    assert stats["n_accept"] == ref["n_accept"]
    assert stats["n_reject"] == ref["n_reject"]
    assert stats["n_rhs"] == ref["n_rhs"]
    assert stats["t"] == 0.6
    assert np.abs(got - ref["u"]).max() <= 1e-12 * np.abs(ref["u"]).max()
    s.close()


def test_integrate_dp5_matches_oracle_controller(ns):
    """Adaptive DP5 (graph replay) with the Sec. 2.2.1 controller: same
    accepted/rejected sequence, right-hand-side count and final state as the
    oracle (FP64 RHS)."""
    n, nu = 16, 0.01
    announce("integrate dp5 n=%d fp64" % n)
    u0 = inputs.random_isotropic(n, 23)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    ref = control.integrate(rhs, u0, t_end=0.6, h0=0.3, atol=1e-8, rtol=1e-8, tab=tableaux.DP5)
    s = mk(ns, n, "fp64", nu)
    s.set_state(u0[None])
    stats = s.integrate(0.6, 0.3, 1e-8, 1e-8, method="dp5")[0]
    got = s.get_state().cpu().numpy()[0]
    assert (stats["n_accept"], stats["n_reject"], stats["n_rhs"]) == \
        (ref["n_accept"], ref["n_reject"], ref["n_rhs"])
    assert stats["t"] == 0.6
    assert np.abs(got - ref["u"]).max() <= 1e-12 * np.abs(ref["u"]).max()
    s.close()


def test_tgv_c1_fp64_rk4_and_bs5(ns):
    """3D TGV 32^3, nu = 1/1600, RK4 dt = 0.01 and adaptive BS5 at
    atol = rtol = 1e-8 to T = 1, FP64 throughout; every velocity component
    (w, zero at t = 0, holds about 30% of the norm of u at T = 1)."""
    n, nu = 32, 1.0 / 1600
    announce("tgv 32^3 rk4+bs5 to T=1")
    u0 = inputs.tgv3d(n)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    ref_rk4, nsteps = control.rk4_fixed(rhs, u0, 1.0, 0.01)
    s = mk(ns, n, "fp64", nu)
    s.set_state(u0[None])
    for _ in range(nsteps):
        s.step_rk4(0.01)
    got = s.get_state().cpu().numpy()[0]
    assert max(per_field_rel_l2(got, ref_rk4)) <= 1e-12
    s.close()
    ref = control.integrate(rhs, u0, 1.0, 0.01, 1e-8, 1e-8)
    s = mk(ns, n, "fp64", nu)
    s.set_state(u0[None])
    stats = s.integrate(1.0, 0.01, 1e-8, 1e-8)[0]
    got = s.get_state().cpu().numpy()[0]
    assert (stats["n_accept"], stats["n_reject"]) == (ref["n_accept"], ref["n_reject"])
    assert max(per_field_rel_l2(got, ref["u"])) <= 1e-12
    s.close()


def test_bs5_attempts_256_full_size_autotuned(ns):
    """Two BS5 attempts at 256^3 with an FP32 right-hand side, in the launch
    configuration the throughput benchmark times (autotuned passes, the host
    step path, FSAL k1 and FP32 stage-derivative copies on the second
    attempt), against the oracle's FP64 attempts on a field that fills the
    2/3-rule band.  The embedded estimate carries the FP32 rounding of the
    stage derivatives, about h * sum|b - b^| * 1e-6 * |k| per mode, at most a
    few percent of the difference per mode at this h; being uncorrelated with
    it, that noise moves the root-mean-square norm by about half its squared
    ratio (< 5e-4), so the estimate is compared at 1e-3."""
    n, nu, h, tol = 256, 1.0 / 1600, 0.02, 1e-6
    announce("bs5 attempts full n=%d fp32 autotuned" % n)
    u0 = inputs.random_isotropic(n, 1810, k0=n / 8.0)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    s = mk(ns, n, "fp32", nu)
    s.set_state(u0[None])
    s.autotune(reps=1)
    ref1 = stepping.bs5_attempt(rhs, u0, h, tol, tol)
    ref2 = stepping.bs5_attempt(rhs, ref1["u_new"], h, tol, tol, k1=ref1["k"][-1])
    for ref in (ref1, ref2):
        st, errs = s.step_bs5(h, tol, tol)
        assert st == ns.NS_OK
        got = s.get_state().cpu().numpy()[0]
        e = per_field_rel_l2(got, ref["u_new"])
        print("u_new rel L2", e, "err", errs[0], "oracle", ref["err"])
        assert max(e) <= 1e-6, e
        assert abs(errs[0] / ref["err"] - 1) <= 1e-3, (errs[0], ref["err"])
    s.close()


def test_fp32_rhs_against_fp64_tgv256_to_t1(ns):
    """Mixed precision at full size: the 256^3 Taylor-Green vortex to T = 1
    with an FP32 right-hand side stays within 1e-5 per-field relative L2 of
    the FP64 path, for RK4 and for BS5, both at the fixed step 0.01 (the same
    steps for both precisions; two adaptive runs would also differ by their
    own step sequences, and the Sec. 2.2.1 norm averages over every
    half-spectrum entry, so for a field whose energy sits in a few modes it
    lets those modes carry errors far above the tolerance)."""
    n, nu, T = 256, 1.0 / 1600, 1.0
    announce("fp32 vs fp64 tgv %d^3 to T=1" % n)
    u0 = inputs.tgv3d(n)[None]
    rk4, bs5 = {}, {}
    for prec in ("fp64", "fp32"):
        s = mk(ns, n, prec, nu)
        s.set_state(u0)
        for _ in range(100):
            s.step_rk4(0.01)
        rk4[prec] = s.get_state().cpu().numpy()[0]
        s.set_state(u0)
        for _ in range(100):
            s.step_bs5(0.01, 1e-8, 1e-8, force=True)
        bs5[prec] = s.get_state().cpu().numpy()[0]
        s.close()
    e_rk4 = per_field_rel_l2(rk4["fp32"], rk4["fp64"])
    e_bs5 = per_field_rel_l2(bs5["fp32"], bs5["fp64"])
    print("per-field rel L2 (u, v, w): RK4", e_rk4, "BS5", e_bs5)
    assert max(e_rk4) <= 1e-5, e_rk4
    assert max(e_bs5) <= 1e-5, e_bs5


def test_fp32_rhs_against_oracle_tgv64_to_t1(ns):
    """Mixed precision against the FP64 oracle itself: the 64^3 Taylor-Green
    vortex (nu = 1/1600) to T = 1 with RK4 and with fixed-step BS5 at
    dt = 0.01, FP32 right-hand side and FP64 state on the GPU, the oracle's
    FP64 trajectory on the CPU; per-field relative L2 (u, v, w) <= 1e-5."""
    n, nu, T, dt = 64, 1.0 / 1600, 1.0, 0.01
    announce("fp32 vs oracle tgv %d^3 to T=1" % n)
    u0 = inputs.tgv3d(n)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    ref_rk4, steps = control.rk4_fixed(rhs, u0, T, dt)
    ref_bs5, _ = control.fixed_steps(rhs, u0, [dt] * steps)
    s = mk(ns, n, "fp32", nu)
    s.set_state(u0[None])
    for _ in range(steps):
        s.step_rk4(dt)
    got_rk4 = s.get_state().cpu().numpy()[0]
    s.set_state(u0[None])
    for _ in range(steps):
        s.step_bs5(dt, 1e-8, 1e-8, force=True)
    got_bs5 = s.get_state().cpu().numpy()[0]
    s.close()
    e_rk4 = per_field_rel_l2(got_rk4, ref_rk4)
    e_bs5 = per_field_rel_l2(got_bs5, ref_bs5)
    print("per-field rel L2 vs oracle (u, v, w): RK4", e_rk4, "BS5", e_bs5)
    assert max(e_rk4) <= 1e-5, e_rk4
    assert max(e_bs5) <= 1e-5, e_bs5
