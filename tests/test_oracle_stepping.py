"""Pins of the oracle's RK4 / BS5 steppers and the embedded error norm
(Sec. 2.2, 2.2.1; Appendix A.3) against closed forms and convergence rates."""
from fractions import Fraction as F
from math import factorial

import numpy as np
import pytest

from oracle import control, diagnostics, spectral, stepping, tableaux
from paper_1810_10197_amd import inputs

# Stability polynomials of the pair written out (exact rationals): the
# b solution is the Taylor polynomial through z^5 plus two tail terms, the
# b_hat solution through z^4 plus four.
R_BS5 = [F(1, factorial(j)) for j in range(6)] + [F(17291, 12418560), F(269, 1379840)]
RH_BS5 = [F(1, factorial(j)) for j in range(5)] + [
    F(269672, 32164209), F(2349047, 1715424480), F(1309661503, 6916591503360),
    F(885817, 768510167040)]
R_RK4 = [F(1, factorial(j)) for j in range(5)]
# R - R_hat as one polynomial, so that its value keeps full relative accuracy
D_BS5 = [a - b for a, b in zip(R_BS5 + [F(0)], RH_BS5)]
# DP5 (Appendix A.1): the b solution's stability polynomial is the Taylor
# polynomial through z^5 plus z^6/600 (the published value for this pair).
R_DP5 = [F(1, factorial(j)) for j in range(6)] + [F(1, 600)]


def peval(c, z):
    return sum(float(ci) * z ** j for j, ci in enumerate(c))


@pytest.mark.parametrize("h", [0.3, 1.0])
def test_linear_tgv_rk4_and_bs5_closed_form(h):
    """On the 2D TGV f = -2 nu u exactly, so each step multiplies the state
    by R(-2 nu h) and the embedded difference is (R - R_hat) u_n."""
    n, nu = 8, 0.05
    u0 = inputs.tgv2d_in3d(n)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    z = -2 * nu * h
    u = u0.copy()
    for step in range(3):
        u = stepping.rk4_step(rhs, u, h)
        assert np.abs(u - peval(R_RK4, z) ** (step + 1) * u0).max() < 1e-15
    atol, rtol = 1e-7, 1e-5
    u = u0.copy()
    for step in range(3):
        res = stepping.bs5_attempt(rhs, u, h, atol, rtol)
        R, D = peval(R_BS5, z), peval(D_BS5, z)
        assert np.abs(res["u_new"] - R * u).max() < 1e-15
        assert np.abs(res["delta"] - D * u).max() < 1e-6 * abs(D) * np.abs(u).max()
        # err in closed form: 2 equal-modulus modes per velocity component
        # (kx = 1, ky = +-1, kz = 0), w identically zero, M = N^2 (N/2+1)
        amp = np.abs(u[0]).max()
        sc = atol + rtol * amp * max(1.0, abs(R))
        m = n * n * (n // 2 + 1)
        expect = np.sqrt(2 * (abs(D) * amp / sc) ** 2 / m)
        assert abs(res["err"] - expect) < 1e-6 * expect
        assert res["errs"][2] == 0.0
        u = res["u_new"]


@pytest.mark.parametrize("h", [0.3, 1.0])
def test_linear_tgv_dp5_closed_form(h):
    """DP5 on the 2D TGV: each attempt multiplies the state by R_DP5(-2 nu h);
    the last stage is f(u_{n+1}) (FSAL)."""
    n, nu = 8, 0.05
    u0 = inputs.tgv2d_in3d(n)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    z = -2 * nu * h
    u = u0.copy()
    for step in range(3):
        res = stepping.embedded_attempt(rhs, u, h, 1e-7, 1e-5, tableaux.DP5)
        assert np.abs(res["u_new"] - peval(R_DP5, z) * u).max() < 1e-15
        assert np.abs(res["k"][-1] - (-2 * nu) * res["u_new"]).max() < 1e-15
        u = res["u_new"]


def test_error_norm_definition_by_hand():
    """err_j on a tiny hand-made array, every number computed by hand."""
    u_old = np.zeros((3, 2, 2), dtype=complex)
    u_new = np.zeros((3, 2, 2), dtype=complex)
    delta = np.zeros((3, 2, 2), dtype=complex)
    u_old[0, 0, 0] = 3 + 4j          # |.| = 5
    u_new[0, 0, 0] = 1.0
    delta[0, 0, 0] = 0.6j
    delta[1, 1, 1] = -0.2            # sc = atol there
    err, errs = stepping.error_norm(u_old, u_new, delta, atol=0.1, rtol=0.1)
    # comp 0: sc = 0.1 + 0.1*5 = 0.6 -> |0.6j/0.6|^2 = 1 over M = 4 -> 0.5
    # comp 1: sc = 0.1 -> |0.2/0.1|^2 = 4 over 4 -> 1.0
    assert errs == pytest.approx([0.5, 1.0, 0.0], abs=1e-15)
    assert err == pytest.approx(1.0, abs=1e-15)


def _tgv_problem():
    n, nu = 16, 0.01
    u0 = inputs.tgv3d(n)
    return u0, (lambda u: spectral.rhs_ns3d(u, nu))


@pytest.mark.slow
def test_convergence_orders_tgv():
    """Halving h cuts the error by ~2^4 (RK4) and ~2^5 (fixed-step BS5)."""
    u0, rhs = _tgv_problem()
    T = 1.0
    ref, _ = control.fixed_steps(rhs, u0, [0.01] * 100)
    e4, e5 = [], []
    for h in [0.2, 0.1, 0.05]:
        u4, _ = control.rk4_fixed(rhs, u0, T, h)
        u5, _ = control.fixed_steps(rhs, u0, [h] * int(round(T / h)))
        e4.append(np.abs(u4 - ref).max())
        e5.append(np.abs(u5 - ref).max())
    s4 = np.log2(np.array(e4[:-1]) / np.array(e4[1:]))
    s5 = np.log2(np.array(e5[:-1]) / np.array(e5[1:]))
    assert np.all(s4 > 3.6) and s4[-1] > 3.85 and np.all(s4 < 4.3)
    assert np.all(s5 > 4.8) and np.all(s5 < 6.5)


@pytest.mark.slow
def test_inviscid_energy_drift_shrinks_with_order():
    n = 16
    r = inputs.random_isotropic(n, 5)
    rhs0 = lambda u: spectral.rhs_ns3d(u, 0.0)
    E0 = diagnostics.energy(r, 3)
    d4, d5 = [], []
    for h in [0.2, 0.1, 0.05]:
        u4, _ = control.rk4_fixed(rhs0, r, 0.8, h)
        u5, _ = control.fixed_steps(rhs0, r, [h] * int(round(0.8 / h)))
        d4.append(abs(diagnostics.energy(u4, 3) - E0))
        d5.append(abs(diagnostics.energy(u5, 3) - E0))
    for d in (d4, d5):
        s = np.log2(np.array(d[:-1]) / np.array(d[1:]))
        assert np.all(s >= 4.0), s


def test_local_error_estimate_scales_as_h5():
    """The embedded difference of BS5 is O(h^5) on a nonlinear flow."""
    u0, rhs = _tgv_problem()
    d = []
    for h in [0.2, 0.1]:
        res = stepping.bs5_attempt(rhs, u0, h, 1.0, 0.0)
        d.append(np.abs(res["delta"]).max())
    assert 4.6 < np.log2(d[0] / d[1]) < 5.6


@pytest.mark.parametrize("t_end,h,steps,last", [(0.37, 0.1, 4, 0.07), (0.3, 0.1, 3, 0.1),
                                                (0.05, 0.1, 1, 0.05)])
def test_rk4_fixed_clips_the_last_step(t_end, h, steps, last):
    """Fixed-step RK4 to a t_end that is not a multiple of h: ceil(t_end/h)
    steps, the last one shortened to land on t_end.  On the 2D TGV every step
    multiplies the state by R_RK4(-2 nu h), so the end state is
    R(-2 nu h)^(steps-1) R(-2 nu last) u0 exactly."""
    n, nu = 8, 0.5
    u0 = inputs.tgv2d_in3d(n)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    u, count = control.rk4_fixed(rhs, u0, t_end, h)
    assert count == steps
    expect = peval(R_RK4, -2 * nu * h) ** (steps - 1) * peval(R_RK4, -2 * nu * last) * u0
    assert np.abs(u - expect).max() < 1e-15
