"""Pins of the oracle's step-size controller (Sec. 2.2.1) on scripted error
sequences whose factors were worked out by hand."""
import math

import numpy as np
import pytest

from oracle import control, spectral, stepping, tableaux
from paper_1810_10197_amd import inputs


def test_factor_hand_values():
    c = control.Controller(q=4)
    # 0.8 * err^(-1/5), clamped to [0.01, 2]
    assert c.factor(0.5, 1.0, False) == pytest.approx(0.918959, rel=1e-6)
    assert c.factor(40.0, 1.0, False) == pytest.approx(0.382541, rel=1e-5)
    assert c.factor(1e-12, 1.0, False) == 2.0
    assert c.factor(1e12, 1.0, False) == 0.01
    assert c.factor(0.0, 1.0, False) == 2.0
    assert c.factor(0.0, 1.0, True) == 1.0
    assert c.factor(0.2, 1.0, True) == 1.0          # 1.10378 capped at 1
    assert c.factor(0.9, 1.0, True) == pytest.approx(0.817036, rel=1e-5)
    assert c.factor(float("nan"), 1.0, False) == 0.01
    assert c.factor(float("inf"), 1.0, False) == 0.01
    # q = 4 means exponent 1/5: err = 32 gives exactly 0.8 / 2
    assert c.factor(32.0, 1.0, False) == pytest.approx(0.4, rel=1e-15)


class Scripted:
    def __init__(self, errs):
        self.errs = list(errs)
        self.calls = []

    def __call__(self, rhs, u, h, atol, rtol, tab, k1=None):
        self.calls.append(h)
        err = self.errs.pop(0)
        ks = [u.copy() for _ in tab["b"]]
        return {"u_new": u + 1.0, "delta": u * 0, "err": err, "errs": None, "k": ks}


def test_scripted_integration(monkeypatch):
    script = Scripted([0.5, 40.0, 20.0, 0.9, 1e-12, 0.0, float("nan"), 0.2] + [0.01] * 200)
    monkeypatch.setattr(stepping, "embedded_attempt", script)
    u0 = np.zeros(3)
    out = control.integrate(None, u0, t_end=10.0, h0=0.1, atol=1, rtol=1)
    hs = script.calls[:9]
    expect = [0.1]
    expect.append(expect[-1] * 0.918959)     # accepted, err 0.5
    expect.append(expect[-1] * 0.382541)     # rejected, err 40
    expect.append(expect[-1] * 0.439425)     # rejected, err 20
    expect.append(expect[-1] * 0.817036)     # accepted after rejection, err 0.9
    expect.append(expect[-1] * 2.0)          # err 1e-12: clamp at 2
    expect.append(expect[-1] * 2.0)          # err 0: dmax
    expect.append(expect[-1] * 0.01)         # NaN: rejected with dmin
    expect.append(expect[-1] * 1.0)          # err 0.2 after rejection: capped at 1
    assert hs == pytest.approx(expect[:9], rel=2e-5)
    hist = out["history"]
    assert [a for (_, _, _, a) in hist[:9]] == [True, False, False, True, True, True,
                                                False, True, True]


def test_clipping_lands_on_t_end(monkeypatch):
    script = Scripted([0.01] * 50)
    monkeypatch.setattr(stepping, "embedded_attempt", script)
    out = control.integrate(None, np.zeros(2), t_end=1.0, h0=0.3, atol=1, rtol=1)
    assert out["t"] == 1.0
    # 0.3, then 0.6 would overshoot (0.3 + 0.6 < 1 ok), then clipped to 0.1
    assert script.calls[:3] == pytest.approx([0.3, 0.6, 0.1])
    assert out["n_accept"] == 3


def test_proposer_is_bounded_by_controller_factor(monkeypatch):
    """After an accepted step the proposal exp(y) is clamped to
    [0.7 fac, fac] around the controller's factor fac."""
    # err 0.5 -> fac 0.918959; err 40 rejects (fac 0.382541); err 0.9 after
    # the rejection -> fac 0.817036 (dmax = 1); err 1e-12 -> fac 2
    script = Scripted([0.5, 0.5, 40.0, 0.9, 1e-12, 1e-12] + [1e-12] * 200)
    monkeypatch.setattr(stepping, "embedded_attempt", script)
    ys = iter([-5.0, 5.0, 5.0, -5.0, 0.5] + [0.0] * 200)
    control.integrate(None, np.zeros(2), t_end=1.0, h0=0.1, atol=1, rtol=1,
                      proposer=lambda u, h, e: next(ys))
    f05, f40, f09 = 0.918959, 0.382541, 0.817036
    expect = [0.1]
    expect.append(expect[-1] * 0.7 * f05)          # y = -5 -> lower bound 0.7 fac
    expect.append(expect[-1] * f05)                # y = +5 -> upper bound fac
    expect.append(expect[-1] * f40)                # rejection: controller only
    expect.append(expect[-1] * f09)                # y = +5 after rejection: fac (dmax 1)
    expect.append(expect[-1] * 1.4)                # y = -5, fac 2: 0.7 fac = 1.4 (can grow)
    expect.append(expect[-1] * math.exp(0.5))      # inside the bounds: exp(y)
    assert script.calls[:7] == pytest.approx(expect, rel=2e-5)


def test_consecutive_rejections_fail(monkeypatch):
    script = Scripted([1e6] * 60)
    monkeypatch.setattr(stepping, "embedded_attempt", script)
    with pytest.raises(control.StepFailure):
        control.integrate(None, np.zeros(2), t_end=1.0, h0=0.3, atol=1, rtol=1)
    assert len(script.calls) == 50


def test_adaptive_run_on_linear_problem_is_scalar_recursion():
    """2D TGV: f = -2 nu u, so every attempt's err has a closed form in h
    and the whole accepted/rejected sequence follows a scalar recursion."""
    from test_oracle_stepping import D_BS5, R_BS5, peval
    n, nu = 8, 0.2
    u0 = inputs.tgv2d_in3d(n)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    atol = rtol = 1e-9
    out = control.integrate(rhs, u0, t_end=3.0, h0=1.0, atol=atol, rtol=rtol)
    m = n * n * (n // 2 + 1)
    amp = 0.25
    t, h, prev_rej = 0.0, 1.0, False
    for (tt, hh, err, acc) in out["history"]:
        assert tt == pytest.approx(t, rel=1e-9)
        assert hh == pytest.approx(min(h, 3.0 - t), rel=1e-5)
        hc = hh
        z = -2 * nu * hc
        R, D = peval(R_BS5, z), peval(D_BS5, z)
        e = math.sqrt(2 * (abs(D) * amp / (atol + rtol * amp)) ** 2 / m)
        # the stage sum of the embedded difference cancels ~7 digits here
        assert err == pytest.approx(e, rel=1e-4)
        ok = e <= 1.0
        assert acc == ok
        fac = 0.8 * e ** -0.2
        fac = min(1.0 if (ok and prev_rej) else 2.0, max(0.01, fac))
        if ok:
            t += hc
            amp *= R
        prev_rej = not ok
        h = hc * fac
    assert out["n_reject"] >= 1     # the h0 = 1 start is too large for 1e-9
    assert out["n_rhs"] == 1 + 7 * len(out["history"])
