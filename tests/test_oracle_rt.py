"""Physical sanity pin of the oracle's 2D Boussinesq right-hand side
(Sec. 3.2, Eqs. (3a-c), (4a-b); the Rayleigh--Taylor workload): the sign and
direction of the buoyancy term.

A heavy layer (rho = +1) above a light one (rho = -1), interface displaced by
eta0 cos(4x) and the fluid at rest: linear theory for a sharp interface with
buoyancy -Ri rho e_y gives sigma^2 = Ri k (a density jump of 2 Ri; with
Ri = A g this is the classical A g k), and starting from rest the displacement
grows as eta0 cosh(sigma t).  The (kx = 4, ky = 0) coefficient of rho is the
y-average of rho at that x-wavenumber, which for a thin interface is
eta_4 / pi: its growth measures sigma without resolving the profile.  Finite
thickness (here the band-limited representation of the tanh) and diffusion
only lower sigma, by a few percent at N = 128 (+-15% is allowed)."""
import numpy as np
import pytest

from oracle import spectral, stepping
from paper_1810_10197_amd import inputs


def growth_rate(n, ri, t_end, dt=0.01, amp=0.01, nu=1e-4, kappa=1e-4):
    u = inputs.rayleigh_taylor2d(n, amp=amp)
    rhs = lambda x: spectral.rhs_ns2d(x, nu, kappa, ri)
    a0 = u[2, 0, 4].real
    ratios = []
    steps = int(round(t_end / dt))
    for i in range(steps):
        u = stepping.rk4_step(rhs, u, dt)
        if (i + 1) % (steps // 2) == 0:
            ratios.append(((i + 1) * dt, u[2, 0, 4].real / a0))
    return ratios


def test_mode4_grows_at_the_linear_rate():
    ri, k = 0.5, 4
    sigma = np.sqrt(ri * k)                      # 1.414...
    out = growth_rate(128, ri, 0.6)
    rates = []
    for t, r in out:
        assert r > 1.0, "mode 4 of the unstable interface must grow"
        rates.append(np.arccosh(r) / t)
    # cosh(sigma t) from rest: the same rate at both times (linear regime)
    assert abs(rates[0] - rates[1]) < 0.01 * sigma
    assert abs(rates[1] - sigma) < 0.15 * sigma, (rates, sigma)


def test_stable_stratification_does_not_grow():
    """Buoyancy of the opposite sign (light fluid on top) turns the
    interface into a stable one: the mode oscillates instead of growing."""
    out = growth_rate(64, -0.5, 0.6)
    assert all(r < 1.0 for _, r in out)
