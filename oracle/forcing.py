"""Deterministic low-wavenumber forcing for homogeneous isotropic turbulence.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3.3.1: after every (accepted) time step the modes with 0 < |k| <= k_f
are rescaled by one common factor so that the energy lost to dissipation is
replaced.  Read here as holding the total kinetic energy at E0: with E the
total and E_f the energy inside the forcing band,

    alpha = sqrt( max(E0 - (E - E_f), 0) / E_f ),   u_hat <- alpha u_hat on the band.

The forcing sits outside the right-hand side and outside the error estimate.
"""
import numpy as np

from .diagnostics import energy, weights
from .spectral import wavenumbers


def band(n, kf):
    kx, ky, kz = wavenumbers(n, 3)
    k2 = kx * kx + ky * ky + kz * kz
    return (k2 > 0) & (k2 <= kf * kf)


def force(uh, kf, e0):
    n = uh.shape[1]
    b = band(n, kf)
    w = weights(n, 3)
    e_band = 0.5 * float(np.sum((w * b) * np.sum(np.abs(uh[:3]) ** 2, axis=0)))
    e_tot = energy(uh, 3)
    if e_band <= 0.0:
        return uh.copy()
    alpha = np.sqrt(max(e0 - (e_tot - e_band), 0.0) / e_band)
    out = uh.copy()
    out[:, b] *= alpha
    return out
