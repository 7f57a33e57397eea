"""Kinetic energy, dissipation rate and shell spectrum (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3.1 defines the kinetic energy per unit volume from the spectral
velocity and its dissipation rate epsilon = -dE/dt, evaluated in spectral
space by reusing f(u_hat) = d u_hat/dt.  The paper adjusts the sums for the
zero and Nyquist planes of the real DFT; with the half spectrum every entry
off those planes stands for itself and its conjugate twin, so it carries
weight 2, and entries on the kx = 0 and kx = N/2 planes carry weight 1.
Under the normalised convention (u_hat = DFT/N^d):

    E   = 1/2 sum_k w_k |u_hat_k|^2
    eps = - sum_k w_k Re( conj(u_hat_k) . f_k )

Both sums run over the velocity components only (the density of the
Boussinesq system is excluded).  The 16-bin shell spectrum (a feature of the
step-size proposer) sums 1/2 w |u_hat|^2 over modes with
floor(16 |k| / K) = b, the last bin also collecting |k| >= K.
"""
import numpy as np

from .spectral import cutoff, wavenumbers


def weights(n, dim):
    """Half-spectrum multiplicity w (1 on the kx = 0, N/2 planes, else 2)."""
    shape = (n,) * (dim - 1) + (n // 2 + 1,)
    w = np.full(shape, 2.0)
    w[..., 0] = 1.0
    w[..., n // 2] = 1.0
    return w


def _velocity(uh, dim):
    return uh[:dim]


def energy(uh, dim):
    n = uh.shape[1]
    w = weights(n, dim)
    return 0.5 * float(np.sum(w * np.sum(np.abs(_velocity(uh, dim)) ** 2, axis=0)))


def dissipation(uh, f, dim):
    n = uh.shape[1]
    w = weights(n, dim)
    return -float(np.sum(w * np.sum(np.real(np.conj(_velocity(uh, dim)) *
                                            _velocity(f, dim)), axis=0)))


def shell_index(n, dim, nbins=16):
    ks = wavenumbers(n, dim)
    k2 = sum(k * k for k in ks)
    kmag = np.sqrt(k2)
    K = cutoff(n)
    b = np.floor(nbins * kmag / K).astype(np.int64)
    return np.minimum(b, nbins - 1)


def shells(uh, dim, nbins=16):
    n = uh.shape[1]
    w = weights(n, dim)
    e = 0.5 * w * np.sum(np.abs(_velocity(uh, dim)) ** 2, axis=0)
    idx = np.broadcast_to(shell_index(n, dim, nbins), e.shape)
    out = np.zeros(nbins)
    np.add.at(out, idx.ravel(), e.ravel())
    return out
