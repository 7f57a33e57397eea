"""Pins of the oracle's diagnostics (Sec. 3.1 energy; the 16-bin shell
spectrum used as proposer features): hand-built single-mode fields whose bin
and energy are known by hand, and the kinetic energy against the mean of
|u|^2 on the physical grid (Parseval, no half-spectrum weights involved)."""
import numpy as np
import pytest

from oracle import diagnostics, spectral
from paper_1810_10197_amd import inputs


def _single_mode(n, k, amp):
    """Real velocity field with one Fourier pair +-k (kx >= 0), component 0
    scaled by amp; on the kx = 0 plane the conjugate twin is stored too."""
    kx, ky, kz = k
    u = np.zeros((3, n, n, n // 2 + 1), dtype=np.complex128)
    u[0, kz % n, ky % n, kx] = amp
    if kx == 0:
        u[0, (-kz) % n, (-ky) % n, 0] = np.conj(amp)
    return u


# (k, expected bin) at n = 32 (K = 10): bin = floor(16 |k| / 10), capped at 15
CASES = [((1, 0, 0), 1),              # |k| = 1    -> 1.6
         ((0, 3, 4), 8),              # |k| = 5    -> 8.0 exactly (kx = 0 plane)
         ((6, 0, 0), 9),              # |k| = 6    -> 9.6
         ((2, -2, 1), 4),             # |k| = 3    -> 4.8
         ((0, 0, -1), 1),             # kx = 0 plane, negative kz
         ((6, 6, 3), 14),             # |k| = 9    -> 14.4
         ((10, 10, 10), 15),          # |k| = 17.3 >= K: overflow into the last bin
         ((7, -7, 0), 15)]            # |k| = 9.9  -> 15.8


@pytest.mark.parametrize("k,b", CASES)
def test_single_mode_lands_in_its_bin(k, b):
    n, amp = 32, 0.3 - 0.4j
    kmag = np.sqrt(sum(c * c for c in k))
    assert min(int(np.floor(16 * kmag / 10)), 15) == b
    expect_bin = b
    u = _single_mode(n, k, amp)
    sh = diagnostics.shells(u, 3)
    # physical-space energy of the real field: 1/2 <|u|^2>
    phys = spectral.inverse(u, n, 3)
    e_phys = 0.5 * float(np.mean(np.sum(phys * phys, axis=0)))
    # a single pair +-k with coefficient amp carries |amp|^2 of <u^2>
    assert e_phys == pytest.approx(abs(amp) ** 2, rel=1e-13)
    assert sh[expect_bin] == pytest.approx(e_phys, rel=1e-13)
    assert np.count_nonzero(sh) == 1
    assert sh.sum() == pytest.approx(diagnostics.energy(u, 3), rel=1e-14)


def test_bins_are_relative_to_the_cutoff():
    """The same integer mode sits in different bins at different N (bins
    scale with K = (N-1)//3, not with N/2)."""
    k = (0, 3, 4)                           # |k| = 5
    for n, b in [(32, 8), (64, 3), (16, 15)]:   # K = 10, 21, 5
        sh = diagnostics.shells(_single_mode(n, k, 1.0), 3)
        assert np.argmax(sh) == b and np.count_nonzero(sh) == 1, (n, sh)


@pytest.mark.parametrize("n,seed", [(16, 3), (24, 11)])
def test_energy_and_shells_against_physical_space(n, seed):
    u = inputs.random_isotropic(n, seed)
    phys = spectral.inverse(u, n, 3)
    e_phys = 0.5 * float(np.mean(np.sum(phys * phys, axis=0)))
    assert diagnostics.energy(u, 3) == pytest.approx(e_phys, rel=1e-13)
    sh = diagnostics.shells(u, 3)
    assert sh.sum() == pytest.approx(e_phys, rel=1e-13)
    # a shell's energy equals the physical energy of the field restricted to it
    idx = diagnostics.shell_index(n, 3)
    for b in (1, 4, 15):
        part = np.where(idx == b, u, 0.0)
        pp = spectral.inverse(part, n, 3)
        assert sh[b] == pytest.approx(0.5 * float(np.mean(np.sum(pp * pp, axis=0))), rel=1e-12, abs=1e-18)


def test_dissipation_against_physical_gradients():
    """eps = nu <|grad u|^2> for the viscous part: with the nonlinear term
    removed (f = -nu |k|^2 u_hat) the spectral sum equals nu times the mean
    squared velocity gradient on the grid."""
    n, nu = 16, 0.01
    u = inputs.random_isotropic(n, 21)
    kx, ky, kz = spectral.wavenumbers(n, 3)
    f = -nu * (kx * kx + ky * ky + kz * kz) * u
    g = 0.0
    for k in (kx, ky, kz):
        d = spectral.inverse(1j * k * u, n, 3)
        g += float(np.mean(np.sum(d * d, axis=0)))
    assert diagnostics.dissipation(u, f, 3) == pytest.approx(nu * g, rel=1e-13)
