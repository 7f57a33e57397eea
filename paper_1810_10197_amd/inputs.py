"""Seeded synthetic initial fields, shared by the tests, the benchmark and the
oracle-side checks.

This module holds no arithmetic of the time integrator or of the right-hand
side: it only builds initial states in the half-spectrum layout of the C ABI,
complex128 arrays of shape (3, N, N, N//2+1) in 3D ([kz][ky][kx], kx = 0..N/2)
and (C, N, N//2+1) in 2D ([ky][kx]), normalised so that physical values are
sum_k u_hat_k exp(i k.x).  Only modes with every |k_j| <= (N-1)//3 are
populated (random fields take a wider band on request: |k_j| <= N/2 - 1 is
the retained set of the 3/2 rule).

* Taylor--Green vortex (Sec. 3.1): u = sin x cos y cos z,
  v = -cos x sin y cos z, w = 0 -- written from its eight Fourier
  coefficients (+-i/8), no transform involved.
* 2D Taylor--Green (a test field): u = sin x cos y, v = -cos x sin y.
* Random-phase isotropic field (Sec. 3.3, spectrum of the forced-HIT
  workload): for every retained mode a vector of unit-modulus random phases
  times A(|k|) = |k| exp(-(|k|/k0)^2), made solenoidal by taking k_unit x a
  (so k . u_hat = 0 by construction, no projection), Hermitian on the kx = 0
  plane, scaled so that half the mean of |u|^2 over the physical grid is E0.
* Rayleigh--Taylor (Sec. 3.2, 2D workload): u = v = 0 and
  rho = tanh((y - pi + 0.05 cos 4x)/0.02) sampled on the grid, transformed
  with numpy.fft and restricted to the retained modes.

Random numbers come from numpy's PCG64 with the seed given.
"""
import numpy as np


def cutoff(n):
    return (n - 1) // 3


def _kidx(n, K=None):
    """Signed retained wavenumbers and their storage index on a full axis."""
    K = cutoff(n) if K is None else K
    ks = np.arange(-K, K + 1)
    return ks, ks % n


def tgv3d(n):
    if n < 4:
        raise ValueError("n >= 4 required")
    u = np.zeros((3, n, n, n // 2 + 1), dtype=np.complex128)
    for sy in (1, -1):
        for sz in (1, -1):
            iz, iy = sz % n, sy % n
            u[0, iz, iy, 1] = -1j / 8.0
            u[1, iz, iy, 1] = 1j * sy / 8.0
    return u


def tgv2d_in3d(n):
    """z-independent 2D Taylor--Green as a 3D field (w = 0)."""
    u = np.zeros((3, n, n, n // 2 + 1), dtype=np.complex128)
    for sy in (1, -1):
        iy = sy % n
        u[0, 0, iy, 1] = -1j / 4.0
        u[1, 0, iy, 1] = 1j * sy / 4.0
    return u


def tgv2d(n, with_density=False):
    c = 3 if with_density else 2
    u = np.zeros((c, n, n // 2 + 1), dtype=np.complex128)
    for sy in (1, -1):
        iy = sy % n
        u[0, iy, 1] = -1j / 4.0
        u[1, iy, 1] = 1j * sy / 4.0
    return u


def _hermitian_kx0(a, n, K=None):
    """Make the kx = 0 plane of a (C, N, N, h) field Hermitian:
    a(0, -ky, -kz) = conj(a(0, ky, kz)), a(0,0,0) = 0.  The canonical half is
    ky > 0, or ky = 0 and kz > 0."""
    ks, idx = _kidx(n, K)
    for ky, iy in zip(ks, idx):
        for kz, iz in zip(ks, idx):
            if ky > 0 or (ky == 0 and kz > 0):
                a[:, (-kz) % n, (-ky) % n, 0] = np.conj(a[:, iz, iy, 0])
    a[:, 0, 0, 0] = 0.0
    return a


def _energy_scale(u, e0):
    """Scale u so that half the mean of |u|^2 over the physical grid is e0
    (the field is synthesised in physical space by numpy's inverse FFT)."""
    n = u.shape[1]
    phys = np.fft.irfftn(u * float(n) ** 3, s=(n, n, n), axes=(1, 2, 3))
    e = 0.5 * float(np.mean(np.sum(phys * phys, axis=0)))
    return u * np.sqrt(e0 / e)


def random_isotropic(n, seed, k0=3.0, e0=0.125, band=None):
    """Random-phase solenoidal field with shell energy ~ k^4 exp(-2 (k/k0)^2)
    on the modes |k_j| <= band (default (N-1)//3)."""
    K = cutoff(n) if band is None else band
    if not 0 <= K <= n // 2 - 1:
        raise ValueError("band must lie in 0..n/2-1")
    rng = np.random.Generator(np.random.PCG64(seed))
    ks, idx = _kidx(n, K)
    kx = np.arange(0, K + 1)
    KZ, KY, KX = np.meshgrid(ks, ks, kx, indexing="ij")
    kmag = np.sqrt(KX * KX + KY * KY + KZ * KZ)
    amp = kmag * np.exp(-(kmag / k0) ** 2)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=(3,) + KX.shape)
    a = amp * np.exp(1j * phases)
    safe = np.where(kmag == 0, 1.0, kmag)
    ex, ey, ez = KX / safe, KY / safe, KZ / safe
    ux = ey * a[2] - ez * a[1]
    uy = ez * a[0] - ex * a[2]
    uz = ex * a[1] - ey * a[0]
    u = np.zeros((3, n, n, n // 2 + 1), dtype=np.complex128)
    sel = np.ix_(idx, idx, np.arange(K + 1))
    for c, comp in enumerate((ux, uy, uz)):
        u[c][sel] = comp
    u = _hermitian_kx0(u, n, K)
    return _energy_scale(u, e0)


def rayleigh_taylor2d(n, amp=0.05, mode=4, width=0.02):
    """(u, v, rho) with rho = tanh((y - pi + amp cos(mode x))/width)."""
    K = cutoff(n)
    x = 2.0 * np.pi * np.arange(n) / n
    X, Y = np.meshgrid(x, x, indexing="xy")        # [iy][ix]
    rho = np.tanh((Y - np.pi + amp * np.cos(mode * X)) / width)
    rh = np.fft.rfft2(rho) / float(n * n)
    keep = np.zeros(rh.shape, dtype=bool)
    _, idx = _kidx(n)
    keep[np.ix_(idx, np.arange(K + 1))] = True
    out = np.zeros((3, n, n // 2 + 1), dtype=np.complex128)
    out[2] = np.where(keep, rh, 0.0)
    return out


def ensemble_members(count, n, seed=1810):
    """Initial fields and viscosities of a mixed ensemble.

    Member m is a Taylor--Green vortex for even m and a random-phase field
    with seed 10197 + m for odd m; nu_m = 10^(-3 + U_m) with U_m uniform in
    [0, 1) drawn from PCG64(seed).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    nus = 10.0 ** (-3.0 + rng.uniform(0.0, 1.0, size=count))
    fields = []
    for m in range(count):
        if m % 2 == 0:
            fields.append(tgv3d(n))
        else:
            fields.append(random_isotropic(n, 10197 + m))
    return np.stack(fields), nus
