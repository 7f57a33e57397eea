"""Spectral operators and the Navier--Stokes right-hand side, FP64 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Sec. 2 ("Pseudo-spectral discretization of incompressible
Navier--Stokes"): the rotational form of Eq. (1b) with the modified pressure,
the spectral ODE system of Eq. (2) whose nonlinear term u x omega is evaluated
pointwise in physical space and transformed back (Sec. 2.1), and the
Boussinesq system of Eqs. (3a-c), (4a-b) (Sec. 3.2).  Dealiasing uses the
2/3 rule (rhs_ns3d, rhs_ns2d) or the 3/2-rule zero padding of Sec. 2.1.1
(rhs_ns3d_padded, rhs_ns2d_padded).

Every function works on the full half-spectrum layout; shapes are
(C, N, N, N//2+1) in 3D and (C, N, N//2+1) in 2D, complex128.
"""
import numpy as np


def cutoff(n):
    """2/3-rule cutoff K = floor((N-1)/3): the largest retained |k_j|.

    With 3K < N the alias of any product mode (|k| <= 2K) lands outside the
    retained cube, which is what the 2/3 rule requires.
    """
    return (n - 1) // 3


def wavenumbers(n, dim):
    """Integer wavenumber grids broadcastable to the half-spectrum shape.

    Returns (kx, ky) in 2D or (kx, ky, kz) in 3D.  Full axes carry
    0..N/2-1, -N/2..-1; the last (real-DFT) axis carries 0..N/2.
    """
    kfull = np.fft.fftfreq(n, 1.0 / n)
    khalf = np.fft.rfftfreq(n, 1.0 / n)
    if dim == 3:
        kz = kfull[:, None, None]
        ky = kfull[None, :, None]
        kx = khalf[None, None, :]
        return kx, ky, kz
    if dim == 2:
        ky = kfull[:, None]
        kx = khalf[None, :]
        return kx, ky
    raise ValueError("dim must be 2 or 3")


def mask(n, dim):
    """Boolean 2/3-rule mask: True where every |k_j| <= K."""
    K = cutoff(n)
    ks = wavenumbers(n, dim)
    m = np.ones(np.broadcast_shapes(*[k.shape for k in ks]), dtype=bool)
    for k in ks:
        m = m & (np.abs(k) <= K)
    return m


def spectral_shape(n, dim):
    return (n,) * (dim - 1) + (n // 2 + 1,)


# ---------------------------------------------------------------------------
# Transforms.  The normalised convention u_hat = DFT(u)/N^d reads the paper's
# kinetic-energy formula (Sec. 3.1), E = (1/2N^6)||u_hat||^2 for the
# unnormalised transform, as E = 1/2 sum w |u_hat|^2 for this one.
# ---------------------------------------------------------------------------

def forward(u, dim):
    """Physical (..., N, ..., N) real -> normalised half spectrum."""
    n = u.shape[-1]
    axes = tuple(range(-dim, 0))
    return np.fft.rfftn(u, axes=axes) / float(n) ** dim


def inverse(uh, n, dim):
    """Normalised half spectrum -> physical real values on the N^d grid."""
    axes = tuple(range(-dim, 0))
    return np.fft.irfftn(uh * float(n) ** dim, s=(n,) * dim, axes=axes)


def naive_forward(u):
    """Direct-summation real DFT (no FFT), normalised, for tiny grids.

    u has shape (N,)*d.  Evaluates sum_x u(x) exp(-i k.x) / N^d for every
    half-spectrum k, with x_j = 2 pi j / N.  O(N^(2d)); N <= 8 only.
    """
    dim = u.ndim
    n = u.shape[0]
    out = np.zeros(spectral_shape(n, dim), dtype=np.complex128)
    kfull = [int(k) for k in np.fft.fftfreq(n, 1.0 / n)]
    khalf = list(range(n // 2 + 1))
    grids = np.meshgrid(*([np.arange(n)] * dim), indexing="ij")
    if dim == 3:
        for a, kz in enumerate(kfull):
            for b, ky in enumerate(kfull):
                for c, kx in enumerate(khalf):
                    ph = 2 * np.pi * (kz * grids[0] + ky * grids[1] + kx * grids[2]) / n
                    out[a, b, c] = np.sum(u * np.exp(-1j * ph))
    else:
        for b, ky in enumerate(kfull):
            for c, kx in enumerate(khalf):
                ph = 2 * np.pi * (ky * grids[0] + kx * grids[1]) / n
                out[b, c] = np.sum(u * np.exp(-1j * ph))
    return out / float(n) ** dim


def naive_inverse(uh, n):
    """Direct-summation inverse of a half spectrum (tiny grids only).

    Rebuilds the full Hermitian spectrum and sums u(x) = sum_k uh_k e^{ik.x}.
    Entries on the kx = N/2 plane are summed once, as irfftn does, taking
    their real part's Hermitian completion.
    """
    dim = uh.ndim
    kfull = [int(k) for k in np.fft.fftfreq(n, 1.0 / n)]
    grids = np.meshgrid(*([np.arange(n)] * dim), indexing="ij")
    u = np.zeros((n,) * dim)
    # full spectrum from the half spectrum: F(-k) = conj(F(k))
    full = np.zeros((n,) * dim, dtype=np.complex128)
    half = n // 2 + 1
    if dim == 3:
        for a in range(n):
            for b in range(n):
                for c in range(n):
                    if c < half:
                        full[a, b, c] = uh[a, b, c]
                    else:
                        full[a, b, c] = np.conj(uh[(-a) % n, (-b) % n, (-c) % n])
        for a, kz in enumerate(kfull):
            for b, ky in enumerate(kfull):
                for c, kx in enumerate(kfull):
                    ph = 2 * np.pi * (kz * grids[0] + ky * grids[1] + kx * grids[2]) / n
                    u = u + np.real(full[a, b, c] * np.exp(1j * ph))
    else:
        for b in range(n):
            for c in range(n):
                if c < half:
                    full[b, c] = uh[b, c]
                else:
                    full[b, c] = np.conj(uh[(-b) % n, (-c) % n])
        for b, ky in enumerate(kfull):
            for c, kx in enumerate(kfull):
                ph = 2 * np.pi * (ky * grids[0] + kx * grids[1]) / n
                u = u + np.real(full[b, c] * np.exp(1j * ph))
    return u


# ---------------------------------------------------------------------------
# Right-hand sides
# ---------------------------------------------------------------------------

def curl3(uh, n):
    """omega_hat = i k x u_hat (Sec. 2: omega = curl u)."""
    kx, ky, kz = wavenumbers(n, 3)
    ux, uy, uz = uh
    return np.stack([1j * (ky * uz - kz * uy),
                     1j * (kz * ux - kx * uz),
                     1j * (kx * uy - ky * ux)])


def cross3(a, b):
    """Pointwise a x b for (3, ...) arrays."""
    return np.stack([a[1] * b[2] - a[2] * b[1],
                     a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]])


def rhs_ns3d(uh, nu):
    """f(u_hat) of Eq. (2), 2/3-dealiased, normalised convention.

    1. omega_hat = i k x u_hat;
    2. u, omega in physical space (inverse real DFT);
    3. n = u x omega pointwise;
    4. N_hat = mask * DFT(n) / N^3;
    5. pressure: p_hat = (k . N_hat)/|k|^2, with p_hat(0) = 0 -- the Leray
       projection that eliminates P (the stray factor i in the printed
       projection term is a typo: with it, f would not be real in physical
       space);
    6. f = N_hat - k p_hat - nu |k|^2 u_hat, and f = 0 at k = 0.
    """
    n = uh.shape[1]
    kx, ky, kz = wavenumbers(n, 3)
    m = mask(n, 3)
    u = inverse(uh, n, 3)
    w = inverse(curl3(uh, n), n, 3)
    nl = forward(cross3(u, w), 3) * m
    k2 = kx * kx + ky * ky + kz * kz
    k2safe = np.where(k2 == 0, 1.0, k2)
    p = (kx * nl[0] + ky * nl[1] + kz * nl[2]) / k2safe
    p = np.where(k2 == 0, 0.0, p)
    f = np.stack([nl[0] - kx * p, nl[1] - ky * p, nl[2] - kz * p]) - nu * k2 * uh
    # k = 0: the projection is undefined there; the mean of u x omega over a
    # periodic box vanishes for a solenoidal field, so the mean velocity is
    # held fixed (f(0) = 0) rather than fed with rounding noise.
    f[:, 0, 0, 0] = 0.0
    return f


# ---------------------------------------------------------------------------
# 3/2-rule dealiasing (Sec. 2.1.1): the velocity and vorticity spectra are
# padded with zeros to 3N/2 frequencies per direction, the product is formed
# on the (3N/2)^3 grid, and the result is truncated back to N frequencies.
# ---------------------------------------------------------------------------

def cutoff_padded(n):
    """Largest retained |k_j| of the 3/2 rule on an N grid: N/2 - 1.

    Of the N frequencies -N/2..N/2-1 kept per direction, the Nyquist one
    (-N/2, which has no +N/2 partner) is held at zero: the retained set is
    then symmetric and a real field stays real.
    """
    return n // 2 - 1


def padded_size(n):
    """Points per direction of the padded grid, 3N/2."""
    return 3 * n // 2


def mask_padded(n, dim=3):
    """Boolean mask of the retained modes (every |k_j| <= N/2 - 1)."""
    K = cutoff_padded(n)
    m = True
    for k in wavenumbers(n, dim):
        m = m & (np.abs(k) <= K)
    return m


def _band_index(n, K):
    """Positions of the wavenumbers -K..K along a full axis of length n."""
    return np.arange(-K, K + 1) % n


def _moved(a, src_n, dst_n, K):
    """Copy the modes |k_j| <= K of half spectra a (C, src_n, ..., src_n//2+1)
    into zero half spectra on the dst_n grid; 2D or 3D from a's rank."""
    dim = a.ndim - 1
    out = np.zeros((a.shape[0],) + (dst_n,) * (dim - 1) + (dst_n // 2 + 1,), dtype=np.complex128)
    full_s = [_band_index(src_n, K)] * (dim - 1) + [np.arange(K + 1)]
    full_d = [_band_index(dst_n, K)] * (dim - 1) + [np.arange(K + 1)]
    src, dst = np.ix_(*full_s), np.ix_(*full_d)
    for c in range(a.shape[0]):
        out[c][dst] = a[c][src]
    return out


def pad_spectrum(uh, n, m):
    """N-grid half spectra (C, N, [N,] N//2+1) -> M-grid ones (M > N), zeros
    outside the retained set of the 3/2 rule.  Coefficients are copied
    unscaled: with the normalised convention a mode's value does not depend
    on the grid it is sampled on."""
    return _moved(uh, n, m, cutoff_padded(n))


def truncate_spectrum(vh, m, n):
    """M-grid half spectra -> N-grid ones, keeping the retained set of the
    3/2 rule on N and zeros elsewhere (the inverse of pad_spectrum on it)."""
    return _moved(vh, m, n, cutoff_padded(n))


def rhs_ns3d_padded(uh, nu):
    """f(u_hat) of Eq. (2) with the nonlinear term dealiased by the 3/2 rule.

    1. u_hat restricted to the retained set; omega_hat = i k x u_hat;
    2. both padded with zeros to M = 3N/2 frequencies per direction;
    3. u and omega on the M^3 grid (inverse real DFT); u x omega pointwise;
    4. forward DFT on the M^3 grid (normalised by M^3), truncated to the
       retained set of the N grid;
    5. projection and viscous term as in rhs_ns3d, with f(0) = 0.
    """
    n = uh.shape[1]
    m = padded_size(n)
    keep = mask_padded(n)
    u0 = uh * keep
    up = pad_spectrum(u0, n, m)
    wp = pad_spectrum(curl3(u0, n), n, m)
    u = inverse(up, m, 3)
    w = inverse(wp, m, 3)
    nl = truncate_spectrum(forward(cross3(u, w), 3), m, n)
    kx, ky, kz = wavenumbers(n, 3)
    k2 = kx * kx + ky * ky + kz * kz
    k2safe = np.where(k2 == 0, 1.0, k2)
    p = (kx * nl[0] + ky * nl[1] + kz * nl[2]) / k2safe
    p = np.where(k2 == 0, 0.0, p)
    f = np.stack([nl[0] - kx * p, nl[1] - ky * p, nl[2] - kz * p]) - nu * k2 * u0
    f[:, 0, 0, 0] = 0.0
    return f


def rhs_ns2d_padded(uh, nu, kappa=0.0, ri=0.0):
    """The 2D right-hand side of rhs_ns2d (plain or Boussinesq) with every
    product -- v omega, -u omega and, with the scalar, rho u, rho v -- formed
    by the 3/2 rule: the factors padded with zeros to M = 3N/2 frequencies
    per direction, multiplied on the M^2 grid, transformed back (normalised
    by M^2) and truncated to |k_j| <= N/2 - 1.  The linear terms (projection,
    buoyancy, diffusion) then act on the N grid as in rhs_ns2d."""
    n = uh.shape[1]
    m = padded_size(n)
    keep = mask_padded(n, 2)
    u0 = uh * keep
    kx, ky = wavenumbers(n, 2)
    k2 = kx * kx + ky * ky
    k2safe = np.where(k2 == 0, 1.0, k2)

    def phys(a):
        return inverse(pad_spectrum(a[None], n, m)[0], m, 2)

    def spec(a):
        return truncate_spectrum(forward(a, 2)[None], m, n)[0]

    u, v = phys(u0[0]), phys(u0[1])
    om = phys(1j * (kx * u0[1] - ky * u0[0]))
    nx = spec(v * om)
    ny = spec(-u * om)
    if uh.shape[0] == 3:
        rho = phys(u0[2])
        qx = spec(rho * u)
        qy = spec(rho * v)
        ny = ny - ri * u0[2]
    p = (kx * nx + ky * ny) / k2safe
    fu = np.where(k2 == 0, 0.0, nx - kx * p) - nu * k2 * u0[0]
    fv = np.where(k2 == 0, 0.0, ny - ky * p) - nu * k2 * u0[1]
    if uh.shape[0] == 2:
        return np.stack([fu, fv])
    frho = -1j * (kx * qx + ky * qy) - kappa * k2 * u0[2]
    frho[0, 0] = 0.0
    return np.stack([fu, fv, frho])


def rhs_ns2d(uh, nu, kappa=0.0, ri=0.0):
    """2D right-hand side; with three components it is the Boussinesq system.

    Components: (u, v) for plain 2D NS, (u, v, rho) for Boussinesq
    (Eqs. (3a-c) and (4a-b) of Sec. 3.2, in two dimensions with gravity
    along -y).  omega = dv/dx - du/dy; the rotational nonlinear term is
    n = u x omega = (v omega, -u omega).  The momentum RHS is
    P(N_hat - Ri rho_hat e_y) - nu |k|^2 u_hat with P = I - k k^T/|k|^2 and
    zero at k = 0; the density RHS is -i k.(rho u)^ - kappa |k|^2 rho_hat.
    """
    n = uh.shape[1]
    kx, ky = wavenumbers(n, 2)
    m = mask(n, 2)
    k2 = kx * kx + ky * ky
    k2safe = np.where(k2 == 0, 1.0, k2)
    u = inverse(uh[0], n, 2)
    v = inverse(uh[1], n, 2)
    om = inverse(1j * (kx * uh[1] - ky * uh[0]), n, 2)
    nx = forward(v * om, 2) * m
    ny = forward(-u * om, 2) * m
    if uh.shape[0] == 3:
        rho = inverse(uh[2], n, 2)
        qx = forward(rho * u, 2) * m
        qy = forward(rho * v, 2) * m
        ny = ny - ri * uh[2]
    p = (kx * nx + ky * ny) / k2safe
    fu = np.where(k2 == 0, 0.0, nx - kx * p) - nu * k2 * uh[0]
    fv = np.where(k2 == 0, 0.0, ny - ky * p) - nu * k2 * uh[1]
    if uh.shape[0] == 2:
        return np.stack([fu, fv])
    frho = -1j * (kx * qx + ky * qy) - kappa * k2 * uh[2]
    frho[0, 0] = 0.0
    return np.stack([fu, fv, frho])


def divergence3(uh):
    """k . u_hat (zero for a divergence-free field)."""
    n = uh.shape[1]
    kx, ky, kz = wavenumbers(n, 3)
    return kx * uh[0] + ky * uh[1] + kz * uh[2]


# ---------------------------------------------------------------------------
# Right-hand side of a state with few modes, by direct convolution (no grid).
# ---------------------------------------------------------------------------

def rhs_ns3d_modes(modes, nu, K):
    """f of Eq. (2) for a real velocity with finitely many nonzero modes.

    modes: {(kx, ky, kz): complex 3-vector u_hat(k)} containing every nonzero
    mode together with its conjugate partner -k (a real field), all with
    |k_j| <= K.  The nonlinear term is the exact product of the Fourier
    series, (u x omega)^(k) = sum_{p+q=k} u_hat(p) x (i q x u_hat(q)), kept on
    the retained cube |k_j| <= K (what the dealiased pseudo-spectral product
    gives there, alias-free); then the projection and the viscous term, with
    f(0) = 0.  Returns {k: f(k)} for every k with kx >= 0 where f can be
    nonzero (all other retained entries are zero).
    """
    keys = list(modes)
    prod = {}
    for p in keys:
        up = np.asarray(modes[p], dtype=np.complex128)
        for q in keys:
            k = (p[0] + q[0], p[1] + q[1], p[2] + q[2])
            if k[0] < 0 or max(abs(k[0]), abs(k[1]), abs(k[2])) > K:
                continue
            uq = np.asarray(modes[q], dtype=np.complex128)
            qv = np.array(q, dtype=float)
            wq = 1j * np.cross(qv, uq)
            prod[k] = prod.get(k, 0.0) + np.cross(up, wq)
    out = {}
    for k in set(prod) | {m for m in keys if m[0] >= 0}:
        kv = np.array(k, dtype=float)
        kk = float(kv @ kv)
        if kk == 0.0:
            out[k] = np.zeros(3, dtype=np.complex128)
            continue
        nl = prod.get(k, np.zeros(3, dtype=np.complex128))
        u = np.asarray(modes.get(k, np.zeros(3)), dtype=np.complex128)
        out[k] = nl - kv * (kv @ nl) / kk - nu * kk * u
    return out
