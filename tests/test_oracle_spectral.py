"""Pins of the oracle's transforms and right-hand sides (Sec. 2, Eq. (2);
Sec. 3.2, Eqs. (4a-b)) against direct summation, closed forms and exact
invariants of the dealiased semi-discrete system."""
import numpy as np
import pytest

from oracle import diagnostics, spectral
from paper_1810_10197_amd import inputs


def grid(n, dim):
    x = 2 * np.pi * np.arange(n) / n
    return np.meshgrid(*([x] * dim), indexing="ij")   # [z][y][x] / [y][x]


@pytest.mark.parametrize("n,dim", [(4, 3), (6, 3), (8, 2), (6, 2)])
def test_forward_matches_direct_dft(n, dim):
    rng = np.random.default_rng(n + dim)
    u = rng.standard_normal((n,) * dim)
    assert np.abs(spectral.forward(u, dim) - spectral.naive_forward(u)).max() < 1e-13


@pytest.mark.parametrize("n,dim", [(4, 3), (6, 2), (8, 2)])
def test_inverse_matches_direct_sum(n, dim):
    rng = np.random.default_rng(7)
    u = rng.standard_normal((n,) * dim)
    uh = spectral.forward(u, dim)
    # direct summation reproduces the grid values
    assert np.abs(spectral.naive_inverse(uh, n) - u).max() < 1e-12
    assert np.abs(spectral.inverse(uh, n, dim) - u).max() < 1e-12


def test_parseval_weights():
    n = 8
    rng = np.random.default_rng(1)
    u = rng.standard_normal((n, n, n))
    uh = spectral.forward(u, 3)
    w = diagnostics.weights(n, 3)
    assert abs(np.sum(w * np.abs(uh) ** 2) - np.mean(u * u)) < 1e-14


def test_tgv_energy_and_dissipation_closed_form():
    """E0 = 1/8, eps0 = 3 nu / 4 for the 3D Taylor--Green vortex."""
    n, nu = 16, 1.0 / 1600
    u = inputs.tgv3d(n)
    f = spectral.rhs_ns3d(u, nu)
    assert abs(diagnostics.energy(u, 3) - 0.125) < 1e-15
    assert abs(diagnostics.dissipation(u, f, 3) - 0.75 * nu) < 1e-15


def test_tgv_generator_matches_sampled_field():
    n = 12
    Z, Y, X = grid(n, 3)
    up = np.stack([np.sin(X) * np.cos(Y) * np.cos(Z),
                   -np.cos(X) * np.sin(Y) * np.cos(Z), 0 * X])
    assert np.abs(spectral.forward(up, 3) - inputs.tgv3d(n)).max() < 1e-15
    Y2, X2 = grid(n, 2)
    up2 = np.stack([np.sin(X2) * np.cos(Y2), -np.cos(X2) * np.sin(Y2)])
    assert np.abs(spectral.forward(up2, 2) - inputs.tgv2d(n)).max() < 1e-15


@pytest.mark.parametrize("n", [16, 24])
def test_2d_tgv_is_exact_viscous_decay(n):
    """The 2D TGV is a steady Euler flow: f = -2 nu u_hat exactly (3D and 2D)."""
    nu = 0.013
    u3 = inputs.tgv2d_in3d(n)
    f3 = spectral.rhs_ns3d(u3, nu)
    assert np.abs(f3 + 2 * nu * u3).max() < 1e-12 * 2 * nu * np.abs(u3).max() + 1e-17
    u2 = inputs.tgv2d(n)
    f2 = spectral.rhs_ns2d(u2, nu)
    assert np.abs(f2 + 2 * nu * u2).max() < 1e-12 * 2 * nu * np.abs(u2).max() + 1e-17


@pytest.mark.parametrize("n,seed", [(16, 1), (18, 2), (32, 3)])
def test_projection_and_mask(n, seed):
    u = inputs.random_isotropic(n, seed)
    f = spectral.rhs_ns3d(u, 0.01)
    div = np.abs(spectral.divergence3(f)).max()
    assert div <= 1e-13 * np.abs(f).max()
    m = np.broadcast_to(spectral.mask(n, 3), f.shape[1:])
    assert np.all(f[:, ~m] == 0.0)


@pytest.mark.parametrize("n,seed", [(16, 4), (20, 5)])
def test_inviscid_invariants(n, seed):
    """With nu = 0 the dealiased rotational nonlinear term conserves energy
    and helicity exactly: sum w Re(conj(u).f) = 0 = sum w Re(conj(omega).f)."""
    u = inputs.random_isotropic(n, seed)
    f = spectral.rhs_ns3d(u, 0.0)
    w = diagnostics.weights(n, 3)
    om = spectral.curl3(u, n)
    scale = np.sqrt(np.sum(w * np.abs(u) ** 2)) * np.sqrt(np.sum(w * np.abs(f) ** 2))
    e_rate = np.sum(w * np.real(np.conj(u) * f).sum(0))
    h_rate = np.sum(w * np.real(np.conj(om) * f).sum(0))
    scale_h = np.sqrt(np.sum(w * np.abs(om) ** 2)) * np.sqrt(np.sum(w * np.abs(f) ** 2))
    assert abs(e_rate) < 1e-14 * scale
    assert abs(h_rate) < 1e-14 * scale_h
    assert np.abs(f).max() > 1e-3          # the nonlinear term is not trivially zero


def test_viscous_dissipation_identity():
    """eps = nu sum w |k|^2 |u_hat|^2 for any solenoidal field."""
    n, nu = 16, 0.02
    u = inputs.random_isotropic(n, 9)
    f = spectral.rhs_ns3d(u, nu)
    kx, ky, kz = spectral.wavenumbers(n, 3)
    k2 = kx * kx + ky * ky + kz * kz
    w = diagnostics.weights(n, 3)
    expect = nu * np.sum(w * k2 * np.sum(np.abs(u) ** 2, axis=0))
    assert abs(diagnostics.dissipation(u, f, 3) - expect) < 1e-14 * expect


def test_rotation_equivariance():
    """Cyclic relabelling of the axes (a proper rotation) commutes with f:
    catches a wrong sign or a transposed operand in the curl or the cross
    product."""
    n, nu = 12, 0.01
    u = inputs.random_isotropic(n, 11)
    up = spectral.inverse(u, n, 3)
    fp = spectral.inverse(spectral.rhs_ns3d(u, nu), n, 3)

    def rot(a):  # v(y, z, x) = (a_y, a_z, a_x)(x, y, z)
        return np.stack([a[1].transpose(2, 0, 1), a[2].transpose(2, 0, 1),
                         a[0].transpose(2, 0, 1)])
    v = spectral.forward(rot(up), 3)
    fv = spectral.inverse(spectral.rhs_ns3d(v, nu), n, 3)
    assert np.abs(fv - rot(fp)).max() < 1e-13


def test_nonlinear_term_against_direct_derivatives():
    """On a field with a handful of modes, u x omega computed by hand."""
    n = 16
    Z, Y, X = grid(n, 3)
    a, b = 0.3, 0.7
    # u = (a sin(2y), b sin(z), 0): omega = (-b cos z, 0, -2a cos 2y)
    up = np.stack([a * np.sin(2 * Y), b * np.sin(Z), 0 * X])
    om = np.stack([-b * np.cos(Z), 0 * X, -2 * a * np.cos(2 * Y)])
    nl = np.stack([up[1] * om[2] - up[2] * om[1],
                   up[2] * om[0] - up[0] * om[2],
                   up[0] * om[1] - up[1] * om[0]])
    uh = spectral.forward(up, 3)
    nh = spectral.forward(nl, 3) * spectral.mask(n, 3)
    kx, ky, kz = spectral.wavenumbers(n, 3)
    k2 = kx * kx + ky * ky + kz * kz
    p = np.where(k2 == 0, 0, (kx * nh[0] + ky * nh[1] + kz * nh[2]) / np.where(k2 == 0, 1, k2))
    expect = nh - np.stack([kx * p, ky * p, kz * p])
    assert np.abs(spectral.rhs_ns3d(uh, 0.0) - expect).max() < 1e-13 * np.abs(expect).max()


def test_boussinesq_hydrostatic_and_budgets():
    n, nu, kappa, ri = 32, 1e-3, 2e-3, 0.5
    # stratification rho(y) only, u = 0: hydrostatic balance, pure diffusion
    Y, X = grid(n, 2)
    rho = spectral.forward(np.cos(Y) + 0.3 * np.sin(2 * Y), 2)
    st = np.zeros((3, n, n // 2 + 1), dtype=complex)
    st[2] = rho
    f = spectral.rhs_ns2d(st, nu, kappa, ri)
    kx, ky = spectral.wavenumbers(n, 2)
    k2 = kx * kx + ky * ky
    assert np.abs(f[:2]).max() < 1e-16
    assert np.abs(f[2] + kappa * k2 * rho).max() < 1e-16
    # general field: density variance budget and energy budget
    rng = np.random.default_rng(3)
    m = spectral.mask(n, 2)
    st = np.zeros((3, n, n // 2 + 1), dtype=complex)
    psi = spectral.forward(rng.standard_normal((n, n)), 2) * m
    st[0] = 1j * ky * psi / np.where(k2 == 0, 1, k2)
    st[1] = -1j * kx * psi / np.where(k2 == 0, 1, k2)
    st[2] = spectral.forward(rng.standard_normal((n, n)), 2) * m
    st = spectral.forward(spectral.inverse(st, n, 2), 2)    # Hermitian-clean
    f = spectral.rhs_ns2d(st, nu, kappa, ri)
    w = diagnostics.weights(n, 2)
    rho_rate = np.sum(w * np.real(np.conj(st[2]) * f[2]))
    assert abs(rho_rate + kappa * np.sum(w * k2 * np.abs(st[2]) ** 2)) < 1e-13
    e_rate = -diagnostics.dissipation(st, f, 2)
    expect = (-nu * np.sum(w * k2 * (np.abs(st[0]) ** 2 + np.abs(st[1]) ** 2))
              - ri * np.sum(w * np.real(np.conj(st[1]) * st[2])))
    assert abs(e_rate - expect) < 1e-13
    assert np.abs(kx * f[0] + ky * f[1]).max() < 1e-14


def _pad(uh, n, m):
    """Embed an N half spectrum into an M > N half spectrum (zero padding)."""
    out = np.zeros(uh.shape[:-3] + (m, m, m // 2 + 1), dtype=complex)
    K = n // 2 - 1
    ks = np.arange(-K, K + 1)
    src = np.ix_(ks % n, ks % n, np.arange(K + 1))
    dst = np.ix_(ks % m, ks % m, np.arange(K + 1))
    for c in range(uh.shape[0]):
        out[c][dst] = uh[c][src]
    return out


@pytest.mark.parametrize("n,seed", [(18, 2), (16, 3)])
def test_dealiased_product_is_exact_truncation(n, seed):
    """The 2/3 rule is alias-free: on every retained mode the masked
    pseudo-spectral product equals the exact product of the band-limited
    fields (computed on a 2N grid, where no alias can reach a retained
    mode), then truncated."""
    rng = np.random.default_rng(seed)
    msk = spectral.mask(n, 3)
    uh = (rng.standard_normal((3,) + msk.shape) + 1j * rng.standard_normal((3,) + msk.shape)) * msk
    uh = spectral.forward(spectral.inverse(uh, n, 3), 3) * msk      # a real field
    m = 2 * n
    up = _pad(uh, n, m)
    u = spectral.inverse(up, m, 3)
    w = spectral.inverse(spectral.curl3(up, m), m, 3)
    exact_big = spectral.forward(spectral.cross3(u, w), 3)
    K = spectral.cutoff(n)
    ks = np.arange(-K, K + 1)
    src = np.ix_(ks % m, ks % m, np.arange(K + 1))
    dst = np.ix_(ks % n, ks % n, np.arange(K + 1))
    exact = np.zeros_like(uh)
    for c in range(3):
        exact[c][dst] = exact_big[c][src]
    kx, ky, kz = spectral.wavenumbers(n, 3)
    k2 = kx * kx + ky * ky + kz * kz
    p = np.where(k2 == 0, 0, (kx * exact[0] + ky * exact[1] + kz * exact[2]) / np.where(k2 == 0, 1, k2))
    expect = exact - np.stack([kx * p, ky * p, kz * p])
    expect[:, 0, 0, 0] = 0.0          # mean mode held fixed
    assert np.abs(spectral.rhs_ns3d(uh, 0.0) - expect).max() < 1e-13 * np.abs(expect).max()


# ---------------------------------------------------------------- 3/2 rule
def _real_band_limited(n, K, seed):
    """A random real solenoidal velocity with every |k_j| <= K (half spectrum)."""
    rng = np.random.default_rng(seed)
    kx, ky, kz = spectral.wavenumbers(n, 3)
    keep = (np.abs(kx) <= K) & (np.abs(ky) <= K) & (np.abs(kz) <= K)
    shape = (3,) + keep.shape
    uh = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * keep
    uh = spectral.forward(spectral.inverse(uh, n, 3), 3) * keep     # a real field
    k2 = kx * kx + ky * ky + kz * kz
    div = (kx * uh[0] + ky * uh[1] + kz * uh[2]) / np.where(k2 == 0, 1, k2)
    return uh - np.stack([kx * div, ky * div, kz * div])


def _full_cube(uh, n, K):
    """Coefficients c[:, kz+K, ky+K, kx+K] of every mode with |k_j| <= K,
    the kx < 0 half from conj(u_hat(-k)) of a real field."""
    ks = range(-K, K + 1)
    L = 2 * K + 1
    out = np.zeros((uh.shape[0], L, L, L), dtype=complex)
    for a, kz in enumerate(ks):
        for b, ky in enumerate(ks):
            for c, kx in enumerate(ks):
                if kx >= 0:
                    out[:, a, b, c] = uh[:, kz % n, ky % n, kx]
                else:
                    out[:, a, b, c] = np.conj(uh[:, (-kz) % n, (-ky) % n, -kx])
    return out


@pytest.mark.parametrize("n,seed", [(8, 21), (10, 22)])
def test_padded_rhs_against_direct_convolution(n, seed):
    """The 3/2 rule forms the product of the two truncated Fourier series
    exactly: on every retained mode the nonlinear term equals the direct
    convolution sum_{p+q=k} u_hat(p) x omega_hat(q) over the retained set
    (no transform involved), followed by the projection and the viscous
    term of Eq. (2)."""
    K = n // 2 - 1
    L = 2 * K + 1
    uh = _real_band_limited(n, K, seed)
    U = _full_cube(uh, n, K)
    k = np.arange(-K, K + 1)
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    W = 1j * np.stack([KY * U[2] - KZ * U[1], KZ * U[0] - KX * U[2], KX * U[1] - KY * U[0]])
    conv = np.zeros_like(U)
    for a in range(L):
        za, zb = max(0, a - K), min(L, a + K + 1)
        for b in range(L):
            ya, yb = max(0, b - K), min(L, b + K + 1)
            for c in range(L):
                xa, xb = max(0, c - K), min(L, c + K + 1)
                p = U[:, a, b, c]
                q = W[:, za - a + K:zb - a + K, ya - b + K:yb - b + K, xa - c + K:xb - c + K]
                conv[:, za:zb, ya:yb, xa:xb] += np.stack([p[1] * q[2] - p[2] * q[1],
                                                          p[2] * q[0] - p[0] * q[2],
                                                          p[0] * q[1] - p[1] * q[0]])
    nu = 0.03
    expect = np.zeros_like(uh)
    for a, kz in enumerate(k):
        for b, ky in enumerate(k):
            for c in range(K, L):
                kx = c - K
                nl = conv[:, a, b, c]
                kk = kx * kx + ky * ky + kz * kz
                if kk == 0:
                    continue                      # mean mode held fixed
                kv = np.array([kx, ky, kz], dtype=float)
                expect[:, kz % n, ky % n, kx] = nl - kv * (kv @ nl) / kk - nu * kk * uh[:, kz % n, ky % n, kx]
    got = spectral.rhs_ns3d_padded(uh, nu)
    assert np.abs(got - expect).max() < 1e-13 * np.abs(expect).max()
    # the Nyquist planes and everything past K stay zero
    assert np.all(got[:, ~spectral.mask_padded(n)] == 0.0)


def test_padded_rhs_equals_two_thirds_rule_on_the_padded_grid():
    """(3N/2 - 1)/3 rounds down to N/2 - 1, so the 2/3 rule on the 3N/2 grid
    keeps the same modes and forms the same product: both right-hand sides
    agree once moved onto a common grid."""
    n = 16
    m = spectral.padded_size(n)
    uh = _real_band_limited(n, n // 2 - 1, 31)
    assert spectral.cutoff(m) == spectral.cutoff_padded(n)
    big = spectral.rhs_ns3d(spectral.pad_spectrum(uh, n, m), 0.02)
    got = spectral.rhs_ns3d_padded(uh, 0.02)
    assert np.abs(spectral.truncate_spectrum(big, m, n) - got).max() < 1e-13 * np.abs(got).max()


def test_padded_rhs_inviscid_invariants():
    """The 3/2-rule system is a Galerkin truncation: with nu = 0 it conserves
    energy and helicity exactly."""
    n = 16
    u = _real_band_limited(n, n // 2 - 1, 41) * 0.1
    f = spectral.rhs_ns3d_padded(u, 0.0)
    w = diagnostics.weights(n, 3)
    om = spectral.curl3(u, n)
    scale = np.sqrt(np.sum(w * np.abs(u) ** 2)) * np.sqrt(np.sum(w * np.abs(f) ** 2))
    scale_h = np.sqrt(np.sum(w * np.abs(om) ** 2)) * np.sqrt(np.sum(w * np.abs(f) ** 2))
    assert abs(np.sum(w * np.real(np.conj(u) * f).sum(0))) < 1e-14 * scale
    assert abs(np.sum(w * np.real(np.conj(om) * f).sum(0))) < 1e-14 * scale_h


def _real_band_limited_2d(n, K, seed, ncomp):
    """Random real 2D state with every |k_j| <= K: a solenoidal velocity from a
    stream function, and (ncomp = 3) a scalar."""
    rng = np.random.default_rng(seed)
    kx, ky = spectral.wavenumbers(n, 2)
    keep = (np.abs(kx) <= K) & (np.abs(ky) <= K)
    psi = spectral.forward(rng.standard_normal((n, n)), 2) * keep
    st = np.zeros((ncomp, n, n // 2 + 1), dtype=complex)
    st[0] = 1j * ky * psi
    st[1] = -1j * kx * psi
    if ncomp == 3:
        st[2] = spectral.forward(rng.standard_normal((n, n)), 2) * keep
    return st


def _full_square(a, n, K):
    """Coefficients c[ky+K, kx+K] of a real 2D field's modes |k_j| <= K."""
    L = 2 * K + 1
    out = np.zeros((L, L), dtype=complex)
    for b, ky in enumerate(range(-K, K + 1)):
        for c, kx in enumerate(range(-K, K + 1)):
            out[b, c] = a[ky % n, kx] if kx >= 0 else np.conj(a[(-ky) % n, -kx])
    return out


def _conv2(A, B, K):
    """Direct convolution sum_{p+q=k} A(p) B(q) over the retained square."""
    L = 2 * K + 1
    out = np.zeros((L, L), dtype=complex)
    for b in range(L):
        ya, yb = max(0, b - K), min(L, b + K + 1)
        for c in range(L):
            xa, xb = max(0, c - K), min(L, c + K + 1)
            out[ya:yb, xa:xb] += A[b, c] * B[ya - b + K:yb - b + K, xa - c + K:xb - c + K]
    return out


@pytest.mark.parametrize("n,ncomp,seed", [(8, 2, 51), (10, 3, 52), (8, 3, 53)])
def test_padded_rhs2d_against_direct_convolution(n, ncomp, seed):
    """2D 3/2 rule (plain and Boussinesq): every product is the exact
    truncated convolution of the retained modes; the projection, buoyancy
    and diffusion then follow Eqs. (4a-b)."""
    K = n // 2 - 1
    L = 2 * K + 1
    st = _real_band_limited_2d(n, K, seed, ncomp)
    nu, kappa, ri = 0.02, 0.03, 0.7
    k = np.arange(-K, K + 1)
    KY, KX = np.meshgrid(k, k, indexing="ij")
    U, V = _full_square(st[0], n, K), _full_square(st[1], n, K)
    W = 1j * (KX * V - KY * U)
    nx, ny = _conv2(V, W, K), -_conv2(U, W, K)
    if ncomp == 3:
        R = _full_square(st[2], n, K)
        qx, qy = _conv2(R, U, K), _conv2(R, V, K)
    expect = np.zeros_like(st)
    for b, ky in enumerate(k):
        for c in range(K, L):
            kx = c - K
            kk = kx * kx + ky * ky
            idx = (ky % n, kx)
            if kk == 0:
                continue
            bx, by = nx[b, c], ny[b, c] - (ri * st[2][idx] if ncomp == 3 else 0.0)
            p = (kx * bx + ky * by) / kk
            expect[0][idx] = bx - kx * p - nu * kk * st[0][idx]
            expect[1][idx] = by - ky * p - nu * kk * st[1][idx]
            if ncomp == 3:
                expect[2][idx] = -1j * (kx * qx[b, c] + ky * qy[b, c]) - kappa * kk * st[2][idx]
    got = (spectral.rhs_ns2d_padded(st, nu, kappa, ri) if ncomp == 3
           else spectral.rhs_ns2d_padded(st, nu))
    assert np.abs(got - expect).max() < 1e-13 * np.abs(expect).max()
    assert np.all(got[:, ~spectral.mask_padded(n, 2)] == 0.0)


@pytest.mark.parametrize("ncomp", [2, 3])
def test_padded_rhs2d_equals_two_thirds_rule_on_the_padded_grid(ncomp):
    n = 32
    m = spectral.padded_size(n)
    st = _real_band_limited_2d(n, n // 2 - 1, 61 + ncomp, ncomp)
    args = (1e-3, 2e-3, 0.5) if ncomp == 3 else (1e-3,)
    big = spectral.rhs_ns2d(spectral.pad_spectrum(st, n, m), *args)
    got = spectral.rhs_ns2d_padded(st, *args)
    assert np.abs(spectral.truncate_spectrum(big, m, n) - got).max() < 1e-13 * np.abs(got).max()


def test_padded_rhs2d_inviscid_budgets():
    """nu = kappa = 0: the scalar variance is conserved and the kinetic energy
    changes only by the buoyancy work -Ri <v, rho>."""
    n, ri = 16, 0.8
    st = _real_band_limited_2d(n, n // 2 - 1, 71, 3)
    f = spectral.rhs_ns2d_padded(st, 0.0, 0.0, ri)
    w = diagnostics.weights(n, 2)
    rho_rate = np.sum(w * np.real(np.conj(st[2]) * f[2]))
    e_rate = np.sum(w * np.real(np.conj(st[0]) * f[0] + np.conj(st[1]) * f[1]))
    work = -ri * np.sum(w * np.real(np.conj(st[1]) * st[2]))
    scale = np.sqrt(np.sum(w * np.abs(st) ** 2) * np.sum(w * np.abs(f) ** 2))
    assert abs(rho_rate) < 1e-13 * scale
    assert abs(e_rate - work) < 1e-13 * scale


def _sparse_state(n, K, count, seed):
    """A real solenoidal velocity with `count` random modes (and their
    conjugate partners) in |k_j| <= K, as a mode dict and as a half spectrum."""
    rng = np.random.default_rng(seed)
    modes = {}
    while len(modes) < 2 * count:
        k = tuple(int(x) for x in rng.integers(-K, K + 1, size=3))
        if k == (0, 0, 0) or k in modes:
            continue
        kv = np.array(k, dtype=float)
        a = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        a = a - kv * (kv @ a) / (kv @ kv)               # solenoidal
        if k[0] == 0 and (-k[0], -k[1], -k[2]) in modes:
            continue
        modes[k] = a
        modes[(-k[0], -k[1], -k[2])] = np.conj(a)
    uh = np.zeros((3, n, n, n // 2 + 1), dtype=complex)
    for k, a in modes.items():
        if k[0] >= 0:
            uh[:, k[2] % n, k[1] % n, k[0]] = a
    return modes, uh


@pytest.mark.parametrize("n,seed", [(16, 81), (20, 82)])
def test_direct_mode_rhs_matches_pseudo_spectral(n, seed):
    """The few-mode direct convolution gives the same f as the dealiased
    pseudo-spectral right-hand side, on every retained entry (kx = 0
    included)."""
    K = spectral.cutoff(n)
    nu = 0.015
    modes, uh = _sparse_state(n, K, 9, seed)
    ref = spectral.rhs_ns3d(uh, nu)
    got = np.zeros_like(ref)
    for k, f in spectral.rhs_ns3d_modes(modes, nu, K).items():
        got[:, k[2] % n, k[1] % n, k[0]] = f
    # on the kx = 0 plane only one of k, -k is stored; the direct sum writes both
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
