"""Pins of the oracle's step-size proposer network (gradients by central
finite differences, Adam against its closed form under a constant gradient),
of the HIT forcing (Sec. 3.3.1) and of the seeded input fields."""
import numpy as np
import pytest

from oracle import diagnostics, forcing, mlp, spectral
from paper_1810_10197_amd import inputs


def test_param_count():
    assert mlp.NPARAM == 20 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 5569


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(rng)
    p += 0.05 * rng.standard_normal(p.shape)
    z = rng.standard_normal((7, 20))
    t = rng.standard_normal(7)
    loss, g = mlp.loss_and_grad(p, z, t)
    idx = rng.choice(p.size, 200, replace=False)
    idx = np.concatenate([idx, [5568, 5567, 0, 1343]])    # b3, W3, W1, b1 corners
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = eps
        lp, _ = mlp.loss_and_grad(p + e, z, t)
        lm, _ = mlp.loss_and_grad(p - e, z, t)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_forward_by_hand_small_weights():
    """With W2 = 0 the output is b3 + W3 . tanh(b2) regardless of x."""
    p = np.zeros(mlp.NPARAM)
    d = mlp.unpack(p)
    d["b2"][...] = np.linspace(-1, 1, 64)
    d["W3"][...] = 0.5
    d["b3"][...] = 0.25
    y, _ = mlp.forward(p, np.ones((2, 20)))
    assert y == pytest.approx([0.25 + 0.5 * np.sum(np.tanh(np.linspace(-1, 1, 64)))] * 2,
                              rel=1e-14)


def test_adam_constant_gradient_closed_form():
    """Under a constant gradient g, m_hat = g and v_hat = g^2 at every step,
    so each update is lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 6):
        p, m, v = mlp.adam_step(p, g, m, v, t, lr=1e-2)
    expect = -5 * 1e-2 * g / (np.abs(g) + 1e-8)
    assert p == pytest.approx(expect, rel=1e-12, abs=1e-18)


def test_features_layout():
    sh = np.full(16, 0.125 / 16)
    x = mlp.features(sh, 0.125, [1e-2, 0.5])
    assert x.shape == (20,)
    assert x[:16] == pytest.approx([np.log10(1 / 16 + 1e-30)] * 16)
    assert x[16:] == pytest.approx([0.0, 0.0, -2.0, np.log10(0.5)])


@pytest.mark.parametrize("n,seed", [(16, 1810), (24, 7)])
def test_random_isotropic_field(n, seed):
    u = inputs.random_isotropic(n, seed)
    assert np.abs(spectral.divergence3(u)).max() < 1e-15
    # the oracle's half-spectrum energy against the physical-space mean (Parseval)
    phys = spectral.inverse(u, n, 3)
    assert 0.5 * float(np.mean(np.sum(phys * phys, axis=0))) == pytest.approx(0.125, rel=1e-14)
    assert diagnostics.energy(u, 3) == pytest.approx(0.125, rel=1e-14)
    # real-valued in physical space: round trip is exact
    back = spectral.forward(spectral.inverse(u, n, 3), 3)
    assert np.abs(back - u).max() < 1e-15
    m = np.broadcast_to(spectral.mask(n, 3), u.shape[1:])
    assert np.all(u[:, ~m] == 0)
    again = inputs.random_isotropic(n, seed)
    assert np.array_equal(u.view(np.float64), again.view(np.float64))


def test_random_isotropic_spectrum_shape():
    """Shell energy follows k^4 exp(-2 (k/k0)^2) up to sampling noise."""
    n = 48
    u = inputs.random_isotropic(n, 3)
    kx, ky, kz = spectral.wavenumbers(n, 3)
    kmag = np.sqrt(kx * kx + ky * ky + kz * kz)
    w = diagnostics.weights(n, 3)
    e = 0.5 * w * np.sum(np.abs(u) ** 2, axis=0)
    shells = np.array([e[(kmag >= k - 0.5) & (kmag < k + 0.5)].sum() for k in range(1, 9)])
    model = np.array([k ** 4 * np.exp(-2 * (k / 3.0) ** 2) for k in range(1, 9)])
    ratio = (shells / shells.sum()) / (model / model.sum())
    assert np.all(np.abs(ratio[1:] - 1) < 0.35), ratio


def test_forcing_restores_energy():
    n, kf, e0 = 16, 2.0, 0.125
    u = inputs.random_isotropic(n, 5)
    u_decayed = u * 0.9
    out = forcing.force(u_decayed, kf, e0)
    assert diagnostics.energy(out, 3) == pytest.approx(e0, rel=1e-14)
    band = forcing.band(n, kf)
    assert np.array_equal(out[:, ~band], u_decayed[:, ~band])
    ratio = out[:, band] / np.where(u_decayed[:, band] == 0, 1, u_decayed[:, band])
    nz = u_decayed[:, band] != 0
    assert np.allclose(ratio[nz], ratio[nz][0])


def test_rayleigh_taylor_field():
    n = 64
    s = inputs.rayleigh_taylor2d(n)
    assert np.all(s[:2] == 0)
    rho = spectral.inverse(s[2], n, 2)
    # heavy (rho ~ +1) above the interface at y ~ pi, light below
    assert rho[3 * n // 4, :].mean() > 0.9 and rho[n // 4, :].mean() < -0.9
    m = spectral.mask(n, 2)
    assert np.all(s[2][~m] == 0)


def test_ensemble_members():
    fields, nus = inputs.ensemble_members(4, 16)
    assert fields.shape == (4, 3, 16, 16, 9)
    assert np.all((nus >= 1e-3) & (nus <= 1e-2))
    assert np.array_equal(fields[0], inputs.tgv3d(16))
    assert np.array_equal(fields[1], inputs.random_isotropic(16, 10198))
