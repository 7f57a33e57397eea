"""GPU parity of the right-hand side f(u_hat) of Eq. (2) through the C ABI
against the CPU FP64 oracle."""
import numpy as np
import pytest

from gpu_util import announce, per_field_rel_l2, rel_l2
from oracle import spectral
from paper_1810_10197_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ns():
    from paper_1810_10197_amd import ns as mod
    return mod


def solver(ns, n, prec, nu=0.01, batch=1):
    return ns.Solver(dim=3, n=n, batch=batch, nu=nu, rhs_precision=prec)


def band_field(n, seed):
    """Random solenoidal field whose spectrum peaks at k0 = n/8, so that the
    modes on the faces of the retained cube (some |k_j| = K) carry energy."""
    return inputs.random_isotropic(n, seed, k0=n / 8.0)


def faces(n):
    """Half-spectrum entries on the faces of the retained cube: every
    |k_j| <= K and max_j |k_j| = K."""
    K = spectral.cutoff(n)
    kx, ky, kz = spectral.wavenumbers(n, 3)
    m = spectral.mask(n, 3)
    return m & (np.maximum(np.maximum(np.abs(kx), np.abs(ky)), np.abs(kz)) == K)


def fp32_tol(u, n):
    """Per-field relative L2 bound of an FP32 right-hand side: unit roundoff
    2^-24 times log2(n) passes, times (1 + |omega|/|u|) because u_z shares a
    complex transform with omega_x (the pairing puts the rounding of the
    larger partner on the smaller), times 2 for margin."""
    kx, ky, kz = spectral.wavenumbers(n, 3)
    k2 = kx * kx + ky * ky + kz * kz
    ratio = np.sqrt(np.sum(k2 * np.abs(u) ** 2) / np.sum(np.abs(u) ** 2))   # |omega| / |u|
    return 2.0 * 2.0 ** -24 * np.log2(n) * (1.0 + ratio)


def check_faces(got, ref, n, rel):
    """The face entries on their own: a dropped or mis-indexed outer band
    leaves errors there of the size of f itself."""
    fm = np.broadcast_to(faces(n), got.shape[1:])
    fr = ref[:, fm]
    assert np.linalg.norm(fr) > 1e-3 * np.linalg.norm(ref), "input does not reach the faces"
    err = np.abs(got[:, fm] - fr).max() / np.abs(fr).max()
    assert err <= rel, err


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128])
def test_state_roundtrip_is_exact(ns, n):
    announce("roundtrip n=%d" % n)
    u = inputs.random_isotropic(n, 5)
    junk = u.copy()
    junk[:, n // 2, :, :] = 7.0            # non-retained entries must be dropped
    s = solver(ns, n, "fp32")
    s.set_state(junk[None])
    back = s.get_state().cpu().numpy()[0]
    assert np.array_equal(back.view(np.float64), u.view(np.float64))
    s.close()


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128])
def test_rhs_fp64_matches_oracle(ns, n):
    announce("rhs fp64 n=%d" % n)
    nu = 0.013
    for u in (inputs.random_isotropic(n, 100 + n), band_field(n, 150 + n)):
        s = solver(ns, n, "fp64", nu=nu)
        got = s.rhs(u[None]).cpu().numpy()[0]
        ref = spectral.rhs_ns3d(u, nu)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        s.close()
    check_faces(got, ref, n, 1e-12)


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128])
def test_rhs_fp32_matches_oracle(ns, n):
    announce("rhs fp32 n=%d" % n)
    nu = 0.013
    u = inputs.random_isotropic(n, 200 + n)
    s = solver(ns, n, "fp32", nu=nu)
    got = s.rhs(u[None]).cpu().numpy()[0]
    ref = spectral.rhs_ns3d(u, nu)
    errs = per_field_rel_l2(got, ref)
    assert max(errs) <= 2e-6, errs
    m = np.broadcast_to(spectral.mask(n, 3), got.shape[1:])
    assert np.all(got[:, ~m] == 0)
    # a field that fills the band: the bound scales with |omega| / |u|
    u = band_field(n, 250 + n)
    got = s.rhs(u[None]).cpu().numpy()[0]
    ref = spectral.rhs_ns3d(u, nu)
    errs = per_field_rel_l2(got, ref)
    tol = fp32_tol(u, n)
    print("band field n=%d: per-field rel L2 %s, bound %.2e" % (n, errs, tol))
    assert max(errs) <= tol, (errs, tol)
    assert np.all(got[:, ~m] == 0)
    check_faces(got, ref, n, 10 * tol)
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-4)])
def test_tgv2d_exact_decay_256(ns, prec, tol):
    """z-independent 2D Taylor--Green: f = -2 nu u_hat exactly (any size).
    The FP32 bound is relative to the viscous term: the nonlinear term
    (|u x omega| ~ 0.5, a pure gradient here) leaves FP32 rounding of
    ~1e-8 after the projection, ~3e-5 of 2 nu |u| at nu = 1/1600."""
    n, nu = 256, 1.0 / 1600
    announce("tgv2d exact decay n=%d %s" % (n, prec))
    u = inputs.tgv2d_in3d(n)
    s = solver(ns, n, prec, nu=nu)
    got = s.rhs(u[None]).cpu().numpy()[0]
    expect = -2 * nu * u
    err = np.abs(got - expect).max() / (2 * nu * np.abs(u).max())
    assert err <= tol, err
    s.close()


def test_rhs_fp32_256_full_size(ns):
    """Full-size 256^3 parity (FP32 RHS) against the oracle: the forced-
    turbulence spectrum (k0 = 3) and a field that fills the band (k0 = 32),
    with the face entries checked on their own."""
    n, nu = 256, 1.0 / 1600
    announce("rhs fp32 full n=256")
    u = inputs.random_isotropic(n, 1810)
    s = solver(ns, n, "fp32", nu=nu)
    got = s.rhs(u[None]).cpu().numpy()[0]
    ref = spectral.rhs_ns3d(u, nu)
    errs = per_field_rel_l2(got, ref)
    assert max(errs) <= 5e-6, errs
    u = band_field(n, 1811)
    got = s.rhs(u[None]).cpu().numpy()[0]
    s.close()
    ref = spectral.rhs_ns3d(u, nu)
    errs = per_field_rel_l2(got, ref)
    tol = fp32_tol(u, n)
    print("band field n=256: per-field rel L2 %s, bound %.2e" % (errs, tol))
    assert max(errs) <= tol, (errs, tol)
    check_faces(got, ref, n, 10 * tol)


def test_batch_members_equal_single_runs(ns):
    n = 32
    announce("batch==single n=%d" % n)
    fields, nus = inputs.ensemble_members(3, n)
    sb = solver(ns, n, "fp32", nu=nus, batch=3)
    fb = sb.rhs(fields).cpu().numpy()
    sb.close()
    for m in range(3):
        s1 = solver(ns, n, "fp32", nu=nus[m])
        f1 = s1.rhs(fields[m][None]).cpu().numpy()[0]
        s1.close()
        assert np.array_equal(f1.view(np.float64), fb[m].view(np.float64))


def test_inviscid_energy_conservation_fp32_512(ns):
    """At 512^3 (beyond the oracle's quick range): the inviscid dealiased RHS
    conserves energy, sum w Re(conj(u).f) = 0, and f is solenoidal."""
    n = 512
    announce("inviscid invariants n=512 fp32")
    u = inputs.random_isotropic(n, 3)
    s = solver(ns, n, "fp32", nu=0.0)
    f = s.rhs(u[None]).cpu().numpy()[0]
    s.close()
    from oracle import diagnostics
    w = diagnostics.weights(n, 3)
    rate = np.sum(w * np.real(np.conj(u) * f).sum(0))
    scale = np.sqrt(np.sum(w * np.abs(u) ** 2) * np.sum(w * np.abs(f) ** 2))
    assert abs(rate) < 1e-6 * scale
    div = np.abs(spectral.divergence3(f)).max()
    kx, ky, kz = spectral.wavenumbers(n, 3)
    assert div < 1e-5 * np.abs(f).max() * n


@pytest.mark.parametrize("n", [64, 256])
def test_every_launch_variant_matches_oracle(ns, n):
    """Each autotuner variant (radix plan, column tile) of each pass, and each
    slab size of the y/x/y passes, is a correct right-hand side; the tuner
    then keeps one of them."""
    announce("launch variants n=%d" % n)
    nu = 0.013
    u = band_field(n, 300 + n)                  # the faces of the band carry energy
    ref = spectral.rhs_ns3d(u, nu)
    tol = fp32_tol(u, n)
    s = solver(ns, n, "fp32", nu=nu)
    for v in range(13):
        s.tune([v % 5, v % 5, v % 2, v % 5, v % 5, v])
        got = s.rhs(u[None]).cpu().numpy()[0]
        errs = per_field_rel_l2(got, ref)
        assert max(errs) <= tol, (v, errs, tol)
        check_faces(got, ref, n, 10 * tol)
    s.set_state(u[None])
    variants, ms = s.autotune(reps=2)
    # per pass the fastest variant, or one within 3% of it that won on whole evaluations
    assert all(ms[p][variants[p]] <= 1.03 * min(x for x in ms[p] if x > 0) for p in range(6))
    got = s.rhs(u[None]).cpu().numpy()[0]
    assert max(per_field_rel_l2(got, ref)) <= tol
    s.close()


@pytest.mark.parametrize("prec,rel", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_rhs_512_full_size_against_direct_modes(ns, prec, rel):
    """512^3 (the forced-turbulence size) against the oracle element by
    element: a velocity with few modes, some on the band's faces, whose f the
    oracle forms by direct convolution; every entry of the output compared."""
    from gpu_util import compare_with_modes, modes_to_half_spectrum, sparse_modes
    n, nu = 512, 0.005
    K = spectral.cutoff(n)
    announce("rhs 512 %s vs direct modes" % prec)
    modes = sparse_modes(K, 12, 512 + (prec == "fp32"))
    expect = spectral.rhs_ns3d_modes(modes, nu, K)
    s = solver(ns, n, prec, nu=nu)
    got = s.rhs(modes_to_half_spectrum(modes, n)[None]).cpu().numpy()[0]
    s.close()
    compare_with_modes(got, expect, n, rel)


def test_rhs_1024_full_size_against_direct_modes(ns):
    """1024^3 on one GPU (FP32 right-hand side, about 175 GB of workspace):
    every output entry against the oracle's direct convolution of a few-mode
    velocity, compared on the device (the ABI arrays are 26 GB each)."""
    import torch
    from gpu_util import sparse_modes
    n, nu = 1024, 0.005
    K = spectral.cutoff(n)
    announce("rhs 1024 fp32 vs direct modes")
    modes = sparse_modes(K, 12, 1024)
    expect = spectral.rhs_ns3d_modes(modes, nu, K)
    u = torch.zeros((1, 3, n, n, n // 2 + 1), dtype=torch.complex128, device="cuda")
    for k, a in modes.items():
        if k[0] >= 0:
            u[0, :, k[2] % n, k[1] % n, k[0]] = torch.tensor(a, dtype=torch.complex128)
    s = solver(ns, n, "fp32", nu=nu)
    f = s.rhs(u)
    s.close()
    del s, u
    scale = max(float(np.abs(v).max()) for v in expect.values())
    for k, v in expect.items():
        f[0, :, k[2] % n, k[1] % n, k[0]] -= torch.tensor(v, dtype=torch.complex128, device="cuda")
    err = 0.0
    for z0 in range(0, n, 128):                 # chunks: no full-size temporaries
        err = max(err, float(torch.view_as_real(f[0, :, z0:z0 + 128]).abs().max()))
    assert err / scale <= 2e-5, err / scale
