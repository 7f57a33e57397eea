"""The pins are strong enough: a plausible mistake planted in the oracle (on
the CPU, via monkeypatch) makes at least one of them fail."""
from fractions import Fraction as F

import numpy as np
import pytest

import test_oracle_spectral as ts
import test_oracle_tableaux as tt
from oracle import spectral, tableaux


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_sign_error_in_cross_product_is_caught(monkeypatch):
    def bad_cross(a, b):
        return np.stack([a[1] * b[2] - a[2] * b[1],
                         a[2] * b[0] - a[0] * b[2],
                         a[1] * b[0] - a[0] * b[1]])      # z component flipped
    monkeypatch.setattr(spectral, "cross3", bad_cross)
    assert _fails(ts.test_rotation_equivariance)


def test_transposed_curl_operand_is_caught(monkeypatch):
    orig = spectral.curl3

    def bad_curl(uh, n):
        w = orig(uh, n)
        return np.stack([w[0], w[2], w[1]])
    monkeypatch.setattr(spectral, "curl3", bad_curl)
    assert _fails(ts.test_inviscid_invariants, 16, 4) or _fails(ts.test_rotation_equivariance)


def test_missing_projection_is_caught(monkeypatch):
    orig = spectral.rhs_ns3d

    def no_proj(uh, nu):
        n = uh.shape[1]
        u = spectral.inverse(uh, n, 3)
        w = spectral.inverse(spectral.curl3(uh, n), n, 3)
        kx, ky, kz = spectral.wavenumbers(n, 3)
        k2 = kx * kx + ky * ky + kz * kz
        return spectral.forward(spectral.cross3(u, w), 3) * spectral.mask(n, 3) - nu * k2 * uh
    monkeypatch.setattr(spectral, "rhs_ns3d", no_proj)
    assert _fails(ts.test_projection_and_mask, 16, 1)


def test_wrong_viscous_sign_is_caught(monkeypatch):
    orig = spectral.rhs_ns3d
    monkeypatch.setattr(spectral, "rhs_ns3d", lambda uh, nu: orig(uh, -nu))
    assert _fails(ts.test_tgv_energy_and_dissipation_closed_form)


def test_wrong_mask_cutoff_is_caught(monkeypatch):
    # K = N // 3 gives 3K = N at N = 18: a product mode aliases onto |k| = K
    monkeypatch.setattr(spectral, "cutoff", lambda n: n // 3)
    assert _fails(ts.test_dealiased_product_is_exact_truncation, 18, 2)


def test_mistyped_tableau_entry_is_caught(monkeypatch):
    A = [row[:] for row in tableaux.BS5["A"]]
    A[5][3] = F(58653, 366081)
    bad = dict(tableaux.BS5, A=A)
    assert _fails(tt.test_main_weights_order, bad, 5) or _fails(tt.test_row_sums_equal_c, bad, "x")


def test_unpadded_product_is_caught(monkeypatch):
    # forming the product on the N grid itself lets aliases reach retained modes
    monkeypatch.setattr(spectral, "padded_size", lambda n: n)
    assert _fails(ts.test_padded_rhs_against_direct_convolution, 8, 21)


def test_padding_that_keeps_the_nyquist_mode_is_caught(monkeypatch):
    # a truncation that keeps |k_j| <= N/2 (Nyquist included) breaks the zero pattern
    monkeypatch.setattr(spectral, "cutoff_padded", lambda n: n // 2)
    assert _fails(ts.test_padded_rhs_against_direct_convolution, 8, 21)


def test_unpadded_2d_product_is_caught(monkeypatch):
    monkeypatch.setattr(spectral, "padded_size", lambda n: n)
    assert _fails(ts.test_padded_rhs2d_against_direct_convolution, 10, 3, 52)


def test_shell_bins_scaled_by_half_the_grid_are_caught(monkeypatch):
    # bins relative to N/2 instead of the cutoff K
    import test_oracle_diagnostics as td
    from oracle import diagnostics
    monkeypatch.setattr(diagnostics, "cutoff", lambda n: n // 2)
    assert _fails(td.test_bins_are_relative_to_the_cutoff)
    assert _fails(td.test_single_mode_lands_in_its_bin, (0, 3, 4), 8)


def test_dropped_half_spectrum_weight_is_caught(monkeypatch):
    # every half-spectrum entry counted once (the conjugate twins forgotten)
    import test_oracle_diagnostics as td
    from oracle import diagnostics
    monkeypatch.setattr(diagnostics, "weights",
                        lambda n, dim: np.ones((n,) * (dim - 1) + (n // 2 + 1,)))
    assert _fails(td.test_energy_and_shells_against_physical_space, 16, 3)
    assert _fails(td.test_single_mode_lands_in_its_bin, (6, 0, 0), 9)


def test_flipped_buoyancy_sign_is_caught(monkeypatch):
    # gravity along +y: the heavy-over-light interface becomes stable
    import test_oracle_rt as tr
    orig = spectral.rhs_ns2d
    monkeypatch.setattr(spectral, "rhs_ns2d", lambda uh, nu, kappa=0.0, ri=0.0: orig(uh, nu, kappa, -ri))
    assert _fails(tr.test_mode4_grows_at_the_linear_rate)


def test_unclipped_last_rk4_step_is_caught(monkeypatch):
    # ceil(t_end/h) full steps: the run overshoots t_end
    import math
    import test_oracle_stepping as tst
    from oracle import control, stepping

    def overshoot(rhs, u0, t_end, h):
        n = max(1, int(math.ceil(t_end / h - 1e-9)))
        u = u0.copy()
        for _ in range(n):
            u = stepping.rk4_step(rhs, u, h)
        return u, n
    monkeypatch.setattr(control, "rk4_fixed", overshoot)
    assert _fails(tst.test_rk4_fixed_clips_the_last_step, 0.37, 0.1, 4, 0.07)
