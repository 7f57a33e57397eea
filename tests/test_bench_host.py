"""Host-side logic of the benchmark's studies, on the CPU: the reference
curve and error of the Re = 280 Taylor--Green test (Sec. 3.1), and the byte
model of the roofline."""
import math

import numpy as np
import pytest

import bench


def test_quadratic_interpolant_is_exact_on_quadratics():
    tref = np.linspace(0.0, 9.4, 95)              # uneven use below
    q = lambda t: 0.3 - 1.7 * t + 0.25 * t * t
    ref = bench.quadratic_interpolant(tref, q(tref))
    for t in [0.0, 0.013, 1.0, 4.321, 9.39, 9.4]:
        assert ref(t) == pytest.approx(q(t), rel=1e-12, abs=1e-12)


def test_quadratic_interpolant_error_is_third_order():
    """On a smooth curve the local error of the three-point quadratic falls
    as the cube of the sample spacing."""
    errs = []
    for m in (50, 100, 200):
        tref = np.linspace(0.0, 2.0, m + 1)
        ref = bench.quadratic_interpolant(tref, np.sin(3 * tref))
        ts = np.linspace(0.0, 2.0, 997)
        errs.append(max(abs(ref(t) - math.sin(3 * t)) for t in ts))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 7.0 < r1 < 9.0 and 7.0 < r2 < 9.0, errs


def test_max_deviation_uses_the_arms_own_times():
    tref = np.linspace(0.0, 1.0, 11)
    ref = bench.quadratic_interpolant(tref, tref ** 2)
    ts = [0.0, 0.25, 0.5, 1.0]
    ys = [0.0, 0.0625 + 3e-3, 0.25 - 5e-3, 1.0]
    assert bench.max_deviation(ts, ys, ref) == pytest.approx(5e-3, rel=1e-9)
    assert bench.max_deviation(ts, ys[:3] + [float("nan")], ref) == float("inf")


def test_pass_bytes_match_the_pencil_model_at_256():
    """1,715.9 MB per FP32 right-hand side from an FP64 state at 256^3."""
    pb = bench.pass_bytes(256)
    assert sum(pb.values()) == pytest.approx(1.7159e9, rel=1e-4)
    assert pb["yinv"] == 6 * 86 * 171 * 256 * 8 + 6 * 86 * 256 * 256 * 8


def test_pass_bytes_2d_with_fp32_stage_inputs():
    """2D Boussinesq at 1024^2 (K = 341: 342 x 683 retained modes, three
    components; four transformed fields of 1024 x 342 FP32 values): Q1 reads
    the stage input in FP32 (8 bytes) instead of FP64 (16), Q3 too, and writes
    f in FP64 plus its FP32 copy in six of seven evaluations."""
    mr, col = 342 * 683, 4 * 1024 * 342 * 8
    pb64 = bench.pass_bytes_2d(1024)
    pb32 = bench.pass_bytes_2d(1024, stage32=True)
    assert pb64 == {"zinv": 3 * mr * 16 + col, "xpass": 2 * col, "zfwd": col + 6 * mr * 16}
    assert pb32["zinv"] == 3 * mr * 8 + col
    assert pb32["xpass"] == pb64["xpass"]
    assert pb32["zfwd"] == col + 3 * mr * 8 + 3 * mr * 16 + 3 * mr * 8 * 6 // 7
    assert sum(pb64.values()) / 1e6 == pytest.approx(78.46, abs=0.01)
    assert sum(pb32.values()) / 1e6 == pytest.approx(72.05, abs=0.01)
