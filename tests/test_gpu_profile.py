"""The kernel-timing API (a tracing aid around the right-hand side): what each
profile mode brackets, counted over the same sequence of BS5 attempts --
mode 0 the passes (the 3D y/x/y phase as one unit), 1 also every y/x/y
launch, 2 only whole evaluations -- and that the autotuner leaves the mode as
it found it."""
import numpy as np
import pytest

from gpu_util import announce
from paper_1810_10197_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ns():
    from paper_1810_10197_amd import ns as mod
    return mod


def _counts(ns, mode, dim=3, n=64, attempts=3, autotune=False):
    u = inputs.tgv3d(n) if dim == 3 else inputs.tgv2d(n)
    s = ns.Solver(dim=dim, n=n, nu=0.01, rhs_precision="fp32")
    s.set_state(u[None])
    s.profile_mode(mode)
    if autotune:
        s.autotune(reps=1)
    s.profile_start()
    for _ in range(attempts):
        s.step_bs5(0.01, 1e-6, 1e-6)
    out = s.profile_stop()
    s.close()
    return {k: v[1] for k, v in out.items()}, {k: v[0] for k, v in out.items()}


def test_profile_modes_bracket_what_they_say(ns):
    announce("profile modes 3D 64^3")
    c0, ms0 = _counts(ns, 0)
    n_rhs = c0["zinv"]
    assert n_rhs >= 3 * 7 and c0["zfwd"] == n_rhs and c0["slab"] == n_rhs
    assert c0["yinv"] == 0 and c0["rhs"] == 0 and c0["reduce"] == 3 and c0["combine"] > 0
    assert all(ms0[k] > 0 for k in ("zinv", "zfwd", "slab", "combine", "reduce"))
    c1, _ = _counts(ns, 1)
    assert c1["zinv"] == n_rhs and c1["yinv"] >= n_rhs and c1["yinv"] == c1["xpass"] == c1["yfwd"]
    assert c1["rhs"] == 0
    c2, ms2 = _counts(ns, 2)
    assert c2["rhs"] == n_rhs and ms2["rhs"] > 0
    assert c2["zinv"] == c2["zfwd"] == c2["slab"] == c2["yinv"] == 0
    assert c2["reduce"] == 3 and c2["combine"] == c0["combine"]
    # one bracket around each evaluation is no longer than the sum of its parts
    assert ms2["rhs"] / n_rhs <= 1.5 * (ms0["zinv"] + ms0["slab"] + ms0["zfwd"]) / n_rhs


def test_profile_mode_whole_evaluations_2d(ns):
    announce("profile mode 2, 2D 256^2")
    c0, _ = _counts(ns, 0, dim=2, n=256)
    c2, _ = _counts(ns, 2, dim=2, n=256)
    assert c0["zinv"] >= 7 and c2["rhs"] == c0["zinv"] and c2["zinv"] == 0 and c0["rhs"] == 0


def test_autotune_keeps_the_profile_mode(ns):
    announce("autotune keeps profile mode 2")
    c2, _ = _counts(ns, 2, n=256, attempts=1, autotune=True)
    assert c2["rhs"] >= 7 and c2["zinv"] == 0 and c2["slab"] == 0


def test_bad_profile_mode_is_refused(ns):
    s = ns.Solver(dim=3, n=16, nu=0.01, rhs_precision="fp32")
    for mode in (-1, 3):
        with pytest.raises(ns.NsError) as ei:
            s.profile_mode(mode)
        assert ei.value.status == ns.NS_ERR_ARG
    s.close()
