"""Failure handling and determinism on the GPU, with every condition forced
from the host so that all kernels run to completion: a non-finite state is
rejected attempt after attempt until the consecutive-rejection limit stops
the run (Sec. 2.2.1: rejection is the only recovery); a proposer whose output
is not finite falls back to the controller's own factor; and repeated runs
are bitwise equal (fixed-order reductions, no races)."""
import numpy as np
import pytest

from gpu_util import announce
from paper_1810_10197_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ns():
    from paper_1810_10197_amd import ns as mod
    return mod


def test_nonfinite_state_is_rejected_until_the_run_stops(ns):
    n = 16
    announce("nan state: rejections then step failure")
    u = inputs.random_isotropic(n, 3)
    u[0, 1, 2, 3] = np.nan
    s = ns.Solver(dim=3, n=n, nu=0.01, rhs_precision="fp32")
    s.set_state(u[None])
    st, errs = s.step_bs5(0.01, 1e-6, 1e-6)
    assert st == ns.NS_STEP_REJECTED and not np.isfinite(errs[0])
    with pytest.raises(ns.NsError) as ei:
        s.integrate(1.0, 0.01, 1e-6, 1e-6)
    assert ei.value.status == ns.NS_ERR_STEPFAIL
    s.close()


def test_nonfinite_proposer_falls_back_to_the_controller(ns):
    """NaN network weights: every proposal is NaN, so each step uses the
    Sec. 2.2.1 factor -- the run equals the plain controller's bitwise."""
    n, nu = 16, 0.02
    announce("nan proposer == pi")
    u0 = inputs.random_isotropic(n, 8)
    out = []
    for ctl in ("pi", "mlp"):
        s = ns.Solver(dim=3, n=n, nu=nu, rhs_precision="fp64")
        s.mlp_set_weights(np.full(ns.NS_MLP_NWEIGHTS, np.nan, dtype=np.float32))
        s.set_state(u0[None])
        st = s.integrate(0.4, 0.4, 1e-10, 1e-10, controller=ctl)[0]
        out.append((st, s.get_state().cpu().numpy()[0]))
        s.close()
    (s1, u1), (s2, u2) = out
    assert s1["n_reject"] >= 1
    assert (s1["n_accept"], s1["n_reject"], s1["n_rhs"]) == (s2["n_accept"], s2["n_reject"], s2["n_rhs"])
    assert np.array_equal(u1.view(np.float64), u2.view(np.float64))


def test_repeated_runs_are_bitwise_equal(ns):
    """The same right-hand side at 256^3 and the same adaptive ensemble run,
    twice each: identical bits (no LDS race, no order-dependent sum)."""
    announce("run twice: rhs 256 and ensemble integrate")
    u = inputs.random_isotropic(256, 99)
    s = ns.Solver(dim=3, n=256, nu=1.0 / 1600, rhs_precision="fp32")
    f1 = s.rhs(u[None]).cpu().numpy()
    f2 = s.rhs(u[None]).cpu().numpy()
    s.close()
    assert np.array_equal(f1.view(np.float64), f2.view(np.float64))
    fields, nus = inputs.ensemble_members(4, 32)
    res = []
    for _ in range(2):
        s = ns.Solver(dim=3, n=32, batch=4, nu=nus, rhs_precision="fp32")
        s.set_state(fields)
        st = s.integrate(0.3, 0.05, 1e-9, 1e-9)
        res.append((st, s.get_state().cpu().numpy()))
        s.close()
    assert [x["n_rhs"] for x in res[0][0]] == [x["n_rhs"] for x in res[1][0]]
    assert np.array_equal(res[0][1].view(np.float64), res[1][1].view(np.float64))


def test_bad_arguments_are_refused_without_a_launch(ns):
    """Argument errors come back as errors before any kernel runs: a state of
    the wrong shape (the binding), an unsupported size and a non-positive
    step (the C ABI); the solver stays usable afterwards."""
    n = 16
    announce("argument errors")
    with pytest.raises(ValueError):
        ns.Solver(dim=3, n=20, nu=0.01)
    s = ns.Solver(dim=3, n=n, batch=2, nu=0.01, rhs_precision="fp32")
    u = inputs.random_isotropic(n, 2)
    with pytest.raises(ValueError):
        s.set_state(u)                          # one member for a batch of two
    with pytest.raises(ValueError):
        s.set_state(np.stack([u, u]).reshape(2, 3, n, n // 2 + 1, n))   # same size, other shape
    s.set_state(np.stack([u, u]))
    with pytest.raises(ns.NsError) as ei:
        s.step_rk4(-0.1)
    assert ei.value.status == ns.NS_ERR_ARG
    s.step_rk4(0.01)
    got = s.get_state().cpu().numpy()
    assert np.all(np.isfinite(got.view(np.float64)))
    assert np.array_equal(got[0].view(np.float64), got[1].view(np.float64))
    s.close()
