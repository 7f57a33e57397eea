"""The batched ensemble at its workload size (128 independent 64^3 runs, even
members Taylor--Green, odd members random-phase fields, nu log-uniform in
[1e-3, 1e-2]) against the FP64 oracle, member by member: one BS5 attempt of
the whole batch (Appendix A.3, Eq. (8)) and a short adaptive run with the
Sec. 2.2.1 controller replayed as a HIP graph."""
import numpy as np
import pytest

from gpu_util import announce, per_field_rel_l2
from oracle import control, spectral, stepping
from paper_1810_10197_amd import inputs

pytestmark = pytest.mark.gpu

N, B = 64, 128


@pytest.fixture(scope="module")
def ns():
    from paper_1810_10197_amd import ns as mod
    return mod


@pytest.fixture(scope="module")
def members():
    fields, nus = inputs.ensemble_members(B, N)
    even, odd = np.arange(0, B, 2), np.arange(1, B, 2)
    # both field types, each at the smallest and the largest viscosity drawn
    picks = [int(even[np.argmin(nus[even])]), int(even[np.argmax(nus[even])]),
             int(odd[np.argmin(nus[odd])]), int(odd[np.argmax(nus[odd])])]
    return fields, nus, picks


def test_ensemble_bs5_attempt_against_oracle(ns, members):
    """One BS5 attempt of all 128 members at h = 0.02: the FP32 right-hand
    side (the workload's precision) within 1e-6 per-field relative L2 of the
    oracle's FP64 attempt, and the FP64 right-hand side within 1e-12 with the
    embedded error estimate of every picked member within 1e-6 (the estimate
    is a difference of stage sums that cancel to about 1e-8 of their size for
    the low-viscosity Taylor--Green members, so FP64 rounding of the sums,
    summed in another order than the oracle's, shows at about 1e-8 of it)."""
    fields, nus, picks = members
    h, tol = 0.02, 1e-6
    announce("ensemble %d x %d^3 bs5 attempt, members %s" % (B, N, picks))
    got = {}
    for prec in ("fp32", "fp64"):
        s = ns.Solver(dim=3, n=N, batch=B, nu=nus, rhs_precision=prec)
        s.set_state(fields)
        st, errs = s.step_bs5(h, tol, tol, force=True)
        u = s.get_state()
        got[prec] = (u[picks].cpu().numpy(), np.asarray(errs)[picks])
        s.close()
        del u
    for j, m in enumerate(picks):
        ref = stepping.bs5_attempt(lambda x: spectral.rhs_ns3d(x, nus[m]), fields[m], h, tol, tol)
        e32 = per_field_rel_l2(got["fp32"][0][j], ref["u_new"])
        e64 = np.abs(got["fp64"][0][j] - ref["u_new"]).max() / np.abs(ref["u_new"]).max()
        print("member %d (nu %.4g): fp32 per-field rel L2 %s, fp64 max rel %.2e, err %.6e vs %.6e"
              % (m, nus[m], e32, e64, got["fp64"][1][j], ref["err"]))
        assert max(e32) <= 1e-6, (m, e32)
        assert e64 <= 1e-12, (m, e64)
        assert abs(got["fp64"][1][j] / ref["err"] - 1) <= 1e-6, (m, got["fp64"][1][j], ref["err"])


def test_ensemble_adaptive_run_against_oracle(ns, members):
    """The whole batch integrated to t = 0.3 from h0 = 0.3 at tol 1e-9 (too
    long a first step for the random-phase members, which reject it), FP64
    right-hand side, one
    captured attempt replayed per step: the picked members take exactly the
    oracle controller's decisions (accepted, rejected, right-hand sides) and
    end on its state."""
    fields, nus, picks = members
    t_end, h0, tol = 0.3, 0.3, 1e-9
    announce("ensemble %d x %d^3 adaptive run, members %s" % (B, N, picks))
    s = ns.Solver(dim=3, n=N, batch=B, nu=nus, rhs_precision="fp64")
    s.set_state(fields)
    stats = s.integrate(t_end, h0, tol, tol)
    u = s.get_state()
    got = u[picks].cpu().numpy()
    s.close()
    del u
    assert all(st["t"] == t_end for st in stats)
    rejected = 0
    for j, m in enumerate(picks):
        ref = control.integrate(lambda x: spectral.rhs_ns3d(x, nus[m]), fields[m], t_end, h0, tol, tol)
        st = stats[m]
        print("member %d: gpu (%d, %d, %d) oracle (%d, %d, %d)" % (
            m, st["n_accept"], st["n_reject"], st["n_rhs"], ref["n_accept"], ref["n_reject"], ref["n_rhs"]))
        assert (st["n_accept"], st["n_reject"], st["n_rhs"]) == (ref["n_accept"], ref["n_reject"], ref["n_rhs"])
        assert np.abs(got[j] - ref["u"]).max() <= 1e-12 * np.abs(ref["u"]).max()
        rejected += ref["n_reject"]
    assert rejected >= 1, "no picked member rejected a step: the controller's retry is not exercised"
