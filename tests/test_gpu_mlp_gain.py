"""What the trained step-size proposer gains over the plain Sec. 2.2.1
controller (the network is trained on the GPU by the library's own forward,
backward and Adam kernels).  Rows come from controller-driven runs of a
64 x 64^3 training ensemble (Taylor--Green and random-phase members, nu
log-uniform in [1e-3, 1e-2]); 16 held-out members of the same distribution
are then integrated to T = 2 at tol 1e-5 with each controller.  The proposer
exists to cut rejected steps (Sec. 4 motivates better controllers); on these
members it must reject fewer steps, spend no more right-hand sides, and end
within 10% of the controller's error against a tight-tolerance FP64 run.
(On the 256^3 Taylor-Green run the controller rejects only about 2 steps in
345, so there the proposer has nothing to cut and gains nothing.)"""
import numpy as np
import pytest

from gpu_util import announce
from paper_1810_10197_amd import inputs

pytestmark = pytest.mark.gpu


def test_trained_proposer_cuts_rejections_on_held_out_members():
    import bench
    from paper_1810_10197_amd import ns
    n, train_members, held_out, T, tol = 64, 64, 16, 2.0, 1e-5
    announce("mlp gain: train on %d x %d^3, test %d held-out members" % (train_members, n, held_out))
    w, info = bench.train_proposer(ns, inputs, members=train_members, n=n, t_end=T, iters=2000)
    print("training:", {k: info[k] for k in ("rows", "loss_first", "loss_last")})
    assert info["loss_last"] < info["loss_first"]
    fields, nus = inputs.ensemble_members(train_members + held_out, n)
    fields, nus = fields[train_members:], nus[train_members:]
    ref = ns.Solver(dim=3, n=n, batch=held_out, nu=nus, rhs_precision="fp64")
    ref.set_state(fields)
    ref.integrate(T, 1e-3, 1e-12, 1e-12)
    uref = ref.get_state().cpu().numpy()
    ref.close()
    res = {}
    for ctl in ("pi", "mlp"):
        s = ns.Solver(dim=3, n=n, batch=held_out, nu=nus, rhs_precision="fp32")
        s.mlp_set_weights(w)
        s.set_state(fields)
        st = s.integrate(T, 1e-3, tol, tol, controller=ctl)
        u = s.get_state().cpu().numpy()
        s.close()
        assert all(x["t"] == T for x in st)
        err = np.linalg.norm((u - uref).reshape(held_out, -1), axis=1) / \
            np.linalg.norm(uref.reshape(held_out, -1), axis=1)
        res[ctl] = (sum(x["n_reject"] for x in st), sum(x["n_rhs"] for x in st), float(err.max()))
    print("held-out (rejections, RHS, max rel L2 error): PI %s, proposer %s" % (res["pi"], res["mlp"]))
    assert res["mlp"][0] < res["pi"][0]
    assert res["mlp"][1] <= res["pi"][1]
    assert res["mlp"][2] <= 1.1 * res["pi"][2]
