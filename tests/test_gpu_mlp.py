"""GPU parity of the step-size proposer's hand-written kernels (forward,
gradient, Adam) against the FP64 oracle, its use inside the controller, and
the collection of training rows from accepted steps."""
import math

import numpy as np
import pytest

from gpu_util import announce
from oracle import control, diagnostics, mlp, spectral
from paper_1810_10197_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ns():
    from paper_1810_10197_amd import ns as mod
    return mod


def weights(seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(rng) + 0.05 * rng.standard_normal(mlp.NPARAM)
    mean = rng.standard_normal(20)
    scale = 0.5 + rng.uniform(0, 1, 20)
    return p, mean, scale


def packed(p, mean, scale):
    return np.concatenate([p, mean, scale]).astype(np.float32)


def f64(w32):
    return w32[:mlp.NPARAM].astype(np.float64), w32[mlp.NPARAM:mlp.NPARAM + 20].astype(np.float64), \
        w32[mlp.NPARAM + 20:].astype(np.float64)


@pytest.fixture(scope="module")
def solver(ns):
    s = ns.Solver(dim=3, n=8, nu=0.01, rhs_precision="fp32")
    yield s
    s.close()


def test_forward_matches_oracle(solver):
    announce("mlp forward")
    w = packed(*weights(1))
    solver.mlp_set_weights(w)
    p, mean, scale = f64(w)
    x = np.random.default_rng(2).standard_normal((33, 20)).astype(np.float32)
    y = solver.mlp_forward(x)
    ref, _ = mlp.forward(p, (x.astype(np.float64) - mean) / scale)
    assert np.abs(y - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())


def test_gradient_matches_oracle(solver):
    announce("mlp gradient")
    w = packed(*weights(3))
    solver.mlp_set_weights(w)
    p, mean, scale = f64(w)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((57, 20)).astype(np.float32)
    t = rng.standard_normal(57).astype(np.float32)
    loss, g = solver.mlp_grad(x, t)
    rl, rg = mlp.loss_and_grad(p, (x.astype(np.float64) - mean) / scale, t.astype(np.float64))
    assert loss == pytest.approx(rl, rel=1e-5)
    assert np.abs(g - rg).max() <= 1e-4 * np.abs(rg).max()
    assert np.linalg.norm(g - rg) <= 1e-5 * np.linalg.norm(rg) * 10


def test_adam_step_matches_oracle(solver):
    announce("mlp adam")
    w = packed(*weights(5))
    solver.mlp_set_weights(w)
    solver.mlp_reset_optimizer()
    p, mean, scale = f64(w)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((40, 20)).astype(np.float32)
    t = rng.standard_normal(40).astype(np.float32)
    z = (x.astype(np.float64) - mean) / scale
    pref, m, v = p.copy(), np.zeros_like(p), np.zeros_like(p)
    for it in range(1, 4):
        solver.mlp_train_batch(x, t, 1e-3)
        _, g = mlp.loss_and_grad(pref, z, t.astype(np.float64))
        pref, m, v = mlp.adam_step(pref, g, m, v, it, lr=1e-3)
    got = solver.mlp_get_weights()[:mlp.NPARAM].astype(np.float64)
    # an Adam step moves every parameter by ~lr; FP32 vs FP64 differ far less
    assert np.abs(got - pref).max() <= 2e-5


@pytest.mark.parametrize("b3", [math.log(1.5), -5.0, 5.0])
def test_mlp_controller_matches_oracle_proposer(ns, b3):
    """Network with W = 0 and output bias b3: after every accepted step the
    proposal is exp(b3), clamped around the controller's factor (the large
    |b3| cases run on the bounds)."""
    n, nu = 16, 0.01
    announce("mlp controller n=%d b3=%g" % (n, b3))
    w = np.zeros(ns.NS_MLP_NWEIGHTS, dtype=np.float32)
    w[mlp.NPARAM - 1] = b3
    w[mlp.NPARAM + 20:] = 1.0
    u0 = inputs.random_isotropic(n, 12)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    y = float(np.float32(b3))
    ref = control.integrate(rhs, u0, 0.6, 0.05, 1e-9, 1e-9, proposer=lambda u, h, e: y)
    s = ns.Solver(dim=3, n=n, nu=nu, rhs_precision="fp64")
    s.mlp_set_weights(w)
    s.set_state(u0[None])
    st = s.integrate(0.6, 0.05, 1e-9, 1e-9, controller="mlp")[0]
    got = s.get_state().cpu().numpy()[0]
    s.close()
    assert (st["n_accept"], st["n_reject"]) == (ref["n_accept"], ref["n_reject"])
    assert np.abs(got - ref["u"]).max() <= 1e-12 * np.abs(ref["u"]).max()


def test_collected_rows_are_pi_trajectory(ns):
    """Rows: features after accepted step n and label log(h_{n+1} / h_n)."""
    n, nu = 16, 0.01
    announce("mlp collect n=%d" % n)
    u0 = inputs.random_isotropic(n, 13)
    rhs = lambda u: spectral.rhs_ns3d(u, nu)
    rows = []

    def record(u, h, errs):
        e = diagnostics.energy(u, 3)
        rows.append((mlp.features(diagnostics.shells(u, 3), e, errs), h))
        return None
    ref = control.integrate(rhs, u0, 0.6, 0.05, 1e-8, 1e-8, proposer=record)
    s = ns.Solver(dim=3, n=n, nu=nu, rhs_precision="fp64")
    s.set_state(u0[None])
    s.mlp_collect(True)
    st = s.integrate(0.6, 0.05, 1e-8, 1e-8)[0]
    x, y, cnt = s.mlp_rows()
    s.close()
    # the last accepted step is clipped to t_end and gives no label
    assert cnt == len(rows) - 2
    for i in range(cnt):
        assert np.abs(x[i] - rows[i][0]).max() <= 1e-5 * max(1.0, np.abs(rows[i][0]).max())
        assert y[i] == pytest.approx(math.log(rows[i + 1][1] / rows[i][1]), abs=1e-6)


def test_pushed_rows_append_to_ring(ns):
    """Rows pushed from the host follow the recorded ones in ring order."""
    announce("mlp push rows")
    rng = np.random.default_rng(5)
    s = ns.Solver(dim=3, n=8, nu=0.01, rhs_precision="fp32")
    x1, y1 = rng.standard_normal((37, 20)).astype(np.float32), rng.standard_normal(37).astype(np.float32)
    x2, y2 = rng.standard_normal((5, 20)).astype(np.float32), rng.standard_normal(5).astype(np.float32)
    s.mlp_push_rows(x1, y1)
    s.mlp_push_rows(x2, y2)
    x, y, cnt = s.mlp_rows()
    s.close()
    assert cnt == 42
    assert np.array_equal(x, np.concatenate([x1, x2])) and np.array_equal(y, np.concatenate([y1, y2]))
