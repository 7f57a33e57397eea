"""Automatic step-size control and the adaptive integration loop (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.2.1: with err the scaled error estimate of the attempted step h,

    h_new = h * min(dmax, max(dmin, delta * (1/err)^(1/(q+1))))

with dmax = 2, dmin = 0.01, delta = 0.8 and q the order of the embedded
method (q = 4 for b_hat of BS5).  The step is accepted iff err <= 1 and the
integration continues with h_new; otherwise it is retried from the same
state with h_new.  dmax is 1 for the first step after a rejection (read as:
the h_new produced by the first accepted attempt after a rejection may not
grow).  The initial h is supplied by the caller.

Additions (readings where the paper is silent): err = 0 gives the factor dmax; a
non-finite err rejects with the factor dmin; 50 consecutive rejections stop
the run; the final step is clipped to land on t_end.  An optional PI term
err_prev^beta (beta = 0 reproduces the paper exactly) and an optional
proposer callable (the MLP of the step-size proposer) are supported; after an
accepted step the proposer's factor exp(y) replaces the controller's factor
fac, clamped to [0.7 fac, fac]: the proposer can only shorten a step (to avoid
a rejection), and since 0.7 dmax > 1 a proposer that is wrong cannot hold the
step down (at worst about 1.4 times the controller's steps).
"""
import math

import numpy as np

from . import stepping, tableaux


class StepFailure(RuntimeError):
    pass


class Controller:
    def __init__(self, q=4, safety=0.8, fac_min=0.01, fac_max=2.0, beta=0.0):
        self.alpha = 1.0 / (q + 1)
        self.safety = safety
        self.fac_min = fac_min
        self.fac_max = fac_max
        self.beta = beta

    def factor(self, err, err_prev, cap_at_one):
        """Step-size factor for an attempt with error err.

        cap_at_one: the attempt was accepted right after a rejection.
        Returns the clamped factor; non-finite err returns fac_min.
        """
        if not math.isfinite(err):
            return self.fac_min
        fmax = 1.0 if cap_at_one else self.fac_max
        if err == 0.0:
            return fmax
        fac = self.safety * err ** (-self.alpha)
        if self.beta != 0.0:
            fac *= err_prev ** self.beta
        return min(fmax, max(self.fac_min, fac))


def integrate(rhs, u0, t_end, h0, atol, rtol, tab=tableaux.BS5,
              controller=None, proposer=None, post_step=None,
              max_reject=50):
    """Adaptive integration of d u/dt = rhs(u) from t = 0 to t_end.

    proposer(u_new, h, accepted_errs) -> y, proposed log(h_next / h); used
    after accepted steps (with the controller as fallback when y is not
    finite).  post_step(u) -> u is applied after every accepted step (the
    HIT forcing); it invalidates the FSAL stage.

    Returns a dict with the final state 'u', 't', counters 'n_rhs',
    'n_accept', 'n_reject' and 'history' = list of (t, h, err, accepted).
    """
    ctl = controller or Controller(q=tab.get("order_hat", 4))
    fsal = all(a == b for a, b in zip(tab["A"][-1], tab["b"]))
    u = u0.copy()
    t = 0.0
    h = float(h0)
    k1 = None
    prev_rejected = False
    consec = 0
    err_prev = 1.0
    acc_errs = []
    hist = []
    n_rhs = n_acc = n_rej = 0
    while t < t_end:
        last = h >= t_end - t
        hc = (t_end - t) if last else h
        res = stepping.embedded_attempt(rhs, u, hc, atol, rtol, tab, k1=k1)
        n_rhs += len(tab["b"]) - (1 if k1 is not None else 0)
        if k1 is None:
            k1 = res["k"][0]
        err = res["err"]
        accept = math.isfinite(err) and err <= 1.0
        fac = ctl.factor(err, err_prev, cap_at_one=accept and prev_rejected)
        h_new = hc * fac
        hist.append((t, hc, err, accept))
        if accept:
            t = t_end if last else t + hc
            u = res["u_new"]
            k1 = res["k"][-1] if fsal else None
            if post_step is not None:
                u = post_step(u)
                k1 = None
            acc_errs.append(err)
            if proposer is not None:
                y = proposer(u, hc, list(acc_errs))
                if y is not None and math.isfinite(y):
                    # the proposer may only shorten the controller's step,
                    # by at most 30%: exp(y) is clamped to [0.7 fac, fac]
                    h_new = hc * min(fac, max(0.7 * fac, math.exp(y)))
            err_prev = err
            prev_rejected = False
            consec = 0
            n_acc += 1
            h = h_new
        else:
            prev_rejected = True
            consec += 1
            n_rej += 1
            if consec >= max_reject:
                raise StepFailure("too many consecutive rejections")
            h = h_new
    return {"u": u, "t": t, "n_rhs": n_rhs, "n_accept": n_acc,
            "n_reject": n_rej, "history": hist}


def fixed_steps(rhs, u0, hs, tab=tableaux.BS5, atol=1.0, rtol=1.0):
    """Integrate with a prescribed list of step sizes, always committing.

    Used for fixed-step BS5 and for replaying an accepted-step sequence.
    Returns (u, errs) with the error estimate of every step.
    """
    u = u0.copy()
    k1 = None
    errs = []
    fsal = all(a == b for a, b in zip(tab["A"][-1], tab["b"]))
    for h in hs:
        res = stepping.embedded_attempt(rhs, u, h, atol, rtol, tab, k1=k1)
        u = res["u_new"]
        k1 = res["k"][-1] if fsal else None
        errs.append(res["err"])
    return u, np.array(errs)


def rk4_fixed(rhs, u0, t_end, h):
    """Classical RK4 with a fixed step h; n = ceil(t_end/h) steps, the last
    one shortened so that the run ends exactly at t_end."""
    n = max(1, int(math.ceil(t_end / h - 1e-9)))
    u = u0.copy()
    for i in range(n):
        hc = h if i < n - 1 else t_end - (n - 1) * h
        u = stepping.rk4_step(rhs, u, hc)
    return u, n
