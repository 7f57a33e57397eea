"""One explicit Runge--Kutta step and the embedded error estimate (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.2 compares explicit RK methods on the ODE system d u_hat/dt = f(u_hat)
of Eq. (2).  Stage i is U_i = u_n + h sum_{j<i} a_ij k_j, k_i = f(U_i); the
solution is u_{n+1} = u_n + h sum_i b_i k_i and the embedded solution
v_{n+1} = u_n + h sum_i bhat_i k_i.  The error measure of Sec. 2.2.1 is

    sc_j(k) = TOL_abs + TOL_rel * max(|u_j^(n)(k)|, |u_j^(n+1)(k)|)
    err_j   = sqrt( (1/M) sum_k |(u_j^(n+1)(k) - v_j^(n+1)(k)) / sc_j(k)|^2 )
    err     = max_j err_j

where M is the number of half-spectrum entries (N^2 (N/2+1) in 3D, N (N/2+1)
in 2D), the sum runs over all of them and |.| is the complex modulus.
"""
import numpy as np

from . import tableaux


def rk_stages(rhs, u, h, tab, k1=None):
    """All stage derivatives k_1..k_s of the tableau at (u, h)."""
    A, b, bh, c = tableaux.as_float(tab)
    s = len(b)
    ks = []
    for i in range(s):
        if i == 0:
            ks.append(rhs(u) if k1 is None else k1)
            continue
        Ui = u.copy()
        for j in range(i):
            if A[i][j] != 0.0:
                Ui = Ui + (h * A[i][j]) * ks[j]
        ks.append(rhs(Ui))
    return ks


def rk4_step(rhs, u, h):
    """One step of classical RK4 with fixed step h."""
    ks = rk_stages(rhs, u, h, tableaux.RK4)
    _, b, _, _ = tableaux.as_float(tableaux.RK4)
    out = u.copy()
    for bi, ki in zip(b, ks):
        out = out + (h * bi) * ki
    return out


def error_norm(u_old, u_new, delta, atol, rtol):
    """Per-component err_j and err = max_j err_j of Sec. 2.2.1.

    u_old, u_new, delta have shape (C, ...): delta = u_new - v_new.
    """
    ncomp = u_old.shape[0]
    m = u_old[0].size
    errs = np.zeros(ncomp)
    for j in range(ncomp):
        sc = atol + rtol * np.maximum(np.abs(u_old[j]), np.abs(u_new[j]))
        errs[j] = np.sqrt(np.sum(np.abs(delta[j] / sc) ** 2) / m)
    return float(np.max(errs)), errs


def embedded_attempt(rhs, u, h, atol, rtol, tab=tableaux.BS5, k1=None):
    """One attempt of an embedded pair (BS5 by default).

    Returns a dict with the candidate solution 'u_new' (the b solution),
    the embedded difference 'delta' = u_new - v_new, 'err' and 'errs' of
    Sec. 2.2.1, and 'k' (all stage derivatives).  For an FSAL pair
    (last row of A equal to b) the last stage derivative is f(u_new).
    """
    ks = rk_stages(rhs, u, h, tab, k1=k1)
    _, b, bh, _ = tableaux.as_float(tab)
    u_new = u.copy()
    for bi, ki in zip(b, ks):
        if bi != 0.0:
            u_new = u_new + (h * bi) * ki
    delta = np.zeros_like(u)
    for bi, bhi, ki in zip(b, bh, ks):
        if bi != bhi:
            delta = delta + (h * (bi - bhi)) * ki
    err, errs = error_norm(u, u_new, delta, atol, rtol)
    return {"u_new": u_new, "delta": delta, "err": err, "errs": errs, "k": ks}


def bs5_attempt(rhs, u, h, atol, rtol, k1=None):
    """One BS5 attempt; see embedded_attempt."""
    return embedded_attempt(rhs, u, h, atol, rtol, tableaux.BS5, k1=k1)
