"""Runge--Kutta coefficients as exact rationals (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* RK4: the classical four-stage method (Sec. 2.2).  The paper does not print
  its tableau; the textbook coefficients are used.
* BS5: the Bogacki--Shampine 5(4) pair, Appendix A.3, Eq. (8).  The solution
  is advanced with b; the embedded weights b_hat (not b*) estimate the error
  (Sec. 2.2).  The last row of A equals b, so the pair is FSAL.
* DP5: the Dormand--Prince 5(4) pair, Appendix A.1, Eq. (7).

Each tableau is a dict with keys 'A' (s x s, strictly lower triangular),
'b', 'bhat' (embedded, None for RK4) and 'c'; entries are Fractions.
"""
from fractions import Fraction as F


def _pad(rows, s):
    out = []
    for r in rows:
        out.append([F(x) for x in r] + [F(0)] * (s - len(r)))
    return out


RK4 = {
    "A": _pad([[], [F(1, 2)], [0, F(1, 2)], [0, 0, 1]], 4),
    "b": [F(1, 6), F(1, 3), F(1, 3), F(1, 6)],
    "bhat": None,
    "c": [F(0), F(1, 2), F(1, 2), F(1)],
    "order": 4,
}

BS5 = {
    "A": _pad([
        [],
        [F(1, 6)],
        [F(2, 27), F(4, 27)],
        [F(183, 1372), F(-162, 343), F(1053, 1372)],
        [F(68, 297), F(-4, 11), F(42, 143), F(1960, 3861)],
        [F(597, 22528), F(81, 352), F(63099, 585728), F(58653, 366080),
         F(4617, 20480)],
        [F(174197, 959244), F(-30942, 79937), F(8152137, 19744439),
         F(666106, 1039181), F(-29421, 29068), F(482048, 414219)],
        [F(587, 8064), F(0), F(4440339, 15491840), F(24353, 124800),
         F(387, 44800), F(2152, 5985), F(7267, 94080)],
    ], 8),
    "b": [F(587, 8064), F(0), F(4440339, 15491840), F(24353, 124800),
          F(387, 44800), F(2152, 5985), F(7267, 94080), F(0)],
    "bhat": [F(2479, 34992), F(0), F(123, 416), F(612941, 3411720),
             F(43, 1440), F(2272, 6561), F(79937, 1113912), F(3293, 556956)],
    "c": [F(0), F(1, 6), F(2, 9), F(3, 7), F(2, 3), F(3, 4), F(1), F(1)],
    "order": 5,
    "order_hat": 4,
}

DP5 = {
    "A": _pad([
        [],
        [F(1, 5)],
        [F(3, 40), F(9, 40)],
        [F(44, 45), F(-56, 15), F(32, 9)],
        [F(19372, 6561), F(-25360, 2187), F(64448, 6561), F(-212, 729)],
        [F(9017, 3168), F(-355, 33), F(46732, 5247), F(49, 176),
         F(-5103, 18656)],
        [F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784),
         F(11, 84)],
    ], 7),
    "b": [F(35, 384), F(0), F(500, 1113), F(125, 192), F(-2187, 6784),
          F(11, 84), F(0)],
    "bhat": [F(5179, 57600), F(0), F(7571, 16695), F(393, 640),
             F(-92097, 339200), F(187, 2100), F(1, 40)],
    "c": [F(0), F(1, 5), F(3, 10), F(4, 5), F(8, 9), F(1), F(1)],
    "order": 5,
    "order_hat": 4,
}


def as_float(tab):
    """The same tableau with float entries (A, b, bhat, c)."""
    A = [[float(x) for x in row] for row in tab["A"]]
    b = [float(x) for x in tab["b"]]
    bh = None if tab["bhat"] is None else [float(x) for x in tab["bhat"]]
    c = [float(x) for x in tab["c"]]
    return A, b, bh, c
