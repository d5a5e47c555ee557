"""Exact rational cubic spline, from the textbook definition -- a test-side pin.

A cubic spline through knots x_0 < ... < x_{n-1} with values y_j is the
piecewise cubic p_i(t) = a_i + b_i t + c_i t^2 + d_i t^3 (t = x - x_i on
[x_i, x_{i+1}]) that

  * interpolates both ends of every piece,
  * has continuous first and second derivatives at the interior knots,
  * meets one condition at each end: zero second derivative (natural) or a
    prescribed first derivative (clamped).

This module sets up those 4(n-1) conditions as a dense linear system and
solves it in exact rational arithmetic.  It uses nothing of the paper's
tridiagonal rows or of its solver, so it pins the oracle's rows, its band
solver and its evaluation formula at once.  The end conditions are those the
paper derives in "Start and End Derivatives" (y'(x_0) = y'_1, y'(x_{n-1}) =
y'_n), and natural ends follow its sentinel (derivative > 0.99e30).
"""
from __future__ import annotations

from fractions import Fraction


def _solve(A, b):
    """Gauss-Jordan elimination over the rationals (any nonzero pivot)."""
    n = len(A)
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        p = M[col][col]
        M[col] = [v / p for v in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [u - f * v for u, v in zip(M[r], M[col])]
    return [M[r][n] for r in range(n)]


def _natural(d) -> bool:
    return float(d) > 0.99e30


class ExactSpline:
    def __init__(self, x, y, start_deriv, end_deriv):
        X = [Fraction(float(v)) for v in x]
        Y = [Fraction(float(v)) for v in y]
        n = len(X)
        assert n >= 3 and all(X[i + 1] > X[i] for i in range(n - 1))
        P = n - 1
        N = 4 * P
        A = []
        b = []

        def row():
            return [Fraction(0)] * N

        H = [X[i + 1] - X[i] for i in range(P)]
        for i in range(P):
            r = row(); r[4 * i] = Fraction(1); A.append(r); b.append(Y[i])
            r = row()
            r[4 * i], r[4 * i + 1], r[4 * i + 2], r[4 * i + 3] = 1, H[i], H[i] ** 2, H[i] ** 3
            A.append(r); b.append(Y[i + 1])
        for i in range(P - 1):
            # p_i'(h_i) = p_{i+1}'(0)
            r = row()
            r[4 * i + 1], r[4 * i + 2], r[4 * i + 3] = 1, 2 * H[i], 3 * H[i] ** 2
            r[4 * (i + 1) + 1] = -1
            A.append(r); b.append(Fraction(0))
            # p_i''(h_i) = p_{i+1}''(0)
            r = row()
            r[4 * i + 2], r[4 * i + 3] = 2, 6 * H[i]
            r[4 * (i + 1) + 2] = -2
            A.append(r); b.append(Fraction(0))
        r = row()
        if _natural(start_deriv):
            r[2] = 2; b.append(Fraction(0))
        else:
            r[1] = 1; b.append(Fraction(float(start_deriv)))
        A.append(r)
        r = row()
        i = P - 1
        if _natural(end_deriv):
            r[4 * i + 2], r[4 * i + 3] = 2, 6 * H[i]; b.append(Fraction(0))
        else:
            r[4 * i + 1], r[4 * i + 2], r[4 * i + 3] = 1, 2 * H[i], 3 * H[i] ** 2
            b.append(Fraction(float(end_deriv)))
        A.append(r)
        coef = _solve(A, b)
        self.X, self.Y, self.H = X, Y, H
        self.coef = [coef[4 * i:4 * i + 4] for i in range(P)]

    def second_derivatives(self):
        out = [2 * c[2] for c in self.coef]
        a, b, c, d = self.coef[-1]
        out.append(2 * c + 6 * d * self.H[-1])
        return out

    def piece(self, q: Fraction) -> int:
        """Left interval at interior knots, end pieces outside [x_0, x_{n-1}]."""
        cnt = sum(1 for v in self.X if v < q)
        return min(max(cnt - 1, 0), len(self.X) - 2)

    def value(self, q) -> Fraction:
        q = Fraction(float(q)) if not isinstance(q, Fraction) else q
        i = self.piece(q)
        a, b, c, d = self.coef[i]
        t = q - self.X[i]
        return a + t * (b + t * (c + t * d))

    def deriv1(self, q) -> Fraction:
        q = Fraction(float(q)) if not isinstance(q, Fraction) else q
        i = self.piece(q)
        a, b, c, d = self.coef[i]
        t = q - self.X[i]
        return b + t * (2 * c + 3 * t * d)

    def deriv2(self, q) -> Fraction:
        q = Fraction(float(q)) if not isinstance(q, Fraction) else q
        i = self.piece(q)
        a, b, c, d = self.coef[i]
        t = q - self.X[i]
        return 2 * c + 6 * t * d
