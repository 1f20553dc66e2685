"""Exact rational brute force for tiny inputs (test infrastructure only).

Inverse and determinant of a 3x3 Hermitian matrix with Gaussian-rational
entries (re + i im, re and im ``fractions.Fraction``), from the plain
definition A X = I by Gauss-Jordan elimination in exact arithmetic, so the
result carries no rounding at all.  Used to pin the floating-point oracle
and to write the stored worked example.
"""
from __future__ import annotations

from fractions import Fraction as F


class Q:
    """Exact complex rational."""

    __slots__ = ("re", "im")

    def __init__(self, re, im=0):
        self.re, self.im = F(re), F(im)

    def __add__(self, o):
        return Q(self.re + o.re, self.im + o.im)

    def __sub__(self, o):
        return Q(self.re - o.re, self.im - o.im)

    def __mul__(self, o):
        return Q(self.re * o.re - self.im * o.im, self.re * o.im + self.im * o.re)

    def conj(self):
        return Q(self.re, -self.im)

    def __truediv__(self, o):
        den = o.re * o.re + o.im * o.im
        p = self * o.conj()
        return Q(p.re / den, p.im / den)

    def is_zero(self):
        return self.re == 0 and self.im == 0

    def __eq__(self, o):
        return self.re == o.re and self.im == o.im

    def __repr__(self):
        return f"Q({self.re}, {self.im})"


def unpack(p) -> list[list[Q]]:
    """9 packed components (a, d, f, Re b, Im b, Re c, Im c, Re e, Im e)."""
    a, d, f, br, bi, cr, ci, er, ei = (F(x) for x in p)
    b, c, e = Q(br, bi), Q(cr, ci), Q(er, ei)
    return [[Q(a), b, c], [b.conj(), Q(d), e], [c.conj(), e.conj(), Q(f)]]


def pack(X) -> list[F]:
    return [X[0][0].re, X[1][1].re, X[2][2].re, X[0][1].re, X[0][1].im,
            X[0][2].re, X[0][2].im, X[1][2].re, X[1][2].im]


def inv_det(A):
    """Exact (X, det) by Gauss-Jordan on [A | I]; pivot = first nonzero."""
    M = [[A[r][c] for c in range(3)] + [Q(1 if r == c else 0) for c in range(3)] for r in range(3)]
    det = Q(1)
    for k in range(3):
        p = next((r for r in range(k, 3) if not M[r][k].is_zero()), None)
        if p is None:
            return None, Q(0)
        if p != k:
            M[k], M[p] = M[p], M[k]
            det = Q(0) - det
        piv = M[k][k]
        det = det * piv
        M[k] = [x / piv for x in M[k]]
        for r in range(3):
            if r != k:
                fct = M[r][k]
                M[r] = [x - fct * y for x, y in zip(M[r], M[k])]
    return [row[3:] for row in M], det
