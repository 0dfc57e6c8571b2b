"""Exact sign of the Sylvester resultant Res_u(a(., v), b(., v)) of two
bivariate polynomials with FP64 coefficients, at a dyadic v.

Pin helper, independent of the oracle: every coefficient and v are taken as
the exact rationals their doubles denote, each univariate polynomial in u is
scaled by a positive power of two to integer coefficients (which leaves the
sign of the resultant unchanged), and the resultant is computed in exact
integer arithmetic by sympy's subresultant algorithm.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
from sympy.polys.domains import ZZ
from sympy.polys.euclidtools import dup_resultant


def upoly_at(C: np.ndarray, deg: int, v: float):
    """Integer coefficients (leading first) of sum_{i<=deg} (sum_j C[i,j] v^j) u^i,
    times a positive power of two; None when the u^deg coefficient vanishes."""
    fv = Fraction(v)
    pw = [Fraction(1)]
    for _ in range(C.shape[1]):
        pw.append(pw[-1] * fv)
    cs = []
    for i in range(deg + 1):
        s = Fraction(0)
        for j in range(C.shape[1] - i if C.shape[0] == C.shape[1] else C.shape[1]):
            c = float(C[i, j])
            if c != 0.0:
                s += Fraction(c) * pw[j]
        cs.append(s)
    if cs[deg] == 0:
        return None
    den = 1
    for c in cs:
        den = max(den, c.denominator)
    # every denominator is a power of two, so the largest one is their lcm
    return [ZZ(int(c * den)) for c in reversed(cs)]


def res_sign(A: np.ndarray, B: np.ndarray, ma: int, nb: int, v: float):
    """sgn Res_u(a, b) at v for a of u-degree ma and b of u-degree nb (None when
    a leading coefficient vanishes at v)."""
    pa = upoly_at(A, ma, v)
    pb = upoly_at(B, nb, v)
    if pa is None or pb is None:
        return None
    r = dup_resultant(pa, pb, ZZ)
    return (r > 0) - (r < 0)


def udeg(C: np.ndarray) -> int:
    """Highest power of u with a nonzero coefficient row."""
    rows = np.nonzero(np.any(C != 0.0, axis=1))[0]
    return int(rows.max()) if len(rows) else 0
