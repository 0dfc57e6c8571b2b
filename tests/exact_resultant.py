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


def paired_sign_hp(A: np.ndarray, B: np.ndarray, ma: int, nb: int, v: float, gap: float = 1e-4, dps: int = 60):
    """Product of sgn b(alpha, v) over the real roots alpha of a(., v), two
    consecutive roots closer than gap * max(1, |alpha|) left out, from the
    exact values of the FP64 coefficients, with roots and values to `dps`
    digits (mpmath).  None when a gap lies within a factor 3 of the rule's
    threshold, or a factor is zero to 30 digits."""
    import mpmath as mp

    with mp.workdps(dps):
        fv = Fraction(v)
        mv = mp.mpf(fv.numerator) / fv.denominator

        def coeffs(C, deg):
            out = []
            for i in range(deg + 1):
                s = mp.mpf(0)
                for j in range(C.shape[1] - i):
                    if C[i, j] != 0.0:
                        s += mp.mpf(float(C[i, j])) * mv ** j
                out.append(s)
            return out

        ac, bc = coeffs(A, ma), coeffs(B, nb)
        rts = mp.polyroots(list(reversed(ac)), maxsteps=500, extraprec=4 * dps)
        tiny = mp.mpf(10) ** (-dps // 2)
        real = sorted(mp.re(r) for r in rts if abs(mp.im(r)) <= tiny * max(1, abs(r)))
        sign = 1
        k = 0
        while k < len(real):
            al = real[k]
            if k + 1 < len(real):
                g = (real[k + 1] - al) / max(1, abs(al))
                if gap / 3 < g < gap * 3:
                    return None
                if g <= gap:
                    k += 2
                    continue
            val = mp.polyval(list(reversed(bc)), al)
            if abs(val) <= tiny * mp.polyval([abs(c) for c in reversed(bc)], abs(al)):
                return None
            if val < 0:
                sign = -sign
            k += 1
        return sign
