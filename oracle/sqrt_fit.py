"""Oracle-side piecewise rational square-root fit (Sec. 4.4).

TEST INFRASTRUCTURE: used only by the test-suite and the oracle wrapper.

The paper approximates sqrt(x) on [0,1] by six pieces, each a (1,1) rational
function (c0 + c1 x)/(d0 + d1 x), with error below 1e-3; its coefficient table
is in a supplement that is not available.  Reading: the pieces are the
breakpoints below and each piece is the best (minimax) (1,1) rational
approximation of sqrt on it, normalised to d0 = 1.  The minimax approximation
is unique and is characterised by an error curve that equioscillates at four
points (Chebyshev alternation for numerator and denominator degree 1), which is
what this Remez exchange computes and what the tests check.
"""
from __future__ import annotations

import numpy as np

BREAKPOINTS = (0.0, 5.0e-4, 9.2e-3, 6.1e-2, 0.256, 0.809, 1.0)


def _grid(a: float, b: float, n: int = 40001) -> np.ndarray:
    t = np.linspace(0.0, 1.0, n)
    return a + (b - a) * t * t if a == 0.0 else a + (b - a) * t


def _err(c, x):
    c0, c1, d1 = c
    return (c0 + c1 * x) / (1.0 + d1 * x) - np.sqrt(x)


def _solve_reference(xr, guess):
    """Newton on c0 + c1 x_k - (sqrt(x_k) + (-1)^k E)(1 + d1 x_k) = 0, k = 0..3."""
    z = np.asarray(guess, dtype=np.float64)  # c0, c1, d1, E
    s = np.array([1.0, -1.0, 1.0, -1.0])
    f = np.sqrt(xr)
    for _ in range(100):
        c0, c1, d1, E = z
        g = c0 + c1 * xr - (f + s * E) * (1.0 + d1 * xr)
        J = np.stack([np.ones(4), xr, -(f + s * E) * xr, -s * (1.0 + d1 * xr)], axis=1)
        dz = np.linalg.solve(J, g)
        z = z - dz
        if np.max(np.abs(dz)) < 1e-16 * (1.0 + np.max(np.abs(z))):
            break
    return z


def _alternating_extrema(x, e):
    # candidate points: ends and interior local extrema of e
    idx = [0]
    de = np.diff(e)
    for i in range(1, len(e) - 1):
        if de[i - 1] * de[i] <= 0:
            idx.append(i)
    idx.append(len(e) - 1)
    idx = np.asarray(sorted(set(idx)))
    # merge consecutive same-sign candidates keeping the largest |e|
    keep = []
    for i in idx:
        if keep and np.sign(e[i]) == np.sign(e[keep[-1]]):
            if abs(e[i]) > abs(e[keep[-1]]):
                keep[-1] = i
        else:
            keep.append(i)
    # choose 4 consecutive with the largest minimum |e|
    best, bi = -1.0, 0
    for k in range(0, max(1, len(keep) - 3)):
        m = min(abs(e[j]) for j in keep[k:k + 4]) if len(keep) >= 4 else 0
        if m > best:
            best, bi = m, k
    return np.asarray([x[j] for j in keep[bi:bi + 4]])


def fit_piece(a: float, b: float, iters: int = 30):
    """Minimax (1,1) rational fit of sqrt on [a,b]: returns (c0, c1, d0=1, d1), max error."""
    xr = a + (b - a) * (1.0 - np.cos(np.arange(4) * np.pi / 3.0)) / 2.0
    # start from interpolation through three inner points with E = 0
    x3 = xr[:3]
    A = np.stack([np.ones(3), x3, -np.sqrt(x3) * x3], axis=1)
    c0, c1, d1 = np.linalg.solve(A, np.sqrt(x3))
    z = np.array([c0, c1, d1, 0.0])
    x = _grid(a, b)
    for _ in range(iters):
        z = _solve_reference(xr, z)
        e = _err(z[:3], x)
        nxr = _alternating_extrema(x, e)
        if len(nxr) < 4:
            break
        if np.max(np.abs(nxr - xr)) <= 1e-15 * max(b, 1e-300):
            xr = nxr
            break
        xr = nxr
    z = _solve_reference(xr, z)
    e = _err(z[:3], x)
    return (float(z[0]), float(z[1]), 1.0, float(z[2])), float(np.max(np.abs(e)))


def fit_table(breakpoints=BREAKPOINTS):
    """[(c0, c1, d0, d1)] per piece and the per-piece max errors."""
    coefs, errs = [], []
    for i in range(len(breakpoints) - 1):
        c, e = fit_piece(breakpoints[i], breakpoints[i + 1])
        coefs.append(c)
        errs.append(e)
    return np.asarray(coefs, dtype=np.float64), np.asarray(errs)
