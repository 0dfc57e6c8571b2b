"""Pins of the two-bounce (TT) oracle.

* piecewise rational sqrt fit (Sec. 4.4): error below the paper's 1e-3 bound on
  every piece, and equioscillation at four points (Chebyshev alternation, which
  characterises the minimax (1,1) rational fit);
* structural degrees of the bivariate TT system;
* sign of det R(v) (Eq. eq_bezout, Gaussian elimination) against the sign of the
  exact Sylvester resultant computed by sympy: their ratio is a constant in v;
* flat parallel slab: the unique refraction path from a 1-D monotone equation.
"""
import math

import numpy as np
import pytest
import sympy as sp

import oracle
import sqrt_fit
from paper_2405_13409_amd import scenes


def test_sqrt_fit_error_bound_and_alternation():
    coefs, errs = sqrt_fit.fit_table()
    bp = sqrt_fit.BREAKPOINTS
    assert len(coefs) == 6
    for i in range(6):
        a, b = bp[i], bp[i + 1]
        x = np.linspace(a, b, 400001)
        c0, c1, d0, d1 = coefs[i]
        e = (c0 + c1 * x) / (d0 + d1 * x) - np.sqrt(x)
        assert np.max(np.abs(e)) < 1e-3
        # four alternating extrema of (nearly) equal magnitude
        ext = sqrt_fit._alternating_extrema(x, e)
        assert len(ext) == 4
        ee = (c0 + c1 * ext) / (d0 + d1 * ext) - np.sqrt(ext)
        assert np.all(np.sign(ee[1:]) == -np.sign(ee[:-1]))
        assert np.max(np.abs(ee)) - np.min(np.abs(ee)) < 1e-3 * np.max(np.abs(ee))


def _slab(h=0.3, size=4.0):
    P = np.array([[-size, -size, 0.0], [size, -size, 0.0], [0.0, size, 0.0],
                  [-size, -size, h], [size, -size, h], [0.0, size, h]])
    N = np.array([[0, 0, -1.0]] * 3 + [[0, 0, 1.0]] * 3)
    tri = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    return P, N, tri


def _slab_path(x0, x3, h, eta):
    """Unique path through a slab 0 <= z <= h with IOR eta inside: the in-plane
    offset equation a tan(t) + c tan(t) + h tan(asin(sin t/eta)) = L, monotone in t."""
    a = -x0[2]
    c = x3[2] - h
    L = np.linalg.norm(x3[:2] - x0[:2])
    e = (x3[:2] - x0[:2]) / L

    def g(t):
        return (a + c) * math.tan(t) + h * math.tan(math.asin(math.sin(t) / eta)) - L

    lo, hi = 0.0, math.pi / 2 - 1e-12
    for _ in range(300):
        m = 0.5 * (lo + hi)
        if not (lo < m < hi):
            break
        if g(m) < 0:
            lo = m
        else:
            hi = m
    t = 0.5 * (lo + hi)
    s1 = a * math.tan(t)
    s2 = h * math.tan(math.asin(math.sin(t) / eta))
    x1 = np.array([*(x0[:2] + s1 * e), 0.0])
    x2 = np.array([*(x0[:2] + (s1 + s2) * e), h])
    return x1, x2


def _bary(P3, x):
    A = np.stack([P3[1] - P3[0], P3[2] - P3[0]], 1)
    uv, *_ = np.linalg.lstsq(A, x - P3[0], rcond=None)
    return uv


def _tri_around(rng, x, z, size):
    """A random triangle in the plane z = const whose interior holds x."""
    ang = np.sort(rng.uniform(0, 2 * np.pi, 3))
    while np.max(np.diff(np.concatenate([ang, [ang[0] + 2 * np.pi]]))) > 0.8 * 2 * np.pi / 2:
        ang = np.sort(rng.uniform(0, 2 * np.pi, 3))
    r = size * rng.uniform(0.6, 1.0, 3)
    P = np.stack([x[0] + r * np.cos(ang), x[1] + r * np.sin(ang), np.full(3, z)], 1)
    return P


@pytest.mark.parametrize("seed", range(16))
def test_flat_slab_unique_path(seed):
    rng = np.random.default_rng(50 + seed)
    h = 0.3
    x0 = np.array([rng.uniform(-0.8, 0.8), rng.uniform(-0.8, 0.8), -rng.uniform(0.5, 1.5)])
    x3 = np.array([rng.uniform(-0.8, 0.8), rng.uniform(-0.8, 0.8), h + rng.uniform(0.5, 1.5)])
    x1, x2 = _slab_path(x0, x3, h, 1.5)
    P1 = _tri_around(rng, x1, 0.0, 0.4)
    P2 = _tri_around(rng, x2, h, 0.4)
    P = np.concatenate([P1, P2])
    N = np.array([[0, 0, -1.0]] * 3 + [[0, 0, 1.0]] * 3)
    tri = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    uv1 = _bary(P1, x1)
    uv2 = _bary(P2, x2)
    if min(uv1.min(), 1 - uv1.sum(), uv2.min(), 1 - uv2.sum()) < 1e-3:
        pytest.skip("path too close to an edge")
    sols, diag = oracle.solve_tt(P, N, tri, x0[None], x3[None], [0], [0], [0], [1])
    assert len(sols) == 1
    s = sols[0]
    assert abs(s["u1"] - uv1[0]) < 1e-10 and abs(s["v1"] - uv1[1]) < 1e-10
    assert abs(s["u2"] - uv2[0]) < 1e-10 and abs(s["v2"] - uv2[1]) < 1e-10


def test_tt_structural_degrees():
    mesh = scenes.caustic_sphere()
    x0 = np.array([0.05, -0.02, -1.0])
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE[0]
    # a bottom triangle and a (non-antipodal) top triangle; an antipodal pair has
    # parallel planes, which cancels the top u-powers (as for the slab below)
    c = mesh.P[mesh.tri].mean(1)
    t1 = int(np.argmin(c[:, 2]))
    t2 = int(np.argmax(c[:, 2] + 0.4 * c[:, 0]))
    A, B, n, fl = oracle.coeffs_tt(mesh.P, mesh.N, mesh.tri, t1, t2, x0, x3)
    # sphere normals equal position/radius: the top u-powers cancel (14 and 40)
    assert A.shape[0] - 1 == 16 and B.shape[0] - 1 == 46 and n == 40
    P, N, tri = _slab()
    A, B, n, fl = oracle.coeffs_tt(P, N, tri, 0, 1, np.array([0.1, 0.2, -1.0]), np.array([0.0, 0.1, 1.5]))
    # parallel flat planes cancel the top u-powers exactly (degrees 5 and 14)
    assert A.shape[0] - 1 == 7 and B.shape[0] - 1 == 20 and n == 14


def _sympy_res_sign(A, B, n, v):
    u = sp.symbols("u")
    vv = sp.Rational(v)

    def upoly(C, deg):
        cs = []
        for i in range(deg + 1):
            s = sp.Integer(0)
            for j in range(C.shape[0] - i):
                if C[i, j] != 0.0:
                    s += sp.Rational(float(C[i, j])) * vv ** j
            cs.append(s)
        return sp.Poly(list(reversed(cs)), u)

    pa = upoly(A, A.shape[0] - 1)
    pb = upoly(B, n)
    r = sp.resultant(pa, pb)
    return int(sp.sign(r))


@pytest.mark.parametrize("seed", range(6))
def test_det_sign_matches_exact_resultant(seed):
    """Gaussian-elimination sign of det R(v) vs the sign of the exact Sylvester
    resultant: det R = +- lc_u(b)^(n - deg a) Res_u(a, b), so the sign ratio is
    constant in v.  Random well-conditioned bivariate a (deg 3) and b (deg 6)."""
    rng = np.random.default_rng(40 + seed)
    A = np.zeros((4, 4))
    B = np.zeros((7, 7))
    for i in range(4):
        for j in range(4 - i):
            A[i, j] = rng.normal()
    for i in range(7):
        for j in range(7 - i):
            B[i, j] = rng.normal()
    B[6, 0] = 1.0 + abs(B[6, 0])   # constant leading coefficient in u
    n = 6
    ratios = set()
    for v in np.linspace(0.0137, 0.9871, 15):
        s_det = oracle.det_sign(A, B, n, float(v))
        s_res = _sympy_res_sign(A, B, n, float(v))
        if s_res != 0:
            ratios.add(s_det * s_res)
    assert len(ratios) == 1
