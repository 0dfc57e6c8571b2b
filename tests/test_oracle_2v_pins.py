"""Pins of the oracle's two-vertex chains with a reflection (RR, RT, TR; Sec.
4.5 with the reflected direction of Eq. eq_431_di and the product form of Eq.
eq_pf_result at a reflecting second vertex).

* flat triangles: closed forms by mirror images (a reflection unfolds the
  path) plus, for a refraction, the 1-D monotone Snell equation;
* structural degrees of the mapped systems;
* curved (interpolated-normal) mirror-gap scene: every forward-traced path is
  found, and on the tuples around each path the oracle's set equals the
  brute-force set (tests/bruteforce_tt.py) wherever the 100-piece scan agrees
  with a 10^4-piece scan;
* det sign: the product formula against the exact resultant sign.
"""
import math

import numpy as np
import pytest

import bruteforce_tt as bt
import exact_resultant as er
import oracle
import twovertex_cases as tc


def _mirror(x, p, n):
    return x - 2.0 * ((x - p) @ n) * n


def _plane_hit(a, b, p, n):
    """Point where the segment a -> b crosses the plane (p, n), or None."""
    da, db = (a - p) @ n, (b - p) @ n
    if da * db >= 0:
        return None
    s = da / (da - db)
    return a + s * (b - a)


def _snell_point(xa, xb, p, n, eta_a, eta_b):
    """Refraction point on the plane (p, n) of the path xa -> xb (opposite sides)."""
    ha, hb = (xa - p) @ n, (xb - p) @ n
    if ha * hb >= 0:
        return None
    pa, pb = xa - ha * n, xb - hb * n
    L = np.linalg.norm(pb - pa)
    e = (pb - pa) / L
    ha, hb = abs(ha), abs(hb)

    def f(s):
        return eta_a * s / math.hypot(s, ha) - eta_b * (L - s) / math.hypot(L - s, hb)

    lo, hi = 0.0, L
    for _ in range(200):
        m = 0.5 * (lo + hi)
        if not (lo < m < hi):
            break
        if f(m) < 0:
            lo = m
        else:
            hi = m
    return pa + 0.5 * (lo + hi) * e


def _tri_around(rng, x, p, n, size=0.5):
    """A random triangle in the plane (p, n) whose interior holds x."""
    a = np.cross(n, [1.0, 0, 0] if abs(n[0]) < 0.9 else [0, 1.0, 0])
    a /= np.linalg.norm(a)
    b = np.cross(n, a)
    ang = np.sort(rng.uniform(0, 2 * np.pi, 3))
    while np.max(np.diff(np.concatenate([ang, [ang[0] + 2 * np.pi]]))) > 0.8 * np.pi:
        ang = np.sort(rng.uniform(0, 2 * np.pi, 3))
    r = size * rng.uniform(0.6, 1.0, 3)
    return np.stack([x + r[k] * (math.cos(ang[k]) * a + math.sin(ang[k]) * b) for k in range(3)])


def _bary(P3, x):
    A = np.stack([P3[1] - P3[0], P3[2] - P3[0]], 1)
    uv, *_ = np.linalg.lstsq(A, x - P3[0], rcond=None)
    return uv


def _planar_case(chain, rng):
    """Random flat planes M1, M2 and endpoints with the closed-form path."""
    n1 = np.array([rng.uniform(-0.6, 0.6), rng.uniform(-0.6, 0.6), 1.0])
    n1 /= np.linalg.norm(n1)
    n2 = np.array([rng.uniform(-0.6, 0.6), rng.uniform(-0.6, 0.6), -1.0])
    n2 /= np.linalg.norm(n2)
    p1 = np.array([0.0, 0.0, 0.0])
    p2 = np.array([0.0, 0.0, 1.0])
    z0, z3, eta = tc.SETUPS[chain]
    x0 = np.array([rng.uniform(-1.0, 1.0), rng.uniform(-1.0, 1.0), z0])
    x3 = np.array([rng.uniform(-1.0, 1.0), rng.uniform(-1.0, 1.0), z3])
    if chain == "RR":
        x3p = _mirror(x3, p2, n2)
        x3pp = _mirror(x3p, p1, n1)
        x1 = _plane_hit(x0, x3pp, p1, n1)
        x2 = None if x1 is None else _plane_hit(x1, x3p, p2, n2)
    elif chain == "RT":
        x0p = _mirror(x0, p1, n1)
        x2 = _snell_point(x0p, x3, p2, n2, eta[1], eta[2])
        x1 = None if x2 is None else _plane_hit(x0p, x2, p1, n1)
    else:  # TR
        x3p = _mirror(x3, p2, n2)
        x1 = _snell_point(x0, x3p, p1, n1, eta[0], eta[1])
        x2 = None if x1 is None else _plane_hit(x1, x3p, p2, n2)
    if x1 is None or x2 is None:
        return None
    # generic position: no vertex near normal incidence, where the square
    # form's true and superfluous roots merge into a near-double root of the
    # resultant that a 100-piece scan cannot separate
    for xp, x, n in ((x0, x1, n1), (x1, x2, n2)):
        d = (x - xp) / np.linalg.norm(x - xp)
        if np.linalg.norm(np.cross(d, n)) < 0.15:
            return None
    if chain == "TR":
        # leaving the denser medium at x1: keep clear of the critical angle on
        # the whole triangle, where beta/S of Sec. 4.4 stays inside the square
        # root's fitted range [0, 1]
        P1 = _tri_around(rng, x1, p1, n1, 0.2)
        for y in P1:
            d = (y - x0) / np.linalg.norm(y - x0)
            if 1.0 - (eta[0] / eta[1]) ** 2 * np.linalg.norm(np.cross(d, n1)) ** 2 < 0.2:
                return None
    else:
        P1 = _tri_around(rng, x1, p1, n1)
    P2 = _tri_around(rng, x2, p2, n2)
    uv1, uv2 = _bary(P1, x1), _bary(P2, x2)
    if min(uv1.min(), 1 - uv1.sum(), uv2.min(), 1 - uv2.sum()) < 1e-3:
        return None
    P = np.concatenate([P1, P2])
    N = np.array([n1] * 3 + [n2] * 3)
    tri = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    return P, N, tri, x0, x3, eta, uv1, uv2


@pytest.mark.parametrize("chain", ["RR", "RT", "TR"])
def test_flat_closed_form(chain):
    rng = np.random.default_rng({"RR": 71, "RT": 72, "TR": 73}[chain])
    done = 0
    while done < 12:
        case = _planar_case(chain, rng)
        if case is None:
            continue
        P, N, tri, x0, x3, eta, uv1, uv2 = case
        s, _ = oracle.solve_2v(P, N, tri, x0[None], x3[None], [0], [0], [0], [1], chain, eta)
        assert len(s) == 1, (chain, done, s)
        assert abs(s["u1"][0] - uv1[0]) < 1e-10 and abs(s["v1"][0] - uv1[1]) < 1e-10
        assert abs(s["u2"][0] - uv2[0]) < 1e-10 and abs(s["v2"][0] - uv2[1]) < 1e-10
        done += 1


@pytest.mark.parametrize("chain,da,db", [("RR", 8, 15), ("RT", 8, 22), ("TR", 16, 31), ("TT", 16, 46)])
def test_structural_degrees(chain, da, db):
    mesh, x0, x3, t1, t2, _ = tc.trace_paths(chain, 1, 3)
    A, B, n, _ = oracle.coeffs_2v(mesh.P, mesh.N, mesh.tri, t1[0], t2[0], x0[0], x3[0], chain, tc.SETUPS[chain][2])
    assert A.shape[0] - 1 == da and B.shape[0] - 1 == db
    assert n == max(er.udeg(A), er.udeg(B))


@pytest.mark.parametrize("chain", ["RR", "RT", "TR"])
def test_traced_paths_found(chain):
    mesh, x0, x3, t1, t2, uv = tc.trace_paths(chain, 40, 11)
    n = len(t1)
    s, _ = oracle.solve_2v(mesh.P, mesh.N, mesh.tri, x0, x3, np.arange(n), np.arange(n), t1, t2, chain,
                           tc.SETUPS[chain][2])
    for k in range(n):
        r = s[s["query"] == k]
        d = [max(abs(x["u1"] - uv[k, 0]), abs(x["v1"] - uv[k, 1]), abs(x["u2"] - uv[k, 2]), abs(x["v2"] - uv[k, 3]))
             for x in r]
        assert len(d) and min(d) < 1e-8, (chain, k, r, uv[k])


def _key(s):
    return np.array([[r["u1"], r["v1"], r["u2"], r["v2"]] for r in s]).reshape(-1, 4)


@pytest.mark.parametrize("chain", ["RR", "RT", "TR"])
def test_neighbourhoods_match_bruteforce(chain):
    mesh, x0, x3, t1, t2, _ = tc.trace_paths(chain, 2, 21)
    eta = tc.SETUPS[chain][2]
    prm = oracle.default_params(True)
    prm.pieces = 10000
    compared = paths = 0
    for k in range(len(t1)):
        tup = tc.neighbourhood(mesh, t1[k], t2[k], 0.12)
        n = len(tup)
        args = (mesh.P, mesh.N, mesh.tri, x0[k][None], x3[k][None], np.zeros(n), np.zeros(n), tup[:, 0], tup[:, 1],
                chain, eta)
        s100, _ = oracle.solve_2v(*args)
        s1e4, _ = oracle.solve_2v(*args, params=prm)
        bf = bt.solve_many(mesh.P, mesh.N, mesh.tri, x0[k], x3[k], tup[:, 0], tup[:, 1], eta, chain=chain)
        for q in range(n):
            a, b = _key(s100[s100["query"] == q]), _key(s1e4[s1e4["query"] == q])
            if len(a) != len(b) or (len(a) and np.abs(a - b).max() > 1e-9):
                continue
            compared += 1
            paths += len(a)
            assert len(bf[q]) == len(a), (chain, k, q, tup[q], bf[q], a)
            if len(a):
                assert np.abs(bf[q] - a).max() < 1e-7
    print(chain, "compared tuples", compared, "paths", paths)
    assert paths >= 2


@pytest.mark.parametrize("chain", ["RR", "RT", "TR", "TT"])
def test_paired_sign_matches_high_precision(chain):
    """The two-vertex det sign (product of sgn b over the real roots of a(., v),
    near-double root pairs left out) equals the same product taken with the
    roots and values of the FP64 coefficients computed to 60 digits, at every
    sample."""
    mesh, x0, x3, t1, t2, _ = tc.trace_paths(chain, 3, 31)
    eta = tc.SETUPS[chain][2]
    checked = 0
    for k in range(len(t1)):
        for pair in ((t1[k], t2[k]), (t1[k], t2[(k + 1) % len(t2)])):
            A, B, n, _ = oracle.coeffs_2v(mesh.P, mesh.N, mesh.tri, pair[0], pair[1], x0[k], x3[k], chain, eta)
            ma, nb = er.udeg(A), er.udeg(B)
            for v in [round((j + 0.5) / 12 * 4096) / 4096 for j in range(12)]:
                ref = er.paired_sign_hp(A, B, ma, nb, v)
                if ref is None:
                    continue
                assert oracle.res_sign_paired(A, B, ma, v) == ref, (chain, k, v)
                checked += 1
    assert checked >= 40
