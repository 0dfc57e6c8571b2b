"""Pins of the FP64 oracle against what geometry and algebra fix independently of it.

* closed-form planar mirror (face normals, Sec. 4.3 Table 1 F case),
* Snell's law on a flat interface, solved as a monotone 1-D equation,
* Bezout determinant (Eq. eq_bezout) + Laplace expansion vs. sympy's
  Sylvester resultant:  det B = +- lc_u(b)^(n - deg_u a) Res_u(a, b),
* recursive root isolation (Sec. 5.2) vs. numpy eigenvalue roots,
* brute-force Newton / grid search on tiny heightfields,
* invariants: endpoint swap (reciprocity), rigid motion.
"""
import math

import numpy as np
import pytest
import sympy as sp

import bruteforce
import oracle
from paper_2405_13409_amd import scenes


def _rot(seed):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _one_tri(P3, N3):
    P = np.asarray(P3, dtype=np.float64)
    N = np.asarray(N3, dtype=np.float64)
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    return P, N, tri


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("seed", range(40))
def test_planar_mirror_closed_form(seed):
    rng = np.random.default_rng(1000 + seed)
    P = rng.uniform(-1, 1, (3, 3))
    m = np.cross(P[1] - P[0], P[2] - P[0])
    m /= np.linalg.norm(m)
    N = np.tile(m, (3, 1))
    c = P.mean(0)
    side = 1.0 if rng.random() < 0.5 else -1.0
    x0 = c + side * (0.5 + rng.random()) * m + rng.uniform(-1, 1, 3) * 0.8
    x2 = c + side * (0.5 + rng.random()) * m + rng.uniform(-1, 1, 3) * 0.8
    # force both strictly on the same side
    if np.dot(x0 - P[0], m) * side < 0.1:
        x0 += side * m
    if np.dot(x2 - P[0], m) * side < 0.1:
        x2 += side * m
    # mirror image construction
    x0m = x0 - 2 * np.dot(x0 - P[0], m) * m
    d = x2 - x0m
    t = np.dot(P[0] - x0m, m) / np.dot(d, m)
    x1 = x0m + t * d
    # barycentrics of x1
    A = np.stack([P[1] - P[0], P[2] - P[0]], 1)
    uv, *_ = np.linalg.lstsq(A, x1 - P[0], rcond=None)
    inside = uv[0] >= 0 and uv[1] >= 0 and uv.sum() <= 1
    Pm, Nm, tri = _one_tri(P, N)
    sols, diag = oracle.solve_1bounce(Pm, Nm, tri, x0[None], x2[None], [0], [0], [0], "R")
    margin = min(uv[0], uv[1], 1 - uv.sum())
    if abs(margin) < 1e-9:
        pytest.skip("on an edge")
    if inside:
        assert len(sols) == 1
        assert abs(sols["u1"][0] - uv[0]) < 1e-10 and abs(sols["v1"][0] - uv[1]) < 1e-10
    else:
        assert len(sols) == 0


def _snell_1d(x0, x2, p0, m, eta0, eta1):
    """Path x0 -> plane(p0, m) -> x2 with x0, x2 on opposite sides: bisection on the
    in-plane offset of x1 (monotone), to full double precision."""
    a = abs(np.dot(x0 - p0, m))
    c = abs(np.dot(x2 - p0, m))
    f0 = x0 - np.dot(x0 - p0, m) * m   # foot points on the plane
    f2 = x2 - np.dot(x2 - p0, m) * m
    L = np.linalg.norm(f2 - f0)
    e = (f2 - f0) / L if L > 0 else np.zeros(3)

    def g(s):  # eta0 sin(t0) - eta1 sin(t1), increasing in s
        return eta0 * s / math.hypot(s, a) - eta1 * (L - s) / math.hypot(L - s, c)

    lo, hi = 0.0, L
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if not (lo < mid < hi):
            break
        if g(mid) < 0:
            lo = mid
        else:
            hi = mid
    return f0 + 0.5 * (lo + hi) * e


@pytest.mark.parametrize("seed", range(40))
def test_snell_flat_interface(seed):
    rng = np.random.default_rng(2000 + seed)
    P = rng.uniform(-1, 1, (3, 3))
    m = np.cross(P[1] - P[0], P[2] - P[0])
    m /= np.linalg.norm(m)
    N = np.tile(m, (3, 1))
    c = P.mean(0)
    eta0, eta1 = (1.5, 1.0) if seed % 2 else (1.0, 1.33)
    x0 = c + (0.3 + rng.random()) * m + rng.uniform(-0.6, 0.6, 3)
    x2 = c - (0.3 + rng.random()) * m + rng.uniform(-0.6, 0.6, 3)
    if np.dot(x0 - P[0], m) < 0.1:
        x0 += m
    if np.dot(x2 - P[0], m) > -0.1:
        x2 -= m
    x1 = _snell_1d(x0, x2, P[0], m, eta0, eta1)
    A = np.stack([P[1] - P[0], P[2] - P[0]], 1)
    uv, *_ = np.linalg.lstsq(A, x1 - P[0], rcond=None)
    inside = uv[0] >= 0 and uv[1] >= 0 and uv.sum() <= 1
    if abs(min(uv[0], uv[1], 1 - uv.sum())) < 1e-9:
        pytest.skip("on an edge")
    # total internal reflection cannot occur here (solution found by the 1-D solve)
    Pm, Nm, tri = _one_tri(P, N)
    sols, _ = oracle.solve_1bounce(Pm, Nm, tri, x0[None], x2[None], [0], [0], [0], "T", eta0, eta1)
    if inside:
        assert len(sols) == 1
        assert abs(sols["u1"][0] - uv[0]) < 1e-10 and abs(sols["v1"][0] - uv[1]) < 1e-10
    else:
        assert len(sols) == 0
    # same-side endpoints admit no refraction path
    x2s = x2 + 2 * abs(np.dot(x2 - P[0], m)) * m
    s2, _ = oracle.solve_1bounce(Pm, Nm, tri, x0[None], x2s[None], [0], [0], [0], "T", eta0, eta1)
    assert len(s2) == 0


# ---------------------------------------------------------------- elimination vs textbook resultant

def _to_sympy(C):
    u, v = sp.symbols("u v")
    d = C.shape[0] - 1
    return sum(sp.Rational(float(C[i, j])) * u ** i * v ** j for i in range(d + 1) for j in range(d + 1 - i)
               if C[i, j] != 0.0), u, v


@pytest.mark.parametrize("event,flat,seed", [("R", False, 0), ("R", False, 1), ("T", False, 2), ("T", False, 3),
                                             ("R", True, 4), ("T", True, 5)])
def test_bezout_laplace_equals_sylvester_resultant(event, flat, seed):
    rng = np.random.default_rng(seed)
    P = rng.uniform(-1, 1, (3, 3))
    N = rng.uniform(-1, 1, (3, 3)) + np.array([0, 0, 2.0])
    if flat:
        N = np.tile(N[0], (3, 1))
    x0 = rng.uniform(-1, 1, 3) + np.array([0, 0, 2.0])
    x2 = rng.uniform(-1, 1, 3) + np.array([0, 0, 2.0 if event == "R" else -2.0])
    Pm, Nm, tri = _one_tri(P, N)
    A, B, n, fl = oracle.coeffs_1bounce(Pm, Nm, tri, 0, x0, x2, event, 1.5 if event == "T" else 1.0, 1.0)
    r = oracle.resultant_laplace(A, B, n)
    a, u, v = _to_sympy(A)
    # structurally-zero leading u-terms are dropped exactly (the oracle never uses them)
    Bt = B.copy()
    Bt[n + 1:, :] = 0.0
    b, _, _ = _to_sympy(Bt)
    res = sp.Poly(sp.resultant(sp.Poly(a, u), sp.Poly(b, u)).as_expr(), v)
    lcb = sp.Poly(sp.Poly(b, u).all_coeffs()[0], v)
    m = sp.degree(a, u)
    ref = sp.Poly((lcb ** (n - m) * res).as_expr(), v)
    rc = np.array([float(c) for c in reversed(ref.all_coeffs())])
    k = max(len(rc), len(r))
    rc = np.pad(rc, (0, k - len(rc)))
    rr = np.pad(r, (0, k - len(r)))
    scale = np.max(np.abs(rc))
    s = 1.0 if np.dot(rc, rr) >= 0 else -1.0
    assert np.max(np.abs(s * rr - rc)) <= 1e-9 * scale


def test_structural_degrees_one_bounce():
    rng = np.random.default_rng(7)
    P = rng.uniform(-1, 1, (3, 3))
    N = rng.uniform(-1, 1, (3, 3)) + np.array([0, 0, 2.0])
    x0 = np.array([0.1, 0.2, 2.0])
    x2 = np.array([-0.3, 0.1, 2.5])
    Pm, Nm, tri = _one_tri(P, N)
    A, B, n, fl = oracle.coeffs_1bounce(Pm, Nm, tri, 0, x0, x2, "R")
    assert A.shape[0] - 1 == 2 and B.shape[0] - 1 == 4  # Sec. 4.5: degrees 2 and 4
    assert n == (4 if fl & oracle.F_EDGE2 else 3)
    if not fl & oracle.F_EDGE2:
        # the u^4 coefficient of the product form with t = n x e1 vanishes
        assert abs(B[4, 0]) <= 1e-12 * np.max(np.abs(B))
    A, B, n, fl = oracle.coeffs_1bounce(Pm, Nm, tri, 0, x0, x2 * np.array([1, 1, -1]), "T", 1.5, 1.0)
    assert A.shape[0] - 1 == 2 and B.shape[0] - 1 == 6 and n == 6  # degrees 2 and 6


# ---------------------------------------------------------------- isolation

@pytest.mark.parametrize("seed", range(25))
def test_isolation_known_roots(seed):
    rng = np.random.default_rng(seed)
    k = rng.integers(1, 9)
    while True:
        r = np.sort(rng.uniform(0.0, 1.0, k))
        if k == 1 or np.min(np.diff(r)) > 1e-3:
            break
    extra = rng.uniform(1.2, 3.0, rng.integers(0, 4)) * rng.choice([-1, 1])
    c = np.polynomial.polynomial.polyfromroots(np.concatenate([r, extra]))
    c *= rng.uniform(0.5, 2.0)
    found = oracle.isolate(c, 0.0, 1.0)
    assert len(found) == k
    # first-order perturbation bound of a simple root under coefficient rounding
    dc = np.polynomial.polynomial.polyder(c)
    cond = np.polynomial.polynomial.polyval(r, np.abs(c)) / np.abs(np.polynomial.polynomial.polyval(r, dc))
    tol = np.maximum(1e-13, 8 * len(c) * np.finfo(float).eps * cond)
    assert np.all(np.abs(found - r) <= tol)


@pytest.mark.parametrize("seed", range(25))
def test_isolation_vs_companion_eigenvalues(seed):
    rng = np.random.default_rng(100 + seed)
    d = int(rng.integers(2, 13))
    c = rng.normal(size=d + 1)
    ev = np.polynomial.polynomial.polyroots(c)
    real = np.sort(ev[(np.abs(ev.imag) < 1e-9) & (ev.real >= 0) & (ev.real <= 1)].real)
    if len(real) > 1 and np.min(np.diff(real)) < 1e-6:
        pytest.skip("clustered roots")
    found = oracle.isolate(c, 0.0, 1.0)
    assert len(found) == len(real)
    if len(real):
        assert np.max(np.abs(found - real)) < 1e-8


# ---------------------------------------------------------------- brute force on tiny meshes

def _bf_compare(mesh, x0s, x2, event, eta0, eta1, band=1e-7):
    nt = mesh.nt
    qp, qt = scenes.all_pairs(len(x0s), nt)
    sols, diag = oracle.solve_1bounce(mesh.P, mesh.N, mesh.tri, x0s, x2[None], qp, np.zeros_like(qp), qt,
                                      event, eta0, eta1)
    n_checked = 0
    for q in range(len(qt)):
        t = qt[q]
        ids = mesh.tri[t]
        bf = bruteforce.solve(mesh.P[ids], mesh.N[ids], x0s[qp[q]], x2, event, eta0, eta1)
        orc = np.stack([sols["u1"][sols["query"] == q], sols["v1"][sols["query"] == q]], 1)

        def keep(s):
            return s[np.minimum(np.minimum(s[:, 0], s[:, 1]), 1 - s[:, 0] - s[:, 1]) > band] if len(s) else s

        bf, orc = keep(bf), keep(orc)
        assert len(bf) == len(orc), (q, bf, orc)
        for p in bf:
            assert np.min(np.abs(orc - p).sum(1)) < 1e-8
        n_checked += len(bf)
    return n_checked


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_bruteforce_tiny_heightfield_R(seed):
    mesh = scenes.heightfield(2, 0.15, 3, 0.5, 1.5, seed)
    x0s = scenes.points_uniform(4, -1.0, 1.0, 0.6, 300 + seed)
    x2 = np.array([0.3, -0.2, 1.2])
    _bf_compare(mesh, x0s, x2, "R", 1.0, 1.0)


@pytest.mark.parametrize("seed", [6, 7, 8])
def test_bruteforce_tiny_heightfield_T(seed):
    mesh = scenes.heightfield(2, 0.15, 3, 0.5, 1.5, seed)
    x0s = scenes.points_uniform(4, -1.0, 1.0, 0.6, 300 + seed)
    x2 = np.array([0.1, 0.2, -1.0])
    _bf_compare(mesh, x0s, x2, "T", 1.0, 1.5)


@pytest.mark.parametrize("seed", [11, 12])
def test_bruteforce_4x4_heightfield_R(seed):
    mesh = scenes.heightfield(4, 0.08, 3, 1.0, 3.0, seed)
    x0s = scenes.points_uniform(2, -1.0, 1.0, 0.8, 400 + seed)
    x2 = np.array([0.3, -0.2, 1.5])
    _bf_compare(mesh, x0s, x2, "R", 1.0, 1.0)


# ---------------------------------------------------------------- invariants

def test_reciprocity_and_rigid_motion():
    w = scenes.glints_small()
    sel = np.arange(0, len(w.q_tri), 7)
    args = (w.q_x0[sel], w.q_x2[sel], w.q_tri[sel])
    s1, _ = oracle.solve_1bounce(w.mesh.P, w.mesh.N, w.mesh.tri, w.x0, w.x2, *args, "R")
    # swap endpoints: every x0 becomes the light and the light the shading point
    qs = np.arange(len(sel), dtype=np.int32)
    x0sw = np.repeat(w.x2, len(sel), 0)
    x2sw = w.x0[args[0]]
    s2, _ = oracle.solve_1bounce(w.mesh.P, w.mesh.N, w.mesh.tri, x0sw, x2sw, np.zeros_like(qs), qs, args[2], "R")
    assert len(s1) == len(s2)
    assert np.allclose(s1["u1"], s2["u1"], atol=1e-9) and np.allclose(s1["v1"], s2["v1"], atol=1e-9)
    # rigid motion + uniform scale of the whole scene
    R = _rot(5)
    t = np.array([0.3, -1.2, 0.7])
    k = 1.7
    P = (w.mesh.P @ R.T) * k + t
    N = w.mesh.N @ R.T
    s3, _ = oracle.solve_1bounce(P, N, w.mesh.tri, (w.x0 @ R.T) * k + t, (w.x2 @ R.T) * k + t, *args, "R")
    keep = lambda s: s[s["edge"] > 1e-7]  # noqa: E731
    a, b = keep(s1), keep(s3)
    assert len(a) == len(b)
    assert np.allclose(a["u1"], b["u1"], atol=1e-9) and np.allclose(a["v1"], b["v1"], atol=1e-9)
