"""Pins of the two-vertex det-sign reading that leaves out the roots of
a(., v) at which x2 is at infinity (det_method 3, the oracle's default).

With the rational coordinate mapping onto T2 (Eq. eq_rct), x2 = X2 / kappa,
where kappa = (Dt x e2) . e1 vanishes when the mapped ray from x1 runs
parallel to T2's plane.  When T2 is flat (M2 = kappa n0) or its vertex
normals are proportional to its positions about a centre (a sphere: M2 is
X2 - kappa c over the radius), kappa divides both a and b, so the resultant
vanishes identically and the sign of the product formula's factor at such a
root is rounding noise.  These tests show the common factor on the oracle's
own expanded polynomials, with kappa computed here from the reflected
direction (a chain that reflects at x1 has the exact mapped direction
Dt = |n1|^2 d0 - 2 (d0 . n1) n1), and pin the effect on two tuples of the
caustic workload."""
import numpy as np
import pytest

import oracle
from paper_2405_13409_amd import scenes


def _tri(P, N, tri, t):
    p = P[tri[t]]
    n = N[tri[t]]
    return p[0], p[1] - p[0], p[2] - p[0], n[0], n[1] - n[0], n[2] - n[0]


def _kappa_roots(P, N, tri, t1, t2, x0, v):
    """Roots u of kappa(u, v) for a reflection at x1 (kappa is a polynomial of
    degree <= 5 in u: sampled at 9 points and interpolated)."""
    p1, e11, e12, n10, dn11, dn12 = _tri(P, N, tri, t1)
    _, e21, e22, _, _, _ = _tri(P, N, tri, t2)
    us = np.linspace(-3, 3, 9)
    ks = []
    for u in us:
        x1 = p1 + u * e11 + v * e12
        n1 = n10 + u * dn11 + v * dn12
        d0 = x1 - x0
        Dt = (n1 @ n1) * d0 - 2 * (d0 @ n1) * n1
        ks.append(np.cross(Dt, e22) @ e21)
    c = np.polyfit(us, ks, 8)
    r = np.roots(c)
    return np.sort(r[np.abs(r.imag) < 1e-9].real)


def _eval(C, u, v):
    d = C.shape[0] - 1
    val = sum(C[i, j] * u ** i * v ** j for i in range(d + 1) for j in range(d + 1 - i))
    scale = sum(abs(C[i, j]) * abs(u) ** i * abs(v) ** j for i in range(d + 1) for j in range(d + 1 - i))
    return val, scale


def _common_factor_case(mesh, t1, t2, x0, x3, chain, eta):
    A, B, _, _ = oracle.coeffs_2v(mesh.P, mesh.N, mesh.tri, t1, t2, x0, x3, chain, eta)
    on, off = [], []
    for v in (0.1, 0.35, 0.6, 0.85):
        for u in _kappa_roots(mesh.P, mesh.N, mesh.tri, t1, t2, x0, v):
            if abs(u) > 6:
                continue
            for C in (A, B):
                val, sc = _eval(C, u, v)
                on.append(abs(val) / sc)
                val, sc = _eval(C, u + 0.37, v)
                off.append(abs(val) / sc)
    return np.array(on), np.array(off)


def test_kappa_divides_a_and_b_with_flat_t2():
    """RR chain from a gently curved floor triangle to a flat vertical
    triangle at x = 2: kappa = 0 where the reflected ray has no x component,
    a line through the floor triangle."""
    P = np.array([[-1, -1, 0], [1, -1, 0.05], [-1, 1, -0.05], [2, -1, 0.2], [2, 1, 0.5], [2, 0, 1.5]], dtype=float)
    N = np.array([[-0.1, -0.1, 1], [0.1, -0.1, 1], [-0.1, 0.1, 1], [-1, 0, 0], [-1, 0, 0], [-1, 0, 0]], dtype=float)
    N[:3] /= np.linalg.norm(N[:3], axis=1, keepdims=True)
    mesh = scenes.Mesh(P, N, np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32))
    x0 = np.array([0.2, 0.1, 1.0])
    x3 = np.array([1.0, 0.3, 2.0])
    on, off = _common_factor_case(mesh, 0, 1, x0, x3, "RR", (1.0, 1.0, 1.0))
    assert len(on) >= 4
    assert on.max() < 1e-11 and np.median(off) > 1e-6


def test_kappa_divides_a_and_b_on_a_sphere():
    """RR chain on two triangles of the icosphere (normals proportional to
    positions)."""
    mesh = scenes.caustic_sphere()
    c = mesh.P[mesh.tri].mean(1)
    t1 = int(np.argmax(c[:, 0]))
    t2 = int(np.argmax(c[:, 1]))
    x0 = np.array([2.0, 0.3, 0.2])
    x3 = np.array([0.3, 2.0, -0.1])
    on, off = _common_factor_case(mesh, t1, t2, x0, x3, "RR", (1.0, 1.0, 1.0))
    assert len(on) >= 4
    assert on.max() < 1e-11 and np.median(off) > 1e-6


def _slice_case(rec_index, t1, t2):
    mesh = scenes.caustic_sphere()
    rec = scenes.caustic_receivers()[::64]
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    return mesh, rec[rec_index][None], x3, np.array([0]), np.array([0]), np.array([t1]), np.array([t2])


@pytest.mark.parametrize("method", [2, 3])
def test_det_sign_on_a_caustic_tuple_with_a_clean_crossing(method):
    """Receiver 12 of every 64th on the caustic grid, T1 888, T2 321: the
    resultant has one real crossing, at v = 0.0231 of a path through both
    triangles.  Leaving out the kappa roots shows exactly that crossing;
    with them the scan sees dozens of rounding sign changes and misses it."""
    mesh, x0, x3, a, b, t1, t2 = _slice_case(12, 888, 321)
    prm = oracle.default_params(True)
    prm.det_method = method
    s, d = oracle.solve_tt(mesh.P, mesh.N, mesh.tri, x0, x3, a, b, t1, t2, params=prm)
    if method == 3:
        assert d["n_vroots"][0] == 1 and len(s) == 1
        assert abs(s["v1"][0] - 0.0230882) < 1e-6 and s["residual"][0] < 1e-12
    else:
        assert d["n_vroots"][0] > 10


def test_det_sign_quiet_where_only_kappa_roots_vary():
    """Receiver 6, T1 888, T2 96: every factor but the kappa roots keeps its
    sign over [0,1], so the scan reports no sign change at all (the paired
    product without the reading reports rounding changes)."""
    mesh, x0, x3, a, b, t1, t2 = _slice_case(6, 888, 96)
    prm = oracle.default_params(True)
    s, d = oracle.solve_tt(mesh.P, mesh.N, mesh.tri, x0, x3, a, b, t1, t2, params=prm)
    assert d["n_vroots"][0] == 0 and len(s) == 0
    prm.det_method = 2
    _, d2 = oracle.solve_tt(mesh.P, mesh.N, mesh.tri, x0, x3, a, b, t1, t2, params=prm)
    assert d2["n_vroots"][0] > 0
