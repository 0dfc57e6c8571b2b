"""Pins of the tail oracle (visibility and contribution of validated paths,
Sec. 5.3) against facts that do not come from the oracle itself: Fresnel's
special angles, an orientation-based segment/triangle test, image-source
closed forms for flat mirrors, the closed form of a point source seen through
one flat interface, and conservation of energy over a curved facet."""
import numpy as np
import pytest

import oracle


# ------------------------------------------------------------------ Fresnel

@pytest.mark.parametrize("n1,n2", [(1.0, 1.5), (1.5, 1.0), (1.0, 2.4), (1.33, 1.0)])
def test_fresnel_normal_incidence(n1, n2):
    assert oracle.fresnel_t(n1, n2, 1.0) == pytest.approx(4 * n1 * n2 / (n1 + n2) ** 2, rel=1e-14)


@pytest.mark.parametrize("n1,n2", [(1.0, 1.5), (1.5, 1.0), (1.0, 2.4)])
def test_fresnel_brewster(n1, n2):
    # at Brewster's angle the p wave is fully transmitted and
    # r_s = -sin(ti - tt) / sin(ti + tt) = (n1^2 - n2^2) / (n1^2 + n2^2)
    tb = np.arctan2(n2, n1)
    R = 0.5 * ((n1 ** 2 - n2 ** 2) / (n1 ** 2 + n2 ** 2)) ** 2
    assert oracle.fresnel_t(n1, n2, np.cos(tb)) == pytest.approx(1 - R, rel=1e-13)


def test_fresnel_reciprocity_and_limits():
    n1, n2 = 1.0, 1.5
    for ti in np.linspace(0.01, 1.5, 30):
        tt = np.arcsin(n1 / n2 * np.sin(ti))
        assert oracle.fresnel_t(n1, n2, np.cos(ti)) == pytest.approx(oracle.fresnel_t(n2, n1, np.cos(tt)), rel=1e-12)
    assert oracle.fresnel_t(1.5, 1.0, np.cos(np.arcsin(1 / 1.5) + 1e-3)) == 0.0   # past the critical angle
    assert oracle.fresnel_t(1.0, 1.5, 1e-9) < 1e-8                               # grazing


# ------------------------------------------------------------------ segment / triangle

def _orient(a, b, c, d):
    return np.einsum("ij,ij->i", np.cross(b - a, c - a), d - a)


def test_seg_tri_against_orientation_tests():
    """A segment pq crosses triangle abc iff a, b, c lie on the same side of
    each plane through pq and an edge, and p, q lie on opposite sides of the
    triangle's plane."""
    rng = np.random.default_rng(11)
    n = 20000
    p, q = rng.normal(size=(n, 3)), rng.normal(size=(n, 3))
    a, b, c = (rng.normal(size=(n, 3)) * 0.8 for _ in range(3))
    s1, s2, s3 = _orient(p, q, a, b), _orient(p, q, b, c), _orient(p, q, c, a)
    same = ((s1 > 0) & (s2 > 0) & (s3 > 0)) | ((s1 < 0) & (s2 < 0) & (s3 < 0))
    opp = _orient(a, b, c, p) * _orient(a, b, c, q) < 0
    ref = same & opp
    hit, margin = oracle.seg_tri(p, q, a, b, c, 0.0)
    ok = margin > 1e-9
    assert ok.mean() > 0.99 and 0.05 < ref.mean() < 0.5
    np.testing.assert_array_equal(hit[ok], ref[ok])


def test_seg_tri_endpoint_band():
    a, b, c = np.array([[0, 0, 0.0]]), np.array([[1, 0, 0.0]]), np.array([[0, 1, 0.0]])
    q = np.array([[0.2, 0.2, 1.0]])
    for z0, expect in ((-1e-3, True), (-1e-8, False), (1e-8, False)):
        hit, _ = oracle.seg_tri(np.array([[0.2, 0.2, z0]]), q, a, b, c, 1e-6)
        assert bool(hit[0]) is expect, z0


# ------------------------------------------------------------------ closed forms

def _quad_mesh(z, normal, half=5.0):
    """Two triangles covering [-half, half]^2 at height z, constant normal."""
    P = np.array([[-half, -half, z], [half, -half, z], [half, half, z], [-half, half, z]], dtype=float)
    tri = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    if normal[2] < 0:
        tri = tri[:, ::-1].copy()
    return P, np.tile(np.asarray(normal, float), (4, 1)), tri


def _bary(P, tri, t, x):
    p0, p1, p2 = P[tri[t]]
    M = np.stack([p1 - p0, p2 - p0], 1)
    uv, *_ = np.linalg.lstsq(M, x - p0, rcond=None)
    assert np.linalg.norm(M @ uv + p0 - x) < 1e-12
    return uv


def _locate(P, tri, x, tris):
    for t in tris:
        u, v = _bary(P, tri, t, x)
        if u >= 0 and v >= 0 and u + v <= 1:
            return t, u, v
    raise AssertionError("point outside the mesh")


def test_flat_mirror_image_source():
    """A point light seen in a flat mirror is its mirror image: the reflected
    beam is a sphere of radius L (the unfolded path length), E = I rho / L^2."""
    P, N, tri = _quad_mesh(0.0, (0, 0, 1))
    L = np.array([[0.3, -0.2, 1.5]])
    rng = np.random.default_rng(5)
    x0s = np.column_stack([rng.uniform(-2, 2, 40), rng.uniform(-2, 2, 40), rng.uniform(0.2, 3, 40)])
    img = L[0] * [1, 1, -1]
    rows = []
    for x0 in x0s:
        s = x0[2] / (x0[2] - img[2])
        rows.append(_locate(P, tri, x0 + s * (img - x0), [0, 1]))
    rows = np.array(rows)
    r = oracle.tail(P, N, tri, x0s, L, np.arange(40), np.zeros(40), rows[:, 0], rows[:, 1], rows[:, 2], "R",
                    (1.0, 1.0), intensity=2.0, rho=0.9)
    Ltot = np.linalg.norm(x0s - img, axis=1)
    np.testing.assert_allclose(r["E"], 2.0 * 0.9 / Ltot ** 2, rtol=1e-8)
    assert np.all(r["mask"] == 0) and np.all(r["fresnel"] == 0.9)


def test_periscope_two_mirrors():
    """Floor z = 0 and ceiling z = 2, both mirrors: a light between them seen
    after floor-then-ceiling reflections (x1 on the floor) is the floor image
    of its ceiling image; E = I rho^2 / L^2."""
    Pa, Na, ta = _quad_mesh(0.0, (0, 0, 1))
    Pb, Nb, tb = _quad_mesh(2.0, (0, 0, -1))
    P, N, tri = np.vstack([Pa, Pb]), np.vstack([Na, Nb]), np.vstack([ta, tb + 4])
    L = np.array([[0.1, 0.2, 1.1]])
    LB = L[0] * [1, 1, -1] + [0, 0, 4.0]        # image in the ceiling
    LBA = LB * [1, 1, -1]                       # then in the floor
    rng = np.random.default_rng(6)
    x0s = np.column_stack([rng.uniform(-2.5, 2.5, 30), rng.uniform(-2.5, 2.5, 30), rng.uniform(0.3, 1.7, 30)])
    T, U, V = [], [], []
    for x0 in x0s:
        x1 = x0 + (0 - x0[2]) / (LBA[2] - x0[2]) * (LBA - x0)
        x2 = x1 + (2 - x1[2]) / (LB[2] - x1[2]) * (LB - x1)
        r1, r2 = _locate(P, tri, x1, [0, 1]), _locate(P, tri, x2, [2, 3])
        T.append([r1[0], r2[0]]); U.append([r1[1], r2[1]]); V.append([r1[2], r2[2]])
    r = oracle.tail(P, N, tri, x0s, L, np.arange(30), np.zeros(30), T, U, V, "RR", (1.0, 1.0, 1.0), rho=0.8)
    np.testing.assert_allclose(r["E"], 0.64 / np.linalg.norm(x0s - LBA, axis=1) ** 2, rtol=1e-8)
    assert np.all(r["mask"] == 0)


def test_flat_refraction_closed_form():
    """Light at height h1 above a flat interface (index 1), receiver at depth
    h2 below (index 1.5).  By symmetry about the vertical through the light,
    dA_horizontal / dw = r (dr/dth1) / sin th1 with r = h1 tan th1 + h2 tan th2
    and dth2/dth1 = n1 cos th1 / (n2 cos th2); the area normal to the arriving
    ray is cos th2 times the horizontal one."""
    P, N, tri = _quad_mesh(0.0, (0, 0, 1), half=8.0)
    h1, h2, n1, n2 = 1.3, 0.7, 1.0, 1.5
    L = np.array([[0.0, 0.0, h1]])
    th1 = np.linspace(0.05, 1.3, 25)
    th2 = np.arcsin(n1 / n2 * np.sin(th1))
    r = h1 * np.tan(th1) + h2 * np.tan(th2)
    phi = np.linspace(0, 2 * np.pi, 25, endpoint=False)
    x0s = np.column_stack([r * np.cos(phi), r * np.sin(phi), np.full(25, -h2)])
    x1s = np.column_stack([h1 * np.tan(th1) * np.cos(phi), h1 * np.tan(th1) * np.sin(phi), np.zeros(25)])
    rows = np.array([_locate(P, tri, x1, [0, 1]) for x1 in x1s])
    res = oracle.tail(P, N, tri, x0s, L, np.arange(25), np.zeros(25), rows[:, 0], rows[:, 1], rows[:, 2], "T",
                      (n2, n1))
    drdth = h1 / np.cos(th1) ** 2 + h2 / np.cos(th2) ** 2 * (n1 * np.cos(th1) / (n2 * np.cos(th2)))
    dA_dw = np.cos(th2) * r * drdth / np.sin(th1)
    TF = np.array([oracle.fresnel_t(n1, n2, np.cos(t)) for t in th1])
    np.testing.assert_allclose(res["E"], TF / dA_dw, rtol=1e-7)
    np.testing.assert_allclose(res["fresnel"], TF, rtol=1e-14)


# ------------------------------------------------------------------ energy over a curved facet

def _facet(bulge):
    P = np.array([[-0.5, -0.4, 0.0], [0.5, -0.4, 0.0], [0.0, 0.5, 0.0]])
    N = np.column_stack([bulge * P[:, 0], bulge * P[:, 1], np.ones(3)])
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    return P, N, np.array([[0, 1, 2]], dtype=np.int32)


def _window(u, v):
    return (u * v * (1 - u - v)) ** 2


def _solid_angle_integral(P, L, f):
    """Integral over the facet of f(u, v, x, w) dw (w: unit direction from
    the light), by the midpoint rule on a fine barycentric grid."""
    m = 600
    i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    keep = i + j < m - 1
    u, v = (i[keep] + 1 / 3) / m, (j[keep] + 1 / 3) / m
    u2, v2 = (i + 2 / 3) / m, (j + 2 / 3) / m
    u = np.concatenate([u, u2[i + j < m - 1]])
    v = np.concatenate([v, v2[i + j < m - 1]])
    e1, e2 = P[1] - P[0], P[2] - P[0]
    x = P[0] + u[:, None] * e1 + v[:, None] * e2
    d = x - L
    r = np.linalg.norm(d, axis=1)
    dw = np.abs(d @ np.cross(e1, e2)) / r ** 3 / (2 * m * m)
    return np.sum(f(u, v, x, d / r[:, None]) * dw)


def _plane_sum(P, N, tri, L, zr, event, eta, half, n=220):
    g = (np.arange(n) + 0.5) / n * 2 * half - half
    X, Y = np.meshgrid(g, g, indexing="ij")
    x0s = np.column_stack([X.ravel(), Y.ravel(), np.full(n * n, zr)])
    nq = len(x0s)
    sols, _ = oracle.solve_1bounce(P, N, tri, x0s, L, np.arange(nq), np.zeros(nq), np.zeros(nq), event, *eta)
    res = oracle.tail(P, N, tri, x0s, L, sols["query"], np.zeros(len(sols)), np.zeros(len(sols)), sols["u1"],
                      sols["v1"], event, eta)
    x1 = P[0] + sols["u1"][:, None] * (P[1] - P[0]) + sols["v1"][:, None] * (P[2] - P[0])
    w0 = x1 - x0s[sols["query"]]
    cos0 = np.abs(w0[:, 2]) / np.linalg.norm(w0, axis=1)
    assert np.all(np.maximum(np.abs(x0s[sols["query"], 0]), np.abs(x0s[sols["query"], 1])) < half - 2 * half / n), \
        "the beam reaches the edge of the receiver grid"
    return np.sum(res["E"] * cos0 * _window(sols["u1"], sols["v1"])) * (2 * half / n) ** 2, len(sols)


def test_energy_conservation_curved_mirror():
    """Flux that leaves the light toward the facet, weighted by a window that
    vanishes on the facet's edges, equals the weighted irradiance summed over
    a receiver plane that catches the whole reflected beam (no folds: the
    facet's normals spread outward)."""
    P, N, tri = _facet(0.35)
    L = np.array([0.4, 0.2, 2.0])
    rho = 1.0
    lhs, n = _plane_sum(P, N, tri, L[None], 1.0, "R", (1.0, 1.0), 2.6)
    rhs = rho * _solid_angle_integral(P, L, lambda u, v, x, w: _window(u, v))
    assert n > 2000
    assert lhs == pytest.approx(rhs, rel=1e-5)


def test_energy_conservation_curved_interface():
    """The same balance through a refracting facet (index 1 above, 1.5 below,
    normals tilted inward so the transmitted beam spreads), with the
    unpolarised Fresnel transmittance weighting the light side."""
    P, N, tri = _facet(-0.35)
    L = np.array([0.3, -0.25, 1.6])
    n1, n2 = 1.0, 1.5

    def tf(u, v, x, w):
        nn = N[0] + u[:, None] * (N[1] - N[0]) + v[:, None] * (N[2] - N[0])
        nn /= np.linalg.norm(nn, axis=1, keepdims=True)
        ci = np.abs(np.sum(w * nn, axis=1))
        ct = np.sqrt(1 - (n1 / n2) ** 2 * (1 - ci ** 2))
        rs = (n1 * ci - n2 * ct) / (n1 * ci + n2 * ct)
        rp = (n2 * ci - n1 * ct) / (n2 * ci + n1 * ct)
        return _window(u, v) * (1 - 0.5 * (rs ** 2 + rp ** 2))

    lhs, n = _plane_sum(P, N, tri, L[None], -0.8, "T", (n2, n1), 2.0)
    rhs = _solid_angle_integral(P, L, tf)
    assert n > 2000
    assert lhs == pytest.approx(rhs, rel=1e-5)


# ------------------------------------------------------------------ visibility of whole paths

def test_path_mask_against_orientation_brute_force():
    """Random paths through a cluttered scene: the oracle's blocked-segment
    mask equals the orientation-test brute force over every other triangle."""
    rng = np.random.default_rng(9)
    nt = 60
    c = rng.uniform(-1, 1, (nt, 3))
    P = (c[:, None, :] + rng.normal(scale=0.25, size=(nt, 3, 3))).reshape(-1, 3)
    tri = np.arange(3 * nt, dtype=np.int32).reshape(nt, 3)
    N = np.tile([0, 0, 1.0], (len(P), 1))
    n = 400
    x0s, L = rng.uniform(-1.5, 1.5, (n, 3)), rng.uniform(-1.5, 1.5, (1, 3))
    T = rng.integers(0, nt, (n, 2))
    T[T[:, 0] == T[:, 1], 1] = (T[T[:, 0] == T[:, 1], 1] + 1) % nt
    U = rng.uniform(0.05, 0.45, (n, 2))
    V = rng.uniform(0.05, 0.45, (n, 2))
    r = oracle.tail(P, N, tri, x0s, L, np.arange(n), np.zeros(n), T, U, V, "RR", (1.0, 1.0, 1.0), teps=0.0)
    X1 = P[tri[T[:, 0], 0]] + U[:, :1] * (P[tri[T[:, 0], 1]] - P[tri[T[:, 0], 0]]) + \
        V[:, :1] * (P[tri[T[:, 0], 2]] - P[tri[T[:, 0], 0]])
    X2 = P[tri[T[:, 1], 0]] + U[:, 1:] * (P[tri[T[:, 1], 1]] - P[tri[T[:, 1], 0]]) + \
        V[:, 1:] * (P[tri[T[:, 1], 2]] - P[tri[T[:, 1], 0]])
    segs = [(x0s, X1, [T[:, 0]]), (X1, X2, [T[:, 0], T[:, 1]]), (X2, np.repeat(L, n, 0), [T[:, 1]])]
    ref = np.zeros(n, dtype=np.int32)
    for s, (p, q, skip) in enumerate(segs):
        for t in range(nt):
            a, b, cc = (np.repeat(P[tri[t, j]][None], n, 0) for j in range(3))
            s1, s2, s3 = _orient(p, q, a, b), _orient(p, q, b, cc), _orient(p, q, cc, a)
            same = ((s1 > 0) & (s2 > 0) & (s3 > 0)) | ((s1 < 0) & (s2 < 0) & (s3 < 0))
            hit = same & (_orient(a, b, cc, p) * _orient(a, b, cc, q) < 0)
            for sk in skip:
                hit &= sk != t
            ref |= hit.astype(np.int32) << s
    ok = r["margin"] > 1e-9
    assert ok.mean() > 0.95 and 0.1 < (ref != 0).mean() < 0.9
    np.testing.assert_array_equal(r["mask"][ok], ref[ok])
