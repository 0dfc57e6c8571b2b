"""Pins of the two-vertex determinant sign and of the det-method choice.

det R(v) of the Bezout matrix (Eq. eq_bezout) equals, up to a constant factor
and a power of lc_u(b), the resultant Res_u(a, b) (Sec. 5.1), whose sign is what
the bisection of Sec. 5.2 tracks.  The resultant's product formula gives that
sign as the product of sgn b over the real roots of a(., v) (det_method 1).
These tests compare it with the EXACT sign of the Sylvester resultant of the
same FP64 coefficients (exact rational arithmetic, tests/exact_resultant.py):
on curved sphere tuples around traced caustic paths and on random systems up
to degrees (16, 40), the ratio of the two signs must be one constant per
system.  The oracle's default (det_method 2) leaves near-double root pairs
of a out of the product; it is pinned against a 60-digit evaluation in
test_oracle_2v_pins.py.  They also check that Gaussian elimination on the
numeric Bezout matrix (the paper's literal procedure, det_method 0) and the
product formulas give the same valid paths where elimination is well
conditioned (flat parallel slab), and record how they compare on the sphere.
"""
import numpy as np
import pytest

import exact_resultant as er
import oracle
import ttcases
from paper_2405_13409_amd import scenes

OFFSETS = ([0.05, 0.02, 0.0], [-0.12, 0.07, 0.0], [0.2, -0.15, 0.0])


def _vgrid(n=24, bits=12):
    """n dyadic sample points in (0,1), away from 0 and 1."""
    return [round((k + 0.5) / n * (1 << bits)) / (1 << bits) for k in range(n)]


def _sphere_tuples():
    mesh = scenes.caustic_sphere()
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE[0]
    c = mesh.P[mesh.tri].mean(1)
    out = []
    for off in OFFSETS:
        x0, q, p = ttcases.traced_receiver(np.array(off))
        tup = ttcases.tuples_near(mesh, x0, x3, q, p, r=0.2)
        # the tuple the traced path crosses (nearest centroids), plus two others
        best = int(np.argmin(np.linalg.norm(c[tup[:, 0]] - q, axis=1) + np.linalg.norm(c[tup[:, 1]] - p, axis=1)))
        for i in (best, len(tup) // 3):
            out.append((x0, x3, int(tup[i, 0]), int(tup[i, 1])))
    return mesh, out


def test_product_sign_matches_exact_resultant_on_sphere_tuples():
    mesh, tuples = _sphere_tuples()
    assert len(tuples) >= 5
    ge_agree = 0
    total = 0
    for x0, x3, t1, t2 in tuples:
        A, B, n, _ = oracle.coeffs_tt(mesh.P, mesh.N, mesh.tri, t1, t2, x0, x3)
        ma, nb = er.udeg(A), er.udeg(B)
        assert n == max(ma, nb) and nb % 2 == 0
        ratios = set()
        for v in _vgrid():
            s_ex = er.res_sign(A, B, ma, nb, v)
            assert s_ex in (-1, 1)
            ratios.add(s_ex * oracle.res_sign(A, B, ma, v))
            ge_agree += s_ex * oracle.det_sign(A, B, n, v) == 1
            total += 1
        assert len(ratios) == 1, (t1, t2, ratios)
    # Gaussian elimination on this Bezout matrix is no better than a coin toss
    print(f"GE sign == exact resultant sign at {ge_agree}/{total} samples")


@pytest.mark.parametrize("da,db,seed", [(3, 6, 1), (8, 20, 2), (12, 31, 3), (16, 40, 4)])
def test_product_sign_matches_exact_resultant_random(da, db, seed):
    """Random bivariate systems of total degrees (da, db): the u^da and u^db
    coefficients are constants, so sgn Res = sgn(lc a)^db * prod sgn b(alpha),
    with a constant first factor.  The product formula must track the rest."""
    rng = np.random.default_rng(900 + seed)
    A = np.zeros((da + 1, da + 1))
    B = np.zeros((db + 1, db + 1))
    for i in range(da + 1):
        A[i, : da + 1 - i] = rng.normal(size=da + 1 - i)
    for i in range(db + 1):
        B[i, : db + 1 - i] = rng.normal(size=db + 1 - i)
    A[da, 0] = 0.5 + abs(A[da, 0])
    B[db, 0] = 0.5 + abs(B[db, 0])
    ratios = set()
    for v in _vgrid(20):
        s_ex = er.res_sign(A, B, da, db, v)
        assert s_ex in (-1, 1)
        ratios.add(s_ex * oracle.res_sign(A, B, da, v))
    assert len(ratios) == 1, ratios


def test_res_sign_known_roots():
    """a = (u - v)(u + 2), b = u - 1/2 + c: Res_u = b(v) b(-2) up to lc powers,
    which changes sign exactly where v = 1/2 - c."""
    A = np.zeros((3, 3))
    # a(u,v) = u^2 + 2u - uv - 2v
    A[2, 0] = 1.0
    A[1, 0] = 2.0
    A[1, 1] = -1.0
    A[0, 1] = -2.0
    B = np.zeros((2, 2))
    B[1, 0] = 1.0
    B[0, 0] = -0.3   # b = u - 0.3: sign change of b(v) at v = 0.3
    signs = [oracle.res_sign(A, B, 2, v) for v in (0.1, 0.2, 0.29, 0.31, 0.5, 0.9)]
    assert signs[:3] == [signs[0]] * 3 and signs[3:] == [-signs[0]] * 3


def _params(method, pieces=100):
    p = oracle.default_params(True)
    p.det_method = method
    p.pieces = pieces
    return p


@pytest.mark.parametrize("seed", range(8))
def test_det_methods_agree_on_flat_slab(seed):
    """On two parallel flat triangles (Bezout size 14, well conditioned) the
    literal Gaussian-elimination sign and the product formula find the same
    valid path."""
    import test_oracle_tt_pins as pins

    rng = np.random.default_rng(50 + seed)
    h = 0.3
    x0 = np.array([rng.uniform(-0.8, 0.8), rng.uniform(-0.8, 0.8), -rng.uniform(0.5, 1.5)])
    x3 = np.array([rng.uniform(-0.8, 0.8), rng.uniform(-0.8, 0.8), h + rng.uniform(0.5, 1.5)])
    x1, x2 = pins._slab_path(x0, x3, h, 1.5)
    P = np.concatenate([pins._tri_around(rng, x1, 0.0, 0.4), pins._tri_around(rng, x2, h, 0.4)])
    N = np.array([[0, 0, -1.0]] * 3 + [[0, 0, 1.0]] * 3)
    tri = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    s0, d0 = oracle.solve_tt(P, N, tri, x0[None], x3[None], [0], [0], [0], [1], params=_params(0))
    for m in (1, 2, 3):
        s1, d1 = oracle.solve_tt(P, N, tri, x0[None], x3[None], [0], [0], [0], [1], params=_params(m))
        assert len(s0) == len(s1) == 1
        for k in ("u1", "v1", "u2", "v2"):
            assert abs(s0[k][0] - s1[k][0]) < 1e-12


def test_det_methods_on_sphere_neighbourhood():
    """Around a traced caustic path on the sphere, elimination and the product
    formula find the same valid paths, while elimination reports far more sign
    changes (its sign is dominated by rounding, see the exact-sign test)."""
    mesh = scenes.caustic_sphere()
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE[0]
    x0, q, p = ttcases.traced_receiver(np.array(OFFSETS[0]))
    tup = ttcases.tuples_near(mesh, x0, x3, q, p, r=0.12)
    n = len(tup)
    args = (mesh.P, mesh.N, mesh.tri, x0[None], x3[None], np.zeros(n), np.zeros(n), tup[:, 0], tup[:, 1])
    s0, d0 = oracle.solve_tt(*args, params=_params(0))
    s1, d1 = oracle.solve_tt(*args, params=_params(1))
    s2, d2 = oracle.solve_tt(*args, params=_params(2))
    s3, d3 = oracle.solve_tt(*args, params=_params(3))
    print(f"{n} tuples: sign changes GE {d0['n_vroots'].sum()} product {d1['n_vroots'].sum()} "
          f"paired {d2['n_vroots'].sum()} chain {d3['n_vroots'].sum()}; valid GE {len(s0)} product {len(s1)} "
          f"paired {len(s2)} chain {len(s3)}")
    assert len(s1) >= 1
    k0 = {(int(s['query']), round(s['u1'], 8), round(s['v1'], 8)) for s in s0}
    k1 = {(int(s['query']), round(s['u1'], 8), round(s['v1'], 8)) for s in s1}
    k2 = {(int(s['query']), round(s['u1'], 8), round(s['v1'], 8)) for s in s2}
    k3 = {(int(s['query']), round(s['u1'], 8), round(s['v1'], 8)) for s in s3}
    assert k0 == k1 == k2 == k3
    assert d3["n_vroots"].sum() <= d2["n_vroots"].sum()
    assert d0["n_vroots"].sum() > d1["n_vroots"].sum()
