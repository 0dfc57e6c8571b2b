"""Host check of the two-level cull's tile bound (no GPU): wherever the tile
test rejects a (tile, triangle), the per-pair test rejects every pair of the
tile.  Both tests are written out here in float64 with the kernel's formulas
and safety factors; the float32 kernel itself is compared with the FP64 cull
twin and with a row-ordered run on the GPU.  A tile radius that is too small (half
of it) fails here; the angle-versus-chord distinction of the tile side only
matters in rare edge cases that random tiles do not reach."""
import numpy as np
import pytest


def _side(c, rad, p, eta):
    a = p - c
    d2 = (a * a).sum(-1)
    ok = d2 > (rad * 1.0001) ** 2
    ia = 1.0 / np.sqrt(np.where(ok, d2, 1.0))
    sa = np.minimum(rad * ia * 1.000001, 1.0)
    chord = sa * (1.0 + 0.41422 * sa * sa) * 1.000001
    return ok, eta * ia[..., None] * a, eta * chord


def _tile_side(c, rad, P, rho, eta):
    a = P - c
    d2 = (a * a).sum(-1)
    r = rad + rho
    ia = 1.0 / np.sqrt(np.where(d2 > 0, d2, 1.0))
    sa = r * ia * 1.000001
    ok = (d2 > (r * 1.0001) ** 2) & (sa < 1.0)
    return ok, eta * ia[..., None] * a, eta * sa * (1.0 + 0.5708 * sa * sa) * 1.001


def _meet(an, cth, sth, ha, da, hb, db):
    H = ha + hb
    iL = 1.0 / np.sqrt((H * H).sum(-1))
    delta = (da + db) * 1.0001 + 1e-6
    sphi = delta * iL * 1.000001
    big = ~(sphi < 1.0)
    cphi = np.sqrt(np.maximum(0.0, 1.0 - sphi * sphi))
    clim = cth * cphi - sth * sphi
    wide = ~(clim > 1e-4)
    cdot = np.abs((an * H).sum(-1)) * iL
    return big | wide | (cdot >= clim * (1.0 - 4e-6))


@pytest.mark.parametrize("eta", [(1.0, 1.0), (1.5, 1.0)])
def test_tile_rejection_implies_pair_rejection(eta):
    rng = np.random.default_rng(17)
    e0, e1 = eta
    nt, margin = 3000, 1e-3
    # triangles near z = 0 on [-1,1]^2, sphere radius ~ a glints cell, tilted normal cones
    c = np.column_stack([rng.uniform(-1, 1, nt), rng.uniform(-1, 1, nt), rng.normal(0, 0.01, nt)])
    rad = rng.uniform(0.005, 0.03, nt)
    tilt = rng.uniform(0, 0.4, nt)
    az = rng.uniform(0, 2 * np.pi, nt)
    an = np.column_stack([np.sin(tilt) * np.cos(az), np.sin(tilt) * np.sin(az), np.cos(tilt)])
    thn = rng.uniform(0.0, 0.08, nt)
    thm = thn + margin
    allk = ~(thm < 1.5707)
    cth, sth = np.cos(np.minimum(thm, 1.5707)), np.sin(np.minimum(thm, 1.5707))
    light = np.array([0.0, 0.0, 4.0])
    n_rej = n_pairs_kept = 0
    for tile in range(60):
        z = 2.0 if e0 == e1 else -2.0
        step = rng.choice([2.0 / 256, 2.0 / 64])
        o = rng.uniform(-1, 1 - 16 * step, 2)
        g = np.arange(16) * step
        X, Y = np.meshgrid(o[0] + g, o[1] + g)
        pts = np.column_stack([X.ravel(), Y.ravel(), np.full(256, z)])
        P = pts.mean(0)
        rho = np.sqrt(((pts - P) ** 2).sum(-1).max()) * 1.0001 + 1e-6
        # tile test, every triangle
        oka, ha, da = _tile_side(c, rad, P[None, :], rho, e0)
        okb, hb, db = _tile_side(c, rad, light[None, :], 1e-6, e1)
        coarse = allk | ~oka | ~okb | _meet(an, cth, sth, ha, da, hb, db)
        rej = np.nonzero(~coarse)[0]
        n_rej += len(rej)
        # per-pair test of every pair of the rejected triangles
        cc, rr = c[rej][:, None, :], rad[rej][:, None]
        pa_ok, pha, pda = _side(cc, rr, pts[None, :, :], e0)
        pb_ok, phb, pdb = _side(cc, rr, light[None, None, :], e1)
        fine = allk[rej][:, None] | ~pa_ok | ~pb_ok | _meet(an[rej][:, None, :], cth[rej][:, None], sth[rej][:, None],
                                                          pha, pda, phb, pdb)
        assert not fine.any(), f"tile {tile}: a pair kept by the per-pair test of a rejected triangle"
        # and the per-pair test keeps something among the triangles the tile test passes
        kept = np.nonzero(coarse)[0]
        ck, rk = c[kept][:, None, :], rad[kept][:, None]
        qa_ok, qha, qda = _side(ck, rk, pts[None, :, :], e0)
        qb_ok, qhb, qdb = _side(ck, rk, light[None, None, :], e1)
        n_pairs_kept += int((allk[kept][:, None] | ~qa_ok | ~qb_ok |
                             _meet(an[kept][:, None, :], cth[kept][:, None], sth[kept][:, None], qha, qda, qhb, qdb)).sum())
    # not vacuous: most (tile, triangle) tests reject, and pairs are kept elsewhere
    assert n_rej > 0.5 * 60 * nt
    assert n_pairs_kept > 1000
