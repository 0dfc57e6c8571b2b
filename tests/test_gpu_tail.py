"""GPU parity of the path-phase tail (visibility through the device BVH and
the contribution of each chain, Sec. 5.3) against the tail oracle, through
the C ABI.  Chains come from the oracle's own solves (inputs may flow from
the oracle to the GPU, never back); the end-to-end case compares the image
of a GPU solve + tail with the oracle's solve + tail."""
import numpy as np
import pytest
import torch

import oracle
import ttcases
import twovertex_cases as tc
from paper_2405_13409_amd import scenes

pytestmark = pytest.mark.gpu

MARGIN = 1e-9      # visibility decisions closer than this to flipping are not compared
E_RTOL = 1e-6      # contribution: exact derivatives (GPU) vs central differences of a trace (oracle)
E_STABLE = 1e-7    # ... where the oracle's difference quotient is stable to this


@pytest.fixture(scope="module")
def sp():
    from paper_2405_13409_amd import spoly

    spoly.load_library()
    return spoly


@pytest.fixture(scope="module")
def ctx(sp):
    c = sp.Context(0)
    yield c
    c.close()


def _tag(name):
    print(f"[gpu-case] {name}", flush=True)


def _i32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def _records(sp, sols, qtris, k):
    """Oracle solutions (SOL_DTYPE) as spoly_solution records; qtris [nq, k]."""
    r = np.zeros(len(sols), dtype=sp.SOLUTION_DTYPE)
    r["query"] = sols["query"]
    r["tri"][:, 0] = qtris[sols["query"], 0]
    r["tri"][:, 1] = qtris[sols["query"], 1] if k == 2 else -1
    r["u"][:, 0], r["v"][:, 0] = sols["u1"], sols["v1"]
    if k == 2:
        r["u"][:, 1], r["v"][:, 1] = sols["u2"], sols["v2"]
    return r


def _oracle_tail(mesh, x0s, xls, q0, ql, qtris, sols, chain, eta, **kw):
    k = len(chain)
    ptri = qtris[sols["query"]][:, :k]
    pu = np.column_stack([sols["u1"], sols["u2"]])[:, :k]
    pv = np.column_stack([sols["v1"], sols["v2"]])[:, :k]
    return oracle.tail(mesh.P, mesh.N, mesh.tri, x0s, xls, q0[sols["query"]], ql[sols["query"]], ptri, pu, pv,
                       chain, eta, **kw)


def _gpu_tail(sp, ctx, mesh, x0s, xls, q0, ql, recs, chain, eta, params=None, image=False, bvh=None, dm=None):
    dm = dm or sp.DeviceMesh(mesh.P, mesh.N, mesh.tri)
    bvh = bvh or sp.Bvh(ctx, dm)
    img = torch.zeros(len(x0s), dtype=torch.float64, device="cuda") if image else None
    m, e, img = ctx.path_tail(dm, bvh, chain, eta, sp.DevicePoints(x0s), sp.DevicePoints(xls), _i32(q0), _i32(ql),
                              sp.solutions_to_device(recs), params=params, image=img)
    torch.cuda.synchronize()
    n = len(recs)
    return m.cpu().numpy()[:n], e.cpu().numpy()[:n], (img.cpu().numpy() if image else None)


def _compare(gm, ge, ot, k, min_blocked=0.0):
    ok = ot["margin"] > MARGIN
    seg = (1 << (k + 1)) - 1
    np.testing.assert_array_equal(gm[ok] & seg, ot["mask"][ok])
    sing = (gm & (1 << 30)) != 0
    st = ok & ~sing & (ot["E_change"] < E_STABLE) & (ot["E"] > 0)
    rel = np.abs(ge[st] - ot["E"][st]) / ot["E"][st]
    blocked = float((ot["mask"] != 0).mean()) if len(ot) else 0.0
    print(f"paths {len(ot)}: mask compared {int(ok.sum())}, blocked {blocked:.3f}; E compared {int(st.sum())}, "
          f"max rel {rel.max() if len(rel) else 0:.2e}, singular {int(sing.sum())}")
    assert ok.mean() > 0.99 and st.mean() > 0.95
    assert blocked >= min_blocked
    if len(rel):
        assert rel.max() <= E_RTOL, rel.max()
    return int(st.sum())


def _one_vertex_case(case):
    """(mesh, x0, light, q_x0, q_light, q_tri [n,1], oracle solutions, eta) of
    a one-vertex tail case: the small glints heightfield with 32x32 shading
    points (refraction: mirrored below the surface), the same with three
    occluding strips, or the self-shadowing steep heightfield.  Candidates
    from the oracle's own cone cull."""
    if case == "R-shadowed":
        w = scenes.shadowed_glints()
        mesh, x0, xl, ev = w.mesh, w.x0, w.x2, "R"
    else:
        w = scenes.glints_small()
        ev = case[0]
        mesh = scenes.with_occluders(w.mesh, scenes.GLINT_STRIPS) if "strips" in case else w.mesh
        x0 = scenes.points_grid(32, -1.0, 1.0, 1.0 if ev == "R" else -1.0)
        xl = w.x2
    eta = (1.0, 1.0) if ev == "R" else (1.5, 1.0)
    keep = oracle.cull_1bounce(mesh.P, mesh.N, mesh.tri, x0, xl, *eta, margin=1e-3)
    j0, jl, t = np.nonzero(keep.reshape(len(x0), len(xl), mesh.nt))
    sols, _ = oracle.solve_1bounce(mesh.P, mesh.N, mesh.tri, x0, xl, j0, jl, t, ev, *eta)
    return mesh, x0, xl, j0.astype(np.int32), jl.astype(np.int32), t[:, None].astype(np.int32), sols, eta


@pytest.mark.parametrize("case", ["R", "T", "R-strips", "R-shadowed"])
def test_tail_one_vertex_vs_oracle(sp, ctx, case):
    _tag(f"tail one vertex {case}")
    ev = case[0]
    mesh, x0, xl, q0, ql, qt, sols, eta = _one_vertex_case(case)
    ot = _oracle_tail(mesh, x0, xl, q0, ql, qt, sols, ev, eta, rho=0.9)
    gm, ge, _ = _gpu_tail(sp, ctx, mesh, x0, xl, q0, ql, _records(sp, sols, qt, 1), ev, eta,
                          params=sp.tail_default_params(reflectance=0.9))
    n = _compare(gm, ge, ot, 1, min_blocked=0.2 if case in ("R-strips", "R-shadowed") else 0.0)
    assert n >= 250


def test_tail_tt_traced_vs_oracle(sp, ctx):
    _tag("tail TT traced receivers")
    mesh = scenes.caustic_sphere()
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    g = np.linspace(-0.35, 0.35, 6)
    x0s, Q = [], []
    for ox in g:
        for oy in g:
            x0, entry, exit_ = ttcases.traced_receiver((ox, oy, 0.0))
            tp = ttcases.tuples_near(mesh, x0, x3[0], entry, exit_, 0.06)
            Q.append(np.column_stack([np.full(len(tp), len(x0s)), tp]))
            x0s.append(x0)
    x0s = np.asarray(x0s)
    Q = np.concatenate(Q).astype(np.int32)
    z = np.zeros(len(Q), dtype=np.int32)
    sols, _ = oracle.solve_tt(mesh.P, mesh.N, mesh.tri, x0s, x3, Q[:, 0], z, Q[:, 1], Q[:, 2])
    eta = (1.0, 1.5, 1.0)
    ot = _oracle_tail(mesh, x0s, x3, Q[:, 0], z, Q[:, 1:], sols, "TT", eta)
    gm, ge, _ = _gpu_tail(sp, ctx, mesh, x0s, x3, Q[:, 0], z, _records(sp, sols, Q[:, 1:], 2), "TT", eta)
    assert _compare(gm, ge, ot, 2) >= 20
    assert np.all((ot["fresnel"] > 0.5) & (ot["fresnel"] < 1.0))


@pytest.mark.parametrize("chain", ["RR", "RT", "TR"])
def test_tail_two_vertex_chains_vs_oracle(sp, ctx, chain):
    _tag(f"tail chain {chain}")
    mesh, x0, x3, t1, t2, uv = tc.trace_paths(chain, 40, 101)
    eta = tc.SETUPS[chain][2]
    Q = []
    for k in range(len(t1)):
        tup = tc.neighbourhood(mesh, t1[k], t2[k], 0.15)
        Q.append(np.column_stack([np.full(len(tup), k), tup]))
    Q = np.concatenate(Q).astype(np.int32)
    sols, _ = oracle.solve_2v(mesh.P, mesh.N, mesh.tri, x0, x3, Q[:, 0], Q[:, 0], Q[:, 1], Q[:, 2], chain, eta)
    ot = _oracle_tail(mesh, x0, x3, Q[:, 0], Q[:, 0], Q[:, 1:], sols, chain, eta, rho=0.95)
    gm, ge, _ = _gpu_tail(sp, ctx, mesh, x0, x3, Q[:, 0], Q[:, 0], _records(sp, sols, Q[:, 1:], 2), chain, eta,
                          params=sp.tail_default_params(reflectance=0.95))
    assert _compare(gm, ge, ot, 2) >= 30


@pytest.mark.parametrize("nt,size,n", [(3000, 0.03, 20000), (50000, 0.008, 2000)])
def test_bvh_visibility_random_soup(sp, ctx, nt, size, n):
    """Visibility masks of random two-vertex 'chains' (vertices at random
    points of random triangles) in a soup of small random triangles: the BVH
    traversal against the oracle's test of every triangle, every combination
    of blocked segments present."""
    _tag(f"bvh random soup {nt}")
    rng = np.random.default_rng(21)
    c = rng.uniform(-1, 1, (nt, 3))
    P = (c[:, None, :] + rng.normal(scale=size, size=(nt, 3, 3))).reshape(-1, 3)
    tri = np.arange(3 * nt, dtype=np.int32).reshape(nt, 3)
    N = rng.normal(size=P.shape)
    mesh = scenes.Mesh(P, N, tri)
    x0s, xl = rng.uniform(-1.3, 1.3, (n, 3)), rng.uniform(-1.3, 1.3, (1, 3))
    T = rng.integers(0, nt, (n, 2))
    U, V = rng.uniform(0.05, 0.45, (n, 2)), rng.uniform(0.05, 0.45, (n, 2))
    sols = np.zeros(n, dtype=oracle.SOL_DTYPE)
    sols["query"] = np.arange(n)
    sols["u1"], sols["v1"], sols["u2"], sols["v2"] = U[:, 0], V[:, 0], U[:, 1], V[:, 1]
    q0, ql = np.arange(n, dtype=np.int32), np.zeros(n, dtype=np.int32)
    ot = _oracle_tail(mesh, x0s, xl, q0, ql, T, sols, "RR", (1.0, 1.0, 1.0))
    gm, _, _ = _gpu_tail(sp, ctx, mesh, x0s, xl, q0, ql, _records(sp, sols, T, 2), "RR", (1.0, 1.0, 1.0))
    ok = ot["margin"] > MARGIN
    np.testing.assert_array_equal(gm[ok] & 7, ot["mask"][ok])
    assert not np.any(gm & (1 << 29))
    combos = np.bincount(ot["mask"], minlength=8)
    print(f"soup {nt}: {n} chains, compared {int(ok.sum())}, masks by value {combos.tolist()}")
    assert ok.mean() > 0.99 and np.all(combos[:8] > 0)


def test_single_triangle_mesh_and_count_limit(sp, ctx):
    """A one-triangle mesh (no internal nodes) and a device count below the
    record count: records past the count are left untouched."""
    _tag("tail single triangle")
    P = np.array([[-0.5, -0.4, 0.0], [0.5, -0.4, 0.0], [0.0, 0.5, 0.0]])
    N = np.column_stack([0.3 * P[:, 0], 0.3 * P[:, 1], np.ones(3)])
    mesh = scenes.Mesh(P, N, np.array([[0, 1, 2]], dtype=np.int32))
    x0 = scenes.points_grid(24, -1.2, 1.2, 1.0)
    xl = np.array([[0.4, 0.2, 2.0]])
    nq = len(x0)
    sols, _ = oracle.solve_1bounce(P, N, mesh.tri, x0, xl, np.arange(nq), np.zeros(nq), np.zeros(nq), "R")
    qt = np.zeros((nq, 1), dtype=np.int32)
    ot = _oracle_tail(mesh, x0, xl, np.arange(nq), np.zeros(nq, np.int32), qt, sols, "R", (1.0, 1.0))
    gm, ge, _ = _gpu_tail(sp, ctx, mesh, x0, xl, np.arange(nq), np.zeros(nq), _records(sp, sols, qt, 1), "R",
                          (1.0, 1.0))
    _compare(gm, ge, ot, 1)
    dm = sp.DeviceMesh(P, N, mesh.tri)
    bvh = sp.Bvh(ctx, dm)
    m = torch.full((len(sols),), -7, dtype=torch.int32, device="cuda")
    cnt = torch.tensor([len(sols) // 2], dtype=torch.int64, device="cuda")
    ctx.path_tail(dm, bvh, "R", (1.0, 1.0), sp.DevicePoints(x0), sp.DevicePoints(xl), _i32(np.arange(nq)),
                  _i32(np.zeros(nq)), sp.solutions_to_device(_records(sp, sols, qt, 1)), sol_count=cnt, mask=m)
    m = m.cpu().numpy()
    assert np.all(m[: len(sols) // 2] != -7) and np.all(m[len(sols) // 2:] == -7)


def test_tail_image_end_to_end(sp, ctx):
    """GPU solve then GPU tail into an image of the receivers, against the
    oracle's solve and tail (receivers with an edge-band or near-threshold
    solution on either side left out)."""
    _tag("tail image end to end")
    w = scenes.glints_small()
    mesh = scenes.with_occluders(w.mesh, scenes.GLINT_STRIPS)
    x0, xl = w.x0, w.x2
    qp, qt = scenes.all_pairs(len(x0), mesh.nt)
    z = np.zeros_like(qp)
    dm = sp.DeviceMesh(mesh.P, mesh.N, mesh.tri)
    d0, dl = sp.DevicePoints(x0), sp.DevicePoints(xl)
    gs = ctx.solve_1bounce(dm, d0, dl, _i32(qp), _i32(z), _i32(qt), "R", 1.0, 1.0)
    bvh = sp.Bvh(ctx, dm)
    img = torch.zeros(len(x0), dtype=torch.float64, device="cuda")
    prm = sp.tail_default_params(rcv_normal=(0.0, 0.0, 1.0))
    ctx.path_tail(dm, bvh, "R", (1.0, 1.0), d0, dl, _i32(qp), _i32(z), sp.solutions_to_device(gs), params=prm,
                  image=img)
    gi = img.cpu().numpy()
    os_, _ = oracle.solve_1bounce(mesh.P, mesh.N, mesh.tri, x0, xl, qp, z, qt, "R")
    ot = _oracle_tail(mesh, x0, xl, qp, z, qt[:, None], os_, "R", (1.0, 1.0))
    x1 = mesh.P[mesh.tri[qt[os_["query"]], 0]]
    e1 = mesh.P[mesh.tri[qt[os_["query"]], 1]] - x1
    e2 = mesh.P[mesh.tri[qt[os_["query"]], 2]] - x1
    x1 = x1 + os_["u1"][:, None] * e1 + os_["v1"][:, None] * e2
    wdir = x1 - x0[qp[os_["query"]]]
    cosz = np.abs(wdir[:, 2]) / np.linalg.norm(wdir, axis=1)
    oi = np.bincount(qp[os_["query"]], weights=ot["E"] * cosz * (ot["mask"] == 0), minlength=len(x0))
    bad = np.zeros(len(x0), dtype=bool)
    for s in (os_, gs):
        amb = (s["edge"] < 1e-9) | ((s["residual"] > 1e-7) & (s["residual"] < 1e-5))
        bad[qp[s["query"][amb]]] = True
    bad[qp[os_["query"][(ot["margin"] <= MARGIN) | (ot["E_change"] >= E_STABLE)]]] = True
    ok = ~bad
    rel = np.abs(gi[ok] - oi[ok]) / np.maximum(oi[ok], 1e-300)
    print(f"image: {int(ok.sum())} of {len(x0)} receivers compared, total {oi.sum():.4e}, max rel {rel.max():.2e}")
    assert ok.sum() >= 0.9 * len(x0)
    assert np.all(rel[oi[ok] > 0] <= E_RTOL)
    assert np.all(gi[ok][oi[ok] == 0] == 0)
