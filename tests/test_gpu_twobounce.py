"""GPU parity of the two-vertex (TT) path against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import ttcases
from paper_2405_13409_amd import scenes

pytestmark = pytest.mark.gpu


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


def _gpu_tt(sp, ctx, mesh, x0s, x3s, q0, q3, qt, eta=(1.0, 1.5, 1.0), diag=False):
    dm = sp.DeviceMesh(mesh.P, mesh.N, mesh.tri)
    d0, d3 = sp.DevicePoints(x0s), sp.DevicePoints(x3s)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()  # noqa: E731
    cnt = torch.zeros(4, dtype=torch.int64, device="cuda")
    dq = torch.zeros(2 * len(q0), dtype=torch.int32, device="cuda") if diag else None
    s = ctx.solve_2bounce(dm, d0, d3, t(q0), t(q3), t(qt), eta, counters=cnt, diag=dq)
    torch.cuda.synchronize()
    if diag:
        return s, cnt.cpu().numpy(), dq.cpu().numpy().reshape(-1, 2)
    return s, cnt.cpu().numpy()


def _compare_tt(g, o, nq, tol=1e-10, band=1e-9, tau=1e-6):
    bad = np.zeros(nq, dtype=bool)
    bad[o["query"][(o["edge"] < band) | ((o["residual"] > tau / 10) & (o["residual"] < 10 * tau))]] = True
    bad[g["query"][(g["edge"] < band) | ((g["residual"] > tau / 10) & (g["residual"] < 10 * tau))]] = True
    g = g[~bad[g["query"]]]
    o = o[~bad[o["query"]]]
    g = g[np.lexsort((g["u"][:, 0], g["v"][:, 0], g["query"]))]
    o = o[np.lexsort((o["u1"], o["v1"], o["query"]))]
    gq, oq = np.bincount(g["query"], minlength=nq), np.bincount(o["query"], minlength=nq)
    mism = np.nonzero(gq != oq)[0]
    assert len(mism) == 0, f"{len(mism)} tuples differ: q={mism[:5]} gpu={gq[mism[:5]]} oracle={oq[mism[:5]]}"
    if len(g):
        err = max(np.abs(g["u"][:, 0] - o["u1"]).max(), np.abs(g["v"][:, 0] - o["v1"]).max(),
                  np.abs(g["u"][:, 1] - o["u2"]).max(), np.abs(g["v"][:, 1] - o["v2"]).max())
        assert err <= tol, err
    return len(o), int(bad.sum())


def test_tt_traced_paths_parity(sp, ctx):
    _tag("tt traced paths")
    mesh = scenes.caustic_sphere()
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    x0s, Q = [], []
    for i, off in enumerate([(0.12, -0.07, 0.0), (-0.15, 0.05, 0.0), (0.05, 0.18, 0.0)]):
        x0, entry, exit_ = ttcases.traced_receiver(off)
        x0s.append(x0)
        tp = ttcases.tuples_near(mesh, x0, x3[0], entry, exit_, 0.15)
        Q.append(np.column_stack([np.full(len(tp), i), tp]))
    x0s = np.asarray(x0s)
    Q = np.concatenate(Q)
    q0, qt = Q[:, 0].astype(np.int32), Q[:, 1:].astype(np.int32)
    z = np.zeros_like(q0)
    o, od = oracle.solve_tt(mesh.P, mesh.N, mesh.tri, x0s, x3, q0, z, qt[:, 0], qt[:, 1])
    g, cnt = _gpu_tt(sp, ctx, mesh, x0s, x3, q0, z, qt)
    n, nb = _compare_tt(g, o, len(q0))
    print("tt compared", n, "excluded", nb, "oracle sign changes", od["n_vroots"].sum(), "gpu", cnt[0])
    assert cnt[3] == 0  # no tuple with more paths than the four kept
    assert n >= 3


def test_tt_random_culled_tuples_parity(sp, ctx):
    _tag("tt random culled")
    mesh = scenes.caustic_sphere()
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    R = scenes.caustic_receivers()
    x0s = R[np.random.default_rng(2).choice(len(R), 3, replace=False)]
    keep = oracle.cull_tt(mesh.P, mesh.N, mesh.tri, x0s, x3)
    j0, j3, t1, t2 = np.nonzero(keep)
    s = np.sort(np.random.default_rng(3).choice(len(j0), 3000, replace=False))
    q0, q3, qt = j0[s].astype(np.int32), j3[s].astype(np.int32), np.stack([t1[s], t2[s]], 1).astype(np.int32)
    o, od = oracle.solve_tt(mesh.P, mesh.N, mesh.tri, x0s, x3, q0, q3, qt[:, 0], qt[:, 1])
    g, cnt = _gpu_tt(sp, ctx, mesh, x0s, x3, q0, q3, qt)
    n, nb = _compare_tt(g, o, len(q0))
    print("random tt compared", n, "excluded", nb, "sign changes oracle/gpu", od["n_vroots"].sum(), cnt[0])
    # random culled tuples rarely hold a path: every tuple's (empty or not) set is compared
    assert len(q0) - nb >= 0.99 * len(q0)


def test_tt_traced_receivers_parity(sp, ctx):
    """64 receivers where traced rays through the exact sphere land; the tuples
    within 0.06 of each path's entry and exit: at least 50 compared paths,
    sign-change counts per tuple compared as a diagnostic."""
    _tag("tt 64 traced receivers")
    mesh = scenes.caustic_sphere()
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    g = np.linspace(-0.35, 0.35, 8)
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
    o, od = oracle.solve_tt(mesh.P, mesh.N, mesh.tri, x0s, x3, Q[:, 0], z, Q[:, 1], Q[:, 2])
    gs, cnt, dq = _gpu_tt(sp, ctx, mesh, x0s, x3, Q[:, 0], z, Q[:, 1:], diag=True)
    n, nb = _compare_tt(gs, o, len(Q))
    rec = len(np.unique(Q[o["query"], 0]))
    same = int(np.sum(dq[:, 0] == od["n_vroots"]))
    print(f"{len(Q)} tuples of {len(x0s)} receivers: compared {n} paths ({rec} receivers), excluded {nb}; "
          f"sign changes oracle {od['n_vroots'].sum()} gpu {dq[:, 0].sum()}, equal on {same} tuples")
    assert n >= 50 and rec >= 20


def test_tt_light_inside_sphere_has_no_paths(sp, ctx):
    _tag("tt negative control")
    mesh = scenes.caustic_sphere()
    x3 = scenes.CAUSTIC_LIGHT_INSIDE
    R = scenes.caustic_receivers()[::613]
    c = mesh.P[mesh.tri].mean(1)
    rng = np.random.default_rng(4)
    Q = np.stack([rng.integers(0, len(R), 4000), rng.integers(0, mesh.nt, 4000), rng.integers(0, mesh.nt, 4000)], 1)
    Q = Q[Q[:, 1] != Q[:, 2]].astype(np.int32)
    z = np.zeros(len(Q), dtype=np.int32)
    g, _ = _gpu_tt(sp, ctx, mesh, R, x3, Q[:, 0], z, Q[:, 1:])
    assert len(g) == 0
    del c


def test_tt_cull_bounds_against_oracle_twin(sp, ctx):
    _tag("tt cull")
    mesh = scenes.caustic_sphere()
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    R = scenes.caustic_receivers()[::1024]
    dm = sp.DeviceMesh(mesh.P, mesh.N, mesh.tri)
    q0, q3, qt = ctx.cull_2bounce(dm, sp.DevicePoints(R), sp.DevicePoints(x3), (1.0, 1.5, 1.0), 1e-3)
    q0, q3, qt = q0.cpu().numpy(), q3.cpu().numpy(), qt.cpu().numpy()
    gk = np.zeros((len(R), 1, mesh.nt, mesh.nt), dtype=bool)
    gk[q0, q3, qt[:, 0], qt[:, 1]] = True
    assert gk.sum() == len(q0)
    tight = oracle.cull_tt(mesh.P, mesh.N, mesh.tri, R, x3, (1.0, 1.5, 1.0), 0.0)
    loose = oracle.cull_tt(mesh.P, mesh.N, mesh.tri, R, x3, (1.0, 1.5, 1.0), 3e-3)
    assert np.all(gk[tight]), "GPU cull dropped a tuple the FP64 twin keeps"
    assert np.all(loose[gk]), "GPU cull kept a tuple outside the widened FP64 twin"


def test_tt_exhaustive_receivers_parity(sp, ctx):
    """Every GPU-culled tuple of every 512th receiver of the 64x64 caustic
    grid, in the order the benchmark solves them: the whole solution sets
    against the oracle's, and the sign-change count of each tuple's scan."""
    from paper_2405_13409_amd import caustic

    _tag("tt exhaustive receivers")
    mesh = scenes.caustic_sphere()
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    rec = scenes.caustic_receivers()[::512]
    dm = sp.DeviceMesh(mesh.P, mesh.N, mesh.tri)
    d0, dl = sp.DevicePoints(rec), sp.DevicePoints(x3)
    T = caustic.cull_sorted(ctx, dm, d0, dl)
    dq = torch.zeros(2 * T.n, dtype=torch.int32, device="cuda")
    g = ctx.solve_2bounce(dm, d0, dl, T.q0, T.q3, T.qt, diag=dq)
    torch.cuda.synchronize()
    q0, q3, qt = T.q0.cpu().numpy(), T.q3.cpu().numpy(), T.qt.cpu().numpy().reshape(-1, 2)
    threads = oracle.set_threads(16)
    try:
        o, od = oracle.solve_tt(mesh.P, mesh.N, mesh.tri, rec, x3, q0, q3, qt[:, 0], qt[:, 1])
    finally:
        oracle.set_threads(threads)
    n, nb = _compare_tt(g, o, T.n)
    same = float(np.mean(dq.cpu().numpy().reshape(-1, 2)[:, 0] == od["n_vroots"]))
    print(f"{T.n} tuples of {len(rec)} receivers: {len(o)} oracle paths, compared {n}, excluded {nb}; "
          f"sign-change counts equal on {same:.5f} of the tuples")
    assert T.n > 100000 and nb <= 0.001 * T.n and same >= 0.999
