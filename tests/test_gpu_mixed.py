"""The persistent mixed launch returns exactly the union of the separate
one- and two-vertex solves, for every queue order and shape, eagerly and when
replayed from a captured graph; the autotuner caches its choice."""
import numpy as np
import pytest
import torch

import ttcases
from paper_2405_13409_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    from paper_2405_13409_amd import spoly

    spoly.load_library()
    return spoly


@pytest.fixture(scope="module")
def problem(sp):
    ctx = sp.Context(0)
    w = scenes.glints_small()
    rng = np.random.default_rng(4)
    sel = np.sort(rng.choice(len(w.q_tri), 6000, replace=False))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()  # noqa: E731
    m1 = sp.DeviceMesh(w.mesh.P, w.mesh.N, w.mesh.tri)
    p1 = (sp.DevicePoints(w.x0), sp.DevicePoints(w.x2))
    q1 = (t(w.q_x0[sel]), t(w.q_x2[sel]), t(w.q_tri[sel]))
    mesh = scenes.caustic_sphere()
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    x0s, Q = [], []
    for i, off in enumerate([(0.12, -0.07, 0.0), (-0.15, 0.05, 0.0)]):
        x0, entry, exit_ = ttcases.traced_receiver(off)
        x0s.append(x0)
        tp = ttcases.tuples_near(mesh, x0, x3[0], entry, exit_, 0.12)
        Q.append(np.column_stack([np.full(len(tp), i), tp]))
    Q = np.concatenate(Q)
    m2 = sp.DeviceMesh(mesh.P, mesh.N, mesh.tri)
    p2 = (sp.DevicePoints(np.asarray(x0s)), sp.DevicePoints(x3))
    q2 = (t(Q[:, 0]), t(np.zeros(len(Q))), t(Q[:, 1:]))
    yield ctx, m1, p1, q1, m2, p2, q2
    ctx.close()


def _key(s):
    s = s[np.lexsort((s["u"][:, 0], s["v"][:, 0], s["query"]))]
    return s


def _separate(sp, ctx, m1, p1, q1, m2, p2, q2):
    a = ctx.solve_1bounce(m1, p1[0], p1[1], *q1, "R", 1.0, 1.0, sp.SPOLY_FP32_POLISH64)
    b = ctx.solve_2bounce(m2, p2[0], p2[1], *q2)
    b = b.copy()
    b["query"] += int(q1[2].numel())
    return _key(np.concatenate([a, b]))


def test_mixed_equals_separate(sp, problem):
    print("[gpu-case] mixed vs separate", flush=True)
    ctx, m1, p1, q1, m2, p2, q2 = problem
    ref = _separate(sp, ctx, m1, p1, q1, m2, p2, q2)
    assert len(ref) > 10 and np.any(ref["tri"][:, 1] >= 0)
    for shape in [(1, 64, 0), (2, 256, 1), (4, 1024, 2), (8, 64, 2)]:
        got = _key(ctx.solve_mixed(m1, *p1, *q1, "R", 1.0, 1.0, m2, *p2, *q2,
                                   shape=sp.MixedShape(shape[0], shape[1], shape[2], 0)))
        assert got.tobytes() == ref.tobytes(), shape


def test_mixed_graph_replay(sp, problem):
    print("[gpu-case] mixed graph", flush=True)
    ctx, m1, p1, q1, m2, p2, q2 = problem
    ref = _separate(sp, ctx, m1, p1, q1, m2, p2, q2)
    cap = 4 * len(ref) + 64
    out = torch.zeros(cap * sp.SOLUTION_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    queue = torch.zeros(1, dtype=torch.int64, device="cuda")
    shape = sp.MixedShape(2, 256, 0, 0)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        cnt.zero_()
        queue.zero_()
        ctx.solve_mixed(m1, *p1, *q1, "R", 1.0, 1.0, m2, *p2, *q2, shape=shape, out=out, out_count=cnt,
                        queue=queue, sync=False)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cnt.zero_()
        queue.zero_()
        ctx.solve_mixed(m1, *p1, *q1, "R", 1.0, 1.0, m2, *p2, *q2, shape=shape, out=out, out_count=cnt,
                        queue=queue, sync=False)
    for rep in range(3):
        out.fill_(0)
        g.replay()
        torch.cuda.synchronize()
        n = int(cnt.item())
        got = _key(out[: n * sp.SOLUTION_DTYPE.itemsize].cpu().numpy().view(sp.SOLUTION_DTYPE))
        assert got.tobytes() == ref.tobytes(), rep
        # eager work between replays
        _separate(sp, ctx, m1, p1, q1, m2, p2, q2)


def test_autotuner_picks_and_caches(sp, problem, tmp_path):
    print("[gpu-case] autotune", flush=True)
    from paper_2405_13409_amd import autotune

    ctx, m1, p1, q1, m2, p2, q2 = problem
    out = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    queue = torch.zeros(1, dtype=torch.int64, device="cuda")

    def run(shape):
        cnt.zero_()
        queue.zero_()
        ctx.solve_mixed(m1, *p1, *q1, "R", 1.0, 1.0, m2, *p2, *q2, shape=shape, out=out, out_count=cnt,
                        queue=queue, sync=False)

    path = str(tmp_path / "tune.json")
    cand = {"workgroups_per_cu": (1, 4), "r_tile": (64, 256), "order": (0, 1)}
    best, t, cached = autotune.tune(run, "test", path, reps=1, candidates=cand)
    assert not cached and len(t) == 8
    best2, _, cached2 = autotune.tune(run, "test", path, reps=1, candidates=cand)
    assert cached2 and (best2.workgroups_per_cu, best2.r_tile, best2.order) == (best.workgroups_per_cu, best.r_tile,
                                                                                 best.order)


def test_mixed_2m_instances_graph_vs_separate_and_oracle(sp):
    """2M instances (70% one-vertex R from the 16x16 heightfield scene, 30% TT
    tuples drawn from the canonical culled list of the 64x64 caustic grid) in
    one captured persistent launch: identical to the separate solves, and the
    one-vertex part within the FP32-path tolerance of the FP64 oracle on a
    seeded sample of instances."""
    print("[gpu-case] mixed 2M", flush=True)
    import oracle
    import parity
    from paper_2405_13409_amd import caustic

    ctx = sp.Context(0)
    w = scenes.glints_small()
    m1 = sp.DeviceMesh(w.mesh.P, w.mesh.N, w.mesh.tri)
    p1 = (sp.DevicePoints(w.x0), sp.DevicePoints(w.x2))
    sph = scenes.caustic_sphere()
    m2 = sp.DeviceMesh(sph.P, sph.N, sph.tri)
    r2 = sp.DevicePoints(scenes.caustic_receivers())
    l2 = sp.DevicePoints(scenes.CAUSTIC_LIGHT_OUTSIDE)
    T = caustic.cull_sorted(ctx, m2, r2, l2)
    i1, i2 = scenes.mixed_draw(len(w.q_tri), T.n, 2_000_000, 0.7, 4)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()  # noqa: E731
    q1 = (dev(w.q_x0[i1]), dev(w.q_x2[i1]), dev(w.q_tri[i1]))
    Q2 = T.take(torch.from_numpy(i2).cuda())
    del T
    prec = sp.SPOLY_FP32_POLISH64
    a = ctx.solve_1bounce(m1, *p1, *q1, "R", 1.0, 1.0, prec)
    b = ctx.solve_2bounce(m2, r2, l2, Q2.q0, Q2.q3, Q2.qt).copy()
    b["query"] += len(i1)
    ref = _key(np.concatenate([a, b]))
    cap = len(ref) + 4096
    out = torch.zeros(cap * sp.SOLUTION_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    queue = torch.zeros(1, dtype=torch.int64, device="cuda")
    shape = sp.MixedShape(2, 1024, 2, 0)

    def launch():
        cnt.zero_()
        queue.zero_()
        ctx.solve_mixed(m1, *p1, *q1, "R", 1.0, 1.0, m2, r2, l2, Q2.q0, Q2.q3, Q2.qt, precision=prec, shape=shape,
                        out=out, out_count=cnt, queue=queue, sync=False)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        launch()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        launch()
    for rep in range(2):
        g.replay()
        torch.cuda.synchronize()
        n = int(cnt.item())
        got = _key(out[: n * sp.SOLUTION_DTYPE.itemsize].cpu().numpy().view(sp.SOLUTION_DTYPE))
        assert got.tobytes() == ref.tobytes(), rep
    # one-vertex part against the FP64 oracle on a seeded sample of 20000 instances
    smp = np.sort(np.random.default_rng(44).choice(len(i1), 20000, replace=False))
    j = i1[smp]
    orc, diag = oracle.solve_1bounce(w.mesh.P, w.mesh.N, w.mesh.tri, w.x0, w.x2, w.q_x0[j], w.q_x2[j], w.q_tri[j],
                                     "R")
    g1 = got[got["query"] < len(i1)]
    pos = np.searchsorted(smp, g1["query"])
    hit = (pos < len(smp)) & (smp[np.minimum(pos, len(smp) - 1)] == g1["query"])
    g1 = g1[hit].copy()
    g1["query"] = pos[hit]
    st = parity.compare_onebounce(g1, orc, diag, len(smp), **parity.FP32)
    print("mixed 2M: paths", len(got), "R sample vs oracle", st, flush=True)
    assert st["compared"] > 20
    # two-vertex part against the FP64 oracle: every tuple with a GPU path plus a seeded sample of 20000
    g2 = got[got["query"] >= len(i1)].copy()
    g2["query"] -= len(i1)
    q0h, q3h, qth = Q2.q0.cpu().numpy(), Q2.q3.cpu().numpy(), Q2.qt.cpu().numpy().reshape(-1, 2)
    smp2 = np.union1d(np.unique(g2["query"]), np.random.default_rng(45).choice(len(i2), 20000, replace=False))
    o2, _ = oracle.solve_tt(sph.P, sph.N, sph.tri, scenes.caustic_receivers(), scenes.CAUSTIC_LIGHT_OUTSIDE,
                            q0h[smp2], q3h[smp2], qth[smp2, 0], qth[smp2, 1])
    pos = np.searchsorted(smp2, g2["query"])
    g2["query"] = pos
    n2 = _compare_tt_sets(g2, o2, len(smp2))
    print("mixed 2M: TT sample vs oracle: tuples", len(smp2), "paths compared", n2, flush=True)
    assert n2 >= 10
    ctx.close()


def _compare_tt_sets(g, o, nq, tol=1e-10, band=1e-9, tau=1e-6):
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
    return len(o)
