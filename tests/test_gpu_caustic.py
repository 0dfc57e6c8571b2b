"""The learned tuple pruner on the caustic scene: labels agree with the FP64
oracle, training resumes bit for bit from a checkpoint, and the packaged
network keeps >= 99.9% of the positive tuples of unseen receivers while the
pruned solve beats the exhaustive one."""
import os

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


@pytest.fixture(scope="module")
def scene(sp):
    mesh = scenes.caustic_sphere()
    return mesh, sp.DeviceMesh(mesh.P, mesh.N, mesh.tri), sp.DevicePoints(scenes.CAUSTIC_LIGHT_OUTSIDE)


def test_exhaustive_labels_match_oracle(sp, ctx, scene):
    """Labels (>= 1 admissible path per tuple) from the GPU exhaustive solve
    against the oracle's solution sets, on traced-path neighbourhoods plus
    random tuples of the oracle's own cone-cull twin."""
    print("[gpu-case] labels vs oracle", flush=True)
    from paper_2405_13409_amd import pruner

    mesh, dm, dl = scene
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    x0s, Q = [], []
    for i, off in enumerate([(0.1, 0.1, 0.0), (-0.2, -0.05, 0.0)]):
        x0, entry, exit_ = ttcases.traced_receiver(off)
        x0s.append(x0)
        tp = ttcases.tuples_near(mesh, x0, x3[0], entry, exit_, 0.1)
        Q.append(np.column_stack([np.full(len(tp), i), tp]))
    R = scenes.caustic_receivers()
    x0s.append(R[2100])
    keep = oracle.cull_tt(mesh.P, mesh.N, mesh.tri, np.asarray(x0s[-1:]), x3)
    _, _, t1, t2 = np.nonzero(keep)
    s = np.random.default_rng(6).choice(len(t1), 1500, replace=False)
    Q.append(np.column_stack([np.full(len(s), 2), t1[s], t2[s]]))
    Q = np.concatenate(Q).astype(np.int32)
    x0s = np.asarray(x0s)
    z = np.zeros(len(Q), dtype=np.int32)
    o, _ = oracle.solve_tt(mesh.P, mesh.N, mesh.tri, x0s, x3, Q[:, 0], z, Q[:, 1], Q[:, 2])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    T = pruner.Tuples(dev(Q[:, 0]), dev(z), dev(Q[:, 1:]))
    lab, nsol, _ = pruner.exhaustive_labels(ctx, dm, sp.DevicePoints(x0s), dl, T)
    g = lab.cpu().numpy() > 0.5
    ol = np.zeros(len(Q), dtype=bool)
    ol[o["query"]] = True
    amb = np.zeros(len(Q), dtype=bool)
    amb[o["query"][(o["edge"] < 1e-9) | ((o["residual"] > 1e-7) & (o["residual"] < 1e-5))]] = True
    print("labels: positives oracle", ol.sum(), "gpu", g.sum(), "ambiguous", amb.sum())
    assert ol.sum() >= 2
    assert np.array_equal(g[~amb], ol[~amb])


def _random_batch(sp, mesh, n, seed):
    from paper_2405_13409_amd import pruner

    rng = np.random.default_rng(seed)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()  # noqa: E731
    q0 = rng.integers(0, 64, n)
    qt = rng.integers(0, mesh.nt, (n, 2))
    T = pruner.Tuples(dev(q0), dev(np.zeros(n)), dev(qt))
    T.labels = torch.from_numpy((rng.random(n) < 0.1).astype(np.float32)).cuda()
    return T


def test_training_resumes_bitwise(sp, ctx, scene, tmp_path):
    """Ten steps, checkpoint, reload into a fresh object, ten more steps: the
    parameters equal those of twenty uninterrupted steps bit for bit."""
    print("[gpu-case] pruner resume", flush=True)
    from paper_2405_13409_amd import pruner

    mesh, dm, dl = scene
    d0 = sp.DevicePoints(scenes.pruner_receivers(64, 9))
    T = _random_batch(sp, mesh, 20000, 3)
    a = pruner.Pruner(7)
    a.train_steps(ctx, dm, d0, dl, T, 20, batch=1024)
    b = pruner.Pruner(7)
    b.train_steps(ctx, dm, d0, dl, T, 10, batch=1024)
    path = str(tmp_path / "ck.npz")
    b.save(path)
    c = pruner.Pruner(123)
    c.load(path)
    c.train_steps(ctx, dm, d0, dl, T, 10, batch=1024)
    torch.cuda.synchronize()
    assert c.step == a.step == 20
    assert torch.equal(a.params, c.params)
    assert torch.equal(a.m, c.m) and torch.equal(a.v, c.v)


def test_training_separates_positives(sp, ctx, scene):
    """A few hundred steps on solver labels of traced-path neighbourhoods:
    the loss falls and every positive tuple scores above the median negative."""
    print("[gpu-case] pruner train small", flush=True)
    from paper_2405_13409_amd import pruner

    mesh, dm, dl = scene
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    rng = np.random.default_rng(11)
    x0s, Q = [], []
    for i in range(12):
        off = np.r_[rng.uniform(-0.25, 0.25, 2), 0.0]
        x0, entry, exit_ = ttcases.traced_receiver(off)
        x0s.append(x0)
        tp = ttcases.tuples_near(mesh, x0, x3[0], entry, exit_, 0.3)
        Q.append(np.column_stack([np.full(len(tp), i), tp]))
    Q = np.concatenate(Q).astype(np.int32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()  # noqa: E731
    T = pruner.Tuples(dev(Q[:, 0]), dev(np.zeros(len(Q))), dev(Q[:, 1:]))
    d0 = sp.DevicePoints(np.asarray(x0s))
    T.labels, nsol, _ = pruner.exhaustive_labels(ctx, dm, d0, dl, T)
    npos = int(T.labels.sum().item())
    assert npos >= 12
    net = pruner.Pruner(1)
    hist = net.train_steps(ctx, dm, d0, dl, T, 400, batch=2048)
    s = net.scores(ctx, dm, d0, dl, T).cpu().numpy()
    y = T.labels.cpu().numpy() > 0.5
    print("tuples", len(Q), "positives", npos, "loss", hist[0], "->", np.mean(hist[-20:]))
    assert np.mean(hist[-20:]) < 0.2 * hist[0]
    assert s[y].min() > np.median(s[~y])


def test_packaged_pruner_recall_and_speedup(sp, ctx, scene):
    """The packaged network on unseen receivers (every 8th of the 64x64 grid,
    offset 5): recall of positive tuples >= 99.9% against the exhaustive solve,
    and score + pruned solve faster than the exhaustive solve."""
    print("[gpu-case] packaged pruner", flush=True)
    from paper_2405_13409_amd import caustic, train_pruner

    assert os.path.exists(train_pruner.DEFAULT_OUT), "trained pruner weights are missing"
    mesh, dm, dl = scene
    net = train_pruner.load()
    rec = scenes.caustic_receivers()[5::8]
    d0 = sp.DevicePoints(rec)
    T = caustic.cull_sorted(ctx, dm, d0, dl)
    r = caustic.prune_vs_exhaustive(ctx, dm, d0, dl, T, net, reps=1)
    print(r.as_dict())
    assert r.positives > 20
    assert r.recall >= 0.999
    assert r.path_recall >= 0.999
    assert r.speedup > 2.0
