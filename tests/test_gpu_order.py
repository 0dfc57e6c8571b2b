"""SPOLY_FLAG_DETERMINISTIC_ORDER through the C ABI: the records a solve
writes come out sorted by (query, v[0], u[0]), the same set as without the
flag, byte-identical from run to run, also when the output capacity cuts the
list; the no-allocation and mixed entry points refuse the flag."""
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
def ctx(sp):
    c = sp.Context(0)
    yield c
    c.close()


def _tag(name):
    print(f"[gpu-case] {name}", flush=True)


def _i32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def _sorted_host(r):
    return r[np.lexsort((r["u"][:, 0], r["v"][:, 0], r["query"]))]


def _assert_sorted(r):
    key = np.lexsort((r["u"][:, 0], r["v"][:, 0], r["query"]))
    assert np.array_equal(key, np.arange(len(r))), "records not in (query, v, u) order"


def _one_vertex(sp, ctx, ordered, cap=None):
    w = scenes.glints_small()
    dm = sp.DeviceMesh(w.mesh.P, w.mesh.N, w.mesh.tri)
    prm = sp.default_params()
    if ordered:
        prm.flags = sp.SPOLY_FLAG_DETERMINISTIC_ORDER
    return ctx.solve_1bounce(dm, sp.DevicePoints(w.x0), sp.DevicePoints(w.x2), _i32(w.q_x0), _i32(w.q_x2),
                             _i32(w.q_tri), "R", 1.0, 1.0, sp.SPOLY_FP64, params=prm, capacity=cap)


def test_one_vertex_sorted_same_set_and_repeatable(sp, ctx):
    _tag("order one vertex")
    plain = _one_vertex(sp, ctx, False)
    a = _one_vertex(sp, ctx, True)
    b = _one_vertex(sp, ctx, True)
    assert len(a) == len(plain) > 20
    _assert_sorted(a)
    assert a.tobytes() == b.tobytes()
    assert _sorted_host(plain).tobytes() == a.tobytes()


def test_two_vertex_sorted_same_set(sp, ctx):
    _tag("order two vertex")
    mesh = scenes.caustic_sphere()
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    x0s, Q = [], []
    for i, off in enumerate([(0.12, -0.07, 0.0), (-0.15, 0.05, 0.0), (0.05, 0.18, 0.0), (0.2, 0.1, 0.0)]):
        x0, entry, exit_ = ttcases.traced_receiver(off)
        x0s.append(x0)
        tp = ttcases.tuples_near(mesh, x0, x3[0], entry, exit_, 0.15)
        Q.append(np.column_stack([np.full(len(tp), i), tp]))
    Q = np.concatenate(Q).astype(np.int32)
    # a shuffled query order, so that the sort has work to do across queries
    Q = Q[np.random.default_rng(5).permutation(len(Q))]
    dm = sp.DeviceMesh(mesh.P, mesh.N, mesh.tri)
    args = (dm, sp.DevicePoints(np.asarray(x0s)), sp.DevicePoints(x3), _i32(Q[:, 0]), _i32(np.zeros(len(Q))),
            _i32(Q[:, 1:]))
    plain = ctx.solve_2bounce(*args)
    prm = sp.tt_default_params()
    prm.flags = sp.SPOLY_FLAG_DETERMINISTIC_ORDER
    a = ctx.solve_2bounce(*args, params=prm)
    b = ctx.solve_2bounce(*args, params=prm)
    assert len(a) == len(plain) >= 3
    _assert_sorted(a)
    assert a.tobytes() == b.tobytes() == _sorted_host(plain).tobytes()


def test_capacity_below_count_sorts_what_was_written(sp, ctx):
    _tag("order capacity")
    w = scenes.glints_small()
    dm = sp.DeviceMesh(w.mesh.P, w.mesh.N, w.mesh.tri)
    prm = sp.default_params()
    prm.flags = sp.SPOLY_FLAG_DETERMINISTIC_ORDER
    cap = 16
    out = torch.zeros(cap * sp.SOLUTION_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.solve_1bounce(dm, sp.DevicePoints(w.x0), sp.DevicePoints(w.x2), _i32(w.q_x0), _i32(w.q_x2), _i32(w.q_tri),
                      "R", 1.0, 1.0, sp.SPOLY_FP64, params=prm, out=out, out_count=cnt, sync=False)
    torch.cuda.synchronize()
    assert int(cnt.item()) > cap
    r = out.cpu().numpy().view(sp.SOLUTION_DTYPE)
    _assert_sorted(r)
    assert np.all(r["query"] >= 0)


def test_noalloc_and_mixed_refuse_the_flag(sp, ctx):
    _tag("order refused")
    import ctypes

    L = sp.load_library()
    w = scenes.glints_small()
    dm = sp.DeviceMesh(w.mesh.P, w.mesh.N, w.mesh.tri)
    d0, d2 = sp.DevicePoints(w.x0), sp.DevicePoints(w.x2)
    prm = sp.default_params()
    prm.flags = sp.SPOLY_FLAG_DETERMINISTIC_ORDER
    out = torch.zeros(64 * sp.SOLUTION_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    q = _i32(w.q_x0[:64]), _i32(w.q_x2[:64]), _i32(w.q_tri[:64])
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    st = L.spoly_solve_1bounce_noalloc(ctypes.byref(dm.c), ctypes.byref(d0.c), ctypes.byref(d2.c), p(q[0]), p(q[1]),
                                       p(q[2]), 64, sp.SPOLY_R, 1.0, 1.0, sp.SPOLY_FP64, ctypes.byref(prm), p(out), 64,
                                       p(cnt), None, None, None)
    assert st == sp.SPOLY_E_UNSUPPORTED
    prm.flags = 1 << 7
    st = L.spoly_solve_1bounce_noalloc(ctypes.byref(dm.c), ctypes.byref(d0.c), ctypes.byref(d2.c), p(q[0]), p(q[1]),
                                       p(q[2]), 64, sp.SPOLY_R, 1.0, 1.0, sp.SPOLY_FP64, ctypes.byref(prm), p(out), 64,
                                       p(cnt), None, None, None)
    assert st == sp.SPOLY_E_INVALID_ARG
