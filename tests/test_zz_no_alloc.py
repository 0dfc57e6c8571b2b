"""spoly_solve_1bounce_noalloc (workspace in a static device array) against
spoly_solve_1bounce (workspace in the context), through the C ABI: the same
solution set, byte for byte, on two calls in a row, the second smaller, for
reflection in FP32 and refraction in FP64 on the glints workload."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2405_13409_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    from paper_2405_13409_amd import spoly

    spoly.load_library()
    return spoly


def _noalloc(sp, mesh, x0s, x2s, q0, q2, qt, ev, e0, e1, prec, cap):
    L = sp.load_library()
    out = torch.empty(cap * sp.SOLUTION_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    prm = sp.default_params()
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    st = L.spoly_solve_1bounce_noalloc(ctypes.byref(mesh.c), ctypes.byref(x0s.c), ctypes.byref(x2s.c), p(q0), p(q2),
                                       p(qt), int(qt.numel()), sp.SPOLY_T if ev == "T" else sp.SPOLY_R, e0, e1, prec,
                                       ctypes.byref(prm), p(out), cap, p(cnt), None, None,
                                       ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, st
    torch.cuda.synchronize()
    n = int(cnt.item())
    assert n <= cap
    return out[: n * sp.SOLUTION_DTYPE.itemsize].cpu().numpy().view(sp.SOLUTION_DTYPE)


@pytest.mark.parametrize("ev,prec,sizes", [("R", 1, (1_900_000, 150_000)), ("T", 0, (440_000, 30_000))])
def test_noalloc_matches_context_entry_point(sp, ev, prec, sizes):
    print(f"[gpu-case] noalloc {ev} prec={prec} sizes={sizes}", flush=True)
    mesh = scenes.glints_large_mesh()
    e0, e1 = (1.0, 1.0) if ev == "R" else (1.5, 1.0)
    x0 = scenes.glints_large_points(ev)[::8]
    x2 = scenes.GLINTS_LARGE_LIGHT
    ctx = sp.Context(0)
    dm = sp.DeviceMesh(mesh.P, mesh.N, mesh.tri)
    d0, d2 = sp.DevicePoints(x0), sp.DevicePoints(x2)
    q0, q2, qt = ctx.cull_1bounce(dm, d0, d2, e0, e1, 1e-3)
    assert qt.numel() >= sizes[0], qt.numel()
    for n in sizes:
        a0, a2, at = q0[:n].contiguous(), q2[:n].contiguous(), qt[:n].contiguous()
        ref = sp.sort_solutions(ctx.solve_1bounce(dm, d0, d2, a0, a2, at, ev, e0, e1, prec))
        got = sp.sort_solutions(_noalloc(sp, dm, d0, d2, a0, a2, at, ev, e0, e1, prec, max(1024, len(ref) + 1024)))
        print(ev, n, "solutions", len(ref))
        assert len(ref) > 100
        assert got.tobytes() == ref.tobytes()
    ctx.close()
