"""Throughput of the one-vertex glints path on one MI355X.

Workload (one step = the whole hot path over one batch): a 128x128 heightfield
(32768 triangles, z = 0.02 * 8 sinusoids of angular frequency 4..32), 256x256
shading points at z = 2 (reflection) and at z = -2 (refraction, IOR 1.5 below
the surface), one point light at (0, 0, 4).  A step runs, for R and for T:
the normal-cone cull over all 65536 x 32768 (point, triangle) pairs, then the
full solve on the kept candidates (coefficients, Bezout + Laplace, isolation, u solve, FP64
polish, validation, compaction).  Inputs are resident in HBM before timing.

Prints one JSON line.  value = candidate solves / s (candidates entering the
solve per second of step time); valid paths / s is reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU = 78.6    # TFLOP/s: 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, fp32 (non-packed) and fp64
PEAK_VALU_PACKED_FP32 = 157.3
METRIC = "candidate solves/s & valid paths/s, pruned vs exhaustive at recall>=99.9%"


# ------------------------------------------------------------------ algorithmic flop model
class _P:
    """Degree-tracking stand-in of a bivariate polynomial; counts the flops of
    the coefficient-phase arithmetic exactly as the kernel performs it."""
    flops = 0

    def __init__(self, d):
        self.d = d

    @staticmethod
    def ts(d):
        return (d + 1) * (d + 2) // 2

    def __mul__(self, o):
        _P.flops += 2 * _P.ts(self.d) * _P.ts(o.d)
        return _P(self.d + o.d)

    def __add__(self, o):
        d = max(self.d, o.d)
        _P.flops += 3 * _P.ts(d)
        return _P(d)

    __sub__ = __add__


def _vdot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _vcross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def coefficient_flops(ev: str) -> int:
    _P.flops = 0
    x1 = [_P(1)] * 3
    n = [_P(1)] * 3
    c = [_P(0)] * 3
    d0 = [x1[k] - c[k] for k in range(3)]
    d1 = [c[k] - x1[k] for k in range(3)]
    _vdot(_vcross(d0, c), n)
    if ev == "R":
        t = _vcross(n, c)
        _vdot(d0, n) * _vdot(d1, t) + _vdot(d0, t) * _vdot(d1, n)
    else:
        l, r = _vcross(d0, n)[0], _vcross(d1, n)[0]
        (_vdot(d1, d1) * (l * l)) + (_vdot(d0, d0) * (r * r))
    return _P.flops


def elimination_flops(ev: str) -> int:
    """2 x (fma + mul) count of the generated Bezout + Laplace code."""
    name = "r_interp" if ev == "R" else "t_interp"
    path = os.path.join(ROOT, "paper_2405_13409_amd", "csrc", "laplace_gen.inc")
    txt = open(path).read()
    body = txt.split(f"elim_{name}(")[1].split("\n}\n")[0]
    return 2 * (body.count("fma(") + body.count(" * "))


def isolation_fixed_flops(ev: str) -> int:
    """Derivative chain plus the sign evaluations at every piece end (the
    data-independent part of the recursive isolation of Sec. 5.2)."""
    D = 9 if ev == "R" else 12
    f = 0
    for d in range(1, D + 1):
        f += d                 # derivative coefficients
        f += (d + 1) * 2 * d   # Horner at d+1 piece ends (upper bound: all breakpoints present)
    return f


def per_instance_flops(ev: str) -> int:
    return coefficient_flops(ev) + elimination_flops(ev) + isolation_fixed_flops(ev)


# ------------------------------------------------------------------ bench
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--res", type=int, default=256, help="shading points per side")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(instances are independent; see the sharding notes in the design document).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2405_13409_amd import scenes, spoly

    spoly.load_library()
    prec = spoly.SPOLY_FP32_POLISH64 if args.precision == "fp32" else spoly.SPOLY_FP64
    ctx = spoly.Context(0)
    mesh = scenes.glints_large_mesh()
    light = scenes.GLINTS_LARGE_LIGHT
    dm = spoly.DeviceMesh(mesh.P, mesh.N, mesh.tri)
    dl = spoly.DevicePoints(light)
    events = [("R", 1.0, 1.0), ("T", 1.5, 1.0)]
    pts = {ev: spoly.DevicePoints(scenes.glints_large_points(ev, args.res)) for ev, _, _ in events}
    L = spoly.load_library()
    import ctypes

    # buffers sized from one untimed pass
    cap_c, cap_s = {}, {}
    for ev, e0, e1 in events:
        q0, q2, qt = ctx.cull_1bounce(dm, pts[ev], dl, e0, e1, 1e-3)
        cap_c[ev] = int(q0.numel() * 1.05) + 1024
        sols = ctx.solve_1bounce(dm, pts[ev], dl, q0, q2, qt, ev, e0, e1, prec)
        cap_s[ev] = int(len(sols) * 1.2) + 1024
        del q0, q2, qt
    buf = {}
    for ev, _, _ in events:
        buf[ev] = dict(q0=torch.empty(cap_c[ev], dtype=torch.int32, device="cuda"),
                       q2=torch.empty(cap_c[ev], dtype=torch.int32, device="cuda"),
                       qt=torch.empty(cap_c[ev], dtype=torch.int32, device="cuda"),
                       ccount=torch.zeros(1, dtype=torch.int64, device="cuda"),
                       out=torch.empty(cap_s[ev] * spoly.SOLUTION_DTYPE.itemsize, dtype=torch.uint8, device="cuda"),
                       scount=torch.zeros(1, dtype=torch.int64, device="cuda"))
    prm = spoly.default_params()
    stream = torch.cuda.current_stream()
    sptr = ctypes.c_void_p(stream.cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    solve_ms = {ev: [] for ev, _, _ in events}

    def step(record: bool):
        tot_inst, tot_sol = 0, 0
        for ev, e0, e1 in events:
            b = buf[ev]
            b["ccount"].zero_()
            b["scount"].zero_()
            st = L.spoly_cull_1bounce(ctx.h, ctypes.byref(dm.c), ctypes.byref(pts[ev].c), ctypes.byref(dl.c), e0, e1,
                                      1e-3, p(b["q0"]), p(b["q2"]), p(b["qt"]), cap_c[ev], p(b["ccount"]), sptr)
            assert st == 0
            nq = int(b["ccount"].item())
            assert nq <= cap_c[ev]
            e_a = torch.cuda.Event(enable_timing=True)
            e_b = torch.cuda.Event(enable_timing=True)
            e_a.record(stream)
            st = L.spoly_solve_1bounce(ctx.h, ctypes.byref(dm.c), ctypes.byref(pts[ev].c), ctypes.byref(dl.c),
                                       p(b["q0"]), p(b["q2"]), p(b["qt"]), nq, 1 if ev == "T" else 0, e0, e1, prec,
                                       ctypes.byref(prm), p(b["out"]), cap_s[ev], p(b["scount"]), None, None, sptr)
            assert st == 0
            e_b.record(stream)
            if record:
                solve_ms[ev].append((e_a, e_b, nq))
            tot_inst += nq
        torch.cuda.synchronize()
        for ev, _, _ in events:
            ns = int(buf[ev]["scount"].item())
            assert ns <= cap_s[ev]
            tot_sol += ns
        return tot_inst, tot_sol

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    inst = sols = 0
    for _ in range(args.steps):
        a, b = step(True)
        inst += a
        sols += b
        print(f"[bench] step done: {a} candidates, {b} valid paths", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = dt / args.steps * 1e3

    # dominant kernel: the R solve (k_onebounce<float/double, R>)
    rec = solve_ms["R"]
    avg_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in rec]))
    n_r = rec[0][2]
    fl = per_instance_flops("R") * n_r
    achieved = fl / (avg_ms * 1e-3) / 1e12
    t_rec = solve_ms["T"]
    avg_ms_t = float(np.mean([a.elapsed_time(b) for a, b, _ in t_rec]))

    out = {
        "metric": METRIC,
        "value": inst / dt,
        "unit": "candidate solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"glints: 128x128 heightfield (32768 tris), {args.res}x{args.res} points at z=+2 (R) and "
                        f"z=-2 (T, IOR 1.5), light (0,0,4); cone cull of all pairs + full solve",
            "precision": "fp32 bulk, fp64 polish" if args.precision == "fp32" else "fp64",
            "candidates_per_step": inst // args.steps,
            "valid_paths_per_step": sols // args.steps,
        },
        "valid_paths_per_s": sols / dt,
        "stage_ms": {"solve_R": avg_ms, "solve_T": avg_ms_t},
        "roofline": {
            "bound": "alu",
            "kernel": "k_onebounce<R>",
            "achieved": achieved,
            "peak": PEAK_VALU,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_VALU,
            "traffic": None,
            "flops_per_instance": per_instance_flops("R"),
            "peak_note": "fp32/fp64 vector FMA without packed fp32 (packed-fp32 peak 157.3)",
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, mesh, light)
    print(json.dumps(out), flush=True)
    ctx.close()


def cpu_baseline(args, mesh, light):
    """The FP64 oracle on the host cores over a bounded sample of the same
    workload: a seeded subset of the shading points, its own FP64 cone cull,
    then the solve of every kept candidate."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle
    from paper_2405_13409_amd import scenes

    oracle.build()
    cores = os.cpu_count() or 1
    rng = np.random.default_rng(12345)
    total_inst = 0.0
    total_t = 0.0
    n_pts = 16
    for ev, e0, e1 in (("R", 1.0, 1.0), ("T", 1.5, 1.0)):
        allp = scenes.glints_large_points(ev, args.res)
        t_budget = args.cpu_seconds / 2
        spent = 0.0
        while spent < t_budget:
            idx = rng.choice(len(allp), n_pts, replace=False)
            x0 = allp[idx]
            t0 = time.perf_counter()
            keep = oracle.cull_1bounce(mesh.P, mesh.N, mesh.tri, x0, light, e0, e1, 0.0)
            j0, j2, jt = np.nonzero(keep)
            oracle.solve_1bounce(mesh.P, mesh.N, mesh.tri, x0, light, j0, j2, jt, ev, e0, e1)
            dt = time.perf_counter() - t0
            spent += dt
            total_t += dt
            total_inst += len(jt)
    return {"value": total_inst / total_t, "unit": "candidate solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{int(total_inst)} candidates from random {n_pts}-point batches of the same workload "
                      f"(R and T, FP64 cull + solve, ~{args.cpu_seconds:.0f} s)"}


if __name__ == "__main__":
    main()
