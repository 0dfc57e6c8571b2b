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
PEAK_HBM = 8000.0   # GB/s

# HBM bytes of one reflection solve (k_ob_front<float,R> + k_ob_back<R> + k_ob_full<R>) on the glints
# workload, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch), scaled by what the same
# counters read for a plain 256 MiB device copy (FETCH x2.0, WRITE x1.0).  Valid only for the kernel
# sources they were taken on (sha256 prefix over the files in _KERNEL_SOURCES, the cull included: it sets
# the order of the candidates); otherwise traffic is null.
TRAFFIC_R = {"sha": "2e33cac3b84d0211", "candidates": 99118956,
             "fetch_kib": 680274.5 + 658461.1 + 34517.1, "write_kib": 1897214.1 + 491000.9 + 41.8,
             "fetch_scale": 262144.0 / 131084.5, "write_scale": 262144.0 / 262144.0}
_KERNEL_SOURCES = ("onebounce.hip", "spoly_dev.hpp", "laplace_gen.inc", "onebounce.hpp", "cull.hip")


def _kernel_sha() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in _KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2405_13409_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_bytes(candidates: int):
    """HBM bytes per reflection-solve launch for `candidates` instances, or None
    if the kernels changed since the counters were taken."""
    t = TRAFFIC_R
    if _kernel_sha() != t["sha"]:
        return None
    per = (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0 / t["candidates"]
    return per * candidates
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
    ap.add_argument("--legs", default="glints,mixed,caustic",
                    help="comma list: glints (the headline line), mixed (2M-instance persistent launch), "
                         "caustic (learned pruner against the exhaustive two-vertex solve)")
    ap.add_argument("--mixed-total", type=int, default=2_000_000)
    ap.add_argument("--caustic-stride", type=int, default=1, help="every k-th receiver of the 64x64 grid")
    ap.add_argument("--pruner", default=None, help="trained pruner .npz (default: the packaged weights)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy 5 times (the reference kernel for scaling "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    legs = set(args.legs.split(","))
    if args.copy_calibration:
        copy_calibration()
        return
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

    # dominant kernel: the reflection solve (front + back + full-list kernels of one spoly_solve_1bounce call)
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
            "kernel": "reflection solve: k_ob_front<float,R> + k_ob_back<R> + k_ob_full<R>",
            "achieved": achieved,
            "peak": PEAK_VALU,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_VALU,
            "traffic": traffic_bytes(n_r),
            "traffic_unit": "bytes per launch (HBM, FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "hbm_GBps": (traffic_bytes(n_r) / (avg_ms * 1e-3) / 1e9) if traffic_bytes(n_r) else None,
            "flops_per_instance": per_instance_flops("R"),
            "peak_note": "fp32/fp64 vector FMA without packed fp32 (packed-fp32 peak 157.3)",
        },
    }
    if "mixed" in legs:
        out["mixed"] = mixed_leg(args, ctx)
    if "caustic" in legs:
        out["pruned_vs_exhaustive"] = caustic_leg(args, ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, mesh, light)
    print(json.dumps(out), flush=True)
    ctx.close()


def copy_calibration(nbytes: int = 256 << 20, reps: int = 5):
    """A plain copy of known size: each launch reads and writes nbytes."""
    import torch

    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}), flush=True)


def mixed_leg(args, ctx):
    """2M instances, 70% drawn from the 32768 one-vertex reflection instances of
    the 16x16 heightfield scene and 30% from the canonical cone-culled TT
    tuples of the 64x64-receiver caustic scene, in one persistent launch
    captured in a graph, with the autotuned shape.  FP32 bulk, FP64 polish."""
    import torch
    from paper_2405_13409_amd import autotune, caustic, scenes, spoly

    w = scenes.glints_small()
    m1 = spoly.DeviceMesh(w.mesh.P, w.mesh.N, w.mesh.tri)
    p1 = (spoly.DevicePoints(w.x0), spoly.DevicePoints(w.x2))
    sph = scenes.caustic_sphere()
    m2 = spoly.DeviceMesh(sph.P, sph.N, sph.tri)
    r2 = spoly.DevicePoints(scenes.caustic_receivers())
    l2 = spoly.DevicePoints(scenes.CAUSTIC_LIGHT_OUTSIDE)
    T = caustic.cull_sorted(ctx, m2, r2, l2)
    i1, i2 = scenes.mixed_draw(len(w.q_tri), T.n, args.mixed_total, 0.7, 4)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()  # noqa: E731
    q1 = (dev(w.q_x0[i1]), dev(w.q_x2[i1]), dev(w.q_tri[i1]))
    Q2 = T.take(torch.from_numpy(i2).cuda())
    n_tt_list = T.n
    del T
    cap = 1 << 20
    out = torch.empty(cap * spoly.SOLUTION_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    queue = torch.zeros(1, dtype=torch.int64, device="cuda")
    prec = spoly.SPOLY_FP32_POLISH64

    def launch(shape):
        cnt.zero_()
        queue.zero_()
        ctx.solve_mixed(m1, *p1, *q1, "R", 1.0, 1.0, m2, r2, l2, Q2.q0, Q2.q3, Q2.qt, precision=prec, shape=shape,
                        out=out, out_count=cnt, queue=queue, sync=False)

    cand = {"workgroups_per_cu": (1, 2, 4), "r_tile": (256, 1024), "order": (0, 2)}
    key = autotune.signature(len(i1), len(i2), "R", prec)
    best, timings, cached = autotune.tune(launch, key, reps=1, candidates=cand)
    print(f"[bench] mixed autotune best {best.workgroups_per_cu}/{best.r_tile}/{best.order} "
          f"(cached={cached})", file=sys.stderr, flush=True)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        launch(best)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        launch(best)
    ms, counts = [], []
    for _ in range(3):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        g.replay()
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
        counts.append(int(cnt.item()))
    assert counts[0] <= cap and len(set(counts)) == 1, counts
    med = float(np.median(ms))
    return {"workload": f"{len(i1)} one-vertex R (16x16 heightfield, 64 points) + {len(i2)} TT tuples drawn from "
                        f"{n_tt_list} culled tuples of the 64x64 caustic grid, seed 4",
            "instances": len(i1) + len(i2), "ms": med, "instances_per_s": (len(i1) + len(i2)) / med * 1e3,
            "valid_paths": counts[0], "valid_paths_per_s": counts[0] / med * 1e3,
            "shape": {"workgroups_per_cu": best.workgroups_per_cu, "r_tile": best.r_tile, "order": best.order},
            "autotune_ms": timings, "graph": True, "precision": "fp32 bulk, fp64 polish (TT fp64)"}


def caustic_leg(args, ctx):
    """Learned pruner against the exhaustive two-vertex solve on a subset of
    the 64x64 receiver grid (every --caustic-stride-th receiver)."""
    from paper_2405_13409_amd import caustic, scenes, spoly, train_pruner

    path = args.pruner or train_pruner.DEFAULT_OUT
    if not os.path.exists(path):
        return {"skipped": f"no trained pruner at {os.path.relpath(path, ROOT)}"}
    net = train_pruner.load(path)
    sph = scenes.caustic_sphere()
    dm = spoly.DeviceMesh(sph.P, sph.N, sph.tri)
    rec = scenes.caustic_receivers()[:: args.caustic_stride]
    d0 = spoly.DevicePoints(rec)
    dl = spoly.DevicePoints(scenes.CAUSTIC_LIGHT_OUTSIDE)
    T = caustic.cull_sorted(ctx, dm, d0, dl)
    r = caustic.prune_vs_exhaustive(ctx, dm, d0, dl, T, net, reps=3, exhaustive_reps=1).as_dict()
    r["exhaustive_solves_per_s"] = r["n_tuples"] / r["ms_exhaustive"] * 1e3
    r["pruned_solves_per_s"] = r["n_tuples"] / r["ms_pruned"] * 1e3
    r["exhaustive_paths_per_s"] = r["paths_exhaustive"] / r["ms_exhaustive"] * 1e3
    r["pruned_paths_per_s"] = r["paths_pruned"] / r["ms_pruned"] * 1e3
    r["workload"] = (f"{len(rec)} receivers (64x64 grid on [-2,2]^2 at z=-1, stride {args.caustic_stride}), "
                     f"icosphere 1280 tris IOR 1.5, light (0.1,0.05,1.5); TT chain")
    r["threshold"] = net.threshold
    r["train"] = train_pruner.load_meta(path)
    return r


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
