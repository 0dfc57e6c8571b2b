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
METRIC = "candidate solves/s & valid paths/s, pruned vs exhaustive at recall>=99.9%"

PEAK_FP32 = 157.3   # TFLOP/s, published FP32 vector peak (packed FP32 instructions)
PEAK_VALU = 78.6    # TFLOP/s: 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, fp32 (non-packed) and fp64
PEAK_BF16 = 2500.0  # TFLOP/s, dense bf16 matrix cores
PEAK_HBM = 8000.0   # GB/s
# wave64 VALU instructions per second if every SIMD (16 lanes, 4 per CU) issues one every 4 cycles; the
# glints front kernel counts 13% more than this (profiles/valu_counters.md), so it is a scale, not a bound
VALU_ISSUE = 256 * 4 * 2.4e9 / 4

# Algorithmic operations per instance by stage (coefficients, elimination, root finding in v, path phase),
# from the oracle's op counter over seeded samples of each workload: profiles/algorithmic_flops.md, written
# by `python oracle/opcount.py`.
OPS = {
    "glints_R": (783, 1264, 440, 71),
    "glints_T": (1439, 7075, 894, 102),
    "caustic_TT": (368162, 936311, 9924, 127),
    "mirror_RR": (17860, 899708, 44109, 704),
}
PRUNER_FLOP = 2 * (42 * 128 + 2 * 128 * 128 + 128)   # multiply-adds of the four dense layers, per tuple

# HBM bytes of the reflection front kernel k_ob_front<float,R> on the glints workload, from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch), scaled by what the same counters read for a plain 256 MiB
# device copy.  Valid only for the one-vertex kernel sources they were taken on (sha256 prefix over
# ONE_VERTEX_SOURCES, the cull included: it sets the order of the candidates); otherwise traffic is null.
ONE_VERTEX_SOURCES = ("onebounce.hip", "spoly_dev.hpp", "laplace_gen.inc", "onebounce.hpp", "cull.hip")
TWO_VERTEX_SOURCES = ("twobounce.hip", "twobounce.hpp", "spoly_dev.hpp")
TRAFFIC_FRONT = {"sha": "1957ee0810a6953e", "candidates": 99118956, "fetch_kib": 682529.5, "write_kib": 1893897.6,
                 "fetch_scale": 262144.0 / 131083.5, "write_scale": 262144.0 / 262144.0}
# VALU wave-instructions (rocprofv3 --pmc SQ_INSTS_VALU) per launch of each one-vertex kernel on the glints
# workload, and per tuple of the two-vertex solve on the RR and TT legs, each group under the source check of
# its own kernels (profiles/valu_counters.md).
VALU_INSTS = {"sha": "1957ee0810a6953e",
              "k_ob_front_R": 2.917e9, "k_ob_back_R": 4.388e8, "k_ob_full_R": 3.702e7,
              "k_ob_coef_T": 6.219e8, "k_ob_iso_T": 1.691e8, "k_ob_back_T": 9.559e7}
VALU_INSTS_TT = {"sha": "3f62131393a90e82",
                 "k_tt_solve_RR_per_tuple": 7.352e11 / 9256723, "k_tt_solve_TT_per_tuple": 4.033e11 / 6477601}


def _kernel_sha(files=ONE_VERTEX_SOURCES) -> str:
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2405_13409_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_bytes(candidates: int):
    """HBM bytes per front launch for `candidates` instances, or None if the
    kernels changed since the counters were taken."""
    t = TRAFFIC_FRONT
    if _kernel_sha() != t["sha"]:
        return None
    per = (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0 / t["candidates"]
    return per * candidates


def valu_insts(kernel: str, instances: int | None = None):
    """VALU wave-instructions of one launch (per-instance figures scaled by
    `instances`), or None if the kernels changed since they were counted."""
    if kernel.startswith("k_tt_solve"):
        t = VALU_INSTS_TT
        if _kernel_sha(TWO_VERTEX_SOURCES) != t["sha"] or instances is None or kernel + "_per_tuple" not in t:
            return None
        return t[kernel + "_per_tuple"] * instances
    t = VALU_INSTS
    if _kernel_sha() != t["sha"]:
        return None
    return t.get(kernel)


def kernel_obj(name, flop, ms, peak, dtype, insts=None, **extra):
    """Roofline object of one kernel: algorithmic flops per launch / its duration."""
    ach = flop / (ms * 1e-3) / 1e12
    o = {"kernel": name, "dtype": dtype, "bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
         "frac": ach / peak, "ms": ms, "algorithmic_flop": flop}
    if insts is not None:
        o["valu_insts"] = insts
        o["valu_insts_per_s"] = insts / (ms * 1e-3)
        o["valu_issue_frac"] = insts / (ms * 1e-3) / VALU_ISSUE
    o.update(extra)
    return o


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
    ap.add_argument("--legs", default="glints,tail,rr,completeness,mixed,caustic",
                    help="comma list: glints (the headline line), tail (visibility + contribution of the headline "
                         "step's paths), rr (two reflections between two wavy mirrors), "
                         "completeness (two-vertex paths found at 10/100/1000/4095 pieces), "
                         "mixed (2M-instance persistent launch), "
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
    mesh = scenes.glints_large_mesh()
    light = scenes.GLINTS_LARGE_LIGHT
    events = [("R", 1.0, 1.0), ("T", 1.5, 1.0)]
    # one context per event, so that each keeps the kernel timings of its own solve
    ctxs = {ev: spoly.Context(0) for ev, _, _ in events}
    dm = spoly.DeviceMesh(mesh.P, mesh.N, mesh.tri)
    dl = spoly.DevicePoints(light)
    pts = {ev: spoly.DevicePoints(scenes.glints_large_points(ev, args.res)) for ev, _, _ in events}
    L = spoly.load_library()
    import ctypes

    # buffers sized from one untimed pass
    cap_c, cap_s = {}, {}
    for ev, e0, e1 in events:
        q0, q2, qt = ctxs[ev].cull_1bounce(dm, pts[ev], dl, e0, e1, 1e-3)
        cap_c[ev] = int(q0.numel() * 1.05) + 1024
        sols = ctxs[ev].solve_1bounce(dm, pts[ev], dl, q0, q2, qt, ev, e0, e1, prec)
        cap_s[ev] = int(len(sols) * 1.2) + 1024
        del q0, q2, qt
    buf = {}
    # candidate counts of both events, then solution counts: one fill per step, one read of each pair
    counts = torch.zeros(2 * len(events), dtype=torch.int64, device="cuda")
    for i, (ev, _, _) in enumerate(events):
        buf[ev] = dict(q0=torch.empty(cap_c[ev], dtype=torch.int32, device="cuda"),
                       q2=torch.empty(cap_c[ev], dtype=torch.int32, device="cuda"),
                       qt=torch.empty(cap_c[ev], dtype=torch.int32, device="cuda"),
                       ccount=counts[i:i + 1],
                       out=torch.empty(cap_s[ev] * spoly.SOLUTION_DTYPE.itemsize, dtype=torch.uint8, device="cuda"),
                       scount=counts[len(events) + i:len(events) + i + 1])
    prm = spoly.default_params()
    prm.flags = spoly.SPOLY_FLAG_STAGE_TIMES
    stream = torch.cuda.current_stream()
    sptr = ctypes.c_void_p(stream.cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    solve_ms = {ev: [] for ev, _, _ in events}
    stage_ms = {ev: [] for ev, _, _ in events}
    n_cand = {}

    def step(record: bool):
        # both culls, one read of their counts (the solve takes its count from the host), both solves
        tot_inst, tot_sol = 0, 0
        counts.zero_()
        for ev, e0, e1 in events:
            b = buf[ev]
            st = L.spoly_cull_1bounce(ctxs[ev].h, ctypes.byref(dm.c), ctypes.byref(pts[ev].c), ctypes.byref(dl.c),
                                      e0, e1, 1e-3, p(b["q0"]), p(b["q2"]), p(b["qt"]), cap_c[ev], p(b["ccount"]),
                                      sptr)
            assert st == 0
        nqs = counts[: len(events)].tolist()
        for i, (ev, e0, e1) in enumerate(events):
            b = buf[ev]
            h = ctxs[ev].h
            nq = int(nqs[i])
            assert nq <= cap_c[ev]
            e_a = torch.cuda.Event(enable_timing=True)
            e_b = torch.cuda.Event(enable_timing=True)
            e_a.record(stream)
            st = L.spoly_solve_1bounce(h, ctypes.byref(dm.c), ctypes.byref(pts[ev].c), ctypes.byref(dl.c),
                                       p(b["q0"]), p(b["q2"]), p(b["qt"]), nq, 1 if ev == "T" else 0, e0, e1, prec,
                                       ctypes.byref(prm), p(b["out"]), cap_s[ev], p(b["scount"]), None, None, sptr)
            assert st == 0
            e_b.record(stream)
            if record:
                solve_ms[ev].append((e_a, e_b))
            n_cand[ev] = nq
            tot_inst += nq
        nss = counts[len(events):].tolist()
        for i, (ev, _, _) in enumerate(events):
            ns = int(nss[i])
            assert ns <= cap_s[ev]
            tot_sol += ns
            if record:
                stage_ms[ev].append(ctxs[ev].stage_times())
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

    # per-kernel times (HIP events recorded around each kernel on the launch stream)
    st_r = np.mean(np.array(stage_ms["R"]), axis=0)   # front, back, full list
    st_t = np.mean(np.array(stage_ms["T"]), axis=0)   # coefficients, isolation, back, full list
    call_r = float(np.mean([a.elapsed_time(b) for a, b in solve_ms["R"]]))
    call_t = float(np.mean([a.elapsed_time(b) for a, b in solve_ms["T"]]))
    nr, nt_ = n_cand["R"], n_cand["T"]
    oR, oT = OPS["glints_R"], OPS["glints_T"]
    fp = "f32" if args.precision == "fp32" else "f64"
    front = kernel_obj("k_ob_front<float,R>" if fp == "f32" else "k_ob_front<double,R>",
                       (oR[0] + oR[1] + oR[2]) * nr, float(st_r[0]), PEAK_FP32 if fp == "f32" else PEAK_VALU, fp,
                       valu_insts("k_ob_front_R"),
                       traffic=traffic_bytes(nr), instances=nr,
                       flop_per_instance=oR[0] + oR[1] + oR[2],
                       peak_nonpacked=PEAK_VALU,
                       frac_nonpacked=(oR[0] + oR[1] + oR[2]) * nr / (float(st_r[0]) * 1e-3) / 1e12 / PEAK_VALU,
                       peak_note="FP32 peak counts packed-FP32 FMAs, which this build does not emit; "
                                 "frac_nonpacked is against the 78.6 TFLOP/s non-packed vector rate")
    kernels = [
        front,
        kernel_obj("k_ob_back<R>", oR[3] * nr, float(st_r[1]), PEAK_VALU, "f64", valu_insts("k_ob_back_R"),
                   note="path phase of the candidates with roots (u solve, FP64 polish, validation)"),
        kernel_obj("k_ob_full<R>", oR[3] * nr, float(st_r[2]), PEAK_VALU, "f64", valu_insts("k_ob_full_R"),
                   note="FP64 re-solve of the handed-off candidates; flops counted as the path phase only"),
        kernel_obj("k_ob_coef<double,T>", (oT[0] + oT[1]) * nt_, float(st_t[0]), PEAK_VALU, "f64",
                   valu_insts("k_ob_coef_T")),
        kernel_obj("k_ob_iso<double,T>", oT[2] * nt_, float(st_t[1]), PEAK_VALU, "f64", valu_insts("k_ob_iso_T")),
        kernel_obj("k_ob_back<T>", oT[3] * nt_, float(st_t[2]), PEAK_VALU, "f64", valu_insts("k_ob_back_T")),
    ]
    hbm = traffic_bytes(nr)
    roofline = {"bound": "alu", "kernel": front["kernel"], "achieved": front["achieved"], "peak": front["peak"],
                "unit": "TFLOP/s", "frac": front["frac"], "traffic": hbm,
                "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "hbm_GBps": (hbm / (float(st_r[0]) * 1e-3) / 1e9) if hbm else None,
                "flop_per_instance": front["flop_per_instance"], "instances": nr, "ms": front["ms"],
                "peak_nonpacked": PEAK_VALU, "frac_nonpacked": front["frac_nonpacked"],
                "valu_issue_frac": front.get("valu_issue_frac"),
                "flop_source": "oracle op counter (profiles/algorithmic_flops.md): coefficients + elimination + "
                               "isolation of a reflection candidate"}

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
        "dtype": fp,
        "data": "synthetic",
        "config": {
            "workload": f"glints: 128x128 heightfield (32768 tris), {args.res}x{args.res} points at z=+2 (R) and "
                        f"z=-2 (T, IOR 1.5), light (0,0,4); cone cull of all pairs + full solve",
            "precision": "fp32 bulk, fp64 polish" if args.precision == "fp32" else "fp64",
            "candidates_per_step": inst // args.steps,
            "valid_paths_per_step": sols // args.steps,
        },
        "valid_paths_per_s": sols / dt,
        "stage_ms": {"solve_R": call_r, "solve_T": call_t, "kernels_R": [float(x) for x in st_r],
                     "kernels_T": [float(x) for x in st_t]},
        "roofline": roofline,
        "kernels": kernels,
    }
    tail_sample = None
    if "tail" in legs:
        out["path_tail"], tail_sample = tail_leg(ctxs["R"], spoly, dm, pts, dl, buf)
    for ev in ctxs:
        ctxs[ev].close()
    ctx = spoly.Context(0)
    if "rr" in legs:
        out["two_reflections"] = rr_leg(args, ctx)
    if "completeness" in legs:
        out["solver_completeness"] = completeness_leg(args, ctx)
    if "mixed" in legs:
        out["mixed"] = mixed_leg(args, ctx)
    if "caustic" in legs:
        out["pruned_vs_exhaustive"] = caustic_leg(args, ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, mesh, light, ctx)
        if tail_sample is not None:
            out["cpu_baseline"]["path_tail"] = cpu_tail_baseline(mesh, light, tail_sample)
    print(json.dumps(out), flush=True)
    ctx.close()


TAIL_BYTES = 56 + 8 + 4 + 8 + 8  # per path: record, two query ids, mask, contribution, image add
# HBM bytes per reflection path of k_tail<1> on the glints workload (FETCH_SIZE x2.0 + WRITE_SIZE x1.0,
# KiB per dispatch over 8,824,972 paths; profiles/tail_glints_hbm_counters.md), under a check of the
# tail's own sources
TRAFFIC_TAIL = {"sha": "e96dd6205077e27e", "paths": 8824972, "fetch_kib": 412944.4, "write_kib": 185462.75}


def tail_traffic(paths: int):
    t = TRAFFIC_TAIL
    if _kernel_sha(("tail.hip", "tail.hpp")) != t["sha"]:
        return None
    return (t["fetch_kib"] * 2.0 + t["write_kib"]) * 1024.0 / t["paths"] * paths


def tail_leg(ctx, spoly, dm, pts, dl, buf, reps: int = 5):
    """Visibility (device BVH) and contribution of every valid path of the
    last headline step, R and T, straight from the solve's output buffer and
    device count; the receivers' image accumulated with the z-facing plane
    weight.  Returns the leg's record and a host sample for the oracle."""
    import torch

    t0 = time.perf_counter()
    bvh = spoly.Bvh(ctx, dm)
    build_ms = (time.perf_counter() - t0) * 1e3
    res = {"bvh_build_ms": build_ms, "bvh_triangles": dm.n_tris}
    stream = torch.cuda.current_stream()
    sample = {}
    tot_paths, tot_ms = 0, 0.0
    for ev, eta in (("R", (1.0, 1.0)), ("T", (1.5, 1.0))):
        b = buf[ev]
        n = int(b["scount"].item())
        mask = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        contrib = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
        img = torch.zeros(pts[ev].n, dtype=torch.float64, device="cuda")
        prm = spoly.tail_default_params(rcv_normal=(0.0, 0.0, 1.0))

        def run():
            ctx.path_tail(dm, bvh, ev, eta, pts[ev], dl, b["q0"], b["q2"], b["out"], n_sols=n, sol_count=b["scount"],
                          params=prm, mask=mask, contrib=contrib, image=img)

        run()
        ms = []
        for _ in range(reps):
            img.zero_()
            e_a = torch.cuda.Event(enable_timing=True)
            e_b = torch.cuda.Event(enable_timing=True)
            e_a.record(stream)
            run()
            e_b.record(stream)
            e_b.synchronize()
            ms.append(e_a.elapsed_time(e_b))
        m = float(np.mean(ms))
        mk = mask[:n].cpu().numpy()
        gbps = n * TAIL_BYTES / (m * 1e-3) / 1e9
        res[ev] = {"paths": n, "ms": m, "paths_per_s": n / (m * 1e-3), "blocked_fraction": float((mk != 0).mean()),
                   "singular": int(((mk & spoly.TAIL_SINGULAR) != 0).sum()),
                   "image_total": float(img.sum().item()),
                   "kernel": f"k_tail<1> ({ev})",
                   "roofline": {"bound": "hbm", "achieved": gbps, "peak": PEAK_HBM, "unit": "GB/s",
                                "frac": gbps / PEAK_HBM, "algorithmic_bytes_per_path": TAIL_BYTES,
                                "traffic": tail_traffic(n) if ev == "R" else None,
                                "note": "the BVH, mesh and endpoints stay in L2/MALL; the kernel is bound by "
                                        "dependent node loads of the traversal, not by HBM"}}
        tot_paths += n
        tot_ms += m
        k = min(n, 600)
        recs = b["out"][: k * spoly.SOLUTION_DTYPE.itemsize].cpu().numpy().view(spoly.SOLUTION_DTYPE)
        q = recs["query"]
        sample[ev] = dict(recs=recs, x0=pts[ev], q0=b["q0"][: int(q.max()) + 1].cpu().numpy() if k else None,
                          q2=b["q2"][: int(q.max()) + 1].cpu().numpy() if k else None, eta=eta,
                          mask=mk[:k], contrib=contrib[:k].cpu().numpy())
    res["paths_per_s"] = tot_paths / (tot_ms * 1e-3)
    res["workload"] = "every valid path of one headline step (R and T lists as the solve wrote them)"
    bvh.close()
    return res, sample


def cpu_tail_baseline(mesh, light, sample):
    """The tail oracle (every segment against every triangle; contribution by
    differences of a forward trace) on one core over the first paths of each
    list, and the GPU's agreement with it on those paths."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle

    threads = oracle.set_threads(1)
    out, n_all, t_all = {}, 0, 0.0
    for ev, s in sample.items():
        recs = s["recs"]
        if len(recs) == 0:
            continue
        x0 = np.column_stack([c.cpu().numpy() for c in s["x0"].cols])
        q = recs["query"]
        t0 = time.perf_counter()
        ot = oracle.tail(mesh.P, mesh.N, mesh.tri, x0, light, s["q0"][q], s["q2"][q], recs["tri"][:, :1],
                         recs["u"][:, :1], recs["v"][:, :1], ev, s["eta"])
        dt = time.perf_counter() - t0
        n_all += len(recs)
        t_all += dt
        ok = ot["margin"] > 1e-9
        st = ok & (ot["E_change"] < 1e-7) & (ot["E"] > 0)
        rel = np.abs(s["contrib"][st] - ot["E"][st]) / ot["E"][st]
        out[ev] = {"paths": int(len(recs)), "mask_compared": int(ok.sum()),
                   "mask_mismatches": int(((s["mask"][ok] & 3) != ot["mask"][ok]).sum()),
                   "contrib_compared": int(st.sum()), "contrib_max_rel_err": float(rel.max()) if len(rel) else None}
    oracle.set_threads(threads)
    return {"value": n_all / t_all if t_all else None, "unit": "paths/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_all} paths of the headline step's R and T lists, brute-force visibility over "
                      f"{mesh.nt} triangles per segment", "gpu_agreement": out}


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

    cand = {"workgroups_per_cu": (1, 2, 4, 8), "r_tile": (256, 1024), "order": (0, 2)}
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


def rr_leg(args, ctx):
    """Two reflections (RR, Sec. 4.5) between two wavy mirrors facing each other
    across a gap: every cone-culled (receiver, T1, T2, light) tuple of a 24x24
    receiver grid in the gap, solved in one launch (FP64, 100 pieces x 10
    bisection steps)."""
    import torch
    from paper_2405_13409_amd import scenes, spoly

    mesh = scenes.mirror_gap()
    rec = scenes.points_grid(24, -0.9, 0.9, 0.5)
    dm = spoly.DeviceMesh(mesh.P, mesh.N, mesh.tri)
    d0, dl = spoly.DevicePoints(rec), spoly.DevicePoints(scenes.MIRROR_GAP_LIGHT)
    eta = (1.0, 1.0, 1.0)
    q0, q3, qt = ctx.cull_2bounce(dm, d0, dl, eta, 1e-3)
    n = int(q0.numel())
    first = ctx.solve_2bounce(dm, d0, dl, q0, q3, qt, eta, chain="RR")
    cap = len(first) + 4096
    out = torch.empty(cap * spoly.SOLUTION_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    ms = []
    for _ in range(3):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        ctx.solve_2bounce(dm, d0, dl, q0, q3, qt, eta, chain="RR", out=out, out_count=cnt, sync=False)
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    paths = int(cnt.item())
    med = float(np.median(ms))
    ops = OPS["mirror_RR"]
    return {"workload": f"{len(rec)} receivers (24x24 grid on [-0.9,0.9]^2 at z=0.5) between two 16x16 wavy "
                        f"heightfields (1024 tris) facing each other across a gap of 1, light (0.15,-0.1,0.5); "
                        f"RR chain, {n} cone-culled tuples",
            "tuples": n, "ms": med, "tuples_per_s": n / med * 1e3, "valid_paths": paths,
            "valid_paths_per_s": paths / med * 1e3, "us_per_tuple": med * 1e3 / n,
            "paper_context": "Table 3, RR (bisection solver, RTX 4080, its own two-dragon scene): 4.936 us per "
                             "triangle pair",
            "roofline": kernel_obj("k_tt_solve (RR)", sum(ops) * n, med, PEAK_VALU, "f64",
                                   valu_insts("k_tt_solve_RR", n), flop_per_instance=sum(ops))}


def completeness_leg(args, ctx):
    """Solver completeness (Sec. 6, validation of the bisection solver): the
    same two-vertex tuples solved with 10, 100, 1000 and 4095 pieces of the
    sign scan (10 bisection steps each); the paths each resolution finds
    against the finest one, and the time each takes."""
    import torch
    from paper_2405_13409_amd import scenes, spoly

    sets = []
    sph = scenes.caustic_sphere()
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    rec, ex, en = scenes.caustic_traced(8, 0.35)
    Q = [np.column_stack([np.full(len(t), k), t]) for k, t in
         enumerate(scenes.tuples_near(sph, rec[k], x3[0], ex[k], en[k], 0.1) for k in range(len(rec)))]
    Q = np.concatenate(Q)
    sets.append(("caustic TT: 64 receivers where traced caustic paths land, tuples within 0.1 of the path",
                 "TT", sph, rec, x3, Q[:, 0], np.zeros(len(Q)), Q[:, 1:], (1.0, 1.5, 1.0)))
    gap = scenes.mirror_gap()
    rr = scenes.points_grid(4, -0.6, 0.6, 0.5)
    dm = spoly.DeviceMesh(gap.P, gap.N, gap.tri)
    q0, q3, qt = ctx.cull_2bounce(dm, spoly.DevicePoints(rr), spoly.DevicePoints(scenes.MIRROR_GAP_LIGHT),
                                  (1.0, 1.0, 1.0), 1e-3)
    sets.append(("mirror gap RR: 16 receivers (4x4 grid), every cone-culled tuple", "RR", gap, rr,
                 scenes.MIRROR_GAP_LIGHT, q0.cpu().numpy(), q3.cpu().numpy(), qt.cpu().numpy().reshape(-1, 2),
                 (1.0, 1.0, 1.0)))
    out = {}
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()  # noqa: E731
    for name, chain, mesh, x0, x3_, j0, j3, tt, eta in sets:
        dm = spoly.DeviceMesh(mesh.P, mesh.N, mesh.tri)
        d0, d3 = spoly.DevicePoints(x0), spoly.DevicePoints(x3_)
        a0, a3, at = dev(j0), dev(j3), dev(tt)
        res, ref = {}, None
        for pieces in (4095, 1000, 100, 10):
            prm = spoly.tt_default_params()
            prm.pieces = pieces
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            s = ctx.solve_2bounce(dm, d0, d3, a0, a3, at, eta, params=prm, chain=chain)
            b.record()
            b.synchronize()
            key = {(int(r["query"]), round(float(r["u"][0]), 7), round(float(r["v"][0]), 7)) for r in s}
            if ref is None:
                ref = key
            res[str(pieces)] = {"paths": len(key), "missed_vs_4095": len(ref - key),
                                "not_in_4095": len(key - ref), "ms": a.elapsed_time(b)}
        out[chain] = {"workload": name, "tuples": len(j0), "by_pieces": res}
    return out


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
    ops = OPS["caustic_TT"]
    r["kernels"] = [
        kernel_obj("k_tt_solve (TT, exhaustive)", sum(ops) * r["n_tuples"], r["ms_exhaustive"], PEAK_VALU, "f64",
                   valu_insts("k_tt_solve_TT", r["n_tuples"]), flop_per_instance=sum(ops)),
        dict(kernel_obj("pruner scoring (feature gather + 4 dense layers)", PRUNER_FLOP * r["n_tuples"],
                        r["ms_score"], PEAK_BF16, "bf16"), bound="mfma", flop_per_instance=PRUNER_FLOP),
    ]
    return r


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _errors_vs_oracle(gpu, orc, diag, nq, tau=1e-6, band=1e-4):
    """Per-result error of the GPU solutions against the FP64 oracle's on the
    same candidates: queries whose solution count differs (ambiguous ones
    excluded: a root pair or tangency below the FP32 path's resolution, a
    solution in the edge band or with a residual near tau), and max / p99 of
    |du|, |dv| over the matched solutions."""
    amb = (diag["tangency"] < 1e-5) | (diag["min_gap"] < 1e-4)
    amb[orc["query"][(orc["edge"] < band) | ((orc["residual"] > tau / 10) & (orc["residual"] < 10 * tau))]] = True
    amb[gpu["query"][(gpu["edge"] < band) | ((gpu["residual"] > tau / 10) & (gpu["residual"] < 10 * tau))]] = True
    g = gpu[~amb[gpu["query"]]]
    o = orc[~amb[orc["query"]]]
    g = g[np.lexsort((g["u"][:, 0], g["v"][:, 0], g["query"]))]
    o = o[np.lexsort((o["u1"], o["v1"], o["query"]))]
    gq, oq = np.bincount(g["query"], minlength=nq), np.bincount(o["query"], minlength=nq)
    bad = gq != oq
    ok_g = ~bad[g["query"]]
    ok_o = ~bad[o["query"]]
    du = np.abs(g["u"][ok_g, 0] - o["u1"][ok_o])
    dv = np.abs(g["v"][ok_g, 0] - o["v1"][ok_o])
    return {"compared": int(ok_o.sum()), "count_mismatch_queries": int(bad.sum()),
            "ambiguous_queries": int(amb.sum()), "ambiguous_fraction": float(amb.mean()) if nq else 0.0,
            "max_abs_du": float(du.max(initial=0.0)), "max_abs_dv": float(dv.max(initial=0.0)),
            "p99_abs_du": float(np.percentile(du, 99)) if len(du) else 0.0,
            "p99_abs_dv": float(np.percentile(dv, 99)) if len(dv) else 0.0}


def cpu_baseline(args, mesh, light, ctx):
    """The FP64 oracle on the host cores over a bounded sample of the same
    workload: a seeded subset of the shading points, its own FP64 cone cull,
    then the solve of every kept candidate; also on one core, and the GPU's
    error against it on the same candidates."""
    import torch

    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle
    from paper_2405_13409_amd import scenes, spoly

    oracle.build()
    threads = oracle.set_threads(0)
    rng = np.random.default_rng(12345)
    n_pts = 16
    prec = spoly.SPOLY_FP32_POLISH64 if args.precision == "fp32" else spoly.SPOLY_FP64
    dm = spoly.DeviceMesh(mesh.P, mesh.N, mesh.tri)
    dl = spoly.DevicePoints(light)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()  # noqa: E731

    def run(seconds):
        inst, t_all, errs = 0, 0.0, {}
        for ev, e0, e1 in (("R", 1.0, 1.0), ("T", 1.5, 1.0)):
            allp = scenes.glints_large_points(ev, args.res)
            spent = 0.0
            while spent < seconds / 2:
                x0 = allp[rng.choice(len(allp), n_pts, replace=False)]
                t0 = time.perf_counter()
                keep = oracle.cull_1bounce(mesh.P, mesh.N, mesh.tri, x0, light, e0, e1, 0.0)
                j0, j2, jt = np.nonzero(keep)
                orc, diag = oracle.solve_1bounce(mesh.P, mesh.N, mesh.tri, x0, light, j0, j2, jt, ev, e0, e1)
                dt = time.perf_counter() - t0
                spent += dt
                t_all += dt
                inst += len(jt)
                if ev not in errs or errs[ev]["compared"] < 20000:
                    g = ctx.solve_1bounce(dm, spoly.DevicePoints(x0), dl, dev(j0), dev(j2), dev(jt), ev, e0, e1,
                                          prec)
                    e = _errors_vs_oracle(g, orc, diag, len(jt))
                    if ev in errs:
                        a = errs[ev]
                        for k in ("compared", "count_mismatch_queries", "ambiguous_queries"):
                            a[k] += e[k]
                        for k in ("max_abs_du", "max_abs_dv", "p99_abs_du", "p99_abs_dv"):
                            a[k] = max(a[k], e[k])
                    else:
                        errs[ev] = e
        return inst, t_all, errs

    inst, t_all, errs = run(args.cpu_seconds)
    oracle.set_threads(1)
    inst1, t1, _ = run(max(2.0, args.cpu_seconds / 4))
    oracle.set_threads(threads)
    return {"value": inst / t_all, "unit": "candidate solves/s", "cores": threads, "kind": "oracle",
            "cpu_model": _cpu_model(), "single_core_value": inst1 / t1,
            "sample": f"{int(inst)} candidates from random {n_pts}-point batches of the same workload "
                      f"(R and T, FP64 cull + solve, ~{args.cpu_seconds:.0f} s on {threads} threads; "
                      f"{int(inst1)} more on one thread)",
            "gpu_error_vs_oracle": {"precision": "fp32 bulk, fp64 polish" if args.precision == "fp32" else "fp64",
                                    **{ev: errs[ev] for ev in errs}}}


if __name__ == "__main__":
    main()
