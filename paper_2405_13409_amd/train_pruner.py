"""Train the learned two-vertex tuple pruner on the caustic scene.

    python -m paper_2405_13409_amd.train_pruner --eval --out paper_2405_13409_amd/weights/caustic_pruner.npz

Training data: receivers x0 ~ U([-2,2]^2) at z = -1 (seeded), the light
outside the sphere.  Every cone-culled tuple of every receiver is solved
exhaustively on the GPU; all positive tuples (at least one admissible path) are
kept, and negatives are subsampled uniformly so that the set holds about
`--examples` tuples.  Receivers with index = 0 mod 10 form the validation
split, on which the score threshold is calibrated for the target recall.  The
test set is the fixed 64 x 64 receiver grid, scored by `--eval`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import caustic, scenes, spoly
from . import pruner as pr

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "weights", "caustic_pruner.npz")


def log(msg: str) -> None:
    print(f"[train] {msg}", flush=True)


def label_receivers(ctx, dm, dl, receivers: np.ndarray, n_examples: int, seed: int, chunk: int = 128):
    """Exhaustively label the culled tuples of every receiver; keep all
    positives and a uniform subsample of negatives.  Returns the device
    Tuples (q_x0 indexes `receivers`), the total number of tuples labelled,
    the number of positives and the solver seconds."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    parts = []
    n_seen = n_pos = 0
    p_neg = None
    t_solve = 0.0
    for s in range(0, len(receivers), chunk):
        e = min(len(receivers), s + chunk)
        d0 = spoly.DevicePoints(receivers[s:e])
        T = caustic.cull_sorted(ctx, dm, d0, dl)
        lab, _, dt = pr.exhaustive_labels(ctx, dm, d0, dl, T, caustic.ETA, chunk=1 << 21)
        t_solve += dt
        if p_neg is None:
            est_total = T.n * (len(receivers) / (e - s))
            p_neg = min(1.0, n_examples / max(est_total, 1.0))
        keep = (lab > 0.5) | (torch.rand(T.n, generator=g, device="cuda") < p_neg)
        idx = torch.nonzero(keep).squeeze(1)
        K = T.take(idx)
        K.q0 = (K.q0 + s).contiguous()
        K.labels = lab[idx].contiguous()
        parts.append(K)
        n_seen += T.n
        n_pos += int(lab.sum().item())
        log(f"receivers {e}/{len(receivers)}: {n_seen} tuples labelled, {n_pos} positive, {dt:.2f} s solve")
        del d0, T, lab
    cat = lambda f: torch.cat([getattr(p, f) for p in parts])  # noqa: E731
    return pr.Tuples(cat("q0"), cat("q3"), cat("qt"), cat("labels")), n_seen, n_pos, t_solve


def split_by_receiver(T: pr.Tuples, every: int = 10):
    val = (T.q0 % every) == 0
    return T.take(torch.nonzero(~val).squeeze(1)), T.take(torch.nonzero(val).squeeze(1))


def evaluate(ctx, dm, dl, net: pr.Pruner, receivers: np.ndarray, chunk: int = 256, reps: int = 1):
    """Pruned against exhaustive over all receivers, chunk by chunk."""
    tot = None
    for s in range(0, len(receivers), chunk):
        e = min(len(receivers), s + chunk)
        d0 = spoly.DevicePoints(receivers[s:e])
        T = caustic.cull_sorted(ctx, dm, d0, dl)
        r = caustic.prune_vs_exhaustive(ctx, dm, d0, dl, T, net, reps=reps).as_dict()
        if tot is None:
            tot = {k: 0 for k in ("n_tuples", "n_kept", "positives", "kept_positives", "paths_exhaustive",
                                  "paths_pruned", "ms_exhaustive", "ms_score", "ms_solve_kept")}
        for k in tot:
            tot[k] += r[k]
        log(f"eval receivers {e}/{len(receivers)}: kept {tot['n_kept']}/{tot['n_tuples']}, "
            f"positives {tot['kept_positives']}/{tot['positives']}")
    tot["recall"] = tot["kept_positives"] / tot["positives"] if tot["positives"] else 1.0
    tot["path_recall"] = tot["paths_pruned"] / tot["paths_exhaustive"] if tot["paths_exhaustive"] else 1.0
    tot["speedup"] = tot["ms_exhaustive"] / (tot["ms_score"] + tot["ms_solve_kept"])
    return tot


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--receivers", type=int, default=8192)
    ap.add_argument("--examples", type=int, default=4_000_000)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--pos-weight", type=float, default=20.0)
    ap.add_argument("--pos-frac", type=float, default=0.25)
    ap.add_argument("--recall", type=float, default=0.999)
    ap.add_argument("--slack", type=float, default=0.1)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--eval", action="store_true", help="also measure on the 64x64 receiver grid")
    ap.add_argument("--eval-stride", type=int, default=1, help="use every k-th grid receiver in --eval")
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args(argv)

    spoly.load_library()
    ctx = spoly.Context(0)
    mesh = scenes.caustic_sphere()
    dm = spoly.DeviceMesh(mesh.P, mesh.N, mesh.tri)
    dl = spoly.DevicePoints(scenes.CAUSTIC_LIGHT_OUTSIDE)
    rec = scenes.pruner_receivers(args.receivers, args.seed)
    t0 = time.perf_counter()
    data, n_seen, n_pos, t_solve = label_receivers(ctx, dm, dl, rec, args.examples, args.seed)
    log(f"data: {data.n} examples ({int(data.labels.sum().item())} positive) from {n_seen} labelled tuples, "
        f"{time.perf_counter() - t0:.1f} s")
    train, val = split_by_receiver(data)
    d0 = spoly.DevicePoints(rec)
    net = pr.Pruner(args.seed)
    t1 = time.perf_counter()
    hist = net.train_steps(ctx, dm, d0, dl, train, args.steps, batch=args.batch, lr=args.lr,
                           pos_weight=args.pos_weight, pos_frac=args.pos_frac)
    torch.cuda.synchronize()
    log(f"{args.steps} steps in {time.perf_counter() - t1:.1f} s, loss {hist[0]:.4f} -> {np.mean(hist[-50:]):.4f}")
    sv = net.scores(ctx, dm, d0, dl, val)
    thr = net.calibrate(sv, val.labels, args.recall, args.slack)
    kept_val = float((sv >= thr).float().mean().item())
    rec_val = pr.recall_of(val.labels[sv >= thr], val.labels)
    log(f"threshold {thr:.4g}: validation recall {rec_val:.4f}, kept fraction {kept_val:.4f} "
        f"({int(val.labels.sum().item())} positives)")
    meta = dict(receivers=args.receivers, examples=data.n, labelled=n_seen, positives=n_pos, steps=args.steps,
                batch=args.batch, lr=args.lr, pos_weight=args.pos_weight, pos_frac=args.pos_frac,
                recall_target=args.recall, slack=args.slack, seed=args.seed, threshold=thr,
                val_recall=rec_val, val_kept=kept_val, loss_last=float(np.mean(hist[-50:])), label_s=t_solve)
    if args.eval:
        grid = scenes.caustic_receivers()[:: args.eval_stride]
        meta["test"] = evaluate(ctx, dm, dl, net, grid)
        log(json.dumps(meta["test"]))
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    st = net.state()
    np.savez(args.out, params=st["params"], threshold=np.float64(thr),
             meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))
    log(f"wrote {args.out}")
    ctx.close()
    return meta


def load(path: str = DEFAULT_OUT) -> pr.Pruner:
    """A Pruner with the stored parameters and threshold (no optimiser state)."""
    z = np.load(path, allow_pickle=False)
    net = pr.Pruner(0)
    net.params = torch.from_numpy(z["params"].astype(np.float32)).cuda()
    net.threshold = float(z["threshold"])
    return net


def load_meta(path: str = DEFAULT_OUT) -> dict:
    z = np.load(path, allow_pickle=False)
    return json.loads(bytes(z["meta"]).decode())


if __name__ == "__main__":
    main(sys.argv[1:])
