"""Two-vertex caustic workload: canonical tuple lists, exhaustive labels, and
the pruned-versus-exhaustive measurement of the learned pruner.

Chain x0 (receiver) -> T1 -> T2 -> x3 (light) through a dielectric body, IOR
(1, 1.5, 1) along the chain (Sec. 4.4-4.5).  Every routine here drives the
library through its C ABI; device tensors come from PyTorch.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import pruner as pr
from . import spoly

ETA = (1.0, 1.5, 1.0)
CULL_MARGIN = 1e-3


def cull_sorted(ctx: spoly.Context, dm: spoly.DeviceMesh, d0: spoly.DevicePoints, d3: spoly.DevicePoints,
                eta=ETA, margin: float = CULL_MARGIN) -> pr.Tuples:
    """Cone-culled (x0, x3, T1, T2) tuples in canonical order (sorted by x0,
    x3, T1, T2), so that seeded draws from the list are reproducible although
    the cull compacts in arbitrary order."""
    q0, q3, qt = ctx.cull_2bounce(dm, d0, d3, eta, margin)
    nt = int(dm.c.n_tris)
    n3 = int(d3.c.n)
    key = ((q0.long() * n3 + q3.long()) * nt + qt[:, 0].long()) * nt + qt[:, 1].long()
    order = torch.argsort(key)
    return pr.Tuples(q0[order].contiguous(), q3[order].contiguous(), qt[order].contiguous())


def solve_count(ctx, dm, d0, d3, T: pr.Tuples, out, out_count, eta=ETA):
    """Enqueue the exhaustive solve of T into caller buffers (no host sync)."""
    out_count.zero_()
    return ctx.solve_2bounce(dm, d0, d3, T.q0, T.q3, T.qt, eta, out=out, out_count=out_count, sync=False)


@dataclasses.dataclass
class PruneReport:
    n_tuples: int
    n_kept: int
    positives: int
    kept_positives: int
    paths_exhaustive: int
    paths_pruned: int
    ms_exhaustive: float
    ms_score: float
    ms_solve_kept: float

    @property
    def ms_pruned(self) -> float:
        return self.ms_score + self.ms_solve_kept

    @property
    def recall(self) -> float:
        return self.kept_positives / self.positives if self.positives else 1.0

    @property
    def path_recall(self) -> float:
        return self.paths_pruned / self.paths_exhaustive if self.paths_exhaustive else 1.0

    @property
    def speedup(self) -> float:
        return self.ms_exhaustive / self.ms_pruned if self.ms_pruned > 0 else float("inf")

    def as_dict(self) -> dict:
        d = dataclasses.asdict(self)
        d.update(ms_pruned=self.ms_pruned, recall=self.recall, path_recall=self.path_recall, speedup=self.speedup,
                 recall_lower_95=recall_lower_bound(self.kept_positives, self.positives))
        if getattr(self, "sweep", None) is not None:
            d["threshold_sweep"] = self.sweep
        return d


def _timed(fn, reps: int, warmup: bool = True):
    """Median device time (ms) of fn() over reps runs, after one warm-up run
    unless warmup is False."""
    if warmup:
        fn()
    ms = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    return float(np.median(ms))


def prune_vs_exhaustive(ctx, dm, d0, d3, T: pr.Tuples, net: pr.Pruner, reps: int = 3, eta=ETA,
                        exhaustive_reps: int | None = None) -> PruneReport:
    """Exhaustive solve of every tuple against score + solve of the kept ones.
    Recall is measured against the exhaustive solve's own labels.  With
    exhaustive_reps set, the (long) exhaustive solve runs exactly that many
    times, without a warm-up run."""
    n = T.n
    cap = max(4096, n // 64)
    out = torch.empty(cap * spoly.SOLUTION_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    if exhaustive_reps is None:
        ms_ex = _timed(lambda: solve_count(ctx, dm, d0, d3, T, out, cnt, eta), reps)
    else:
        ms_ex = _timed(lambda: solve_count(ctx, dm, d0, d3, T, out, cnt, eta), exhaustive_reps, warmup=False)
    n_ex = int(cnt.item())
    if n_ex > cap:
        raise spoly.SpolyError(f"solution capacity {cap} < {n_ex}")
    sols = out[: n_ex * spoly.SOLUTION_DTYPE.itemsize].cpu().numpy().view(spoly.SOLUTION_DTYPE)
    lab = np.zeros(n, dtype=bool)
    lab[sols["query"]] = True

    keep = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    kc = torch.zeros(1, dtype=torch.int64, device="cuda")

    def score():
        kc.zero_()
        ctx.prune_score(dm, d0, d3, T.q0, T.q3, T.qt, net.params, net.threshold, keep=keep, keep_count=kc)

    ms_sc = _timed(score, reps)
    nk = int(kc.item())
    kidx = keep[:nk].long()
    K = T.take(kidx)
    ms_kept = _timed(lambda: solve_count(ctx, dm, d0, d3, K, out, cnt, eta), reps)
    n_pr = int(cnt.item())
    kept = np.zeros(n, dtype=bool)
    kept[kidx.cpu().numpy()] = True
    rep = PruneReport(n, nk, int(lab.sum()), int((lab & kept).sum()), n_ex, n_pr, ms_ex, ms_sc, ms_kept)
    rep.sweep = threshold_sweep(ctx, dm, d0, d3, T, net, lab, out, cnt, eta)
    return rep


def recall_lower_bound(k: int, n: int, conf: float = 0.95) -> float:
    """One-sided Clopper-Pearson lower confidence bound on a recall of k/n."""
    if n == 0:
        return 1.0
    if k == 0:
        return 0.0
    from scipy.stats import beta

    return float(beta.ppf(1.0 - conf, k, n - k + 1))


def threshold_sweep(ctx, dm, d0, d3, T: pr.Tuples, net: pr.Pruner, lab: np.ndarray, out, cnt, eta=ETA,
                    factors=(1.0, 0.1, 0.01)):
    """Recall, kept fraction and pruned time at the calibrated threshold times
    each factor (scores from one scoring pass; the kept tuples solved and timed)."""
    n = T.n
    scores = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
    keep = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    kc = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.prune_score(dm, d0, d3, T.q0, T.q3, T.qt, net.params, net.threshold, scores=scores, keep=keep, keep_count=kc)
    sc = scores[:n].cpu().numpy()
    rows = []
    for f in factors:
        th = net.threshold * f
        kept = sc >= th
        K = T.take(torch.from_numpy(np.nonzero(kept)[0]).cuda())
        ms = _timed(lambda: solve_count(ctx, dm, d0, d3, K, out, cnt, eta), 3)
        kp = int((lab & kept).sum())
        rows.append({"threshold": th, "kept": int(kept.sum()), "kept_fraction": float(kept.mean()) if n else 0.0,
                     "positives": int(lab.sum()), "kept_positives": kp,
                     "recall": kp / int(lab.sum()) if lab.sum() else 1.0,
                     "recall_lower_95": recall_lower_bound(kp, int(lab.sum())), "ms_solve_kept": ms})
    return rows
