"""Training, calibration and use of the learned two-vertex tuple pruner.

Labels come from the solver itself: a tuple is positive iff the exhaustive
two-vertex solve (spoly_solve_nbounce) returns at least one admissible path
for it.  The network (spoly_prune_score / spoly_pruner_fwd_bwd /
spoly_pruner_step) is trained on the GPU with class-weighted binary cross
entropy and Adam; the threshold is calibrated on held-out tuples for a target
recall.  The exhaustive solve stays available as the fallback and as the judge
of the pruner's error.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import torch

from . import spoly

IN, HID = 42, 128
SIZES = [("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (HID, HID)),
         ("b3", (HID,)), ("W4", (HID,)), ("b4", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)
assert NPARAMS == spoly.PRUNER_NPARAMS


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights (limit sqrt(6 / fan_in)), zero biases, float32."""
    rng = np.random.default_rng(seed)
    out = []
    for name, shape in SIZES:
        n = int(np.prod(shape))
        if name[0] == "W":
            lim = np.sqrt(6.0 / shape[0])
            out.append(rng.uniform(-lim, lim, n))
        else:
            out.append(np.zeros(n))
    return np.concatenate(out).astype(np.float32)


@dataclasses.dataclass
class Tuples:
    """Device tensors of (x0, x3, T1, T2) tuples and optional labels."""
    q0: torch.Tensor
    q3: torch.Tensor
    qt: torch.Tensor          # [n, 2]
    labels: torch.Tensor | None = None

    @property
    def n(self) -> int:
        return int(self.q0.numel())

    def take(self, idx: torch.Tensor) -> "Tuples":
        return Tuples(self.q0[idx].contiguous(), self.q3[idx].contiguous(), self.qt[idx].contiguous(),
                      None if self.labels is None else self.labels[idx].contiguous())


def exhaustive_labels(ctx: spoly.Context, dm, d0, d3, T: Tuples, eta=(1.0, 1.5, 1.0), chunk: int = 1 << 20):
    """Run the exhaustive two-vertex solve over all tuples; returns (labels
    float32 [n] on the device, number of solutions, seconds)."""
    lab = torch.zeros(T.n, dtype=torch.float32, device="cuda")
    nsol = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(0, T.n, chunk):
        e = min(T.n, s + chunk)
        sols = ctx.solve_2bounce(dm, d0, d3, T.q0[s:e], T.q3[s:e], T.qt[s:e], eta)
        if len(sols):
            q = torch.from_numpy(sols["query"].astype(np.int64) + s).cuda()
            lab[q] = 1.0
        nsol += len(sols)
    torch.cuda.synchronize()
    return lab, nsol, time.perf_counter() - t0


class Pruner:
    """fp32 master parameters and Adam state on the GPU."""

    def __init__(self, seed: int = 0):
        self.params = torch.from_numpy(init_params(seed)).cuda()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.step = 0
        self.rng = np.random.default_rng(seed + 1)
        self.threshold = 0.5

    # ---------------------------------------------------------------- checkpoint / resume
    def state(self) -> dict:
        return {"params": self.params.cpu().numpy(), "m": self.m.cpu().numpy(), "v": self.v.cpu().numpy(),
                "step": np.int64(self.step), "threshold": np.float64(self.threshold),
                "rng": np.frombuffer(repr(self.rng.bit_generator.state).encode(), dtype=np.uint8)}

    def save(self, path: str) -> None:
        np.savez(path, **self.state())

    def load(self, path: str) -> None:
        z = np.load(path, allow_pickle=False)
        self.params = torch.from_numpy(z["params"]).cuda()
        self.m = torch.from_numpy(z["m"]).cuda()
        self.v = torch.from_numpy(z["v"]).cuda()
        self.grads = torch.zeros_like(self.params)
        self.step = int(z["step"])
        self.threshold = float(z["threshold"])
        import ast
        self.rng = np.random.default_rng()
        self.rng.bit_generator.state = ast.literal_eval(bytes(z["rng"]).decode())

    # ---------------------------------------------------------------- training
    def train_steps(self, ctx, dm, d0, d3, T: Tuples, steps: int, batch: int = 4096, lr: float = 1e-3,
                    pos_weight: float = 20.0, pos_frac: float | None = 0.25):
        """`steps` Adam steps on batches drawn from T (labels required).  With
        pos_frac set, each batch holds that share of positives (drawn with
        replacement) so that rare positives are seen every step."""
        lab = T.labels.cpu().numpy() > 0.5
        pos = np.nonzero(lab)[0]
        neg = np.nonzero(~lab)[0]
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        hist = []
        for _ in range(steps):
            if pos_frac is not None and len(pos):
                npos = int(batch * pos_frac)
                idx = np.concatenate([self.rng.choice(pos, npos), self.rng.choice(neg, batch - npos)])
            else:
                idx = self.rng.choice(T.n, batch, replace=False)
            B = T.take(torch.from_numpy(idx.astype(np.int64)).cuda())
            loss.zero_()
            ctx.pruner_fwd_bwd(dm, d0, d3, B.q0, B.q3, B.qt, B.labels, pos_weight, self.params, self.grads, loss)
            self.step += 1
            ctx.pruner_step(self.params, self.grads, self.m, self.v, self.step, lr)
            hist.append(loss)
            loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        return [float(h.item()) for h in hist]

    # ---------------------------------------------------------------- inference
    def scores(self, ctx, dm, d0, d3, T: Tuples) -> torch.Tensor:
        s = torch.empty(T.n, dtype=torch.float32, device="cuda")
        keep = torch.empty(1, dtype=torch.int32, device="cuda")
        ctx.prune_score(dm, d0, d3, T.q0, T.q3, T.qt, self.params, 1.0, scores=s, keep=keep)
        return s

    def calibrate(self, scores: torch.Tensor, labels: torch.Tensor, recall: float = 0.999, slack: float = 0.5):
        """Threshold = `slack` times the (1 - recall) quantile of the positives'
        scores (at most one positive in 1/(1-recall) below it; the slack factor
        keeps margin for unseen receivers)."""
        s = scores.cpu().numpy()
        y = labels.cpu().numpy() > 0.5
        ps = np.sort(s[y])
        if len(ps) == 0:
            self.threshold = 0.0
            return self.threshold
        k = int(np.floor((1.0 - recall) * len(ps)))
        self.threshold = float(ps[k]) * slack
        return self.threshold

    def prune(self, ctx, dm, d0, d3, T: Tuples) -> Tuples:
        keep = torch.empty(max(T.n, 1), dtype=torch.int32, device="cuda")
        kc = torch.zeros(1, dtype=torch.int64, device="cuda")
        ctx.prune_score(dm, d0, d3, T.q0, T.q3, T.qt, self.params, self.threshold, keep=keep, keep_count=kc)
        idx = keep[: int(kc.item())].long()
        idx, _ = torch.sort(idx)
        return T.take(idx)


def recall_of(kept_labels: torch.Tensor, all_labels: torch.Tensor) -> float:
    p = float(all_labels.sum().item())
    return float(kept_labels.sum().item()) / p if p > 0 else 1.0
