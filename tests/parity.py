"""Set comparison between HIP-path solutions and the FP64 oracle.

The result of one instance is a set of (u, v) solutions.  Both sides follow the
same readings of the paper, but a few situations are numerically ambiguous and
are excluded from the exact comparison (their share is reported):
  * a solution within `band` of a triangle edge (closed-triangle test on
    polished values can go either way),
  * a residual within a factor 10 of tau,
  * an instance whose resultant has a near-tangent critical value or two roots
    closer than `gap` (a sign change can be lost or gained by rounding).
Everything else must match exactly in count, and in (u, v) within `tol`.
"""
from __future__ import annotations

import numpy as np

FP64 = dict(tol=1e-10, band=1e-9, tangency=1e-12, gap=1e-8)
FP32 = dict(tol=1e-5, band=1e-4, tangency=1e-5, gap=1e-4)


def compare_onebounce(gpu, orc, diag, nq, tol, band, tangency, gap, tau=1e-6):
    """gpu: SOLUTION_DTYPE records; orc: oracle SOL_DTYPE records; diag: oracle diag [nq].
    Returns a stats dict; raises AssertionError on a mismatch."""
    bad_q = np.zeros(nq, dtype=bool)
    bad_q |= diag["tangency"] < tangency
    bad_q |= diag["min_gap"] < gap
    o_amb = (orc["edge"] < band) | ((orc["residual"] >= tau / 10) & (orc["residual"] <= 10 * tau))
    g_amb = (gpu["edge"] < band) | ((gpu["residual"] >= tau / 10) & (gpu["residual"] <= 10 * tau))
    # an instance with any ambiguous solution on either side is left out entirely
    bad_q[orc["query"][o_amb]] = True
    bad_q[gpu["query"][g_amb]] = True
    go = gpu[~bad_q[gpu["query"]]]
    oo = orc[~bad_q[orc["query"]]]
    go = go[np.lexsort((go["u"][:, 0], go["v"][:, 0], go["query"]))]
    oo = oo[np.lexsort((oo["u1"], oo["v1"], oo["query"]))]
    gq = np.bincount(go["query"], minlength=nq)
    oq = np.bincount(oo["query"], minlength=nq)
    mism = np.nonzero(gq != oq)[0]
    assert len(mism) == 0, f"{len(mism)} instances differ in solution count, e.g. q={mism[:5]} " \
                           f"gpu={gq[mism[:5]]} oracle={oq[mism[:5]]}"
    du = np.abs(go["u"][:, 0] - oo["u1"]) if len(go) else np.zeros(0)
    dv = np.abs(go["v"][:, 0] - oo["v1"]) if len(go) else np.zeros(0)
    err = float(max(du.max(initial=0.0), dv.max(initial=0.0)))
    assert err <= tol, f"max |du|,|dv| = {err} > {tol}"
    assert np.all(go["tri"][:, 0] >= 0)
    return dict(compared=len(oo), excluded_instances=int(bad_q.sum()), max_err=err,
                p99_err=float(np.percentile(np.maximum(du, dv), 99)) if len(du) else 0.0,
                ambiguous_fraction=float(bad_q.sum()) / max(1, nq))
