"""Solver completeness (what the 100-piece, 10-bisection scan of Sec. 5.2
misses), measured against a reference that does not use the scan at all: the
brute-force search of tests/bruteforce_tt.py (damped Gauss-Newton on the
exact constraints at both vertices from dense seeds over T1).  Every tuple
within 0.06 of the entry and exit points of traced caustic paths for a 4x4
grid of receivers: the scan at 10 and 100 pieces finds exactly the reference
set.  (Over 64 receivers, 1316 tuples and 52 paths, 10, 100 and 4095 pieces
all match it too.)"""
import numpy as np
import pytest

import bruteforce_tt as bt
import oracle
import ttcases
from paper_2405_13409_amd import scenes


@pytest.fixture(scope="module")
def case():
    mesh = scenes.caustic_sphere()
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    g = np.linspace(-0.3, 0.3, 4)
    x0s, Q = [], []
    for ox in g:
        for oy in g:
            x0, entry, exit_ = ttcases.traced_receiver((ox, oy, 0.0))
            tp = ttcases.tuples_near(mesh, x0, x3[0], entry, exit_, 0.06)
            Q.append(np.column_stack([np.full(len(tp), len(x0s)), tp]))
            x0s.append(x0)
    x0s = np.asarray(x0s)
    Q = np.concatenate(Q).astype(np.int32)
    ref = [None] * len(Q)
    for k in range(len(x0s)):
        sel = np.nonzero(Q[:, 0] == k)[0]
        for j, z in zip(sel, bt.solve_many(mesh.P, mesh.N, mesh.tri, x0s[k], x3[0], Q[sel, 1], Q[sel, 2])):
            ref[j] = z
    return mesh, x0s, x3, Q, ref


@pytest.mark.parametrize("pieces", [10, 100])
def test_scan_finds_the_brute_force_set(case, pieces):
    mesh, x0s, x3, Q, ref = case
    prm = oracle.default_params(True)
    prm.pieces = pieces
    z = np.zeros(len(Q), dtype=np.int32)
    o, _ = oracle.solve_tt(mesh.P, mesh.N, mesh.tri, x0s, x3, Q[:, 0], z, Q[:, 1], Q[:, 2], params=prm)
    n_ref = sum(len(r) for r in ref)
    missed = extra = 0
    for q in range(len(Q)):
        oq, B = o[o["query"] == q], ref[q]
        for p in B:
            missed += not np.any((np.abs(oq["u1"] - p[0]) < 1e-7) & (np.abs(oq["v1"] - p[1]) < 1e-7))
        for r in oq:
            extra += not (len(B) and np.any((np.abs(B[:, 0] - r["u1"]) < 1e-7) & (np.abs(B[:, 1] - r["v1"]) < 1e-7)))
    print(f"{len(Q)} tuples, {n_ref} reference paths; {pieces} pieces: missed {missed}, not in the reference {extra}")
    assert n_ref >= 10 and missed == 0 and extra == 0
