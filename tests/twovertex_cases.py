"""Seeded two-vertex test cases on the mirror-gap scene (two wavy heightfields
facing each other): paths traced forward from x0 through a random point of a
bottom triangle, with the exact reflection or refraction at each vertex
(interpolated normals), to a light placed on the outgoing ray.  Every traced
tuple has that path; the tuples around it are its neighbourhood."""
from __future__ import annotations

import numpy as np

from paper_2405_13409_amd import scenes

# per chain: height of x0, height of x3, IORs of the segments x0x1, x1x2, x2x3
SETUPS = {
    "RR": (0.5, 0.5, (1.0, 1.0, 1.0)),
    "RT": (0.5, 1.6, (1.0, 1.0, 1.5)),
    "TR": (-0.6, 0.5, (1.5, 1.0, 1.0)),
    "TT": (-0.6, 1.6, (1.5, 1.0, 1.5)),
}


def _nz(x):
    return x / np.linalg.norm(x)


def _bend(d, n, ev, eta_in, eta_out):
    """Outgoing unit direction of unit d at unit normal n (either orientation)."""
    c = d @ n
    if ev == "R":
        return d - 2.0 * c * n
    if c > 0:
        n, c = -n, -c
    r = eta_in / eta_out
    k = 1.0 - r * r * (1.0 - c * c)
    if k < 0:
        return None
    return r * d + (r * -c - np.sqrt(k)) * n


def _hit(mesh, tris, o, d):
    """Nearest hit of the ray o + t d (t > 1e-9) among triangles `tris`: (t, tri, u, v) or None."""
    P0 = mesh.P[mesh.tri[tris, 0]]
    e1 = mesh.P[mesh.tri[tris, 1]] - P0
    e2 = mesh.P[mesh.tri[tris, 2]] - P0
    pv = np.cross(d, e2)
    det = np.einsum("ij,ij->i", e1, pv)
    ok = np.abs(det) > 1e-14
    det = np.where(ok, det, 1.0)
    tv = o - P0
    u = np.einsum("ij,ij->i", tv, pv) / det
    qv = np.cross(tv, e1)
    v = (qv @ d) / det
    t = np.einsum("ij,ij->i", e2, qv) / det
    ok &= (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 1e-9)
    if not ok.any():
        return None
    k = np.argmin(np.where(ok, t, np.inf))
    return t[k], int(tris[k]), u[k], v[k]


def trace_paths(chain: str, n: int, seed: int, mesh=None):
    """n traced paths: arrays x0 [n,3], x3 [n,3], t1, t2 [n], uv [n,4]."""
    mesh = mesh or scenes.mirror_gap()
    z0, z3, eta = SETUPS[chain]
    half = mesh.nt // 2
    bottom, top = np.arange(half), np.arange(half, mesh.nt)
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        x0 = np.array([rng.uniform(-0.6, 0.6), rng.uniform(-0.6, 0.6), z0])
        t1 = int(rng.integers(0, half))
        a, b = rng.uniform(0.05, 0.9, 2)
        if a + b > 0.95:
            continue
        P = mesh.P[mesh.tri[t1]]
        N = mesh.N[mesh.tri[t1]]
        x1 = P[0] + a * (P[1] - P[0]) + b * (P[2] - P[0])
        n1 = _nz(N[0] + a * (N[1] - N[0]) + b * (N[2] - N[0]))
        d1 = _bend(_nz(x1 - x0), n1, chain[0], eta[0], eta[1])
        if d1 is None or d1[2] <= 0.05:
            continue
        h = _hit(mesh, top, x1, d1)
        if h is None:
            continue
        _, t2, u2, v2 = h
        if min(u2, v2, 1 - u2 - v2) < 0.02:
            continue
        Q = mesh.P[mesh.tri[t2]]
        M = mesh.N[mesh.tri[t2]]
        x2 = Q[0] + u2 * (Q[1] - Q[0]) + v2 * (Q[2] - Q[0])
        n2 = _nz(M[0] + u2 * (M[1] - M[0]) + v2 * (M[2] - M[0]))
        d2 = _bend(d1, n2, chain[1], eta[1], eta[2])
        if d2 is None or abs(d2[2]) < 0.05:
            continue
        s = (z3 - x2[2]) / d2[2]
        if s <= 0.05:
            continue
        x3 = x2 + s * d2
        # the light must not see the bottom surface first (keeps the cases clean)
        out.append((x0, x3, t1, t2, np.array([a, b, u2, v2])))
    x0 = np.array([o[0] for o in out])
    x3 = np.array([o[1] for o in out])
    t1 = np.array([o[2] for o in out], dtype=np.int32)
    t2 = np.array([o[3] for o in out], dtype=np.int32)
    uv = np.array([o[4] for o in out])
    return mesh, x0, x3, t1, t2, uv


def neighbourhood(mesh, t1: int, t2: int, r: float = 0.15):
    """Tuples (a, b) with a a bottom triangle within r of t1's centroid and b a
    top triangle within r of t2's."""
    c = mesh.P[mesh.tri].mean(1)
    half = mesh.nt // 2
    a = np.nonzero(np.linalg.norm(c[:half] - c[t1], axis=1) < r)[0]
    b = half + np.nonzero(np.linalg.norm(c[half:] - c[t2], axis=1) < r)[0]
    A, B = np.meshgrid(a, b, indexing="ij")
    return np.stack([A.ravel(), B.ravel()], 1).astype(np.int32)
