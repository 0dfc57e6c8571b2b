"""Brute-force specular path search, independent of the polynomial method.

It solves the path-space constraint h x n = 0 of Eq. (eq_ch) directly: damped
Gauss-Newton from a dense grid of seeds plus local minima of |G| on a fine
grid, where G(u,v) = h^ x n^ with h = eta_in wi + eta_out wo.  Used to pin the
oracle's complete solution sets on tiny meshes.
"""
from __future__ import annotations

import numpy as np


def _norm(a):
    return a / np.linalg.norm(a, axis=-1, keepdims=True)


def residual(tri_P, tri_N, x0, x2, eta0, eta1, u, v):
    """G(u,v) for arrays u, v (any shape) -> [..., 3]."""
    p0, p1, p2 = tri_P
    n0, n1, n2 = tri_N
    w = 1.0 - u - v
    x = w[..., None] * p0 + u[..., None] * p1 + v[..., None] * p2
    n = _norm(w[..., None] * n0 + u[..., None] * n1 + v[..., None] * n2)
    wi = _norm(x0 - x)
    wo = _norm(x2 - x)
    h = _norm(eta0 * wi + eta1 * wo)
    return np.cross(h, n), wi, wo, n


def _gn(tri_P, tri_N, x0, x2, eta0, eta1, u, v, iters=60):
    hstep = 1e-7
    for _ in range(iters):
        G, *_ = residual(tri_P, tri_N, x0, x2, eta0, eta1, u, v)
        Gu, *_ = residual(tri_P, tri_N, x0, x2, eta0, eta1, u + hstep, v)
        Gv, *_ = residual(tri_P, tri_N, x0, x2, eta0, eta1, u, v + hstep)
        Ju = (Gu - G) / hstep
        Jv = (Gv - G) / hstep
        # normal equations of the 3x2 least-squares step
        a = np.sum(Ju * Ju, -1)
        b = np.sum(Ju * Jv, -1)
        c = np.sum(Jv * Jv, -1)
        ru = np.sum(Ju * G, -1)
        rv = np.sum(Jv * G, -1)
        det = a * c - b * b
        det = np.where(np.abs(det) > 1e-300, det, 1e-300)
        du = (c * ru - b * rv) / det
        dv = (a * rv - b * ru) / det
        # damp large steps
        s = np.minimum(1.0, 0.25 / np.maximum(np.abs(du) + np.abs(dv), 1e-300))
        f0 = np.linalg.norm(G, axis=-1)
        for _ls in range(8):
            un, vn = u - s * du, v - s * dv
            Gn, *_ = residual(tri_P, tri_N, x0, x2, eta0, eta1, un, vn)
            better = np.linalg.norm(Gn, axis=-1) <= f0
            if np.all(better):
                break
            s = np.where(better, s, s * 0.5)
        u, v = u - s * du, v - s * dv
        u = np.clip(u, -0.5, 1.5)
        v = np.clip(v, -0.5, 1.5)
    # final exact Newton polish on two tangential components (square system)
    for _ in range(4):
        G, *_ = residual(tri_P, tri_N, x0, x2, eta0, eta1, u, v)
        Gu, *_ = residual(tri_P, tri_N, x0, x2, eta0, eta1, u + hstep, v)
        Gv, *_ = residual(tri_P, tri_N, x0, x2, eta0, eta1, u, v + hstep)
        Ju = (Gu - G) / hstep
        Jv = (Gv - G) / hstep
        a = np.sum(Ju * Ju, -1)
        b = np.sum(Ju * Jv, -1)
        c = np.sum(Jv * Jv, -1)
        ru = np.sum(Ju * G, -1)
        rv = np.sum(Jv * G, -1)
        det = a * c - b * b
        det = np.where(np.abs(det) > 1e-300, det, 1e-300)
        u = u - (c * ru - b * rv) / det
        v = v - (a * rv - b * ru) / det
    return u, v


def solve(tri_P, tri_N, x0, x2, event, eta0=1.0, eta1=1.0, seeds=48, grid=400, tol=1e-11, dedup=1e-7):
    """All admissible (u,v) on one triangle, as an [k,2] array sorted by (v,u)."""
    tri_P = [np.asarray(p, dtype=np.float64) for p in tri_P]
    tri_N = [np.asarray(n, dtype=np.float64) for n in tri_N]
    x0 = np.asarray(x0, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    g = np.linspace(-0.05, 1.05, seeds)
    U, Vv = np.meshgrid(g, g, indexing="ij")
    su, sv = U.ravel(), Vv.ravel()
    # local minima of |G| on a fine grid as extra seeds
    gg = np.linspace(-0.02, 1.02, grid)
    GU, GV = np.meshgrid(gg, gg, indexing="ij")
    G, *_ = residual(tri_P, tri_N, x0, x2, eta0, eta1, GU, GV)
    f = np.linalg.norm(G, axis=-1)
    inner = f[1:-1, 1:-1]
    m = np.ones_like(inner, dtype=bool)
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            if di == 0 and dj == 0:
                continue
            m &= inner <= f[1 + di:grid - 1 + di, 1 + dj:grid - 1 + dj]
    ii, jj = np.nonzero(m)
    su = np.concatenate([su, GU[1:-1, 1:-1][ii, jj]])
    sv = np.concatenate([sv, GV[1:-1, 1:-1][ii, jj]])
    u, v = _gn(tri_P, tri_N, x0, x2, eta0, eta1, su, sv)
    G, wi, wo, n = residual(tri_P, tri_N, x0, x2, eta0, eta1, u, v)
    r = np.linalg.norm(G, axis=-1)
    side = np.sum(wi * n, -1) * np.sum(wo * n, -1)
    ok = (r < tol) & np.isfinite(r)
    ok &= (side > 0) if event == "R" else (side < 0)
    ok &= (u >= -1e-12) & (v >= -1e-12) & (u + v <= 1 + 1e-12)
    pts = np.stack([u[ok], v[ok]], 1)
    out = []
    for p in pts[np.lexsort((pts[:, 0], pts[:, 1]))] if len(pts) else []:
        if not any(abs(p[0] - q[0]) < dedup and abs(p[1] - q[1]) < dedup for q in out):
            out.append(p)
    return np.asarray(out).reshape(-1, 2)
