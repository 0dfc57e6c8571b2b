"""Brute-force search for two-vertex specular paths (x0 -> T1 -> T2 -> x3,
reflection or refraction at each vertex), independent of the polynomial method.

Unknowns z = (u1, v1, u2, v2): barycentric coordinates on both triangles, with
interpolated normals.  The path-space constraints of Eq. (eq_ch) hold at both
vertices: G_i = h_i^ x n_i^ = 0 with h_i = eta_in w_in + eta_out w_out (unit
directions towards the neighbours).  Damped Gauss-Newton on the six residual
components from many seeds: a grid over T1, each seed completed by tracing the
exactly reflected or refracted ray into T2's plane (the laws in vector form),
plus the local minima of the traced residual on a fine grid.  Converged points
that are inside both (closed) triangles and have the right sides at both
vertices (reflection: both neighbours on one side; refraction: opposite sides)
are the paths.
"""
from __future__ import annotations

import numpy as np


def _nz(a):
    return a / np.linalg.norm(a, axis=-1, keepdims=True)


def _interp(T, u, v):
    """T: [..., 3 vertices, 3] (broadcast against u, v)."""
    w = 1.0 - u - v
    return w[..., None] * T[..., 0, :] + u[..., None] * T[..., 1, :] + v[..., None] * T[..., 2, :]


def residual(T1P, T1N, T2P, T2N, x0, x3, eta, z):
    u1, v1, u2, v2 = z[..., 0], z[..., 1], z[..., 2], z[..., 3]
    x1 = _interp(T1P, u1, v1)
    x2 = _interp(T2P, u2, v2)
    n1 = _nz(_interp(T1N, u1, v1))
    n2 = _nz(_interp(T2N, u2, v2))
    a0, a1, a2 = _nz(x0 - x1), _nz(x2 - x1), _nz(x1 - x2)
    a3 = _nz(x3 - x2)
    h1 = _nz(eta[0] * a0 + eta[1] * a1)
    h2 = _nz(eta[1] * a2 + eta[2] * a3)
    G = np.concatenate([np.cross(h1, n1), np.cross(h2, n2)], -1)
    side = np.stack([np.sum(a0 * n1, -1) * np.sum(a1 * n1, -1), np.sum(a2 * n2, -1) * np.sum(a3 * n2, -1)], -1)
    return G, side


def _refract_into(T1P, T1N, T2P, x0, eta, u1, v1, ev1="T"):
    """(u2, v2) where the exactly reflected (ev1 = "R") or refracted ray from
    x1(u1, v1) meets T2's plane."""
    x1 = _interp(T1P, u1, v1)
    n = _nz(_interp(T1N, u1, v1))
    d = _nz(x1 - x0)
    c = np.sum(d * n, -1)
    if ev1 == "R":
        t = d - (2.0 * c)[..., None] * n
        ok = np.ones(c.shape, dtype=bool)
    else:
        n = np.where((c > 0)[..., None], -n, n)
        ci = np.abs(c)
        r = eta[0] / eta[1]
        k = 1.0 - r * r * (1.0 - ci * ci)
        ok = k >= 0
        t = r * d + (r * ci - np.sqrt(np.maximum(k, 0.0)))[..., None] * n
    p0 = T2P[..., 0, :]
    e1, e2 = T2P[..., 1, :] - p0, T2P[..., 2, :] - p0
    m = np.cross(e1, e2)
    dot = lambda a, b: np.sum(a * b, -1)  # noqa: E731
    den = dot(t, m)
    s = dot(p0 - x1, m) / np.where(den != 0, den, 1e-300)
    y = x1 + s[..., None] * t - p0
    # barycentrics of y in (e1, e2) by the 2x2 normal equations
    g11, g12, g22 = dot(e1, e1), dot(e1, e2), dot(e2, e2)
    b1, b2 = dot(y, e1), dot(y, e2)
    dd = g11 * g22 - g12 * g12
    u2 = (g22 * b1 - g12 * b2) / dd
    v2 = (g11 * b2 - g12 * b1) / dd
    ok &= (den != 0) & (s > 0)
    return u2, v2, ok


def _gauss_newton(f, z, iters=50, h=1e-7):
    for _ in range(iters):
        G, _ = f(z)
        J = np.empty(G.shape + (4,))
        for k in range(4):
            zk = z.copy()
            zk[..., k] += h
            J[..., k] = (f(zk)[0] - G) / h
        JT = np.swapaxes(J, -1, -2)
        A = JT @ J + 1e-18 * np.eye(4)
        g = (JT @ G[..., None])[..., 0]
        try:
            dz = np.linalg.solve(A, g[..., None])[..., 0]
        except np.linalg.LinAlgError:
            break
        dz = np.where(np.isfinite(dz), dz, 0.0)
        # damping: at most 0.1 in barycentric units per step, then backtrack
        s = np.minimum(1.0, 0.1 / np.maximum(np.abs(dz).max(-1), 1e-300))
        f0 = np.linalg.norm(G, axis=-1)
        for _ls in range(6):
            zn = z - s[..., None] * dz
            better = np.linalg.norm(f(zn)[0], axis=-1) <= f0
            if np.all(better):
                break
            s = np.where(better, s, 0.5 * s)
        z = np.clip(z - s[..., None] * dz, -0.5, 1.5)
    return z


def solve_many(mesh_P, mesh_N, tri, x0, x3, t1, t2, eta=(1.0, 1.5, 1.0), seeds=10, grid=100, tol=1e-11,
               dedup=1e-7, chain="TT"):
    """All paths of the given chain ("RR", "RT", "TR", "TT") of every tuple
    (t1[k], t2[k]) between the points x0 and x3: a list with one [m, 4] array
    of (u1, v1, u2, v2) per tuple, sorted by (v1, u1)."""
    t1 = np.asarray(t1)
    t2 = np.asarray(t2)
    nt = len(t1)
    T1P, T1N = mesh_P[tri[t1]], mesh_N[tri[t1]]
    T2P, T2N = mesh_P[tri[t2]], mesh_N[tri[t2]]
    x0 = np.asarray(x0, dtype=np.float64)
    x3 = np.asarray(x3, dtype=np.float64)
    # grid seeds over T1 plus the local minima of the traced residual on a fine grid
    g = np.linspace(-0.05, 1.05, seeds)
    gg = np.linspace(-0.02, 1.02, grid)
    GU, GV = np.meshgrid(gg, gg, indexing="ij")
    rows, su, sv = [], [], []
    U, V = np.meshgrid(g, g, indexing="ij")
    for k in range(nt):
        sl = (slice(k, k + 1),)
        u2, v2, ok = _refract_into(T1P[k], T1N[k], T2P[k], x0, eta, GU, GV, chain[0])
        G, _ = residual(T1P[k], T1N[k], T2P[k], T2N[k], x0, x3, eta, np.stack([GU, GV, u2, v2], -1))
        r = np.where(ok, np.linalg.norm(G[..., 3:], axis=-1), np.inf)
        inner = r[1:-1, 1:-1]
        m = np.isfinite(inner)
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                if di or dj:
                    m &= inner <= r[1 + di:grid - 1 + di, 1 + dj:grid - 1 + dj]
        ii, jj = np.nonzero(m)
        cu = np.concatenate([U.ravel(), GU[1:-1, 1:-1][ii, jj]])
        cv = np.concatenate([V.ravel(), GV[1:-1, 1:-1][ii, jj]])
        su.append(cu)
        sv.append(cv)
        rows.append(np.full(len(cu), k))
        del sl
    rows = np.concatenate(rows)
    su = np.concatenate(su)
    sv = np.concatenate(sv)
    A1P, A1N, A2P, A2N = T1P[rows], T1N[rows], T2P[rows], T2N[rows]
    u2, v2, ok = _refract_into(A1P, A1N, A2P, x0, eta, su, sv, chain[0])
    rows, A1P, A1N, A2P, A2N = rows[ok], A1P[ok], A1N[ok], A2P[ok], A2N[ok]
    z = np.stack([su, sv, u2, v2], -1)[ok]
    out = [np.zeros((0, 4)) for _ in range(nt)]
    if len(z) == 0:
        return out

    def f(zz):
        return residual(A1P, A1N, A2P, A2N, x0, x3, eta, zz)

    z = _gauss_newton(f, z)
    G, side = f(z)
    res = np.linalg.norm(G, axis=-1)
    want = np.array([1.0 if c == "R" else -1.0 for c in chain])
    keep = (res < tol) & np.all(side * want > 0, -1)
    e = 1e-12
    keep &= (z[:, 0] >= -e) & (z[:, 1] >= -e) & (z[:, 0] + z[:, 1] <= 1 + e)
    keep &= (z[:, 2] >= -e) & (z[:, 3] >= -e) & (z[:, 2] + z[:, 3] <= 1 + e)
    for k in np.unique(rows[keep]):
        zk = z[keep & (rows == k)]
        acc = []
        for p in zk[np.lexsort((zk[:, 0], zk[:, 1]))]:
            if not any(np.all(np.abs(p - q) < dedup) for q in acc):
                acc.append(p)
        out[k] = np.asarray(acc).reshape(-1, 4)
    return out
