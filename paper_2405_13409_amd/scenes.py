"""Seeded synthetic scenes and query lists.

This module only generates inputs: meshes (vertex positions, vertex normals,
triangle indices), separator points and candidate lists.  It holds none of the
specular-polynomial arithmetic, so both the FP64 oracle and the HIP path can be
fed from it without sharing any part of the method.

Scene recipes (the paper's own scenes are not available; these stand in for
its glint and caustic workloads of Sec. 6):

* ``heightfield(N, A, J, f_lo, f_hi, seed)`` -- a wavy specular surface over
  [-1,1]^2: vertices (-1+2i/N, -1+2j/N, z) with
  z = A * sum_m sin(f_m (cos t_m x + sin t_m y) + p_m),
  f_m ~ U[f_lo, f_hi] (angular frequency, radians per unit length),
  t_m ~ U[0, 2pi), p_m ~ U[0, 2pi) drawn (all f, then all t, then all p) from
  ``numpy.random.default_rng(seed)``.  With the grid sizes used here the
  shortest wavelength spans about 12.6 grid cells, so each triangle is smooth.  Vertex normals come from
  the analytic gradient, normalize(-z_x, -z_y, 1); the interpolated normal of
  Eq. (eq_ni) is formed from them inside each triangle.  Cell (i, j) is split
  into (v_ij, v_i+1j, v_i+1j+1) and (v_ij, v_i+1j+1, v_ij+1), counter-clockwise
  seen from +z.
* ``icosphere(levels, radius)`` -- icosahedron subdivided ``levels`` times with
  midpoints projected to the sphere; smooth normals = position / radius.
  Faces are oriented outward.
* ``mirror_gap(N, gap, ...)`` -- two wavy heightfields facing each other across
  a gap (stand-in for the paper's two-reflection glints scene): the bottom one
  z = h_b(x, y) with normals up (triangles 0 .. nt/2 - 1), the top one
  z = gap - h_t(x, y) with normals down (triangles nt/2 .. nt - 1), both built
  as ``heightfield`` with their own seeds.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Mesh:
    """Triangle mesh: positions ``P`` [nv,3] f64, vertex normals ``N`` [nv,3] f64,
    triangle vertex ids ``tri`` [nt,3] int32."""

    P: np.ndarray
    N: np.ndarray
    tri: np.ndarray

    @property
    def nv(self) -> int:
        return int(self.P.shape[0])

    @property
    def nt(self) -> int:
        return int(self.tri.shape[0])

    def as_f32_exact(self) -> "Mesh":
        """The same mesh with every coordinate rounded to the nearest float32
        (still stored as f64), so an FP32 kernel and an FP64 reference see one
        exactly identical problem."""
        return Mesh(self.P.astype(np.float32).astype(np.float64),
                    self.N.astype(np.float32).astype(np.float64), self.tri.copy())


def heightfield(N: int, A: float, J: int, f_lo: float, f_hi: float, seed: int) -> Mesh:
    rng = np.random.default_rng(seed)
    f = rng.uniform(f_lo, f_hi, J)
    th = rng.uniform(0.0, 2.0 * math.pi, J)
    ph = rng.uniform(0.0, 2.0 * math.pi, J)
    g = -1.0 + 2.0 * np.arange(N + 1) / N
    X, Y = np.meshgrid(g, g, indexing="xy")  # X[j, i] = x_i, Y[j, i] = y_j
    z = np.zeros_like(X)
    zx = np.zeros_like(X)
    zy = np.zeros_like(X)
    for m in range(J):
        c, s = math.cos(th[m]), math.sin(th[m])
        arg = f[m] * (c * X + s * Y) + ph[m]
        z += A * np.sin(arg)
        k = A * f[m] * np.cos(arg)
        zx += k * c
        zy += k * s
    P = np.stack([X.ravel(), Y.ravel(), z.ravel()], axis=1)
    n = np.stack([-zx.ravel(), -zy.ravel(), np.ones(X.size)], axis=1)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    tris = []
    W = N + 1
    for j in range(N):
        for i in range(N):
            v00 = j * W + i
            v10 = j * W + i + 1
            v11 = (j + 1) * W + i + 1
            v01 = (j + 1) * W + i
            tris.append((v00, v10, v11))
            tris.append((v00, v11, v01))
    return Mesh(P.astype(np.float64), n.astype(np.float64), np.asarray(tris, dtype=np.int32))


def icosphere(levels: int = 3, radius: float = 0.5, center=(0.0, 0.0, 0.0)) -> Mesh:
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
         (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    V = [np.asarray(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(levels):
        cache: dict = {}

        def mid(a: int, b: int) -> int:
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]

        nf = []
        for (a, b, c) in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = nf
    U = np.asarray(V)
    tri = np.asarray(F, dtype=np.int32)
    # orient outward
    e = np.cross(U[tri[:, 1]] - U[tri[:, 0]], U[tri[:, 2]] - U[tri[:, 0]])
    flip = np.einsum("ij,ij->i", e, U[tri].mean(axis=1)) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    P = U * radius + np.asarray(center, dtype=np.float64)
    return Mesh(P, U.copy(), tri)


def mirror_gap(N: int = 16, gap: float = 1.0, A: float = 0.05, J: int = 3, f_lo: float = 1.0, f_hi: float = 4.0,
               seed_bottom: int = 6, seed_top: int = 7) -> Mesh:
    lo = heightfield(N, A, J, f_lo, f_hi, seed_bottom)
    hi = heightfield(N, A, J, f_lo, f_hi, seed_top)
    P_hi = hi.P.copy()
    P_hi[:, 2] = gap - P_hi[:, 2]
    # heightfield normals are (-h_x, -h_y, 1)/|.|; the downward normal of z = gap - h is (-h_x, -h_y, -1)/|.|
    N_hi = hi.N * np.array([1.0, 1.0, -1.0])
    tri_hi = hi.tri[:, [0, 2, 1]] + lo.nv   # counter-clockwise seen from below
    return Mesh(np.concatenate([lo.P, P_hi]), np.concatenate([lo.N, N_hi]),
                np.concatenate([lo.tri, tri_hi]).astype(np.int32))


# ---------------------------------------------------------------- workloads

def points_uniform(n: int, lo: float, hi: float, z: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    xy = rng.uniform(lo, hi, (n, 2))
    return np.concatenate([xy, np.full((n, 1), z)], axis=1)


def points_grid(n: int, lo: float, hi: float, z: float, tile: int = 1) -> np.ndarray:
    """n x n cell-centre grid on [lo,hi]^2 at height z.  tile = 1: row-major in
    y, then x.  tile = k (dividing n): k x k pixel tiles in row-major order,
    each row-major inside, so that consecutive points are close in space."""
    g = lo + (np.arange(n) + 0.5) * (hi - lo) / n
    X, Y = np.meshgrid(g, g, indexing="xy")
    P = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], axis=1)
    if tile <= 1:
        return P
    if n % tile:
        raise ValueError(f"tile {tile} does not divide {n}")
    nt = n // tile
    # index [ty, tx, iy, ix] -> row-major pixel (ty*tile+iy, tx*tile+ix)
    ty, tx, iy, ix = np.meshgrid(np.arange(nt), np.arange(nt), np.arange(tile), np.arange(tile), indexing="ij")
    return P[((ty * tile + iy) * n + tx * tile + ix).ravel()]


@dataclasses.dataclass
class OneBounceWorkload:
    """(shading point, light, triangle) queries for one specular vertex."""

    mesh: Mesh
    x0: np.ndarray          # [n0,3] shading points
    x2: np.ndarray          # [n2,3] lights
    q_x0: np.ndarray        # [nq] int32
    q_x2: np.ndarray        # [nq] int32
    q_tri: np.ndarray       # [nq] int32
    event: str              # "R" or "T"
    eta0: float             # IOR on the x0 side
    eta1: float             # IOR on the x2 side


def all_pairs(n_points: int, n_tris: int):
    qp = np.repeat(np.arange(n_points, dtype=np.int32), n_tris)
    qt = np.tile(np.arange(n_tris, dtype=np.int32), n_points)
    return qp, qt


def glints_small(seed_mesh: int = 1, seed_pts: int = 101) -> OneBounceWorkload:
    """16x16 heightfield (512 triangles), z = 0.05 * 3 sinusoids (freq 1..4),
    64 shading points uniform on [-1,1]^2 at z = 1, light (0.3,-0.2,1.5),
    reflection, every (point, triangle) pair: 32768 solves."""
    mesh = heightfield(16, 0.05, 3, 1.0, 4.0, seed_mesh)
    x0 = points_uniform(64, -1.0, 1.0, 1.0, seed_pts)
    x2 = np.asarray([[0.3, -0.2, 1.5]])
    qp, qt = all_pairs(64, mesh.nt)
    return OneBounceWorkload(mesh, x0, x2, qp, np.zeros_like(qp), qt, "R", 1.0, 1.0)


def glints_large_mesh(seed: int = 2) -> Mesh:
    """128x128 heightfield (32768 triangles), z = 0.02 * 8 sinusoids (freq 4..32)."""
    return heightfield(128, 0.02, 8, 4.0, 32.0, seed)


def glints_large_points(event: str, res: int = 256) -> np.ndarray:
    """res x res pixel-centre shading points on [-1,1]^2 in 16 x 16 pixel
    tiles (when 16 divides res); z = 2 for reflection, z = -2 (below the
    interface) for refraction."""
    return points_grid(res, -1.0, 1.0, 2.0 if event == "R" else -2.0, 16 if res % 16 == 0 else 1)


def with_occluders(mesh: Mesh, quads) -> Mesh:
    """The mesh plus axis-aligned horizontal rectangles (x0, x1, y0, y1, z),
    two triangles each with normal +z, appended after the mesh's own."""
    P, N, T = [mesh.P], [mesh.N], [mesh.tri]
    base = len(mesh.P)
    for k, (xa, xb, ya, yb, z) in enumerate(quads):
        P.append(np.array([[xa, ya, z], [xb, ya, z], [xb, yb, z], [xa, yb, z]], dtype=np.float64))
        N.append(np.tile([0.0, 0.0, 1.0], (4, 1)))
        b = base + 4 * k
        T.append(np.array([[b, b + 1, b + 2], [b, b + 2, b + 3]], dtype=np.int32))
    return Mesh(np.vstack(P), np.vstack(N), np.vstack(T).astype(np.int32))


# three strips between the small glints heightfield and its shading points
GLINT_STRIPS = [(-0.9, -0.6, -1.3, 1.3, 0.5), (-0.15, 0.15, -1.3, 1.3, 0.5), (0.5, 0.8, -1.3, 1.3, 0.5)]


def shadowed_glints(res: int = 48) -> OneBounceWorkload:
    """A steep 16x16 heightfield (z = 0.15 * 3 sinusoids, freq 1..4, seed 1)
    lit from low at (1.5, 0.3, 0.5) with res x res shading points on
    [-1,1]^2 at z = 0.5: its bumps hide one another from the light and from
    the shading points.  Reflection; every (point, triangle) pair."""
    mesh = heightfield(16, 0.15, 3, 1.0, 4.0, 1)
    x0 = points_grid(res, -1.0, 1.0, 0.5)
    qp, qt = all_pairs(len(x0), mesh.nt)
    return OneBounceWorkload(mesh, x0, np.asarray([[1.5, 0.3, 0.5]]), qp, np.zeros_like(qp), qt, "R", 1.0, 1.0)


GLINTS_LARGE_LIGHT = np.asarray([[0.0, 0.0, 4.0]])

CAUSTIC_LIGHT_OUTSIDE = np.asarray([[0.1, 0.05, 1.5]])
CAUSTIC_LIGHT_INSIDE = np.asarray([[0.0, 0.0, 0.1]])
MIRROR_GAP_LIGHT = np.asarray([[0.15, -0.1, 0.5]])


def _euler(a: float, b: float, c: float) -> np.ndarray:
    ca, sa, cb, sb, cc, sc = math.cos(a), math.sin(a), math.cos(b), math.sin(b), math.cos(c), math.sin(c)
    Rz = np.array([[ca, -sa, 0], [sa, ca, 0], [0, 0, 1.0]])
    Ry = np.array([[cb, 0, sb], [0, 1.0, 0], [-sb, 0, cb]])
    Rx = np.array([[1.0, 0, 0], [0, cc, -sc], [0, sc, cc]])
    return Rz @ Ry @ Rx


def caustic_sphere() -> Mesh:
    """Level-3 icosphere of radius 0.5 at the origin: 642 vertices, 1280 triangles.
    The tessellation is turned by a fixed generic rotation (Euler z-y-x angles
    0.3, 0.7, 1.1) so that no vertex coordinate is exactly zero: exact zeros would
    make whole rows of polynomial coefficients cancel exactly."""
    m = icosphere(3, 0.5)
    R = _euler(0.3, 0.7, 1.1)
    return Mesh(m.P @ R.T, m.N @ R.T, m.tri)


def caustic_traced(n_side: int = 8, span: float = 0.35, radius: float = 0.5, light=None):
    """Receivers where caustic paths exist: rays from the light aimed at the
    sphere's centre shifted by offsets on an n_side x n_side grid over
    [-span, span]^2, refracted into and out of the exact sphere (IOR 1.5)
    and followed to the receiver plane z = -1.  Returns the receivers [n,3],
    the exit points (receiver side) and the entry points (light side)."""
    x3 = (CAUSTIC_LIGHT_OUTSIDE if light is None else np.asarray(light, dtype=np.float64).reshape(1, 3))[0]

    def nz(x):
        return x / np.linalg.norm(x)

    def refract(d, n, eta):
        c = -d @ n
        k = 1.0 - eta * eta * (1.0 - c * c)
        return eta * d + (eta * c - math.sqrt(k)) * n

    rec, ex, en = [], [], []
    g = np.linspace(-span, span, n_side)
    for ox in g:
        for oy in g:
            d = nz(np.array([ox, oy, 0.0]) - x3)
            b = x3 @ d
            t = -b - math.sqrt(b * b - (x3 @ x3 - radius * radius))
            p = x3 + t * d
            d2 = nz(refract(d, nz(p), 1.0 / 1.5))
            q = p + (-2.0 * (p @ d2)) * d2
            d3 = nz(refract(d2, -nz(q), 1.5))
            rec.append(q + ((-1.0 - q[2]) / d3[2]) * d3)
            ex.append(q)
            en.append(p)
    return np.asarray(rec), np.asarray(ex), np.asarray(en)


def tuples_near(mesh: Mesh, x0, x3, p1, p2, r: float) -> np.ndarray:
    """(T1, T2) pairs with T1's centroid within r of p1 and facing x0, and
    T2's within r of p2 and facing x3 (by the mean vertex normal)."""
    c = mesh.P[mesh.tri].mean(1)
    nc = mesh.N[mesh.tri].mean(1)
    t1 = np.nonzero((((x0 - c) * nc).sum(1) > 0) & (np.linalg.norm(c - p1, axis=1) < r))[0]
    t2 = np.nonzero((((x3 - c) * nc).sum(1) > 0) & (np.linalg.norm(c - p2, axis=1) < r))[0]
    A, B = np.meshgrid(t1, t2, indexing="ij")
    return np.stack([A.ravel(), B.ravel()], 1).astype(np.int32)


def caustic_receivers(res: int = 64) -> np.ndarray:
    """res x res cell-centre receivers on [-2,2]^2 at z = -1."""
    return points_grid(res, -2.0, 2.0, -1.0)


def subsample(n_total: int, n_take: int, seed: int) -> np.ndarray:
    """Seeded uniform subsample of indices (sorted)."""
    rng = np.random.default_rng(seed)
    if n_take >= n_total:
        return np.arange(n_total, dtype=np.int64)
    return np.sort(rng.choice(n_total, n_take, replace=False)).astype(np.int64)


def pruner_receivers(n: int, seed: int = 5) -> np.ndarray:
    """Training receivers of the learned tuple pruner: x0 ~ U([-2,2]^2) at z = -1."""
    return points_uniform(n, -2.0, 2.0, -1.0, seed)


def mixed_draw(n_list_1: int, n_list_2: int, n_total: int = 2_000_000, frac_1: float = 0.7, seed: int = 4):
    """Mixed batch: round(frac_1 * n_total) instances drawn with replacement
    from a list of n_list_1 one-vertex instances, the rest from a list of
    n_list_2 two-vertex tuples.  Returns the two index arrays (int64), each in
    draw order."""
    rng = np.random.default_rng(seed)
    n1 = int(round(frac_1 * n_total))
    i1 = rng.integers(0, n_list_1, n1) if n_list_1 > 0 else np.zeros(0, dtype=np.int64)
    i2 = rng.integers(0, n_list_2, n_total - n1) if n_list_2 > 0 else np.zeros(0, dtype=np.int64)
    return i1.astype(np.int64), i2.astype(np.int64)
