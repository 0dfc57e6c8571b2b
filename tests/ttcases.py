"""Seeded two-vertex (TT) test cases on the caustic sphere: receivers found by
tracing light rays through the exact sphere, and the tuples around each path."""
from __future__ import annotations

import numpy as np

from paper_2405_13409_amd import scenes


def _nz(x):
    return x / np.linalg.norm(x)


def _refract(d, n, eta):
    c = -d @ n
    k = 1 - eta * eta * (1 - c * c)
    return eta * d + (eta * c - np.sqrt(k)) * n


def traced_receiver(offset, light=None, radius=0.5):
    """Shoot a ray from the light towards the sphere centre shifted by `offset`,
    refract through the exact sphere (IOR 1.5) and return where it lands on
    z = -1, with the entry and exit points."""
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE[0] if light is None else light
    d = _nz(-x3 + np.asarray(offset))
    b = x3 @ d
    c = x3 @ x3 - radius * radius
    t = -b - np.sqrt(b * b - c)
    p = x3 + t * d
    d2 = _nz(_refract(d, _nz(p), 1 / 1.5))
    q = p + (-2 * (p @ d2)) * d2
    d3 = _nz(_refract(d2, -_nz(q), 1.5))
    x0 = q + ((-1 - q[2]) / d3[2]) * d3
    return x0, q, p


def tuples_near(mesh, x0, x3, entry, exit_, r=0.2):
    c = mesh.P[mesh.tri].mean(1)
    nc = mesh.N[mesh.tri].mean(1)
    front = np.nonzero(((x0 - c) * nc).sum(1) > 0)[0]
    back = np.nonzero(((x3 - c) * nc).sum(1) > 0)[0]
    t1 = front[np.linalg.norm(c[front] - entry, axis=1) < r]
    t2 = back[np.linalg.norm(c[back] - exit_, axis=1) < r]
    A, B = np.meshgrid(t1, t2, indexing="ij")
    return np.stack([A.ravel(), B.ravel()], 1).astype(np.int32)
