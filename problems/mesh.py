"""Seeded synthetic P1 triangle meshes of a mapped domain (inputs for the grid<->mesh transfers).

A jittered logical lattice of m x m points on (-1,1)^2 is split into triangles along a random
diagonal per quad and mapped through X = T^{-1}; the image T(x_v) of every physical vertex is then
known exactly (it is the lattice point), as the paper assumes for an analytic map (Sec. 2.3.1:
the mesh vertices are mapped through T).  Vertices are randomly permuted so that the mesh has no
grid-aligned numbering.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    xy_p: np.ndarray    # [nv][2] physical vertex coordinates
    xy_c: np.ndarray    # [nv][2] their images T(x) in (-1,1)^2
    tris: np.ndarray    # [nt][3] int32, counter-clockwise in both domains
    dof: np.ndarray     # [nv] bool: False on the physical boundary (Dirichlet)

    @property
    def nv(self):
        return self.xy_p.shape[0]

    @property
    def nt(self):
        return self.tris.shape[0]


def lattice_mesh(mp, m: int, rng: np.random.Generator, jitter: float = 0.15) -> Mesh:
    """m x m lattice, interior points jittered by up to ``jitter`` lattice spacings in each
    coordinate (0.15 keeps every triangle positively oriented), random diagonals, random
    vertex permutation."""
    h = 2.0 / (m - 1)
    g = np.linspace(-1.0, 1.0, m)
    X, Y = np.meshgrid(g, g)
    inner = np.zeros((m, m), dtype=bool)
    inner[1:-1, 1:-1] = True
    X = X + np.where(inner, rng.uniform(-jitter, jitter, size=(m, m)) * h, 0.0)
    Y = Y + np.where(inner, rng.uniform(-jitter, jitter, size=(m, m)) * h, 0.0)
    vid = np.arange(m * m).reshape(m, m)
    a, b = vid[:-1, :-1].ravel(), vid[:-1, 1:].ravel()       # (i,j), (i+1,j)
    c, d = vid[1:, :-1].ravel(), vid[1:, 1:].ravel()         # (i,j+1), (i+1,j+1)
    diag = rng.integers(0, 2, size=a.shape[0]).astype(bool)
    t1 = np.where(diag[:, None], np.stack([a, b, d], 1), np.stack([a, b, c], 1))
    t2 = np.where(diag[:, None], np.stack([a, d, c], 1), np.stack([b, d, c], 1))
    tris = np.concatenate([t1, t2], axis=0)
    xy_c = np.stack([X.ravel(), Y.ravel()], axis=1)
    px, py = mp(xy_c[:, 0], xy_c[:, 1])
    xy_p = np.stack([np.asarray(px), np.asarray(py)], axis=1)
    dof = inner.ravel().copy()
    perm = rng.permutation(m * m)              # new index of old vertex k is inv[k]
    inv = np.empty_like(perm)
    inv[perm] = np.arange(m * m)
    mesh = Mesh(xy_p=xy_p[perm], xy_c=xy_c[perm], tris=inv[tris].astype(np.int32), dof=dof[perm])
    for xy in (mesh.xy_c, mesh.xy_p):
        p = xy[mesh.tris]
        cross = ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                 - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
        if not np.all(cross > 0):
            raise ValueError("lattice mesh produced an inverted triangle")
    return mesh


def mesh_points_for_grid(n: int, alpha: float = 0.28) -> int:
    """Lattice size m whose vertex count is about n^2 / alpha (the paper sizes the computational
    grid as about alpha = 0.28 times the physical DoF, Sec. 4.3)."""
    return int(np.ceil(np.sqrt(n * n / alpha)))
