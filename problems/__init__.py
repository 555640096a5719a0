"""Seeded synthetic workloads for the mapped structured multigrid solve.

Shared by the HIP library's tests/benchmarks and by the oracle: this package produces plain
input data only (map Jacobians at quadrature points, per-cell coefficients, right-hand sides,
targets, meshes) and contains none of the solver's arithmetic.

Workloads (every random draw comes from numpy.random.SeedSequence(root).spawn(...)):
  quarter_annulus(n, seed)   : n x n grid, K = 1, b ~ U(-1,1)         (root 0)
  star(n, seed)              : star domain, log-normal K, b ~ U(-1,1)  (roots 1, 2, 4)
  batch(count, sizes, seed)  : independent star instances of mixed sizes (root 3)
  discontinuous(kind, n)     : unit square, identity map, the discontinuous diffusivities of
                               the paper's variable-coefficient problems, b ~ U(-1,1) (root 5)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .fields import (GAUSS_OFFSETS, grid_coords, lognormal_K, lognormal_at, lognormal_features,
                     sample_jacobian, smooth_target, uniform_rhs)
from .maps import Affine, Identity, QuarterAnnulus, Star, conformal_square_to_disk
from .mesh import Mesh, lattice_mesh, mesh_points_for_grid

__all__ = ["Problem", "quarter_annulus", "star", "identity", "batch", "Affine", "Identity",
           "QuarterAnnulus", "Star", "conformal_square_to_disk", "sample_jacobian", "lognormal_K",
           "uniform_rhs", "smooth_target", "grid_coords", "GAUSS_OFFSETS", "Mesh", "lattice_mesh",
           "mesh_points_for_grid", "streams", "DmgProblem", "star_dmg", "unit_square_K",
           "discontinuous", "discontinuous_dmg", "DISCONTINUOUS"]


@dataclass
class Problem:
    name: str
    nx: int
    ny: int
    map: object
    jac: np.ndarray          # [16][ny-1][nx-1]
    K: np.ndarray            # [ny-1][nx-1]
    b: np.ndarray            # [ny][nx], zero boundary ring
    target: np.ndarray = None
    extra: dict = field(default_factory=dict)

    @property
    def dof(self) -> int:
        return (self.nx - 2) * (self.ny - 2)


def streams(root: int, n: int = 5):
    """Independent generators for (map, K, rhs, target, directions, ...)."""
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(root).spawn(n)]


def quarter_annulus(n: int, seed: int = 0, ny: int | None = None) -> Problem:
    ny = ny or n
    g_map, g_k, g_b, g_t, _ = streams(seed)
    mp = QuarterAnnulus()
    return Problem("quarter_annulus", n, ny, mp, sample_jacobian(mp, n, ny),
                   np.ones((ny - 1, n - 1)), uniform_rhs(n, ny, g_b), smooth_target(n, ny, g_t))


def identity(n: int, seed: int = 0, K: np.ndarray | None = None, ny: int | None = None) -> Problem:
    ny = ny or n
    _, _, g_b, g_t, _ = streams(seed)
    mp = Identity()
    K = np.ones((ny - 1, n - 1)) if K is None else K
    return Problem("identity", n, ny, mp, sample_jacobian(mp, n, ny), K, uniform_rhs(n, ny, g_b),
                   smooth_target(n, ny, g_t))


def star(n: int, seed: int = 1, ny: int | None = None, lognormal: bool = True,
         device: str | None = None) -> Problem:
    ny = ny or n
    g_map, g_k, g_b, g_t, _ = streams(seed)
    mp = Star.random(g_map)
    K = lognormal_K(mp, n, ny, g_k, device=device) if lognormal else np.ones((ny - 1, n - 1))
    return Problem("star", n, ny, mp, sample_jacobian(mp, n, ny), K, uniform_rhs(n, ny, g_b),
                   smooth_target(n, ny, g_t))


@dataclass
class DmgProblem:
    """A physical P1 problem on a mesh of a star domain with its logical grid (two-level method)."""
    grid: Problem            # the n x n grid problem of the same map and field (jac, K)
    mesh: Mesh               # physical mesh (vertices, their images in (-1,1)^2, triangles, dof)
    K_t: np.ndarray          # coefficient per triangle at its physical centroid
    f: np.ndarray            # right-hand side per vertex (0 on Dirichlet vertices)


def star_dmg(n: int, seed: int = 1, m: int | None = None, lognormal: bool = True) -> DmgProblem:
    """Star domain (map and K as star(n, seed)) with a jittered m x m P1 lattice mesh mapped
    through the same map (m about n / sqrt(0.28) by default, the paper's grid-to-mesh size
    ratio), K per triangle from the same log-normal field, f ~ U(-1, 1) on free vertices."""
    grid = star(n, seed=seed, lognormal=lognormal)
    g = streams(seed, 7)
    m = m or mesh_points_for_grid(n)
    mesh = lattice_mesh(grid.map, m, g[5])
    cen = mesh.xy_p[mesh.tris].mean(axis=1)
    if lognormal:
        omega, phase = lognormal_features(streams(seed)[1])
        K_t = lognormal_at(cen[:, 0], cen[:, 1], omega, phase)
    else:
        K_t = np.ones(mesh.tris.shape[0])
    f = np.where(mesh.dof, g[6].uniform(-1.0, 1.0, size=mesh.dof.shape[0]), 0.0)
    return DmgProblem(grid, mesh, K_t, f)


def directions(seed: int, count: int, n_cells: tuple, n_vert: tuple):
    """Finite-difference directions: z_K ~ N(0,1) per cell, z_b ~ N(0,1) per interior vertex."""
    g = streams(seed)[4]
    zK = g.normal(size=(count,) + tuple(n_cells))
    zb = g.normal(size=(count,) + tuple(n_vert))
    zb[:, 0, :] = zb[:, -1, :] = 0.0
    zb[:, :, 0] = zb[:, :, -1] = 0.0
    return zK, zb


def batch_sizes(count: int, choices=(129, 257, 513, 1025), seed: int = 3):
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed).spawn(count + 1)[-1]))
    return [int(c) for c in g.choice(np.asarray(choices), size=count)]


def batch(count: int, choices=(129, 257, 513, 1025), seed: int = 3, lognormal: bool = True,
          device: str | None = None):
    """``count`` independent star instances; instance k uses child seed k of the root."""
    sizes = batch_sizes(count, choices, seed)
    kids = np.random.SeedSequence(seed).spawn(count + 1)
    out = []
    for k, n in enumerate(sizes):
        g_map, g_k, g_b, g_t, _ = [np.random.Generator(np.random.PCG64(s)) for s in kids[k].spawn(5)]
        mp = Star.random(g_map)
        K = lognormal_K(mp, n, n, g_k, device=device) if lognormal else np.ones((n - 1, n - 1))
        out.append(Problem(f"star[{k}]", n, n, mp, sample_jacobian(mp, n, n), K,
                           uniform_rhs(n, n, g_b), None))
    return out


DISCONTINUOUS = ("circle", "checker", "layer")


def unit_square_K(kind: str, x, y) -> np.ndarray:
    """The discontinuous diffusivities of Sec. 4.1's variable-coefficient problems on the unit
    square, at physical points (x, y):
      circle : 100 inside the circle of radius 3/5 about the origin, 1 elsewhere;
      checker: 100 where floor(4x) + floor(4y) is even, 1 elsewhere (a 4 x 4 checkerboard);
      layer  : 1e-10 in the stripe 0 <= x < 0.06, 2 elsewhere."""
    x, y = np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64)
    if kind == "circle":
        return np.where(np.hypot(x, y) < 0.6, 100.0, 1.0)
    if kind == "checker":
        return np.where((np.floor(4 * x) + np.floor(4 * y)) % 2 == 0, 100.0, 1.0)
    if kind == "layer":
        return np.where((x >= 0.0) & (x < 0.06), 1e-10, 2.0)
    raise ValueError(f"unknown coefficient {kind!r}")


def _unit_square():
    # (-1, 1)^2 -> [0, 1]^2: the identity up to a uniform scaling, which leaves the pulled-back
    # operator of a scalar coefficient unchanged (D_c = K I)
    return Affine(0.5 * np.eye(2), np.array([0.5, 0.5]))


SUB = 16  # sub-samples per direction for cell and triangle averages of a discontinuous K


def discontinuous(kind: str, n: int, seed: int = 5, ny: int | None = None) -> Problem:
    """Unit square with the discontinuous diffusivity ``kind``, b ~ U(-1, 1).  A cell's K is the
    cell average of the diffusivity (a 16 x 16 midpoint rule): with the constant metric of this
    affine map, that is what a stiffness quadrature of high order in the coefficient computes,
    which is what a rapidly changing coefficient calls for.  (The grid is not aligned with the
    circle or the stripe; the checkerboard lines fall on grid lines when 4 divides n - 1.)"""
    ny = ny or n
    _, _, g_b, g_t, _ = streams(seed)
    mp = _unit_square()
    xi, eta = grid_coords(n, ny)
    hx, hy = xi[1] - xi[0], eta[1] - eta[0]
    K = np.zeros((ny - 1, n - 1))
    for qy in range(SUB):
        for qx in range(SUB):
            XX, YY = np.meshgrid(xi[:-1] + hx * (qx + 0.5) / SUB, eta[:-1] + hy * (qy + 0.5) / SUB)
            x, y = mp(XX, YY)
            K += unit_square_K(kind, x, y) / SUB ** 2
    return Problem(f"disc_{kind}", n, ny, mp, sample_jacobian(mp, n, ny), K,
                   uniform_rhs(n, ny, g_b), smooth_target(n, ny, g_t))


def triangle_average(kind: str, xy: np.ndarray) -> np.ndarray:
    """Average of unit_square_K over each triangle xy [nt][3][2]: the mean over the centroids of
    its 16 congruent sub-triangles (4 x 4 subdivision)."""
    out = np.zeros(xy.shape[0])
    s = 4
    cnt = 0
    for i in range(s):
        for j in range(s - i):
            # upward sub-triangle (i, j) and, where it exists, the downward one beside it
            cents = [((i + 1 / 3) / s, (j + 1 / 3) / s)]
            if i + j < s - 1:
                cents.append(((i + 2 / 3) / s, (j + 2 / 3) / s))
            for a, b in cents:
                p = xy[:, 0] + a * (xy[:, 1] - xy[:, 0]) + b * (xy[:, 2] - xy[:, 0])
                out += unit_square_K(kind, p[:, 0], p[:, 1])
                cnt += 1
    return out / cnt


def discontinuous_dmg(kind: str, n: int, seed: int = 5, m: int | None = None) -> DmgProblem:
    """The physical P1 problem of ``discontinuous(kind, n)``: a jittered lattice mesh of the unit
    square (about n^2 / 0.28 vertices; not aligned with the discontinuities), K per triangle its
    average over the triangle (triangle_average), f ~ U(-1, 1) on free vertices."""
    grid = discontinuous(kind, n, seed)
    g = streams(seed, 7)
    mesh = lattice_mesh(grid.map, m or mesh_points_for_grid(n), g[5])
    K_t = triangle_average(kind, mesh.xy_p[mesh.tris])
    f = np.where(mesh.dof, g[6].uniform(-1.0, 1.0, size=mesh.dof.shape[0]), 0.0)
    return DmgProblem(grid, mesh, K_t, f)
