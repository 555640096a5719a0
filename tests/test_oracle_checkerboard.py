"""The 4 x 4 checkerboard diffusivity (100 : 1, Sec. 4.1's discontinuous checkerboard problem on
the identity map): what the BoxMG hierarchy of this library does there, pinned.

* Every level's own two-grid cycle (its operator, point smoothing, exact solve on the Galerkin
  level below) contracts the energy norm by at most 0.35 per cycle, at every level: the
  operator-induced interpolation and the Galerkin products work at each scale.
* The V-cycle compounds the levels' corrections.  Its slowest mode is the cross-point mode of
  the checkerboard (about constant on two diagonally touching high-K squares, decaying into the
  low-K ones): near a cross point the solution varies like r^alpha with small alpha, so it has
  structure on every level.  The V-cycle rate still stays bounded as h shrinks: it stays below
  0.75 from 65^2 to 257^2 and each refinement adds less than the one before."""
import numpy as np
import pytest

import problems as pb
from oracle import boxmg, cycle, fem


def _levels(n):
    p = pb.discontinuous("checker", n)
    return p, boxmg.build_hierarchy(fem.assemble_stencil(p.jac, p.K, n, n))


def _vcycle_rate(n):
    p, L = _levels(n)
    _, _, hist, _ = cycle.solve(cycle.Oracle(L), p.b, 1e-10, max_iters=30)
    return cycle.convergence_factor(hist, skip=3)


def test_each_level_two_grid_contracts():
    _, L = _levels(65)
    rng = np.random.default_rng(0)
    for l in range(len(L) - 2):
        o = cycle.Oracle([L[l], boxmg.Level(L[l + 1].S)])
        m = o.levels[0].masks
        inner = m[0] | m[1] | m[2] | m[3]
        u = np.where(inner, rng.uniform(-1, 1, L[l].nx * L[l].ny), 0.0)
        A = L[l].A
        e = []
        for _ in range(12):
            o.vcycle(u, np.zeros_like(u))
            e.append(np.sqrt(u @ (A @ u)))
        rate = (e[-1] / e[2]) ** (1 / 9)
        assert rate <= 0.35, (l, L[l].nx, rate)


def test_vcycle_rate_bounded_with_shrinking_increments():
    r = [_vcycle_rate(n) for n in (65, 129, 257)]
    assert max(r) <= 0.75, r
    assert r[0] < r[1] < r[2] and (r[2] - r[1]) < (r[1] - r[0]), r


def test_smooth_coefficients_converge_fast_on_the_same_grid():
    """Contrast 1 (the same grid, K = 1 everywhere): the usual rate, so the slowdown above is the
    coefficients', not the grid's or the smoother's."""
    n = 65
    p = pb.identity(n)
    L = boxmg.build_hierarchy(fem.assemble_stencil(p.jac, p.K, n, n))
    _, _, hist, _ = cycle.solve(cycle.Oracle(L), p.b, 1e-10, max_iters=30)
    assert cycle.convergence_factor(hist, skip=3) <= 0.15
