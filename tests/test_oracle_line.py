"""Pins of the line-relaxation smoother of the oracle (oracle/cycle.py): exactness on operators
coupled along one direction only, agreement of the solve with a sparse direct solve, symmetry
of the V-cycle, and the convergence behaviour line relaxation exists for (a strongly
anisotropic operator that point smoothing cannot reduce)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

import problems as pb
from oracle import boxmg, cycle, fem


def _S(prob):
    return fem.assemble_stencil(prob.jac, prob.K, prob.nx, prob.ny)


def _one_direction_stencil(n, direction):
    """A 5-plane stencil with couplings along one grid direction only (a stack of independent
    1-D tridiagonal problems): C = 2 + a small shift, the one neighbour coupling -1."""
    S = np.zeros((5, n, n))
    S[0, 1:-1, 1:-1] = 2.5
    if direction == "x":
        S[1, 1:-1, 2:-1] = -1.0     # W coupling, none into the boundary column
    else:
        S[2, 2:-1, 1:-1] = -1.0     # S coupling, none into the boundary row
    return S


@pytest.mark.parametrize("direction", ["x", "y"])
def test_one_line_sweep_solves_a_one_direction_operator(direction):
    n = 17
    levels = boxmg.build_hierarchy(_one_direction_stencil(n, direction))
    orc = cycle.Oracle(levels, smoother="xline" if direction == "x" else "yline")
    rng = np.random.default_rng(1)
    b = np.zeros(n * n)
    m = np.zeros((n, n), bool)
    m[1:-1, 1:-1] = True
    b[m.ravel()] = rng.uniform(-1, 1, m.sum())
    u = np.zeros(n * n)
    for parity in (0, 1):
        orc.line_smooth(0, u, b, direction, parity)
    assert np.abs(orc.residual(0, u, b)).max() < 1e-14
    # a sweep across the coupling direction is a point Jacobi-like update and does not solve it
    other = "y" if direction == "x" else "x"
    w = np.zeros(n * n)
    for parity in (0, 1):
        orc.line_smooth(0, w, b, other, parity)
    assert np.abs(orc.residual(0, w, b)).max() > 1e-3


@pytest.mark.parametrize("smoother", ["xline", "yline", "alt"])
def test_line_smoothed_solve_matches_direct_solve(smoother):
    prob = pb.star(33, seed=2)
    levels = boxmg.build_hierarchy(_S(prob))
    orc = cycle.Oracle(levels, smoother=smoother)
    u, k, hist, _ = cycle.solve(orc, prob.b, rtol=1e-10)
    m = np.zeros((33, 33), bool)
    m[1:-1, 1:-1] = True
    A = levels[0].A.tocsr()
    x = spl.spsolve(A[m.ravel()][:, m.ravel()].tocsc(), prob.b[m])
    assert hist[-1] <= 1e-10 and np.linalg.norm(u[m] - x) / np.linalg.norm(x) < 1e-7


def test_line_smoothed_vcycle_is_symmetric():
    prob = pb.quarter_annulus(33)
    orc = cycle.Oracle(boxmg.build_hierarchy(_S(prob)), smoother="alt")
    rng = np.random.default_rng(3)
    n = 33
    m = np.zeros((n, n), bool)
    m[1:-1, 1:-1] = True
    b1, b2 = np.zeros((2, n * n))
    b1[m.ravel()], b2[m.ravel()] = rng.normal(size=(2, m.sum()))
    v1 = orc.vcycle(np.zeros(n * n), b1.copy())
    v2 = orc.vcycle(np.zeros(n * n), b2.copy())
    assert abs(v1 @ b2 - b1 @ v2) < 1e-13 * abs(v1 @ b2)


def test_line_relaxation_handles_anisotropy():
    """The quarter annulus pulls back to D_c = diag(pi r, 1/(pi r)): coupling along x is up to
    10x the coupling along y.  Point smoothing converges at ~0.65 per cycle; x-line relaxation
    (the strong direction) and alternating lines converge fast, y-lines (the weak one) do not
    help."""
    prob = pb.quarter_annulus(65)
    S = _S(prob)
    rate = {}
    for sm in ("point", "xline", "yline", "alt"):
        orc = cycle.Oracle(boxmg.build_hierarchy(S), smoother=sm)
        _, k, hist, _ = cycle.solve(orc, prob.b, rtol=1e-10, max_iters=200)
        rate[sm] = cycle.convergence_factor(hist)
    assert rate["point"] > 0.6 and rate["yline"] > 0.6
    assert rate["xline"] < 0.2 and rate["alt"] < 0.05
