"""Pins for the oracle's BoxMG pieces: operator-induced interpolation, Galerkin coarse operators,
coarsest solve, four-colour Gauss-Seidel V-cycle and the stationary solve.

Facts used: bilinear interpolation and the coarse Q1 stencil for the Laplacian (textbook);
hand-derived centre weights for a constant tensor with a mixed term; the defining property of the
operator-induced weights (the fine equation they were built from holds exactly); reproduction of
constants where rows sum to zero; agreement with a sparse direct solve; a convergence factor that
stays bounded as h -> 0 (Sec. 4.3 reports h-independent D-MG convergence); symmetry of the
V-cycle operator."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

import problems as pb
from oracle import boxmg, cycle, fem


def _S(prob):
    return fem.assemble_stencil(prob.jac, prob.K, prob.nx, prob.ny)


def _P_entry(P, nx, ncx, i, j, I, J):
    return P[j * nx + i, J * ncx + I]


def test_laplacian_interpolation_is_bilinear():
    n = 17
    S = _S(pb.identity(n))
    P = boxmg.interpolation(S)
    nc = 9
    # x-line point (5, 6): halves to (2,3) and (3,3); centre (5,7): quarters
    assert np.isclose(_P_entry(P, n, nc, 5, 6, 2, 3), 0.5, atol=1e-15)
    assert np.isclose(_P_entry(P, n, nc, 5, 6, 3, 3), 0.5, atol=1e-15)
    assert np.isclose(_P_entry(P, n, nc, 6, 5, 3, 2), 0.5, atol=1e-15)
    for I, J in ((2, 3), (3, 3), (2, 4), (3, 4)):
        assert np.isclose(_P_entry(P, n, nc, 5, 7, I, J), 0.25, atol=1e-15)
    assert np.isclose(_P_entry(P, n, nc, 6, 6, 3, 3), 1.0)
    # next to the boundary the weight toward the boundary coarse point vanishes
    assert _P_entry(P, n, nc, 1, 6, 0, 3) == 0.0 and np.isclose(_P_entry(P, n, nc, 1, 6, 1, 3), 0.5)
    # boundary fine rows are empty
    assert P[0].nnz == 0 and P[n - 1].nnz == 0


def test_mixed_tensor_centre_weights_closed_form():
    """Constant tensor [[a,b],[b,c]] (shear map, a=1.25, b=-0.5, c=1): line weights are 1/2 and
    the centre weights are 1/4 +- 3b/(8(a+c)) (derived by hand from the constant stencil)."""
    n = 17
    S = _S(pb.Problem("shear", n, n, None, pb.sample_jacobian(pb.Affine([[1.0, 0.5], [0.0, 1.0]]), n, n),
                      np.ones((n - 1, n - 1)), np.zeros((n, n))))
    P = boxmg.interpolation(S)
    a, b, c = 1.25, -0.5, 1.0
    d = 3 * b / (8 * (a + c))
    nc = 9
    i, j = 7, 9
    I0, J0 = 3, 4
    assert np.isclose(_P_entry(P, n, nc, i, j, I0, J0), 0.25 + d, atol=1e-14)          # SW
    assert np.isclose(_P_entry(P, n, nc, i, j, I0 + 1, J0), 0.25 - d, atol=1e-14)      # SE
    assert np.isclose(_P_entry(P, n, nc, i, j, I0, J0 + 1), 0.25 - d, atol=1e-14)      # NW
    assert np.isclose(_P_entry(P, n, nc, i, j, I0 + 1, J0 + 1), 0.25 + d, atol=1e-14)  # NE
    assert np.isclose(_P_entry(P, n, nc, 7, 8, 3, 4), 0.5, atol=1e-14)


@pytest.fixture(scope="module")
def star33():
    prob = pb.star(33, seed=1)
    return prob, _S(prob)


def test_centre_rows_of_AP_vanish(star33):
    """The centre weights are defined by the fine point's own equation: (A P)[centre, :] = 0."""
    prob, S = star33
    n = prob.nx
    A = fem.stencil_to_matrix(S)
    P = boxmg.interpolation(S)
    AP = (A @ P).toarray()
    j, i = np.meshgrid(np.arange(1, n - 1, 2), np.arange(1, n - 1, 2), indexing="ij")
    rows = (j * n + i).ravel()
    assert np.abs(AP[rows]).max() < 1e-13 * np.abs(AP).max()


def test_line_weights_satisfy_collapsed_equation(star33):
    prob, S = star33
    n = prob.nx
    st = boxmg.full_stencil(S)
    P = boxmg.interpolation(S)
    nc = (n + 1) // 2
    for j in range(2, n - 1, 2):
        for i in range(3, n - 3, 2):            # x-line points with interior coarse neighbours
            wW = _P_entry(P, n, nc, i, j, (i - 1) // 2, j // 2)
            wE = _P_entry(P, n, nc, i, j, (i + 1) // 2, j // 2)
            lhs = st["C"][j, i] + st["N"][j, i] + st["S"][j, i]
            # collapsed row: (C+N+S) u_f + (W+NW+SW) u_W + (E+NE+SE) u_E = 0 for u_f = wW u_W + wE u_E
            colW = st["W"][j, i] + st["NW"][j, i] + st["SW"][j, i]
            colE = st["E"][j, i] + st["NE"][j, i] + st["SE"][j, i]
            assert abs(lhs * wW + colW) < 1e-13 and abs(lhs * wE + colE) < 1e-13


def test_interpolation_reproduces_constants_where_rows_sum_to_zero(star33):
    prob, S = star33
    n = prob.nx
    P = boxmg.interpolation(S)
    ones = np.ones(P.shape[1])
    v = (P @ ones).reshape(n, n)
    assert np.allclose(v[3:-3, 3:-3], 1.0, atol=1e-13)


def test_galerkin_identity_gives_coarse_q1_at_every_level():
    levels = boxmg.build_hierarchy(_S(pb.identity(65)))
    assert [L.nx for L in levels] == [65, 33, 17, 9, 5, 3]
    for L in levels:
        S = L.S
        assert np.allclose(S[0][1:-1, 1:-1], 8 / 3, atol=1e-12)
        assert np.allclose(S[1][1:-1, 2:-1], -1 / 3, atol=1e-12)
        assert np.allclose(S[2][2:-1, 1:-1], -1 / 3, atol=1e-12)
        assert np.allclose(S[3][2:-1, 2:-1], -1 / 3, atol=1e-12)
        assert np.allclose(S[4][2:-1, 1:-2], -1 / 3, atol=1e-12)


def test_galerkin_storage_round_trip_and_structure(star33):
    prob, S = star33
    levels = boxmg.build_hierarchy(S)
    rng = np.random.default_rng(0)
    for f, c in zip(levels[:-1], levels[1:]):
        AH = fem.stencil_to_matrix(c.S)
        x, y = rng.normal(size=(2, c.nx * c.ny))
        lhs = x @ (AH @ y)
        rhs = (f.P @ x) @ (f.A @ (f.P @ y))
        assert abs(lhs - rhs) < 1e-12 * abs(rhs)
        assert abs(AH - AH.T).max() < 1e-13 * abs(AH).max()
        nnz_row = np.diff(AH.tocsr().indptr)
        assert nnz_row.max() <= 9
        rs = np.asarray(AH.sum(axis=1)).reshape(c.ny, c.nx)
        assert np.allclose(rs[2:-2, 2:-2], 0.0, atol=1e-11 * abs(AH).max())


def test_coarsest_solve_matches_dense_solve():
    levels = boxmg.build_hierarchy(_S(pb.star(33, seed=1)), coarsest_n=9)
    orc = cycle.Oracle(levels)
    last = levels[-1]
    rng = np.random.default_rng(1)
    b = np.zeros(last.nx * last.ny)
    idx = orc.coarse_idx
    b[idx] = rng.normal(size=idx.size)
    u = orc.coarse_solve(b)
    Ad = last.A.toarray()[np.ix_(idx, idx)]
    assert np.allclose(u[idx], np.linalg.solve(Ad, b[idx]), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("maker,n", [(lambda n: pb.star(n, seed=1), 129),
                                     (lambda n: pb.quarter_annulus(n), 65),
                                     (lambda n: pb.identity(n), 65)])
def test_solve_matches_sparse_direct_solve(maker, n):
    prob = maker(n)
    levels = boxmg.build_hierarchy(_S(prob))
    orc = cycle.Oracle(levels)
    u, k, hist, _ = cycle.solve(orc, prob.b, rtol=1e-10)
    assert hist[-1] <= 1e-10
    m = np.zeros((n, n), bool)
    m[1:-1, 1:-1] = True
    A = levels[0].A.tocsr()
    x = spl.spsolve(A[m.ravel()][:, m.ravel()].tocsc(), prob.b[m])
    assert np.linalg.norm(u[m] - x) / np.linalg.norm(x) < 1e-7


@pytest.mark.parametrize("maker,bound", [(lambda n: pb.star(n, seed=1), 0.2),
                                         (lambda n: pb.identity(n), 0.15),
                                         (lambda n: pb.quarter_annulus(n), 0.72)])
def test_convergence_factor_bounded_as_h_shrinks(maker, bound):
    rhos = []
    for n in (33, 65, 129, 257):
        prob = maker(n)
        orc = cycle.Oracle(boxmg.build_hierarchy(_S(prob)))
        _, k, hist, _ = cycle.solve(orc, prob.b, rtol=1e-10)
        rhos.append(cycle.convergence_factor(hist))
    assert max(rhos) < bound, rhos
    assert rhos[-1] < rhos[-2] + 0.05, rhos


def test_vcycle_operator_is_symmetric(star33):
    """With pre order 0,1,2,3, post order 3,2,1,0 and R = P^T, b -> V(0, b) is symmetric."""
    prob, S = star33
    orc = cycle.Oracle(boxmg.build_hierarchy(S))
    rng = np.random.default_rng(2)
    n = prob.nx
    b1, b2 = np.zeros((2, n * n))
    m = np.zeros((n, n), bool)
    m[1:-1, 1:-1] = True
    b1[m.ravel()], b2[m.ravel()] = rng.normal(size=(2, m.sum()))
    v1 = orc.vcycle(np.zeros(n * n), b1.copy())
    v2 = orc.vcycle(np.zeros(n * n), b2.copy())
    assert abs(v1 @ b2 - b1 @ v2) < 1e-13 * abs(v1 @ b2)
    # a same-order post-smoother breaks the symmetry (sanity check of the check)
    orc2 = cycle.Oracle(boxmg.build_hierarchy(S), post=(0, 1, 2, 3))
    w1 = orc2.vcycle(np.zeros(n * n), b1.copy())
    w2 = orc2.vcycle(np.zeros(n * n), b2.copy())
    assert abs(w1 @ b2 - b1 @ w2) > 1e-6 * abs(w1 @ b2)


def test_rectangular_grid_and_general_coarsest():
    prob = pb.star(33, seed=1, ny=65)
    levels = boxmg.build_hierarchy(_S(prob))
    assert [(L.nx, L.ny) for L in levels] == [(33, 65), (17, 33), (9, 17), (5, 9), (3, 5)]
    orc = cycle.Oracle(levels)
    assert orc.coarse_idx.size == 3
    u, k, hist, _ = cycle.solve(orc, prob.b, rtol=1e-10)
    # 2:1 cell aspect ratio makes the operator anisotropic; point smoothing slows down but converges
    assert hist[-1] <= 1e-10 and cycle.convergence_factor(hist) < 0.6


def test_complexities_are_bounded():
    levels = boxmg.build_hierarchy(_S(pb.star(129, seed=1)))
    gc, oc = boxmg.complexities(levels)
    assert 1.0 < gc < 4.0 / 3.0 + 1e-12 and 1.0 < oc < 1.4


def test_odd_dims_coarsen_until_a_dim_turns_even():
    """Dims of the form c 2^k + 1 (c odd): 25 = 3 * 8 + 1 stops at 4; the identity map still
    gives the coarse Q1 stencil at every level (2:1 coarsening with aligned boundaries), and the
    solve equals a sparse direct solve on a grid with the paper's 1.5 aspect ratio."""
    levels = boxmg.build_hierarchy(_S(pb.identity(25)))
    assert [L.nx for L in levels] == [25, 13, 7, 4]
    for L in levels[:-1]:
        S = L.S
        assert np.allclose(S[0][1:-1, 1:-1], 8 / 3, atol=1e-12)
        assert np.allclose(S[1][1:-1, 2:-1], -1 / 3, atol=1e-12)
        assert np.allclose(S[3][2:-1, 2:-1], -1 / 3, atol=1e-12)
    # the coarsest 4 x 4 level (2 x 2 unknowns) is the Galerkin product, solved directly
    assert np.allclose(levels[-1].S[0][1:-1, 1:-1], 8 / 3, atol=1e-12)
    prob = pb.quarter_annulus(33, ny=49)
    levels = boxmg.build_hierarchy(_S(prob))
    assert [(L.nx, L.ny) for L in levels] == [(33, 49), (17, 25), (9, 13), (5, 7), (3, 4)]
    orc = cycle.Oracle(levels)
    u, k, hist, _ = cycle.solve(orc, prob.b, rtol=1e-10)
    m = np.zeros((49, 33), bool)
    m[1:-1, 1:-1] = True
    A = levels[0].A.tocsr()
    x = spl.spsolve(A[m.ravel()][:, m.ravel()].tocsc(), prob.b[m])
    assert hist[-1] <= 1e-10 and np.linalg.norm(u[m] - x) / np.linalg.norm(x) < 1e-7
    # 45 x 67: 67 -> 34 turns even after one coarsening; the 23 x 34 coarsest is solved directly
    levels = boxmg.build_hierarchy(_S(pb.star(45, seed=1, ny=67)))
    assert [(L.nx, L.ny) for L in levels] == [(45, 67), (23, 34)]
