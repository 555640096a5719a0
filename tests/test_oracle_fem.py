"""Pins for the oracle's discretisation (metric tensor, element matrices, stencil assembly).

Each check compares with a fact fixed outside the oracle: textbook Q1 stencils, closed forms
derived by hand for constant tensors and for the quarter annulus of Sec. 4.1, convergence to an
analytic solution, and annihilation of physically harmonic functions."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spl

import problems as pb
from oracle import fem


def _stencil(mp, n, K=None):
    jac = pb.sample_jacobian(mp, n, n)
    K = np.ones((n - 1, n - 1)) if K is None else K
    return fem.assemble_stencil(jac, K, n, n)


def _interior(v, k=2):
    return v[k:-k, k:-k]


def test_identity_map_gives_textbook_q1_laplacian():
    S = _stencil(pb.Identity(), 9)
    assert np.allclose(_interior(S[0], 1), 8.0 / 3.0, atol=1e-14)
    for k in (1, 2, 3, 4):
        assert np.allclose(_interior(S[k]), -1.0 / 3.0, atol=1e-14)
    # boundary rows and couplings into the boundary are zero
    assert not S[:, 0, :].any() and not S[:, :, 0].any() and not S[:, -1, :].any() and not S[:, :, -1].any()
    assert not S[1, :, 1].any() and not S[2, 1, :].any()


def _constant_tensor_stencil(a, b, c):
    """Q1 stiffness stencil of -div([[a,b],[b,c]] grad u) on a uniform square grid (hand-derived
    from the unit-square element matrices; h cancels in 2D)."""
    return dict(C=4 * (a + c) / 3, W=-2 * a / 3 + c / 3, S=a / 3 - 2 * c / 3,
                SW=-(a + c) / 6 - b / 2, SE=-(a + c) / 6 + b / 2)


@pytest.mark.parametrize("A,abc", [
    ([[2.0, 0.0], [0.0, 1.0]], (0.5, 0.0, 2.0)),         # det 2 * diag(1/4, 1)
    ([[1.0, 0.5], [0.0, 1.0]], (1.25, -0.5, 1.0)),       # shear: A^-1 A^-T = [[1.25,-.5],[-.5,1]]
    ([[0.6, -0.8], [0.8, 0.6]], (1.0, 0.0, 1.0)),        # rotation: conformal -> identity tensor
])
def test_affine_map_gives_constant_tensor_stencil(A, abc):
    S = _stencil(pb.Affine(A), 9)
    ref = _constant_tensor_stencil(*abc)
    for k, name in enumerate(("C", "W", "S", "SW", "SE")):
        assert np.allclose(_interior(S[k]), ref[name], atol=1e-13), name


def test_quarter_annulus_metric_closed_form():
    """For the quarter annulus, D_c = diag(pi r, 1/(pi r)) in (xi, eta), r = 1/2 + (xi+1)/4."""
    mp = pb.QuarterAnnulus()
    rng = np.random.default_rng(0)
    xi, eta = rng.uniform(-1, 1, size=(2, 100))
    M11, M12, M22 = fem.metric_tensor(*mp.jacobian(xi, eta))
    r = 0.5 + (xi + 1) / 4
    assert np.allclose(M11, np.pi * r, rtol=1e-14)
    assert np.allclose(M22, 1 / (np.pi * r), rtol=1e-14)
    assert np.allclose(M12, 0.0, atol=1e-14)


def test_assembled_matrix_symmetric_zero_rowsum_positive_diagonal():
    prob = pb.star(33, seed=1)
    G = fem.element_matrices(prob.jac, 33, 33)
    assert np.allclose(G, np.swapaxes(G, -1, -2), atol=1e-14)
    assert np.allclose(G.sum(-1), 0.0, atol=1e-12)              # constants are in the kernel
    A = fem.assemble_matrix(G, prob.K, 33, 33)
    assert abs(A - A.T).max() < 1e-13
    S = fem.matrix_to_stencil_fast(A, 33, 33)
    assert np.all(_interior(S[0], 1) > 0)
    Af = fem.stencil_to_matrix(S)
    assert abs(Af - A).max() < 1e-14                           # 5-value storage is lossless
    rs = np.asarray(A.sum(axis=1)).reshape(33, 33)
    assert np.allclose(_interior(rs), 0.0, atol=1e-11)


def _annulus_load(n, alpha=math.pi / 2, nq=5):
    """b_i = int f phi_i dxi for the pulled-back annulus problem with exact solution
    u = sin(alpha(xi+1)) sin(alpha(eta+1)):  f = -[(pi/4) u_xi + pi r u_xixi + u_etaeta/(pi r)]."""
    xs, ws = np.polynomial.legendre.leggauss(nq)
    xs, ws = 0.5 * (xs + 1), 0.5 * ws
    h = 2.0 / (n - 1)
    b = np.zeros((n, n))
    for qy in range(nq):
        for qx in range(nq):
            s, t = xs[qx], xs[qy]
            XI = -1 + (np.arange(n - 1) + s) * h
            ETA = -1 + (np.arange(n - 1) + t) * h
            X, E = np.meshgrid(XI, ETA)
            r = 0.5 + (X + 1) / 4
            u = np.sin(alpha * (X + 1)) * np.sin(alpha * (E + 1))
            ux = alpha * np.cos(alpha * (X + 1)) * np.sin(alpha * (E + 1))
            f = -((np.pi / 4) * ux + np.pi * r * (-alpha ** 2 * u) + (-alpha ** 2 * u) / (np.pi * r))
            w = ws[qx] * ws[qy] * h * h * f
            b[:-1, :-1] += w * (1 - s) * (1 - t)
            b[:-1, 1:] += w * s * (1 - t)
            b[1:, :-1] += w * (1 - s) * t
            b[1:, 1:] += w * s * t
    return b


def test_quarter_annulus_second_order_convergence():
    errs = []
    for n in (17, 33, 65):
        S = _stencil(pb.QuarterAnnulus(), n)
        A = fem.stencil_to_matrix(S).tocsr()
        m = np.zeros((n, n), bool)
        m[1:-1, 1:-1] = True
        m = m.ravel()
        b = _annulus_load(n).ravel()
        x = spl.spsolve(A[m][:, m].tocsc(), b[m])
        xi, eta = pb.grid_coords(n, n)
        X, E = np.meshgrid(xi, eta)
        ue = (np.sin(np.pi / 2 * (X + 1)) * np.sin(np.pi / 2 * (E + 1))).ravel()[m]
        errs.append(np.max(np.abs(x - ue)))
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(orders) > 1.9, (errs, orders)


def test_star_map_annihilates_physical_harmonics():
    """x and y are harmonic on the physical domain, so the pulled-back operator applied to the
    map's own coordinates vanishes up to the O(h^4) consistency error (away from the conformal
    map's corner singularities).  A transposed or unscaled metric leaves an O(h^2) residual."""
    mp = pb.Star.random(pb.streams(1)[0])
    scaled = []
    for n in (65, 129, 257):
        A = fem.stencil_to_matrix(_stencil(mp, n))
        xi, eta = pb.grid_coords(n, n)
        X, E = np.meshgrid(xi, eta)
        q = n // 8
        worst = 0.0
        for comp in mp(X, E):
            r = (A @ comp.ravel()).reshape(n, n)[q:-q, q:-q]
            worst = max(worst, np.abs(r).max() * n * n)
        scaled.append(worst)
    assert scaled[-1] < 2e-3
    assert scaled[0] / scaled[1] > 3.0 and scaled[1] / scaled[2] > 3.0
