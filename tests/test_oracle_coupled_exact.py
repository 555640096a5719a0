"""Pins of the exact coupled mass (oracle/transfer.py, coupled_mass_exact) against closed forms:
integrals of monomials over a triangle, s^p t^q over the reference triangle = p! q! / (p+q+2)!,
and of products of barycentric coordinates, l^alpha over T = 2|T| alpha! / (|alpha| + 2)!;
bilinear interpolation on the grid reproduces 1, X, Y and XY, so the column moments of C are
integrals of lambda_a times those; the Jacobian factor scales C; the rasterised rule of Sec. 2.3.1
converges to it as its order grows."""
from math import factorial as fact

import numpy as np

import problems as pb
from oracle import transfer


def _ref_monomial(p, q):
    return fact(p) * fact(q) / fact(p + q + 2)


def _poly_integral(c):
    """Integral over the reference triangle of sum c[p, q] s^p t^q."""
    return sum(c[p, q] * _ref_monomial(p, q) for p in range(c.shape[0]) for q in range(c.shape[1]))


def _mul(a, b):
    out = np.zeros((a.shape[0] + b.shape[0] - 1, a.shape[1] + b.shape[1] - 1))
    for p in range(a.shape[0]):
        for q in range(a.shape[1]):
            out[p:p + b.shape[0], q:q + b.shape[1]] += a[p, q] * b
    return out


def test_single_cell_half_matches_monomial_integrals():
    # grid 3 x 3 on [-1, 1]^2 (h = 1); the triangle is the lower-left half of cell (0, 0), so in
    # cell coordinates s = X + 1, t = Y + 1 it is the reference triangle
    xy = np.array([[-1.0, -1.0], [0.0, -1.0], [-1.0, 0.0]])
    tris = np.array([[0, 1, 2]])
    dof = np.ones(3, dtype=bool)
    C = transfer.coupled_mass_exact(xy, xy, tris, dof, 3, 3, drop_grid_boundary=False).toarray()
    one, s, t = np.zeros((2, 2)), np.zeros((2, 2)), np.zeros((2, 2))
    one[0, 0], s[1, 0], t[0, 1] = 1.0, 1.0, 1.0
    lam = [one - s - t, s, t]
    phi = {0: _mul(one - s, one - t), 1: _mul(s, one - t), 3: _mul(one - s, t), 4: _mul(s, t)}
    for a in range(3):
        for g in range(9):
            want = _poly_integral(_mul(lam[a], phi[g])) if g in phi else 0.0
            assert abs(C[a, g] - want) <= 1e-15, (a, g, C[a, g], want)
    # the physical triangle three times larger: |J| = 9 scales every entry
    C9 = transfer.coupled_mass_exact(xy, 3.0 * xy, tris, dof, 3, 3, drop_grid_boundary=False).toarray()
    assert np.allclose(C9, 9.0 * C, rtol=1e-14, atol=0)


def test_multi_cell_triangle_moments():
    n = 5
    xy = np.array([[-0.9, -0.8], [0.7, -0.3], [-0.2, 0.85]])
    tris = np.array([[0, 1, 2]])
    C = transfer.coupled_mass_exact(xy, xy, tris, np.ones(3, dtype=bool), n, n,
                                    drop_grid_boundary=False).toarray()
    g = np.linspace(-1.0, 1.0, n)
    GX, GY = np.meshgrid(g, g)
    X, Y = xy[:, 0], xy[:, 1]
    area = 0.5 * abs((X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]))

    def bary(alpha):   # integral of l0^a0 l1^a1 l2^a2 over the triangle
        return 2 * area * np.prod([fact(k) for k in alpha]) / fact(sum(alpha) + 2)

    for a in range(3):
        e = lambda *idx: tuple(sum(1 for k in idx if k == b) for b in range(3))
        m1 = bary(e(a))
        mx = sum(X[b] * bary(e(a, b)) for b in range(3))
        my = sum(Y[b] * bary(e(a, b)) for b in range(3))
        mxy = sum(X[b] * Y[c] * bary(e(a, b, c)) for b in range(3) for c in range(3))
        row = C[a]
        assert abs(row.sum() - m1) <= 1e-15
        assert abs(row @ GX.ravel() - mx) <= 1e-15
        assert abs(row @ GY.ravel() - my) <= 1e-15
        assert abs(row @ (GX * GY).ravel() - mxy) <= 1e-15
    assert abs(C.sum() - area) <= 1e-15


def test_rasterised_rule_converges_to_exact():
    n = 9
    mesh = pb.lattice_mesh(pb.Star.random(pb.streams(4)[0]), 14, np.random.default_rng(4))
    ex = transfer.coupled_mass(mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, n, n, nq=0)
    errs = []
    for nq in (4, 8, 16, 32):
        C = transfer.coupled_mass(mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, n, n, nq=nq)
        errs.append(abs(C - ex).max() / abs(ex).max())
    assert errs[-1] < 0.02 and errs[-1] < errs[1] < errs[0]
