"""Invariants of the seeded input generators (maps, fields, meshes).

The generators are project-defined inputs; beyond these invariants their values are
"parity unpinned" by construction (there is nothing in the paper to compare them with)."""
import math

import numpy as np
import pytest

import problems as pb
from problems.maps import CONFORMAL_A


def _fd_jacobian(mp, xi, eta, h=1e-6):
    xp, yp = mp(xi + h, eta)
    xm, ym = mp(xi - h, eta)
    xq, yq = mp(xi, eta + h)
    xr, yr = mp(xi, eta - h)
    return (xp - xm) / (2 * h), (xq - xr) / (2 * h), (yp - ym) / (2 * h), (yq - yr) / (2 * h)


MAPS = [pb.Identity(), pb.Affine([[1.0, 0.5], [0.0, 1.0]]), pb.QuarterAnnulus(),
        pb.Star.random(pb.streams(1)[0])]


@pytest.mark.parametrize("mp", MAPS, ids=lambda m: m.name)
def test_jacobian_matches_finite_differences(mp):
    rng = np.random.default_rng(0)
    xi, eta = rng.uniform(-0.95, 0.95, size=(2, 200))
    J = mp.jacobian(xi, eta)
    F = _fd_jacobian(mp, xi, eta)
    for a, b in zip(J, F):
        assert np.max(np.abs(a - b)) < 1e-7
    det = J[0] * J[3] - J[1] * J[2]
    assert np.all(det > 0)


def test_conformal_constant_is_F_of_one():
    from scipy.integrate import quad
    val = quad(lambda t: 1.0 / math.sqrt(1.0 + t ** 4), 0.0, 1.0, epsabs=1e-14)[0]
    assert abs(val - CONFORMAL_A) < 1e-13


def test_conformal_map_boundary_and_conformality():
    t = np.linspace(-1, 1, 101)
    for xi, eta in ((t, np.ones_like(t)), (t, -np.ones_like(t)), (np.ones_like(t), t), (-np.ones_like(t), t)):
        w, _ = pb.conformal_square_to_disk(xi, eta)
        assert np.allclose(np.abs(w), 1.0, atol=1e-12)
    rng = np.random.default_rng(1)
    xi, eta = rng.uniform(-0.9, 0.9, size=(2, 100))
    w, dw = pb.conformal_square_to_disk(xi, eta)
    assert np.all(np.abs(w) < 1.0)
    # Cauchy-Riemann: the real 2x2 derivative is a scaled rotation equal to dw
    h = 1e-6
    wx = (pb.conformal_square_to_disk(xi + h, eta)[0] - pb.conformal_square_to_disk(xi - h, eta)[0]) / (2 * h)
    wy = (pb.conformal_square_to_disk(xi, eta + h)[0] - pb.conformal_square_to_disk(xi, eta - h)[0]) / (2 * h)
    assert np.allclose(wx, dw, atol=1e-7)
    assert np.allclose(wy, 1j * dw, atol=1e-7)
    # symmetry of the square: w(-z) = -w(z), w(i z) = i w(z)
    assert np.allclose(pb.conformal_square_to_disk(-xi, -eta)[0], -w, atol=1e-13)
    assert np.allclose(pb.conformal_square_to_disk(-eta, xi)[0], 1j * w, atol=1e-13)


def test_star_boundary_radius():
    mp = pb.Star.random(pb.streams(1)[0])
    t = np.linspace(-1, 1, 57)
    xi, eta = t, np.ones_like(t)
    x, y = mp(xi, eta)
    w, _ = pb.conformal_square_to_disk(xi, eta)
    assert np.allclose(np.hypot(x, y), mp.boundary_radius(np.angle(w)), atol=1e-12)
    assert np.all(mp.a <= 0.05 / np.arange(1, 9) + 1e-15)


def test_quarter_annulus_matches_paper_T():
    """The map inverts T(x,y) = (2(|x| - 1/2)/(1/2) - 1, (4/pi) atan2(y,x) - 3) (Sec. 4.1)."""
    mp = pb.QuarterAnnulus()
    rng = np.random.default_rng(2)
    xi, eta = rng.uniform(-1, 1, size=(2, 50))
    x, y = mp(xi, eta)
    T1 = 2 * (np.hypot(x, y) - 0.5) / 0.5 - 1
    T2 = 4 / np.pi * np.arctan2(y, x) - 3
    assert np.allclose(T1, xi, atol=1e-13) and np.allclose(T2, eta, atol=1e-13)


def test_jacobian_sampling_layout():
    mp = pb.QuarterAnnulus()
    n = 9
    jac = pb.sample_jacobian(mp, n, n)
    assert jac.shape == (16, n - 1, n - 1)
    xi, eta = pb.grid_coords(n, n)
    h = xi[1] - xi[0]
    j, i, q = 3, 5, 2                      # q = qx + 2 qy -> qx = 0, qy = 1
    J = mp.jacobian(xi[i] + h * pb.GAUSS_OFFSETS[0], eta[j] + h * pb.GAUSS_OFFSETS[1])
    assert np.allclose([jac[4 * q + e, j, i] for e in range(4)], J)


def test_lognormal_K_statistics():
    mp = pb.Star.random(pb.streams(1)[0])
    K = pb.lognormal_K(mp, 129, 129, pb.streams(1)[1])
    g = np.log(K)
    assert K.shape == (128, 128) and np.all(K > 0)
    assert abs(g.mean()) < 0.6 and 0.5 < g.std() < 1.5


def test_rhs_and_target_vanish_on_boundary():
    b = pb.uniform_rhs(17, 33, pb.streams(0)[2])
    t = pb.smooth_target(17, 33, pb.streams(0)[3])
    for v in (b, t):
        assert v.shape == (33, 17)
        assert not v[0].any() and not v[-1].any() and not v[:, 0].any() and not v[:, -1].any()
    assert np.all(np.abs(b) <= 1.0)


def test_lattice_mesh_is_valid():
    mp = pb.Star.random(pb.streams(1)[0])
    mesh = pb.lattice_mesh(mp, 21, np.random.default_rng(3))
    assert mesh.nv == 441 and mesh.nt == 2 * 400
    assert mesh.dof.sum() == 19 * 19
    # every vertex's computational image is in the closed square; boundary vertices on its edge
    assert np.all(np.abs(mesh.xy_c) <= 1.0)
    edge = np.any(np.isclose(np.abs(mesh.xy_c), 1.0), axis=1)
    assert np.array_equal(edge, ~mesh.dof)


def test_batch_sizes_are_seeded():
    s1 = pb.batch_sizes(256)
    assert s1 == pb.batch_sizes(256)
    assert set(s1) <= {129, 257, 513, 1025} and len(set(s1)) == 4


def test_device_batch_reproduces_host_batch():
    """The device path of the star batch draws the same instances as problems.batch."""
    import torch

    from problems.batch_device import star_batch_device

    host = pb.batch(3, choices=(17, 33), seed=5)
    dev = list(star_batch_device(3, choices=(17, 33), seed=5, device="cpu"))
    for p, (n, jac, K, b) in zip(host, dev):
        assert n == p.nx
        assert np.allclose(jac.numpy(), p.jac, rtol=1e-13, atol=1e-14)
        assert np.allclose(K.numpy(), p.K, rtol=1e-12)
        assert np.array_equal(b.numpy(), p.b)


def test_device_star_and_patches_reproduce_host_star():
    """star_device and the patch samplers draw the inputs of problems.star."""
    import torch  # noqa: F401

    from problems.batch_device import star_device
    from problems.fields import lognormal_K_patch, sample_jacobian_patch

    p = pb.star(33, seed=3)
    jac, K, b = star_device(33, seed=3, device="cpu")
    assert np.allclose(jac.numpy(), p.jac, rtol=1e-13, atol=1e-14)
    assert np.allclose(K.numpy(), p.K, rtol=1e-12)
    assert np.array_equal(b.numpy(), p.b)
    assert np.allclose(sample_jacobian_patch(p.map, 33, 6, 10, 8), p.jac[:, 10:18, 6:14], rtol=1e-14, atol=1e-15)
    Kp = lognormal_K_patch(p.map, 33, 6, 10, 8, pb.streams(3)[1])
    assert np.allclose(Kp, p.K[10:18, 6:14], rtol=1e-12)


def test_device_star_dmg_reproduces_host_star_dmg():
    """star_dmg_device draws the inputs of problems.star_dmg (fields evaluated with torch)."""
    from problems.batch_device import star_dmg_device
    P = pb.star_dmg(17, seed=2)
    jac, K, mesh, K_t, f = star_dmg_device(17, seed=2, device="cpu")
    assert np.array_equal(mesh.tris, P.mesh.tris) and np.array_equal(mesh.dof, P.mesh.dof)
    assert np.array_equal(mesh.xy_c, P.mesh.xy_c) and np.array_equal(mesh.xy_p, P.mesh.xy_p)
    assert np.array_equal(f, P.f)
    assert np.allclose(K_t, P.K_t, rtol=1e-12, atol=0)
    assert np.allclose(jac.numpy(), P.grid.jac, rtol=1e-12, atol=1e-14)
    assert np.allclose(K.numpy(), P.grid.K, rtol=1e-12, atol=0)


def test_discontinuous_coefficients():
    """The unit-square problems: the map is the uniform scaling (-1, 1)^2 -> [0, 1]^2 (constant
    Jacobian I / 2) and each cell's K is the mean of the diffusivity at its Gauss points."""
    n = 33
    for kind in pb.DISCONTINUOUS:
        P = pb.discontinuous(kind, n)
        assert P.jac.shape == (16, n - 1, n - 1)
        J = P.jac.reshape(4, 4, n - 1, n - 1)
        assert np.allclose(J[:, 0], 0.5) and np.allclose(J[:, 3], 0.5)
        assert np.allclose(J[:, 1], 0.0) and np.allclose(J[:, 2], 0.0)
    # checkerboard lines fall on grid lines when 4 divides n - 1: cells are pure, half of each
    K = pb.discontinuous("checker", n).K
    assert set(np.unique(K)) == {1.0, 100.0} and np.count_nonzero(K == 100.0) == K.size // 2
    assert K[0, 0] == 100.0 and K[0, (n - 1) // 4] == 1.0
    # circle of radius 3/5 about the corner: a quarter disc, area 0.09 pi of the unit square
    K = pb.discontinuous("circle", 129).K
    frac = (K - 1.0).sum() / (99.0 * K.size)
    assert abs(frac - 0.09 * np.pi) < 5e-3
    # the stripe 0 <= x < 0.06 along the left edge
    K = pb.discontinuous("layer", 129).K
    assert np.allclose(K[:, 0], 1e-10, rtol=1e-12) and np.all(K[:, 10:] == 2.0)
    # triangle averages: triangles wholly inside or outside the stripe keep its value, the
    # others lie in between
    D = pb.discontinuous_dmg("layer", 17)
    xs = D.mesh.xy_p[D.mesh.tris][:, :, 0]
    inside, outside = (xs < 0.06).all(axis=1), (xs >= 0.06).all(axis=1)
    assert inside.any() and outside.any() and (~inside & ~outside).any()
    assert np.allclose(D.K_t[inside], 1e-10, rtol=1e-12) and np.all(D.K_t[outside] == 2.0)
    mixed = D.K_t[~inside & ~outside]
    assert np.all((mixed >= 1e-10) & (mixed <= 2.0))
    # the average over a triangle integrates a linear function exactly: the 16 sub-triangle
    # centroids have the triangle's centroid as their mean
    tri = np.array([[[0.1, 0.2], [0.7, 0.3], [0.4, 0.9]]])
    xs = []
    saved = pb.unit_square_K
    try:
        pb.unit_square_K = lambda kind, x, y: np.asarray(x)      # K(x, y) = x
        avg = pb.triangle_average("linear", tri)
    finally:
        pb.unit_square_K = saved
    assert abs(avg[0] - tri[0, :, 0].mean()) < 1e-15
