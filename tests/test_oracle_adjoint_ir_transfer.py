"""Pins for the oracle's float32-refinement driver, adjoint gradients and grid<->mesh transfers.

Facts used: the float64 residual criterion itself; central finite differences of J with exact
(sparse direct) solves; SciPy's CG with a fixed iteration count; the P1 mass matrix integrating
1 to the domain area; the coupled mass C integrating to the mesh area (partition of unity of
both bases); an exact mass solve reproducing constants (Sec. 2.3 L2 projection)."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spl

import problems as pb
from oracle import adjoint, boxmg, cycle, fem, transfer


def _setup(prob):
    S = fem.assemble_stencil(prob.jac, prob.K, prob.nx, prob.ny)
    levels = boxmg.build_hierarchy(S)
    return S, levels


def test_fp32_refinement_reaches_fp64_tolerance():
    prob = pb.star(129, seed=2)
    S, levels = _setup(prob)
    o64 = cycle.Oracle(levels, np.float64)
    o32 = cycle.Oracle(levels, np.float32)
    u64, k64, h64, _ = cycle.solve(o64, prob.b, 1e-10)
    x1, k1, h1, _ = cycle.solve_ir(o64, o32, prob.b, 1e-10, inner=1)
    x2, k2, h2, _ = cycle.solve_ir(o64, o32, prob.b, 1e-10, inner=2)
    assert h1[-1] <= 1e-10 and h2[-1] <= 1e-10
    assert abs(k1 - k64) <= 2                       # same outer count as float64 cycles
    assert k2 <= (k64 + 1) // 2 + 2                 # two inner cycles roughly halve it
    # both are solutions of the same float64 system to within the residual tolerance
    assert np.linalg.norm(x1 - u64) / np.linalg.norm(u64) < 1e-7


def test_fp32_levels_are_rounded_fp64_setup():
    prob = pb.star(33, seed=2)
    S, levels = _setup(prob)
    o32 = cycle.Oracle(levels, np.float32)
    assert o32.levels[1].A.dtype == np.float32
    assert np.array_equal(o32.levels[1].diag, levels[1].A.diagonal().astype(np.float32))


def _exact_solve(A, rhs, n):
    m = np.zeros((n, n), bool)
    m[1:-1, 1:-1] = True
    m = m.ravel()
    x = np.zeros(n * n)
    x[m] = spl.spsolve(A.tocsr()[m][:, m].tocsc(), rhs.ravel()[m])
    return x.reshape(n, n)


def test_adjoint_gradient_matches_central_differences():
    n = 17
    prob = pb.star(n, seed=4)
    G = fem.element_matrices(prob.jac, n, n)

    def J_of(K, b):
        A = fem.assemble_matrix(G, K, n, n)
        return adjoint.objective(_exact_solve(A, b, n), prob.target)

    A = fem.assemble_matrix(G, prob.K, n, n)
    u = _exact_solve(A, prob.b, n)
    lam = _exact_solve(A, adjoint.objective_grad_u(u, prob.target), n)
    gK = adjoint.grad_K(prob.jac, lam, u, n, n)
    rng = np.random.default_rng(0)
    for _ in range(3):
        zK = prob.K * rng.normal(size=prob.K.shape)
        zb = np.zeros((n, n))
        zb[1:-1, 1:-1] = rng.normal(size=(n - 2, n - 2))
        eps = 1e-5
        fdK = (J_of(prob.K + eps * zK, prob.b) - J_of(prob.K - eps * zK, prob.b)) / (2 * eps)
        fdb = (J_of(prob.K, prob.b + eps * zb) - J_of(prob.K, prob.b - eps * zb)) / (2 * eps)
        assert abs(fdK - np.sum(gK * zK)) < 1e-7 * max(1.0, abs(fdK))
        assert abs(fdb - np.sum(lam * zb)) < 1e-7 * max(1.0, abs(fdb))


def test_adjoint_with_multigrid_solves():
    """The same gradients with the V-cycle solve run to a tight tolerance."""
    n = 33
    prob = pb.star(n, seed=4)
    S, levels = _setup(prob)
    orc = cycle.Oracle(levels)
    u, _, _, _ = cycle.solve(orc, prob.b, 1e-13)
    lam, _, _, _ = cycle.solve(orc, adjoint.objective_grad_u(u, prob.target), 1e-13)
    G = fem.element_matrices(prob.jac, n, n)
    A = fem.assemble_matrix(G, prob.K, n, n)
    u_ex = _exact_solve(A, prob.b, n)
    lam_ex = _exact_solve(A, adjoint.objective_grad_u(u_ex, prob.target), n)
    g1 = adjoint.grad_K(prob.jac, lam, u, n, n)
    g2 = adjoint.grad_K(prob.jac, lam_ex, u_ex, n, n)
    assert np.linalg.norm(g1 - g2) < 1e-9 * np.linalg.norm(g2)


@pytest.fixture(scope="module")
def mesh_star():
    mp = pb.Star.random(pb.streams(1)[0])
    mesh = pb.lattice_mesh(mp, 25, np.random.default_rng(5))
    return mp, mesh


def test_p1_mass_integrates_area():
    mesh = pb.lattice_mesh(pb.Identity(), 11, np.random.default_rng(0))
    M = transfer.p1_mass(mesh.xy_p, mesh.tris, np.ones(mesh.nv, bool))
    assert abs(M.sum() - 4.0) < 1e-13
    x = mesh.xy_p[:, 0]
    assert abs(x @ (M @ np.ones(mesh.nv))) < 1e-13          # int x dx over the square


def test_coupled_mass_integrates_area(mesh_star):
    """sum_ij C_ij = sum_t |tau_p| / |tt| * (quadrature of |tt|) -> area of the mesh, because the
    P1 and Q1 bases are both partitions of unity.  Identity map: the area is exactly 4."""
    mp, mesh = mesh_star
    n = 17
    allv = np.ones(mesh.nv, bool)
    mesh_i = pb.lattice_mesh(pb.Identity(), 25, np.random.default_rng(5))
    Ci = transfer.coupled_mass(mesh_i.xy_c, mesh_i.xy_p, mesh_i.tris, allv, n, n, drop_grid_boundary=False)
    assert abs(Ci.sum() - 4.0) < 2e-3
    p = mesh.xy_p[mesh.tris]
    area = 0.5 * np.sum((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                        - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    Cs = transfer.coupled_mass(mesh.xy_c, mesh.xy_p, mesh.tris, allv, n, n, drop_grid_boundary=False)
    assert abs(Cs.sum() - area) < 2e-3 * area
    # the star's area is pi (1 + sum a_k^2 / 2); the polygonal mesh approximates it to O(h^2)
    assert abs(area - math.pi * (1 + 0.5 * np.sum(mp.a ** 2))) < 2e-2


def test_cg2_matches_scipy_cg(mesh_star):
    mp, mesh = mesh_star
    M = transfer.p1_mass(mesh.xy_p, mesh.tris, mesh.dof)
    rng = np.random.default_rng(1)
    y = rng.normal(size=mesh.nv) * mesh.dof
    x = transfer.cg2(M, y)
    xs, _ = spl.cg(M, y, x0=np.zeros(mesh.nv), rtol=0.0, atol=0.0, maxiter=2)
    assert np.allclose(x, xs, rtol=1e-12, atol=1e-14 * np.abs(xs).max())
    assert np.all(x[~mesh.dof] == 0.0)


def test_coupled_mass_rows_converge_to_mass_rows(mesh_star):
    """sum_g C_ig = int phi_p^i = sum_j (M_p)_ij exactly; the cell quadrature of the element
    indicator converges to it as the rule is refined, and then an exact mass solve reproduces
    constants (P 1 = 1 for the L2 projection of Sec. 2.3)."""
    mp, mesh = mesh_star
    n = 17
    allv = np.ones(mesh.nv, bool)
    M = transfer.p1_mass(mesh.xy_p, mesh.tris, allv)
    rm = np.asarray(M.sum(axis=1)).ravel()
    errs = []
    for nq in (2, 4, 8, 16):
        C = transfer.coupled_mass(mesh.xy_c, mesh.xy_p, mesh.tris, allv, n, n, nq=nq, drop_grid_boundary=False)
        errs.append(np.abs(np.asarray(C.sum(axis=1)).ravel() - rm).max() / rm.max())
    assert errs[0] > errs[1] > errs[2] and errs[3] < 1e-2, errs
    up = spl.spsolve(M.tocsc(), C @ np.ones(n * n))
    far = np.all(np.abs(mesh.xy_c) < 0.5, axis=1)
    assert np.max(np.abs(up[far] - 1.0)) < 2e-2


def test_transfers_are_transposes_for_exact_mass_solve(mesh_star):
    mp, mesh = mesh_star
    n = 17
    M = transfer.p1_mass(mesh.xy_p, mesh.tris, mesh.dof)
    C = transfer.coupled_mass(mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, n, n)
    rng = np.random.default_rng(2)
    uc = np.zeros((n, n))
    uc[1:-1, 1:-1] = rng.normal(size=(n - 2, n - 2))
    rp = rng.normal(size=mesh.nv) * mesh.dof
    up = transfer.from_grid(M, C, uc, iters=200)
    rc = transfer.to_grid(M, C, rp, n, n, iters=200)
    assert abs(up @ rp - np.sum(uc * rc)) < 1e-10 * abs(up @ rp)
