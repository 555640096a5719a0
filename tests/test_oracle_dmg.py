"""Pins of the two-level cycle oracle (oracle/dmg.py) against facts fixed outside it: the
textbook P1 element stiffness, properties of the assembled operator, a valid colouring, the
lumped mass against triangle areas, convergence to a direct solve, and a convergence rate that
does not grow with the problem size (Sec. 4.3's observation for the two-level method)."""
import os

import numpy as np
import pytest
import scipy.sparse as spx
import scipy.sparse.linalg as spl

import problems as pb
from oracle import boxmg, cycle, dmg, fem, transfer

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _setup(n, seed=1, nq=0, mass="lumped"):
    P = pb.star_dmg(n, seed=seed)
    m = P.mesh
    A = dmg.p1_stiffness(m.xy_p, m.tris, m.dof, P.K_t)
    M = transfer.p1_mass(m.xy_p, m.tris, m.dof)
    C = transfer.coupled_mass(m.xy_c, m.xy_p, m.tris, m.dof, n, n, nq=nq)
    orc = cycle.Oracle(boxmg.build_hierarchy(fem.assemble_stencil(P.grid.jac, P.grid.K, n, n)))
    return P, A, M, C, dmg.TwoLevel(A, M, C, orc, n, n, dmg.mesh_colouring(m.tris, m.dof), mass=mass)


def _inner(m):
    """Free vertices all of whose triangle neighbours are free (from the triangles, not from the
    sparsity of an operator whose Dirichlet couplings are removed)."""
    bad = np.zeros(m.nv, dtype=bool)
    tri_free = m.dof[m.tris].all(axis=1)
    bad[m.tris[~tri_free].ravel()] = True
    return m.dof & ~bad


def test_p1_element_stiffness_golden():
    rows = np.loadtxt(os.path.join(GOLDEN, "p1_element_stiffness.txt"), comments="#", ndmin=2)
    for x0, y0, x1, y1, x2, y2, *a in rows:
        G = dmg.p1_element_stiffness(np.array([[x0, y0], [x1, y1], [x2, y2]]))
        ref = np.array([[a[0], a[1], a[2]], [a[1], a[3], a[4]], [a[2], a[4], a[5]]])
        assert np.allclose(G, ref, atol=1e-15)


def test_stiffness_properties_and_colouring():
    P = pb.star_dmg(17, seed=2)
    m = P.mesh
    A = dmg.p1_stiffness(m.xy_p, m.tris, m.dof, P.K_t)
    assert abs(A - A.T).max() < 1e-14
    assert np.all(A.diagonal() > 0)
    # zero row sums where the vertex and all its neighbours are free
    inner = _inner(m)
    assert inner.sum() > m.nv // 2
    assert np.allclose(np.asarray(A.sum(axis=1)).ravel()[inner], 0.0, atol=1e-12)
    col = dmg.mesh_colouring(m.tris, m.dof)
    Ac = A.tocoo()
    off = Ac.row != Ac.col
    assert np.all(col[Ac.row[off]] != col[Ac.col[off]])          # a proper colouring of A_p
    G = dmg.mesh_graph(m.tris, m.dof)
    assert abs(G - G.T).max() == 0 and G.diagonal().sum() == 0
    # every coupling of A_p is a mesh edge, and every mesh edge a coupling (no cancellation here)
    Gp = (abs(A) > 0).astype(float) - spx.eye(m.nv)
    assert abs((Gp != 0).astype(float) - (G != 0).astype(float)).max() == 0
    # a planar graph always has a vertex of degree <= 5, so greedy colouring in smallest-last
    # order needs at most 6 colours
    assert col.max() + 1 <= 6
    assert np.all(col[~m.dof] == 0)                               # isolated Dirichlet vertices
    # the order: brute force over the removals, each of least degree among the vertices left
    # (smallest index among equals); each vertex then takes the smallest colour unused by the
    # neighbours coloured before it
    order = dmg.smallest_last_order(G)
    left = np.ones(m.nv, dtype=bool)
    Gd = (G != 0).toarray()
    for v in order[::-1]:
        deg = (Gd & left[None, :]).sum(axis=1)
        cand = np.nonzero(left)[0]
        best = cand[deg[cand] == deg[cand].min()].min()
        assert v == best
        left[v] = False
    pos = np.empty(m.nv, dtype=np.int64)
    pos[order] = np.arange(m.nv)
    for v in range(0, m.nv, 5):
        nb = G.indices[G.indptr[v]:G.indptr[v + 1]]
        used = set(col[nb[pos[nb] < pos[v]]].tolist())
        assert col[v] == min(set(range(10)) - used)


@pytest.mark.parametrize("edges, expected", [
    # path 0-1-2: 0 leaves first, then 1, then 2; coloured 2, 1, 0
    ([(0, 1), (1, 2)], [0, 1, 0]),
    # triangle 0-1-2 with 3 hanging on 2: removals 3, 0, 1, 2; coloured 2, 1, 0, 3
    ([(0, 1), (1, 2), (0, 2), (2, 3)], [2, 1, 0, 1]),
    # wheel: hub 0 on the 5-cycle 1-2-3-4-5: removals 1, 2, 3, 0, 4, 5; coloured 5, 4, 0, 3, 2, 1
    # (an odd wheel needs 4 colours)
    ([(0, k) for k in range(1, 6)] + [(1, 2), (2, 3), (3, 4), (4, 5), (5, 1)], [2, 3, 1, 0, 1, 0]),
])
def test_smallest_last_colouring_by_hand(edges, expected):
    n = len(expected)
    r = [a for a, b in edges] + [b for a, b in edges]
    c = [b for a, b in edges] + [a for a, b in edges]
    G = spx.coo_matrix((np.ones(len(r)), (r, c)), shape=(n, n)).tocsr()
    col = dmg.greedy_colouring(G, dmg.smallest_last_order(G))
    assert col.tolist() == expected


def test_lumped_mass_is_a_third_of_incident_area():
    P = pb.star_dmg(17, seed=3)
    m = P.mesh
    M = transfer.p1_mass(m.xy_p, m.tris, m.dof)
    ML = dmg.lumped(M)
    p = m.xy_p[m.tris]
    area = 0.5 * np.abs((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                        - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    third = np.bincount(m.tris.ravel(), weights=np.repeat(area / 3, 3), minlength=m.nv)
    # vertices whose neighbours are all free keep their full row sum
    inner = _inner(m)
    assert np.allclose(ML[inner], third[inner], rtol=1e-13)
    assert np.all(ML[~m.dof] == 1.0)


def test_two_level_solves_the_physical_system():
    P, A, M, C, tl = _setup(17)
    u, k, hist, _ = dmg.solve(tl, P.f, rtol=1e-10)
    ue = spl.spsolve(A.tocsc(), P.f)
    assert hist[-1] <= 1e-10 and k < 40
    assert np.linalg.norm(u - ue) / np.linalg.norm(ue) < 1e-8


def test_two_level_rate_does_not_grow_with_size():
    rates, counts = [], []
    for n in (17, 33):
        P, A, M, C, tl = _setup(n)
        u, k, hist, _ = dmg.solve(tl, P.f, rtol=1e-10)
        rates.append(cycle.convergence_factor(hist))
        counts.append(k)
    assert max(rates) < 0.3 and abs(counts[1] - counts[0]) <= 3


def _dense_pencil(n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    Q = g.normal(size=(n, n))
    A = Q @ Q.T + n * np.eye(n)                       # SPD
    B = g.normal(size=(n, n))
    G = B @ B.T                                       # symmetric positive semidefinite
    return A, G, g.normal(size=n)


def test_lanczos_mean_over_the_whole_space_is_the_eigenvalue_mean():
    """k = n steps span the space: T_n is similar to A^{-1} G, so its trace / n is the mean of
    all generalized eigenvalues (scipy.linalg.eigh of the pencil) and its eigenvalues are them."""
    import scipy.linalg as sla
    A, G, v0 = _dense_pencil(8, 3)
    gam, T = dmg.lanczos_mean(lambda x: G @ x, lambda y: np.linalg.solve(A, y), lambda x: A @ x, v0, 8)
    lam = sla.eigh(G, A, eigvals_only=True)
    assert abs(gam - lam.mean()) <= 1e-12 * abs(lam.mean())
    assert np.allclose(np.sort(np.linalg.eigvalsh(T)), lam, rtol=1e-9, atol=1e-12)


def test_lanczos_mean_special_cases():
    A, G, v0 = _dense_pencil(10, 4)
    # G = c A: every generalized eigenvalue is c; the space is invariant after one step
    gam, T = dmg.lanczos_mean(lambda x: 2.5 * (A @ x), lambda y: np.linalg.solve(A, y), lambda x: A @ x, v0, 4)
    assert abs(gam - 2.5) <= 1e-13 and T.shape == (1, 1)
    # k < n: Ritz values lie inside the pencil's spectrum (Cauchy interlacing)
    import scipy.linalg as sla
    lam = sla.eigh(G, A, eigvals_only=True)
    gam, T = dmg.lanczos_mean(lambda x: G @ x, lambda y: np.linalg.solve(A, y), lambda x: A @ x, v0, 5)
    ritz = np.linalg.eigvalsh(T)
    assert ritz.min() >= lam.min() - 1e-12 and ritz.max() <= lam.max() + 1e-12
    assert T.shape == (5, 5) and np.allclose(T, T.T)


def test_coarse_scaling_of_the_two_level_cycle():
    """gamma of the star mesh lies inside the range of the generalized eigenvalues (computed
    independently by scipy's eigsh on the same pencil); with gamma = 0 the cycle drops its coarse
    correction and is two symmetric Gauss-Seidel sweeps."""
    P, A, M, C, tl = _setup(17)
    g = np.random.Generator(np.random.PCG64(9))
    v0 = g.uniform(-1, 1, (17, 17))
    gam, T = dmg.coarse_scaling(tl, v0, 12)
    ii = np.nonzero(np.pad(np.ones((15, 15), bool), 1).ravel())[0]
    Ac = tl.grid.levels[0].A.tocsr()[ii][:, ii]
    Pm = (spx.diags(1.0 / tl.ML) @ tl.C).tocsr()[:, ii]
    Gm = (Pm.T @ tl.A @ Pm).tocsr()
    hi = spl.eigsh(Gm, k=1, M=Ac.tocsc(), which="LA", return_eigenvectors=False)[0]
    lo = spl.eigsh(Gm, k=1, M=Ac.tocsc(), sigma=0.0, which="LM", return_eigenvectors=False)[0]
    assert lo - 1e-10 <= gam <= hi + 1e-10
    assert np.all(np.linalg.eigvalsh(T) <= hi + 1e-10) and np.all(np.linalg.eigvalsh(T) >= lo - 1e-10)
    u0 = np.where(P.mesh.dof, g.uniform(-1, 1, P.mesh.nv), 0.0)
    tl.gamma = 0.0
    u_g0 = tl.cycle(u0.copy(), P.f)
    tl.gamma = 1.0
    u_s = dmg.sgs(tl.A, dmg.sgs(tl.A, u0.copy(), P.f, tl.colour), P.f, tl.colour)
    assert np.array_equal(u_g0, u_s)
    assert not np.allclose(tl.cycle(u0.copy(), P.f), u_s)
