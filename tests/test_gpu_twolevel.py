"""Parity of the two-level cycle on the physical mesh (HIP library through the C ABI) with the
float64 oracle (oracle/dmg.py) on star-domain meshes: the relaxation colours bit for bit, every
iterate entry by entry (1e-12 |ref| + 256 eps max|ref|, tests/entrywise.py) for both mass modes
and both coupled-mass rules, whole solves (cycle counts, residual histories, solutions), the
zero-residual start, the iteration cap, the captured-graph path against the eager one, and the
cycle over the matrix-free coupled mass."""
import numpy as np
import pytest
import torch

import problems as pb
from entrywise import assert_iterate
from oracle import boxmg, cycle, dmg, fem, transfer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2509_08109_amd as m
    m.lib()
    return m


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


_CACHE = {}


def pair(lib, n, seed=1, mass="lumped", nq=0, kind=None, matrix_free=False):
    """(problem, oracle two-level, GPU two-level) on the star mesh of grid size n (or on the unit
    square with the discontinuous diffusivity ``kind``); nq = 0 is the exact coupled mass, nq > 0
    the rasterised rule of that order; matrix_free: the library stores no C."""
    key = (n, seed, mass, nq, kind, matrix_free)
    if key not in _CACHE:
        P = pb.star_dmg(n, seed=seed) if kind is None else pb.discontinuous_dmg(kind, n)
        m = P.mesh
        A = dmg.p1_stiffness(m.xy_p, m.tris, m.dof, P.K_t)
        M = transfer.p1_mass(m.xy_p, m.tris, m.dof)
        Cm = transfer.coupled_mass(m.xy_c, m.xy_p, m.tris, m.dof, n, n, nq=nq)
        grid = cycle.Oracle(boxmg.build_hierarchy(fem.assemble_stencil(P.grid.jac, P.grid.K, n, n)))
        orc = dmg.TwoLevel(A, M, Cm, grid, n, n, dmg.mesh_colouring(m.tris, m.dof),
                           mass="lumped" if mass == "lumped" else 2)
        H = lib.Hierarchy(lib.assemble_stencil(dev(P.grid.jac), dev(P.grid.K)))
        tl = lib.TwoLevel(H, m.xy_c, m.xy_p, m.tris, m.dof, K_t=P.K_t, nq=nq, mass=mass,
                          matrix_free=matrix_free)
        _CACHE[key] = (P, orc, tl)
    return _CACHE[key]


def test_colouring_and_operator_size(lib):
    P, orc, tl = pair(lib, 33)
    nc, nnz, col = tl.info()
    assert np.array_equal(col, orc.colour.astype(np.int32))
    assert nc == int(orc.colour.max()) + 1
    assert nnz == orc.A.nnz


@pytest.mark.parametrize("n,mass,nq", [(17, "lumped", 0), (33, "lumped", 0), (17, "cg2", 0),
                                       (33, "cg2", 0), (33, "lumped", 8), (65, "lumped", 0),
                                       (33, "cg2", 4)])
def test_cycles_match_oracle(lib, n, mass, nq):
    """65 x 65 is the smallest grid whose finest level runs in the strip kernels (smaller grids
    run whole in the one-workgroup coarse kernel).  (cg2, nq = 4) is the paper's own
    configuration: two CG iterations on M_p and the rasterised coupled mass.  On larger star
    meshes that cycle diverges (its coarse correction over-corrects modes whose generalized
    eigenvalue of (P^T A_p P, A_c) exceeds 2), and a divergent iteration multiplies the rounding
    difference of two implementations every cycle, so it is compared here at 33^2 only."""
    P, orc, tl = pair(lib, n, mass=mass, nq=nq)
    g = np.random.Generator(np.random.PCG64(11))
    u0 = np.where(P.mesh.dof, g.uniform(-1, 1, P.mesh.nv), 0.0)
    uo = u0.copy()
    ug = dev(u0)
    fg = dev(P.f)
    for k in range(3):
        orc.cycle(uo, P.f)
        tl.cycle(ug, fg)
        used = assert_iterate(f"cycle {k + 1}", host(ug), uo)
        print(f"[twolevel] n={n} {mass} nq={nq} cycle {k + 1}: worst excess {used:.1f} eps max|u|")


@pytest.mark.parametrize("n,mass,nq", [(33, "lumped", 0), (65, "lumped", 0), (33, "cg2", 4),
                                       (33, "lumped", 8)])
def test_matrix_free_cycles_match_oracle(lib, n, mass, nq):
    """The two-level cycle over the matrix-free coupled mass (no C stored; its action recomputed
    from the overlap sets on every interpolation and restriction) against the oracle's cycle with
    the assembled C, entry by entry, and its solve's cycle count and history."""
    P, orc, tl = pair(lib, n, mass=mass, nq=nq, matrix_free=True)
    g = np.random.Generator(np.random.PCG64(13))
    u0 = np.where(P.mesh.dof, g.uniform(-1, 1, P.mesh.nv), 0.0)
    uo, ug, fg = u0.copy(), dev(u0), dev(P.f)
    for k in range(3):
        orc.cycle(uo, P.f)
        tl.cycle(ug, fg)
        used = assert_iterate(f"matrix-free cycle {k + 1}", host(ug), uo)
        print(f"[twolevel] matrix-free n={n} {mass} nq={nq} cycle {k + 1}: worst excess {used:.1f} eps max|u|")
    if mass == "lumped":
        u, k, rel, hist = tl.solve(fg, rtol=1e-10)
        uo, ko, histo, _ = dmg.solve(orc, P.f, rtol=1e-10)
        assert k == ko and rel <= 1e-10
        assert np.allclose(hist, histo, rtol=1e-6, atol=1e-13)
        assert_iterate("matrix-free solution", host(u), uo)


def test_matrix_free_scaling_estimate_matches_oracle(lib):
    """Sec. 2.4's estimate runs P and R through the matrix-free coupled mass."""
    n = 33
    P, orc, tl = pair(lib, n, matrix_free=True)
    v0 = np.random.Generator(np.random.PCG64(9)).uniform(-1, 1, (n, n))
    go, To = dmg.coarse_scaling(orc, v0, 12)
    gg, Tg = tl.estimate_scaling(dev(v0), 12)
    assert abs(gg - go) <= 1e-9 * abs(go), (gg, go)
    assert np.allclose(Tg, To, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("n", [17, 33])
def test_solve_matches_oracle(lib, n):
    P, orc, tl = pair(lib, n)
    u, k, rel, hist = tl.solve(dev(P.f), rtol=1e-10)
    uo, ko, histo, _ = dmg.solve(orc, P.f, rtol=1e-10)
    assert k == ko and rel <= 1e-10
    assert np.allclose(hist, histo, rtol=1e-6, atol=1e-13)
    assert_iterate("solution", host(u), uo)


def test_solve_from_random_guess_with_zero_rhs(lib):
    """The paper's convergence setting: f = 0 from a random initial guess."""
    P, orc, tl = pair(lib, 33)
    g = np.random.Generator(np.random.PCG64(5))
    u0 = np.where(P.mesh.dof, g.uniform(-1, 1, P.mesh.nv), 0.0)
    f0 = np.zeros(P.mesh.nv)
    u, k, rel, hist = tl.solve(dev(f0), u=dev(u0), rtol=1e-10)
    uo, ko, histo, _ = dmg.solve(orc, f0, u0=u0, rtol=1e-10)
    assert k == ko
    assert np.allclose(hist, histo, rtol=1e-6, atol=1e-13)
    # the iterates decay towards 0: compare against the starting scale
    assert np.max(np.abs(host(u) - uo)) <= 1e-12 * np.max(np.abs(u0))


def test_zero_initial_residual_and_iteration_cap(lib):
    P, orc, tl = pair(lib, 17)
    z = torch.zeros(P.mesh.nv, dtype=torch.float64, device="cuda")
    u, k, rel, hist = tl.solve(torch.zeros_like(z), u=z.clone(), rtol=1e-10)
    assert k == 0 and rel == 0.0 and hist == [] and float(u.abs().max()) == 0.0
    u, k, rel, hist = tl.solve(dev(P.f), rtol=1e-30, max_iters=3, raise_on_fail=False)
    uo, ko, histo, _ = dmg.solve(orc, P.f, rtol=1e-30, max_iters=3)
    assert k == ko == 3 and np.allclose(hist, histo, rtol=1e-6, atol=1e-13)
    assert_iterate("capped solve", host(u), uo)
    with pytest.raises(lib.DmgError):
        tl.solve(dev(P.f), rtol=1e-30, max_iters=2)


def test_graph_path_matches_eager(lib):
    """Solves on a side stream run through captured graphs of four cycles; the default stream
    runs them eagerly.  Both give the same iterate bit for bit."""
    P, orc, tl = pair(lib, 33)
    f = dev(P.f)
    u_e, k_e, _, h_e = tl.solve(f, rtol=1e-10)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):  # the second solve replays the captured graph
            u_g, k_g, _, h_g = tl.solve(f, rtol=1e-10)
    torch.cuda.synchronize()
    assert k_g == k_e and h_g == h_e
    assert torch.equal(u_g, u_e)


@pytest.mark.parametrize("n", [33, 65])
def test_scaling_estimate_matches_oracle(lib, n):
    """gamma and the Lanczos tridiagonal of Sec. 2.4's estimate.  The library solves with A_c by
    the multigrid solve to a relative residual of 1e-13 (the oracle exactly); over 12 steps that
    leaves gamma within 1e-9 and T within 1e-8 relative."""
    P, orc, tl = pair(lib, n)
    v0 = np.random.Generator(np.random.PCG64(9)).uniform(-1, 1, (n, n))
    go, To = dmg.coarse_scaling(orc, v0, 12)
    gg, Tg = tl.estimate_scaling(dev(v0), 12)
    assert Tg.shape == To.shape == (12, 12)
    assert abs(gg - go) <= 1e-9 * abs(go), (gg, go)
    assert np.allclose(Tg, To, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("n,mass", [(33, "lumped"), (17, "cg2")])
def test_scaled_cycles_match_oracle(lib, n, mass):
    P, orc, tl = pair(lib, n, mass=mass)
    g = np.random.Generator(np.random.PCG64(12))
    u0 = np.where(P.mesh.dof, g.uniform(-1, 1, P.mesh.nv), 0.0)
    orc.gamma = 0.7
    tl.set_scaling(0.7)
    try:
        uo, ug, fg = u0.copy(), dev(u0), dev(P.f)
        for k in range(3):
            orc.cycle(uo, P.f)
            tl.cycle(ug, fg)
            assert_iterate(f"scaled cycle {k + 1}", host(ug), uo)
    finally:
        orc.gamma = 1.0
        tl.set_scaling(1.0)


def test_set_scaling_replaces_captured_cycles(lib):
    """A solve captures its cycles in a graph; a new gamma must not replay the old one."""
    P, orc, tl = pair(lib, 33)
    f = dev(P.f)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    try:
        with torch.cuda.stream(s):
            _, k1, _, _ = tl.solve(f, rtol=1e-10)
            tl.set_scaling(0.7)
            u, k, rel, hist = tl.solve(f, rtol=1e-10)
        torch.cuda.synchronize()
        orc.gamma = 0.7
        uo, ko, histo, _ = dmg.solve(orc, P.f, rtol=1e-10)
        assert k == ko and k != k1
        assert np.allclose(hist, histo, rtol=1e-6, atol=1e-13)
    finally:
        orc.gamma = 1.0
        tl.set_scaling(1.0)


def test_scaling_estimate_needs_lumped_mass(lib):
    P, orc, tl = pair(lib, 17, mass="cg2")
    with pytest.raises(lib.DmgError):
        tl.estimate_scaling(torch.ones((17, 17), dtype=torch.float64, device="cuda"), 4)


@pytest.mark.parametrize("kind", ["circle", "checker", "layer"])
def test_discontinuous_cycles_match_oracle(lib, kind):
    """The unit-square problems with discontinuous diffusivity (contrast up to 2e10)."""
    P, orc, tl = pair(lib, 33, kind=kind)
    g = np.random.Generator(np.random.PCG64(13))
    u0 = np.where(P.mesh.dof, g.uniform(-1, 1, P.mesh.nv), 0.0)
    uo, ug, fg = u0.copy(), dev(u0), dev(P.f)
    for k in range(2):
        orc.cycle(uo, P.f)
        tl.cycle(ug, fg)
        assert_iterate(f"{kind} cycle {k + 1}", host(ug), uo)
