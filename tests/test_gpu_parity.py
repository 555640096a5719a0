"""Parity of the HIP library (called through the C ABI) with the float64 CPU oracle, entry by
entry (tests/entrywise.py states each bound and why):
  * setup data (stencils, interpolation weights, Galerkin stencils, gradients): every entry
    within 1e-12 of the magnitude of the terms summed to form it;
  * iterates of V-cycles and solves: every entry within 1e-12 |ref| + 256 eps max|ref|;
  * identical cycle counts, residual histories to 1e-6 relative (late residuals ~1e-10 carry
    the rounding noise of the residual itself)."""
import numpy as np
import pytest
import torch

import problems as pb
from entrywise import (EPS64, assert_entrywise, assert_hierarchy, assert_iterate, assert_stencil)
from oracle import adjoint, boxmg, cycle, fem, transfer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dmg():
    import paper_2509_08109_amd as m
    m.lib()
    return m


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


PROBLEMS = {
    "identity33": lambda: pb.identity(33),
    "annulus65": lambda: pb.quarter_annulus(65),
    "star129": lambda: pb.star(129, seed=1),
    "star65x129": lambda: pb.star(65, seed=1, ny=129),
    # odd dims that are not 2^k + 1: the paper's 1.5 aspect ratio (33 x 49 -> ... -> 3 x 4),
    # 97 = 3 * 32 + 1 (coarsest 4 x 3), and 45 x 67 (coarsest 23 x 34, 672 unknowns)
    "annulus33x49": lambda: pb.quarter_annulus(33, ny=49),
    "star97x65": lambda: pb.star(97, seed=1, ny=65),
    "star45x67": lambda: pb.star(45, seed=1, ny=67),
    # the discontinuous diffusivities of the paper's variable-coefficient problems
    "circle65": lambda: pb.discontinuous("circle", 65),
    "checker65": lambda: pb.discontinuous("checker", 65),
    "layer65": lambda: pb.discontinuous("layer", 65),
}


@pytest.fixture(scope="module", params=list(PROBLEMS))
def case(request, dmg):
    prob = PROBLEMS[request.param]()
    S_or = fem.assemble_stencil(prob.jac, prob.K, prob.nx, prob.ny)
    levels = boxmg.build_hierarchy(S_or)
    return prob, S_or, levels


def hier_levels(h):
    """Every level's (S, P) of a library hierarchy as host arrays."""
    out = []
    for l in range(h.num_levels):
        S, P = h.level(l)
        out.append((host(S), None if P is None else host(P)))
    return out


def test_assembly_matches_oracle(dmg, case):
    prob, S_or, _ = case
    S = dmg.assemble_stencil(dev(prob.jac), dev(prob.K))
    assert_stencil("assembly", host(S), S_or)


def test_hierarchy_matches_oracle(dmg, case):
    prob, S_or, levels = case
    h = dmg.Hierarchy(dev(S_or))
    assert h.num_levels == len(levels)
    assert_hierarchy("hierarchy", hier_levels(h), levels)
    h.close()


def test_vcycle_iterates_match_oracle(dmg, case):
    prob, S_or, levels = case
    h = dmg.Hierarchy(dev(S_or))
    orc = cycle.Oracle(levels)
    b = dev(prob.b)
    u = torch.zeros_like(b)
    uo = np.zeros(prob.nx * prob.ny)
    bo = prob.b.ravel().copy()
    for k in range(8):
        h.vcycle(u, b)
        orc.vcycle(uo, bo)
        assert_iterate(f"iterate {k + 1}", host(u).ravel(), uo)
    h.close()


@pytest.mark.parametrize("name", ["star129", "annulus65", "circle65"])
def test_dense_coarse_operator_matches_coarse_kernel(dmg, name):
    """The cycle below 33 x 33 applied as its dense matrix (coarse_gemv = 1, built at setup
    from unit-vector runs) and run in the one-workgroup coarse kernel (0): the same iterates to
    rounding, each matching the oracle per iterate; also for float32 refinement."""
    prob = PROBLEMS[name]()
    S_or = fem.assemble_stencil(prob.jac, prob.K, prob.nx, prob.ny)
    orc = cycle.Oracle(boxmg.build_hierarchy(S_or))
    b = dev(prob.b)
    hs = [dmg.Hierarchy(dev(S_or), coarse_gemv=g) for g in (0, 1)]
    us = [torch.zeros_like(b) for _ in hs]
    uo = np.zeros(prob.nx * prob.ny)
    for k in range(6):
        for h, u in zip(hs, us):
            h.vcycle(u, b)
        orc.vcycle(uo, prob.b.ravel().copy())
        for g, u in enumerate(us):
            assert_iterate(f"coarse_gemv={g} iterate {k + 1}", host(u).ravel(), uo)
        assert_iterate(f"gemv vs coarse kernel, iterate {k + 1}", host(us[1]), host(us[0]))
    for h in hs:
        h.close()
    xs = []
    for g in (0, 1):
        h = dmg.Hierarchy(dev(S_or), coarse_gemv=g, precision=dmg.DMG_FP32_IR)
        x, k, rel, _ = h.solve(b, rtol=1e-10)
        assert rel <= 1e-10
        xs.append((host(x), k))
        h.close()
    # float32 cycles whose coarse levels differ by float32 rounding: the same outer-step count to
    # one step; both solutions are 1e-10-residual solutions of one system
    assert abs(xs[0][1] - xs[1][1]) <= 1
    assert_iterate("fp32 refinement, gemv vs coarse kernel", xs[1][0], xs[0][0], rtol=1e-7,
                   floor_ulps=int(1e-7 / EPS64))


def test_refresh_replays_a_captured_setup(dmg):
    """Refreshes from one stencil array: the first runs eagerly, the next is captured, later
    ones replay the graph, each reading the array's current contents; every refreshed
    hierarchy solves exactly as a freshly built one."""
    probs = [pb.star(129, seed=21), pb.star(129, seed=22), pb.quarter_annulus(129)]
    Ss = [dmg.assemble_stencil(dev(p.jac), dev(p.K)) for p in probs]
    b = dev(probs[0].b)
    buf = Ss[0].clone()
    h = dmg.Hierarchy(buf)
    for k in (1, 2, 0, 1, 2):
        buf.copy_(Ss[k])
        h.refresh(buf)
        u, it, rel, _ = h.solve(b, rtol=1e-10)
        ref = dmg.Hierarchy(Ss[k])
        u1, it1, rel1, _ = ref.solve(b, rtol=1e-10)
        ref.close()
        assert it == it1 and torch.equal(u, u1)
    h.close()


def test_solve_matches_oracle(dmg, case):
    prob, S_or, levels = case
    h = dmg.Hierarchy(dev(S_or))
    u, k, rel, hist = h.solve(dev(prob.b), rtol=1e-10)
    uo, ko, histo, _ = cycle.solve(cycle.Oracle(levels), prob.b, rtol=1e-10)
    assert rel <= 1e-10 and k == ko
    # late relative residuals (~1e-10) carry rounding noise of order eps * cond-free 1e-15
    assert np.allclose(hist, histo, rtol=1e-6, atol=1e-13)
    assert_iterate("solution", host(u), uo)
    h.close()


@pytest.mark.parametrize("pre,post,nu", [((1, 0, 3, 2), (2, 3, 0, 1), (1, 1)),
                                         ((2, 3, 0, 1), (1, 0, 3, 2), (1, 1)),
                                         ((0, 1, 2, 3), (3, 2, 1, 0), (2, 2)),
                                         ((3, 2, 0, 1), (0, 1, 3, 2), (1, 2))])
def test_colour_orders_and_sweep_counts(dmg, pre, post, nu):
    prob = pb.star(257, seed=5)
    S_or = fem.assemble_stencil(prob.jac, prob.K, prob.nx, prob.ny)
    levels = boxmg.build_hierarchy(S_or)
    h = dmg.Hierarchy(dev(S_or), pre_order=pre, post_order=post, nu_pre=nu[0], nu_post=nu[1])
    orc = cycle.Oracle(levels, pre=pre, post=post, nu_pre=nu[0], nu_post=nu[1])
    b = dev(prob.b)
    u = torch.zeros_like(b)
    uo = np.zeros(prob.nx * prob.ny)
    for k in range(4):
        h.vcycle(u, b)
        orc.vcycle(uo, prob.b.ravel().copy())
        assert_iterate(f"iterate {k + 1}", host(u).ravel(), uo)
    h.close()


@pytest.mark.parametrize("wave", [0, 1])
@pytest.mark.parametrize("pre,post", [((0, 1, 2, 3), (3, 2, 1, 0)), ((2, 3, 1, 0), (0, 1, 3, 2))])
def test_strip_kernel_variants_match_oracle(dmg, wave, pre, post):
    """Both strip-kernel implementations (LDS strips, one-wavefront DPP strips) give the oracle's
    iterates, for both row parities smoothed first."""
    prob = pb.star(513, seed=9)
    S_or = fem.assemble_stencil(prob.jac, prob.K, prob.nx, prob.ny)
    levels = boxmg.build_hierarchy(S_or)
    h = dmg.Hierarchy(dev(S_or), pre_order=pre, post_order=post, tile_rows=8, strip_kernel=wave)
    assert all((bw == 1) == bool(wave) for bw, sh in h.config()["levels"] if bw)
    orc = cycle.Oracle(levels, pre=pre, post=post)
    b = dev(prob.b)
    u = torch.zeros_like(b)
    uo = np.zeros(prob.nx * prob.ny)
    for k in range(3):
        h.vcycle(u, b)
        orc.vcycle(uo, prob.b.ravel().copy())
        assert_iterate(f"iterate {k + 1}", host(u).ravel(), uo)
    x, k, rel, hist = h.solve(b, rtol=1e-10)
    xo, ko, _, _ = cycle.solve(orc, prob.b, 1e-10)
    assert k == ko
    assert_iterate("solution", host(x), xo)
    h.close()


@pytest.mark.parametrize("wave", [0, 1])
@pytest.mark.parametrize("tile_rows", [2, 6, 64])
def test_launch_shape_is_numerically_neutral(dmg, tile_rows, wave):
    """Within one strip-kernel implementation the segment height changes nothing, bitwise."""
    prob = pb.star(513, seed=6)
    S = dmg.assemble_stencil(dev(prob.jac), dev(prob.K))
    b = dev(prob.b)
    ref = dmg.Hierarchy(S, strip_kernel=wave)
    u0, k0, _, _ = ref.solve(b, rtol=1e-10)
    h = dmg.Hierarchy(S, tile_rows=tile_rows, strip_kernel=wave)
    u1, k1, _, _ = h.solve(b, rtol=1e-10)
    assert k0 == k1 and torch.equal(u0, u1)
    h.close()
    ref.close()


@pytest.mark.parametrize("wave", [0, 1])
@pytest.mark.parametrize("tile_rows", [2, 64])
def test_launch_shape_is_numerically_neutral_fp32(dmg, tile_rows, wave):
    """The same for the float32 sweeps of refinement (which also add into the float64
    iterate)."""
    prob = pb.star(513, seed=6)
    S = dmg.assemble_stencil(dev(prob.jac), dev(prob.K))
    b = dev(prob.b)
    ref = dmg.Hierarchy(S, strip_kernel=wave, precision=dmg.DMG_FP32_IR)
    u0, k0, _, _ = ref.solve(b, rtol=1e-10)
    h = dmg.Hierarchy(S, tile_rows=tile_rows, strip_kernel=wave, precision=dmg.DMG_FP32_IR)
    u1, k1, _, _ = h.solve(b, rtol=1e-10)
    assert k0 == k1 and torch.equal(u0, u1)
    h.close()
    ref.close()


def test_autotuned_hierarchy_matches_oracle(dmg):
    """Tuned launch shapes are numerically neutral; a tuned colour order is replayed by the
    oracle."""
    prob = pb.star(513, seed=7)
    S_or = fem.assemble_stencil(prob.jac, prob.K, prob.nx, prob.ny)
    levels = boxmg.build_hierarchy(S_or)
    b = dev(prob.b)
    h = dmg.Hierarchy(dev(S_or), precision=dmg.DMG_FP32_IR)
    cfg = h.autotune(b, tiles=True, colour_order=True, reps=2)
    assert all(bw in (0, 1, 64, 128) for bw, _ in cfg["levels"])   # float64 shapes
    assert cfg["post_order"] == cfg["pre_order"][::-1]
    h64 = dmg.Hierarchy(dev(S_or), pre_order=cfg["pre_order"], post_order=cfg["post_order"])
    h64.autotune(b, tiles=True, reps=2)
    u, k, rel, _ = h64.solve(b, rtol=1e-10)
    orc = cycle.Oracle(levels, pre=cfg["pre_order"], post=cfg["post_order"])
    uo, ko, _, _ = cycle.solve(orc, prob.b, 1e-10)
    assert k == ko
    assert_iterate("tuned solution", host(u), uo)
    x, k32, rel32, _ = h.solve(b, rtol=1e-10)
    assert rel32 <= 1e-10
    h.close()
    h64.close()


def test_solve_on_a_side_stream_uses_graph_chunks(dmg):
    """Solves on a non-default stream run chunks of steps through captured graphs; the step
    count and the iterate are those of the oracle, also when max_iters cuts a chunk short."""
    prob = pb.star(257, seed=8)
    S_or = fem.assemble_stencil(prob.jac, prob.K, prob.nx, prob.ny)
    orc = cycle.Oracle(boxmg.build_hierarchy(S_or))
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        h = dmg.Hierarchy(dev(S_or))
        b = dev(prob.b)
        u, k, rel, hist = h.solve(b, rtol=1e-10)
        for cap in (1, 3, 6):
            u2 = torch.zeros_like(b)
            _, k2, _, _ = h.solve(b, u=u2, rtol=1e-10, max_iters=cap, raise_on_fail=False)
            uo, ko, _, _ = cycle.solve(orc, prob.b, 1e-10, max_iters=cap)
            assert k2 == ko == cap
            assert_iterate(f"max_iters={cap}", host(u2), uo)
    torch.cuda.synchronize()
    uo, ko, histo, _ = cycle.solve(orc, prob.b, 1e-10)
    assert k == ko and np.allclose(hist, histo, rtol=1e-6, atol=1e-13)
    assert_iterate("solution", host(u), uo)
    h.close()


def test_graph_and_eager_solves_are_identical(dmg):
    prob = pb.star(129, seed=1)
    S = dmg.assemble_stencil(dev(prob.jac), dev(prob.K))
    b = dev(prob.b)
    out = []
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    for g in (0, 1):
      with torch.cuda.stream(st):
        h = dmg.Hierarchy(S, use_graph=g)
        u, k, rel, _ = h.solve(b, rtol=1e-10)
        # a second solve on the same arrays replays the captured graph
        u2 = torch.zeros_like(b)
        u2, k2, rel2, _ = h.solve(b, u=u2, rtol=1e-10)
        u3 = torch.zeros_like(b)
        u3, k3, rel3, _ = h.solve(b, u=u3, rtol=1e-10)
        assert k == k2 == k3 and torch.equal(u2, u3)
        out.append((host(u3), k))
        h.close()
    assert out[0][1] == out[1][1] and np.array_equal(out[0][0], out[1][0])


def test_solve_start_tests_the_initial_iterate(dmg):
    """A solve's start tests the initial iterate on the device.  From zero, the first residual
    is b and its pass reads neither the stencil nor u.  From anything else it is formed in full.
    The same captured start (same arrays, so graph replays) is run with a zero guess, a random
    interior guess, a guess that is nonzero only on the boundary ring (a zero residual change, but
    not a zero iterate) and zero again.  Each gives the oracle's step count, history and iterate.
    Float32 refinement from zero gives the same bits before and after a nonzero-guess solve on the
    same arrays."""
    prob = pb.star(257, seed=5)
    S_or = fem.assemble_stencil(prob.jac, prob.K, prob.nx, prob.ny)
    levels = boxmg.build_hierarchy(S_or)
    orc = cycle.Oracle(levels)
    rng = np.random.default_rng(3)
    g_int = np.zeros((prob.ny, prob.nx))
    g_int[1:-1, 1:-1] = rng.uniform(-1.0, 1.0, (prob.ny - 2, prob.nx - 2))
    g_bnd = np.zeros((prob.ny, prob.nx))
    g_bnd[0, :] = 1.0
    g_bnd[:, -1] = -2.0
    zero = np.zeros((prob.ny, prob.nx))
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        h = dmg.Hierarchy(dev(S_or))
        b = dev(prob.b)
        u = torch.zeros_like(b)
        for name, g in (("zero", zero), ("interior guess", g_int), ("boundary-only guess", g_bnd),
                        ("zero again", zero)):
            u.copy_(dev(g))
            x, k, rel, hist = h.solve(b, u=u, rtol=1e-10)
            uo, ko, histo, _ = cycle.solve(orc, prob.b, 1e-10, u0=g.copy())
            assert k == ko, (name, k, ko)
            assert np.allclose(hist, histo, rtol=1e-6, atol=1e-13), name
            # the library writes boundary entries of a solution as 0; the oracle keeps u0's
            assert_iterate(name, host(x)[1:-1, 1:-1].ravel(), np.asarray(uo)[1:-1, 1:-1].ravel())
        h.close()
        h32 = dmg.Hierarchy(dev(S_or), precision=dmg.DMG_FP32_IR, inner_cycles=2)
        x32 = torch.zeros_like(b)
        runs = []
        for g in (zero, g_int, zero):
            x32.copy_(dev(g))
            x, k, rel, _ = h32.solve(b, u=x32, rtol=1e-10)
            assert rel <= 1e-10
            runs.append((x.clone(), k))
        assert torch.equal(runs[0][0], runs[2][0]) and runs[0][1] == runs[2][1]
        u64, _, _, _ = cycle.solve(orc, prob.b, 1e-10)
        err = float(np.linalg.norm(host(runs[1][0]) - u64) / np.linalg.norm(u64))
        assert err < 1e-7, err
        h32.close()
    torch.cuda.synchronize()


def test_grad_K_matches_oracle(dmg):
    """dK_e = -sum_ab lam_a G_e[a,b] u_b per cell, within 1e-12 of sum_ab |lam_a G_ab u_b|."""
    for prob in (pb.star(65, seed=4), pb.quarter_annulus(33, ny=49)):
        nx, ny = prob.nx, prob.ny
        rng = np.random.default_rng(0)
        lam = np.zeros((ny, nx)); lam[1:-1, 1:-1] = rng.normal(size=(ny - 2, nx - 2))
        u = np.zeros((ny, nx)); u[1:-1, 1:-1] = rng.normal(size=(ny - 2, nx - 2))
        g = dmg.grad_K(dev(prob.jac), dev(lam), dev(u))
        go = adjoint.grad_K(prob.jac, lam, u, nx, ny)
        G = fem.element_matrices(prob.jac, nx, ny)
        scale = np.einsum("jia,jiab,jib->ji", np.abs(adjoint.local_values(lam)), np.abs(G),
                          np.abs(adjoint.local_values(u)))
        assert_entrywise("grad_K", host(g), go, scale, 1e-12)


def test_diffsolve_reuses_one_hierarchy_exactly(dmg):
    """Repeated DiffSolve calls share one cached hierarchy, refreshed from each new stencil: every
    call returns bit for bit what a fresh hierarchy's solve from zero returns."""
    n = 65
    prob = pb.star(n, seed=6)
    jac = dev(prob.jac)
    dmg.DiffSolve.clear_cache()
    st = torch.cuda.Stream()                      # a side stream: the solves replay graphs
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        for scale in (1.0, 2.5, 0.3):
            K = dev(prob.K * scale)
            b = dev(prob.b * (1.0 + scale))
            u = dmg.DiffSolve.apply(K, b, jac, 1e-11)
            h = dmg.Hierarchy(dmg.assemble_stencil(jac, K))
            ur, _, _, _ = h.solve(b, rtol=1e-11)
            h.close()
            st.synchronize()
            assert torch.equal(u, ur)
    torch.cuda.synchronize()
    assert len(dmg._DiffSolver._cache) == 1
    dmg.DiffSolve.clear_cache()
    assert len(dmg._DiffSolver._cache) == 0


def test_diffsolve_gradients(dmg):
    n = 33
    prob = pb.star(n, seed=4)
    jac = dev(prob.jac)
    K = dev(prob.K).requires_grad_(True)
    b = dev(prob.b).requires_grad_(True)
    t = dev(prob.target)

    def J_of(Kv, bv):
        u = dmg.DiffSolve.apply(Kv, bv, jac, 1e-13)
        d = (u - t)[1:-1, 1:-1]
        return 0.5 * (d * d).sum()

    J = J_of(K, b)
    J.backward()
    # oracle adjoint gradient
    S_or = fem.assemble_stencil(prob.jac, prob.K, n, n)
    orc = cycle.Oracle(boxmg.build_hierarchy(S_or))
    uo, _, _, _ = cycle.solve(orc, prob.b, 1e-13)
    lo, _, _, _ = cycle.solve(orc, adjoint.objective_grad_u(uo, prob.target), 1e-13)
    gKo = adjoint.grad_K(prob.jac, lo, uo, n, n)
    assert np.linalg.norm(host(K.grad) - gKo) / np.linalg.norm(gKo) <= 1e-6
    assert np.linalg.norm(host(b.grad) - lo) / np.linalg.norm(lo) <= 1e-6
    # entry by entry: both sides solve to 1e-13, so u and lam differ by that solve tolerance
    # times the conditioning (~1e-11 of their size), far below 1e-6
    G = fem.element_matrices(prob.jac, n, n)
    scale = np.einsum("jia,jiab,jib->ji", np.abs(adjoint.local_values(lo)), np.abs(G),
                      np.abs(adjoint.local_values(uo)))
    assert_entrywise("dJ/dK", host(K.grad), gKo, scale, 1e-6)
    assert_iterate("dJ/db", host(b.grad), lo, rtol=1e-6, floor_ulps=int(1e-9 / EPS64))
    # central differences along random directions
    zK, zb = pb.directions(4, 4, (n - 1, n - 1), (n, n))
    with torch.no_grad():
        for d in range(4):
            dK = dev(zK[d] * prob.K)
            db = dev(zb[d])
            eps = 1e-5
            fdK = (J_of(K + eps * dK, b) - J_of(K - eps * dK, b)).item() / (2 * eps)
            fdb = (J_of(K, b + eps * db) - J_of(K, b - eps * db)).item() / (2 * eps)
            adK = float((K.grad * dK).sum())
            adb = float((b.grad * db).sum())
            assert abs(fdK - adK) <= 1e-6 * max(abs(adK), 1e-12)
            assert abs(fdb - adb) <= 1e-6 * max(abs(adb), 1e-12)


def test_diffsolve_reports_non_convergence(dmg):
    """A forward or adjoint solve that stops above rtol raises (unless strict=False, which
    returns the last iterate and reports its residual)."""
    n = 33
    prob = pb.star(n, seed=5)
    jac = dev(prob.jac)
    K = dev(prob.K).requires_grad_(True)
    b = dev(prob.b)
    with pytest.raises(dmg.DmgError) as ei:
        dmg.DiffSolve.apply(K, b, jac, 1e-10, 1)
    assert ei.value.code == 6 and "forward" in str(ei.value)
    u = dmg.DiffSolve.apply(K, b, jac, 1e-10, 1, None, False)
    its, rr = dmg.DiffSolve.last["forward"]
    assert its == 1 and rr > 1e-10
    # b = 0 solves exactly (u = 0, relative residual 0); the adjoint of a loss with a nonzero
    # target cannot reach 1e-16 in three cycles: backward raises
    t = dev(prob.target)
    u = dmg.DiffSolve.apply(K, torch.zeros_like(b), jac, 1e-16, 3)
    assert float(u.detach().abs().max()) == 0.0
    with pytest.raises(dmg.DmgError) as ei:
        ((u - t) ** 2).sum().backward()
    assert "adjoint" in str(ei.value)
    dmg.DiffSolve.clear_cache()


def test_stats_match_oracle_complexities(dmg):
    """Levels, grid complexity and operator complexity (Sec. 4 definitions) against the
    oracle's hierarchy."""
    for prob in (pb.star(129, seed=1), pb.quarter_annulus(33, ny=49), pb.star(45, seed=1, ny=67)):
        S_or = fem.assemble_stencil(prob.jac, prob.K, prob.nx, prob.ny)
        levels = boxmg.build_hierarchy(S_or)
        gc, oc = boxmg.complexities(levels)
        h = dmg.Hierarchy(dev(S_or))
        lv, hgc, hoc = h.stats()
        h.close()
        assert lv == len(levels)
        assert abs(hgc - gc) <= 1e-14 * gc and abs(hoc - oc) <= 1e-14 * oc, (hgc, gc, hoc, oc)


def test_transfer_matches_oracle(dmg):
    mp = pb.Star.random(pb.streams(1)[0])
    n = 33
    mesh = pb.lattice_mesh(mp, 45, np.random.default_rng(7))
    T = dmg.Transfer(mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, n, n, nq=4)
    M = transfer.p1_mass(mesh.xy_p, mesh.tris, mesh.dof)
    Co = transfer.coupled_mass(mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, n, n, nq=4)
    nnzC, nnzM = T.nnz()
    assert nnzC == Co.nnz and nnzM == M.nnz
    rng = np.random.default_rng(3)
    uc = np.zeros((n, n)); uc[1:-1, 1:-1] = rng.normal(size=(n - 2, n - 2))
    rp = rng.normal(size=mesh.nv)
    up = T.from_grid(dev(uc))
    rc = T.to_grid(dev(rp))
    # CG2 is two steps of an iteration: its outputs are compared as iterates
    assert_iterate("from_grid", host(up), transfer.from_grid(M, Co, uc))
    assert_iterate("to_grid", host(rc), transfer.to_grid(M, Co, rp * mesh.dof, n, n))
    T.close()


@pytest.mark.parametrize("nq", [4, 0])
def test_transfer_from_caller_csr_matches_oracle(dmg, nq):
    """The transfer created from the caller's C and M_p (device CSR, caller workspace, C^T formed
    on the device): from_grid = CG2(M_p, C u_c) and to_grid = C^T CG2(M_p, r_p) against the
    oracle's, entry by entry, for the rasterised (nq = 4) and exact (nq = 0) coupled mass; and
    against the transfer the library assembles from the same mesh."""
    mp = pb.Star.random(pb.streams(2)[0])
    n = 33
    mesh = pb.lattice_mesh(mp, 45, np.random.default_rng(8))
    M = transfer.p1_mass(mesh.xy_p, mesh.tris, mesh.dof)
    Co = transfer.coupled_mass(mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, n, n, nq=nq).tocsr()
    T = dmg.Transfer.from_csr(Co, M, n, n)
    assert T.nnz() == (Co.nnz, M.nnz)
    rp, ci, v = T.copy_C()
    assert np.array_equal(rp, Co.indptr) and np.array_equal(ci, Co.indices) and np.array_equal(v, Co.data)
    Tm = dmg.Transfer(mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, n, n, nq=nq)
    rng = np.random.default_rng(4)
    for _ in range(2):
        uc = np.zeros((n, n)); uc[1:-1, 1:-1] = rng.normal(size=(n - 2, n - 2))
        rpv = rng.normal(size=mesh.nv) * mesh.dof
        up = host(T.from_grid(dev(uc)))
        rc = host(T.to_grid(dev(rpv)))
        assert_iterate("from_grid (CSR)", up, transfer.from_grid(M, Co, uc))
        assert_iterate("to_grid (CSR)", rc, transfer.to_grid(M, Co, rpv, n, n))
        assert_iterate("from_grid, CSR vs mesh form", up, host(Tm.from_grid(dev(uc))))
        assert_iterate("to_grid, CSR vs mesh form", rc, host(Tm.to_grid(dev(rpv))))
    T.close()
    Tm.close()
    # a column index beyond the grid is rejected by the device check before C^T is formed
    bad = Co.copy()
    bad.indices[bad.indptr[5]] = n * n + 3
    with pytest.raises(dmg.DmgError) as ei:
        dmg.Transfer.from_csr(bad, M, n, n)
    assert ei.value.code == 1 and "out of range" in str(ei.value)


@pytest.mark.parametrize("nq,nx,ny,m", [(4, 33, 33, 45), (0, 33, 33, 45), (4, 41, 29, 45),
                                        (0, 29, 41, 45), (4, 65, 49, 13), (0, 65, 65, 13)])
def test_matrix_free_transfer_matches_oracle(dmg, nq, nx, ny, m):
    """DMG_MESH_MATRIX_FREE stores no C: every apply recomputes the triangle-cell integrals from
    the overlap sets.  from_grid and to_grid against the oracle's (assembled C) and against the
    library's assembled form of the same mesh, entry by entry; grid boundary values of u_c and
    Dirichlet entries of r_p are ignored as in the assembled form; two applies in a row (the
    buffer between the kernels is rewritten); no C to copy, and less device memory.  m = 13 is a
    mesh coarser than the grid: each triangle's box spans about 5 x 5 cells (rows of C longer
    than the device merge holds, so the assembled form falls back to the host)."""
    mp = pb.Star.random(pb.streams(3)[0])
    mesh = pb.lattice_mesh(mp, m, np.random.default_rng(9))
    M = transfer.p1_mass(mesh.xy_p, mesh.tris, mesh.dof)
    Co = transfer.coupled_mass(mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, nx, ny, nq=nq)
    Tf = dmg.Transfer(mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, nx, ny, nq=nq, matrix_free=True)
    Ta = dmg.Transfer(mesh.xy_c, mesh.xy_p, mesh.tris, mesh.dof, nx, ny, nq=nq)
    assert Tf.nnz() == (0, M.nnz)
    bytes_f, pairs = Tf.memory()
    bytes_a, pairs_a = Ta.memory()
    assert pairs > 0 and pairs_a == 0, (pairs, pairs_a)
    if m > nx:                                           # a mesh finer than the grid
        assert bytes_f < bytes_a, (bytes_f, bytes_a)
    with pytest.raises(dmg.DmgError) as ei:
        Tf.copy_C()
    assert ei.value.code == 8
    rng = np.random.default_rng(5)
    for _ in range(2):
        uc = rng.normal(size=(ny, nx))                   # boundary values too: ignored
        rpv = rng.normal(size=mesh.nv)                   # Dirichlet entries too: ignored
        up = host(Tf.from_grid(dev(uc)))
        rc = host(Tf.to_grid(dev(rpv)))
        assert_iterate("from_grid (matrix-free)", up, transfer.from_grid(M, Co, uc))
        assert_iterate("to_grid (matrix-free)", rc, transfer.to_grid(M, Co, rpv * mesh.dof, nx, ny))
        assert_iterate("from_grid, matrix-free vs assembled", up, host(Ta.from_grid(dev(uc))))
        assert_iterate("to_grid, matrix-free vs assembled", rc, host(Ta.to_grid(dev(rpv))))
    Tf.close()
    Ta.close()


@pytest.mark.parametrize("precision,n,ny", [(0, 257, 193), (1, 257, 193), (0, 33, 33), (1, 45, 67),
                                            (0, 65, 17)])
def test_refresh_assembled_equals_assemble_then_refresh(dmg, precision, n, ny):
    """dmg_refresh_assembled (the fine stencil assembled straight into the hierarchy, planar and
    point-major) against dmg_assemble_stencil + dmg_refresh: every level's stencil and weights bit
    for bit, and the same solve bit for bit; called three times so that the captured setup graph
    is replayed (on a side stream), with new coefficients in between.  Small grids run whole in
    the coarse kernel; widths below and not a multiple of the 64-column assembly tile."""
    p1, p2 = pb.star(n, seed=61, ny=ny), pb.star(n, seed=62, ny=ny)
    jac, K = dev(p1.jac), dev(p1.K)
    b = dev(p1.b)
    S = dmg.assemble_stencil(jac, K)
    ha = dmg.Hierarchy(S, precision=precision)
    hb = dmg.Hierarchy(S, precision=precision)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for rep in range(3):
            if rep == 2:                                  # new coefficients in the same arrays
                jac.copy_(dev(p2.jac))
                K.copy_(dev(p2.K))
            dmg.assemble_stencil(jac, K, out=S)
            ha.refresh(S)
            hb.refresh_assembled(jac, K)
            for l in range(ha.num_levels):
                Sa, Pa = ha.level(l)
                Sb, Pb = hb.level(l)
                assert torch.equal(Sa, Sb), (rep, l)
                assert (Pa is None) == (Pb is None) and (Pa is None or torch.equal(Pa, Pb)), (rep, l)
            xa, ka, _, _ = ha.solve(b, rtol=1e-10)
            xb, kb, _, _ = hb.solve(b, rtol=1e-10)
            assert ka == kb and torch.equal(xa, xb), rep
    torch.cuda.synchronize()
    ha.close()
    hb.close()


def _batch_vs_single(dmg, Ss, bs, bt, us, its, rels, probs=None, orders=None):
    """The batch runs its coarse levels in the one-workgroup coarse kernel: its iterates equal
    single solves with coarse_gemv=0 (and the same colour orders) bitwise, and single solves
    with the whole-GPU dense coarse operator (the default) to rounding.  With `probs`, every
    instance is also solved by the oracle (same colour orders): the same cycle count and the
    solution entry by entry."""
    for k, (S, b, u, it, r) in enumerate(zip(Ss, bs, us, its, rels)):
        pre, post = orders[k] if orders else ((0, 1, 2, 3), (3, 2, 1, 0))
        h = dmg.Hierarchy(S, coarse_gemv=0, pre_order=pre, post_order=post)
        u1, k1, r1, _ = h.solve(b, rtol=1e-10)
        assert it == k1 and r <= 1e-10
        assert abs(r - r1) <= 1e-13 * max(r1, 1e-300) * 10
        assert torch.equal(u, u1)
        h.close()
        h = dmg.Hierarchy(S, pre_order=pre, post_order=post)
        u2, k2, r2, _ = h.solve(b, rtol=1e-10)
        assert k2 == it and r2 <= 1e-10
        assert_iterate(f"instance {k}: dense coarse operator vs batch", host(u2), host(u))
        h.close()
        if probs is not None:
            p = probs[k]
            orc = cycle.Oracle(boxmg.build_hierarchy(fem.assemble_stencil(p.jac, p.K, p.nx, p.ny)),
                               pre=pre, post=post)
            uo, ko, _, _ = cycle.solve(orc, p.b, 1e-10, max_iters=300)
            assert it == ko, (k, it, ko)
            assert_iterate(f"instance {k} ({p.nx}x{p.ny}) vs oracle", host(u), uo)


def test_batch_matches_single_solves(dmg):
    """Uneven sizes (one all-tail instance), different convergence counts: every instance's
    iterate equals its single solve bitwise and the oracle's solution entry by entry."""
    probs = [pb.star(n, seed=10 + k) for k, n in enumerate((33, 65, 129, 65, 257, 129))]
    probs.append(pb.quarter_annulus(65))          # needs many more cycles than the stars
    Ss = [dmg.assemble_stencil(dev(p.jac), dev(p.K)) for p in probs]
    bs = [dev(p.b) for p in probs]
    bt = dmg.BatchSolver(Ss)
    us, its, rels = bt.solve(bs, rtol=1e-10)
    assert len(set(its)) > 1
    _batch_vs_single(dmg, Ss, bs, bt, us, its, rels, probs=probs)
    # a second solve on new arrays rebuilds the schedule; autotuned shapes change no bit
    bt.autotune(bs, reps=1, tiles=True)
    us2, its2, rels2 = bt.solve(bs, rtol=1e-10)
    assert its2 == its and all(torch.equal(a, c) for a, c in zip(us, us2))
    bt.close()


def test_batch_tuned_colour_order_matches_oracle(dmg):
    """The batch tuner picks a colour-order pair per size class by timing whole batched solves;
    each instance then runs its class's pair and equals its single solve with that pair bit for
    bit and the oracle's solve with that pair entry by entry (same cycle counts)."""
    sizes = (129, 65, 257, 129, 65, 33, 257)
    probs = [pb.star(n, seed=40 + k) for k, n in enumerate(sizes)]
    probs.append(pb.quarter_annulus(65))
    Ss = [dmg.assemble_stencil(dev(p.jac), dev(p.K)) for p in probs]
    bs = [dev(p.b) for p in probs]
    bt = dmg.BatchSolver(Ss)
    cfg = bt.autotune(bs, reps=4, tiles=True, colour_order=True)
    orders = cfg["orders"]
    by_class = {}
    for p, (pre, post) in zip(probs, orders):
        assert post == pre[::-1] and sorted(pre) == [0, 1, 2, 3]
        assert by_class.setdefault((p.nx, p.ny), (pre, post)) == (pre, post)  # one pair per class
    print(f"[batch] tuned colour orders per class {by_class}, tail threads {cfg['tail_threads']}")
    assert tuple(cfg["pre_order"]) == orders[0][0]
    us, its, rels = bt.solve(bs, rtol=1e-10)
    assert max(rels) <= 1e-10
    _batch_vs_single(dmg, Ss, bs, bt, us, its, rels, probs=probs, orders=orders)
    bt.close()


def test_batch_with_odd_dims_matches_single_solves(dmg):
    """Odd dims that are not 2^k + 1, rectangular, mixed with a 2^k + 1 instance; two instances
    share every level size (97 x 65)."""
    probs = [pb.star(97, seed=31, ny=65), pb.quarter_annulus(33, ny=49), pb.star(65, seed=32),
             pb.star(45, seed=33, ny=67), pb.star(97, seed=34, ny=65)]
    Ss = [dmg.assemble_stencil(dev(p.jac), dev(p.K)) for p in probs]
    bs = [dev(p.b) for p in probs]
    bt = dmg.BatchSolver(Ss)
    us, its, rels = bt.solve(bs, rtol=1e-10)
    _batch_vs_single(dmg, Ss, bs, bt, us, its, rels, probs=probs)
    bt.close()


@pytest.mark.parametrize("smoother", [1, 3])
def test_batch_line_relaxation_matches_single_solves(dmg, smoother):
    """Zebra line relaxation in the batch (x-lines, alternating): the line steps of one level size
    run as one launch over every instance that has it.  Each instance's solution equals its
    single line-smoothed solve (coarse_gemv = 0) bit for bit with the same cycle count, and the
    oracle's line-smoothed solve entry by entry; autotuning changes nothing."""
    probs = [pb.quarter_annulus(65), pb.quarter_annulus(129, ny=97), pb.star(65, seed=51),
             pb.quarter_annulus(33, ny=49), pb.star(97, seed=52, ny=65), pb.quarter_annulus(65, seed=3)]
    Ss = [dmg.assemble_stencil(dev(p.jac), dev(p.K)) for p in probs]
    bs = [dev(p.b) for p in probs]
    bt = dmg.BatchSolver(Ss, smoother=smoother)
    us, its, rels = bt.solve(bs, rtol=1e-10, max_iters=300)
    assert max(rels) <= 1e-10
    for k, (S, b, u, it, r, p) in enumerate(zip(Ss, bs, us, its, rels, probs)):
        h = dmg.Hierarchy(S, coarse_gemv=0, smoother=smoother)
        u1, k1, r1, _ = h.solve(b, rtol=1e-10, max_iters=300)
        h.close()
        assert it == k1, (k, it, k1)
        assert abs(r - r1) <= 1e-12 * r1, (k, r, r1)    # the norms' partial sums differ
        assert torch.equal(u, u1), k
        orc = cycle.Oracle(boxmg.build_hierarchy(fem.assemble_stencil(p.jac, p.K, p.nx, p.ny)),
                           smoother=LINE[smoother])
        uo, ko, _, _ = cycle.solve(orc, p.b, 1e-10, max_iters=300)
        assert it == ko, (k, it, ko)
        assert_iterate(f"instance {k} ({p.nx}x{p.ny}) line batch vs oracle", host(u), uo)
    cfg = bt.autotune(bs, reps=1, tiles=True, colour_order=True)
    assert cfg["pre_order"] == [0, 1, 2, 3]              # line relaxation visits no colours
    us2, its2, _ = bt.solve(bs, rtol=1e-10, max_iters=300)
    assert its2 == its and all(torch.equal(a, c) for a, c in zip(us, us2))
    bt.close()


def test_batch_zero_rhs_and_limits(dmg):
    probs = [pb.star(n, seed=20 + k) for k, n in enumerate((129, 65, 257))]
    Ss = [dmg.assemble_stencil(dev(p.jac), dev(p.K)) for p in probs]
    bs = [dev(p.b) for p in probs]
    bs[1] = torch.zeros_like(bs[1])
    bt = dmg.BatchSolver(Ss)
    us0 = [torch.ones_like(b) for b in bs]
    us, its, rels = bt.solve(bs, us=us0, rtol=1e-10)
    assert its[1] == 0 and rels[1] == 0.0 and float(us[1].abs().max()) == 0.0
    assert its[0] > 0 and its[2] > 0 and max(rels) <= 1e-10
    # a step budget too small for the tolerance: no convergence reported, counts capped
    with pytest.raises(dmg.DmgError) as ei:
        bt.solve(bs, rtol=1e-10, max_iters=3)
    assert ei.value.code == 6
    _, its3, _ = bt.solve(bs, rtol=1e-10, max_iters=3, raise_on_fail=False)
    assert its3[0] == 3 and its3[2] == 3 and its3[1] == 0
    bt.close()


# ---- edge cases -------------------------------------------------------------------------
@pytest.mark.parametrize("n", [3, 5, 9])
def test_tiny_grids(dmg, n):
    prob = pb.star(n, seed=1)
    S_or = fem.assemble_stencil(prob.jac, prob.K, n, n)
    levels = boxmg.build_hierarchy(S_or)
    h = dmg.Hierarchy(dev(S_or))
    u, k, rel, _ = h.solve(dev(prob.b), rtol=1e-10)
    uo, ko, _, _ = cycle.solve(cycle.Oracle(levels), prob.b, 1e-10)
    assert k == ko
    assert_iterate(f"{n}x{n} solution", host(u), uo)
    h.close()


def test_coarsest_dense_cholesky_larger(dmg):
    prob = pb.star(65, seed=1, ny=129)
    S_or = fem.assemble_stencil(prob.jac, prob.K, 65, 129)
    levels = boxmg.build_hierarchy(S_or, coarsest_n=9)
    h = dmg.Hierarchy(dev(S_or), coarsest_n=9)
    assert h.num_levels == len(levels)
    u, k, rel, _ = h.solve(dev(prob.b), rtol=1e-10)
    uo, ko, _, _ = cycle.solve(cycle.Oracle(levels), prob.b, 1e-10)
    assert k == ko
    assert_iterate("solution", host(u), uo)
    h.close()


def test_zero_rhs_and_failures(dmg):
    prob = pb.star(33, seed=1)
    S = dmg.assemble_stencil(dev(prob.jac), dev(prob.K))
    h = dmg.Hierarchy(S)
    u = torch.ones((33, 33), dtype=torch.float64, device="cuda")
    u, k, rel, _ = h.solve(torch.zeros_like(u), u=u)
    assert k == 0 and torch.count_nonzero(u) == 0
    with pytest.raises(dmg.DmgError) as ei:
        h.solve(dev(prob.b), rtol=1e-10, max_iters=2)
    assert ei.value.code == 6
    bad = dev(prob.b)
    bad[5, 5] = float("nan")
    with pytest.raises(dmg.DmgError) as ei:
        h.solve(bad)
    assert ei.value.code == 5
    # a NaN in the initial guess, inside or on the boundary ring, is not a zero iterate: the
    # start forms the residual in full and reports it
    for where in ((7, 9), (0, 3)):
        u_nan = torch.zeros((33, 33), dtype=torch.float64, device="cuda")
        u_nan[where] = float("nan")
        with pytest.raises(dmg.DmgError) as ei:
            h.solve(dev(prob.b), u=u_nan)
        assert ei.value.code == 5, where
    h.close()
    Sneg = -S
    with pytest.raises(dmg.DmgError) as ei:
        dmg.Hierarchy(Sneg)
    assert ei.value.code == 4


LINE = {1: "xline", 2: "yline", 3: "alt"}


@pytest.mark.parametrize("smoother", [1, 2, 3])
@pytest.mark.parametrize("name", ["annulus65", "star65x129", "star97x65", "layer65"])
def test_line_smoother_matches_oracle(dmg, name, smoother):
    """Zebra line relaxation (x-lines, y-lines, alternating): every V-cycle iterate to 1e-12,
    and the whole solve (cycle count, residual history)."""
    prob = PROBLEMS[name]()
    S_or = fem.assemble_stencil(prob.jac, prob.K, prob.nx, prob.ny)
    orc = cycle.Oracle(boxmg.build_hierarchy(S_or), smoother=LINE[smoother])
    h = dmg.Hierarchy(dev(S_or), smoother=smoother)
    b = dev(prob.b)
    u = torch.zeros_like(b)
    uo = np.zeros(prob.nx * prob.ny)
    for k in range(3):
        h.vcycle(u, b)
        orc.vcycle(uo, prob.b.ravel())
        assert_iterate(f"iterate {k + 1}", host(u).ravel(), uo)
    x, k, rel, hist = h.solve(b, rtol=1e-10, max_iters=300)
    xo, ko, histo, _ = cycle.solve(orc, prob.b, rtol=1e-10, max_iters=300)
    assert k == ko and rel <= 1e-10
    assert np.allclose(hist, histo, rtol=1e-6, atol=1e-13)
    assert_iterate("solution", host(x), xo)
    h.close()


def test_line_smoother_graph_and_limits(dmg):
    prob = pb.quarter_annulus(65)
    S = dmg.assemble_stencil(dev(prob.jac), dev(prob.K))
    h = dmg.Hierarchy(S, smoother=3)
    b = dev(prob.b)
    x_e, k_e, _, h_e = h.solve(b, rtol=1e-10)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(2):          # captured chunks of cycles, then their replay
            x_g, k_g, _, h_g = h.solve(b, rtol=1e-10)
    torch.cuda.synchronize()
    assert k_g == k_e and h_g == h_e and torch.equal(x_g, x_e)
    assert k_e <= 10                # point smoothing needs ~55 cycles here
    # refresh recomputes the line factors: the operator doubled halves every iterate.  Scaling
    # by two commutes with every rounding except the square roots of the coarsest Cholesky
    # factor, whose rounding now reaches every cycle through the dense coarse operators: equal
    # to a few ulps
    h.refresh(2.0 * S)
    x_2, k_2, _, _ = h.solve(b, rtol=1e-10)
    assert k_2 == k_e
    assert float((2.0 * x_2 - x_e).abs().max()) <= 1e-13 * float(x_e.abs().max())
    h.close()
