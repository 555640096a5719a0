"""Whole-grid parity at the benchmark sizes: the 1025 x 1025 star (root seed 1) and the
4097 x 4097 star (root seed 2), in the launch configuration bench.py times (autotuned launch
shapes, and for float32 refinement the tuned number of float32 cycles per step).

The inputs (map Jacobians at the Gauss points, log-normal K, b) come from the seeded on-device
generator bench.py uses; both the library and the oracle receive those same arrays.  Every
comparison is entry by entry over the whole grid (tests/entrywise.py):
  * 1025^2: every level's stencil, Galerkin stencil and interpolation weights; every one of the
    float64 V-cycle iterates to convergence, the solve's cycle count, residual history and
    solution (bitwise equal to the last cycle's iterate); the float32-refined solve step by step
    against the oracle's refinement, and its solution against the float64 oracle solution;
  * 4097^2: every level's stencil and interpolation weights, the float64 solve's cycle count,
    history and solution, and the float32-refined solution against the oracle's refinement and
    against the float64 oracle solution;
  * the 256-instance batch (sizes 129^2 to 1025^2, root seed 3): every instance against its single
    solve bit for bit, and one instance of each size against the oracle;
  * the differentiable solve on the 2049^2 star (root seed 4): dJ/dK per cell and dJ/db against
    the oracle's adjoint gradient of the same arrays.
"""
import numpy as np
import pytest
import torch

from entrywise import EPS32, EPS64, assert_entrywise, assert_hierarchy, assert_iterate, grid_floor_ulps
from oracle import adjoint, boxmg, cycle, fem
from problems.batch_device import star_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dmg():
    import paper_2509_08109_amd as m
    m.lib()
    return m


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _say(msg):
    print(f"[fullsize] {msg}", flush=True)


def _levels(h):
    out = []
    for l in range(h.num_levels):
        S, P = h.level(l)
        out.append((host(S), None if P is None else host(P)))
    return out


def _inputs(dmg, n, seed):
    jac, K, b = star_device(n, seed, "cuda")
    S = dmg.assemble_stencil(jac, K)
    jac_h, K_h, b_h = host(jac), host(K), host(b)
    del jac, K
    return S, b, jac_h, K_h, b_h


def _fp32_check(name, got, ref):
    used = assert_iterate(name, got, ref, rtol=1e-5, eps=EPS32, floor_ulps=64)
    _say(f"{name}: worst excess {used:.2f} eps32 max|x|")
    return used


def test_bench_config_1025_whole_grid(dmg):
    n, seed = 1025, 1
    S, b, jac_h, K_h, b_h = _inputs(dmg, n, seed)
    S_or = fem.assemble_stencil(jac_h, K_h, n, n)
    levels = boxmg.build_hierarchy(S_or)
    h = dmg.Hierarchy(S)
    cfg = h.autotune(b, tiles=True, reps=5)                 # bench.py's float64 configuration
    _say(f"{n}: tuned {cfg['levels']} / {cfg['post_levels']}")
    assert h.num_levels == len(levels)
    w = assert_hierarchy(f"{n}x{n} hierarchy", _levels(h), levels)
    _say(f"{n}: hierarchy worst |got - ref| / scale {w:.2e}")
    orc = cycle.Oracle(levels)
    uo, ko, histo, its = cycle.solve(orc, b_h, 1e-10, keep_iterates=True)
    u = torch.zeros_like(b)
    worst = 0.0
    for k in range(ko):
        h.vcycle(u, b)
        worst = max(worst, assert_iterate(f"{n}x{n} iterate {k + 1}", host(u), its[k],
                                          floor_ulps=grid_floor_ulps(n)))
    _say(f"{n}: {ko} iterates, worst excess {worst:.1f} eps max|u|")
    x, kx, rel, hist = h.solve(b, rtol=1e-10)
    assert kx == ko and rel <= 1e-10
    assert np.allclose(hist, histo, rtol=1e-6, atol=1e-13)
    assert torch.equal(x, u), "the solve's iterate is the last V-cycle's"
    h.close()
    # float32 refinement as bench.py runs it
    h32 = dmg.Hierarchy(S, precision=dmg.DMG_FP32_IR)
    cfg = h32.autotune(b, tiles=True, reps=5, inner_cycles=True)
    m = cfg["inner_cycles"]
    xo, ko32, _, its32 = cycle.solve_ir(orc, cycle.Oracle(levels, np.float32), b_h, 1e-10, inner=m,
                                        keep_iterates=True)
    x32, k32, rel32, _ = h32.solve(b, rtol=1e-10)
    assert k32 == ko32 and rel32 <= 1e-10
    for step in range(1, ko32 + 1):
        xs, _, _, _ = h32.solve(b, rtol=1e-10, max_iters=step, raise_on_fail=False)
        _fp32_check(f"{n}x{n} fp32 (m={m}) step {step}", host(xs), its32[step - 1])
    err = float(np.linalg.norm(host(x32) - uo) / np.linalg.norm(uo))
    _say(f"{n}: fp32-refined m={m}, {k32} steps, error vs float64 oracle solution {err:.2e}")
    assert err < 1e-7
    h32.close()


def test_bench_config_4097_whole_grid(dmg):
    n, seed = 4097, 2
    S, b, jac_h, K_h, b_h = _inputs(dmg, n, seed)
    _say(f"{n}: oracle assembly and hierarchy")
    S_or = fem.assemble_stencil(jac_h, K_h, n, n)
    del jac_h, K_h
    levels = boxmg.build_hierarchy(S_or)
    h = dmg.Hierarchy(S)
    h.autotune(b, tiles=True, reps=5)
    assert h.num_levels == len(levels)
    # the Galerkin triple-product scale is checked at 1025^2; here the sqrt(C_v C_n) scale
    w = assert_hierarchy(f"{n}x{n} hierarchy", _levels(h), levels, galerkin=False)
    _say(f"{n}: hierarchy worst |got - ref| / scale {w:.2e}; oracle solve")
    orc = cycle.Oracle(levels)
    uo, ko, histo, _ = cycle.solve(orc, b_h, 1e-10)
    x, k, rel, hist = h.solve(b, rtol=1e-10)
    assert k == ko and rel <= 1e-10
    assert np.allclose(hist, histo, rtol=1e-6, atol=1e-13)
    used = assert_iterate(f"{n}x{n} float64 solution", host(x), uo, floor_ulps=grid_floor_ulps(n))
    _say(f"{n}: float64 {k} cycles, worst excess {used:.1f} eps max|u|")
    h.close()
    h32 = dmg.Hierarchy(S, precision=dmg.DMG_FP32_IR)
    cfg = h32.autotune(b, tiles=True, reps=5, inner_cycles=True)
    m = cfg["inner_cycles"]
    x32, k32, rel32, _ = h32.solve(b, rtol=1e-10)
    del S
    xo32, ko32, _, _ = cycle.solve_ir(orc, cycle.Oracle(levels, np.float32), b_h, 1e-10, inner=m)
    assert k32 == ko32 and rel32 <= 1e-10
    _fp32_check(f"{n}x{n} fp32-refined solution (m={m})", host(x32), xo32)
    err = float(np.linalg.norm(host(x32) - uo) / np.linalg.norm(uo))
    _say(f"{n}: fp32-refined m={m}, {k32} steps, error vs float64 oracle solution {err:.2e}")
    assert err < 1e-7
    h32.close()


def test_batch_bench_config(dmg):
    """The batch workload bench.py times: 256 star instances, sizes uniform over
    {129, 257, 513, 1025}^2 (root seed 3), tuned as bench.py tunes them (segment heights, tail
    workgroup size, one colour-order pair per size class).  Every instance converges and equals its
    single solve (coarse kernel, the same colour orders) bit for bit; the first instance of each
    size class equals the oracle's solve of the same arrays (cycle count, and the solution entry by
    entry)."""
    from problems.batch_device import star_batch_device

    Ss, bs, sizes, first = [], [], [], {}
    for k, (n, jac, K, b) in enumerate(star_batch_device(256, device="cuda")):
        Ss.append(dmg.assemble_stencil(jac, K))
        bs.append(b)
        sizes.append(n)
        if n not in first:
            first[n] = (k, host(jac), host(K), host(b))
        del jac, K
    _say(f"batch: {len(Ss)} instances, sizes {sorted(set(sizes))}")
    bt = dmg.BatchSolver(Ss)
    cfg = bt.autotune(bs, reps=2, tiles=True, colour_order=True)
    orders = cfg["orders"]
    us, its, rels = bt.solve(bs, rtol=1e-10)
    assert max(rels) <= 1e-10
    _say(f"batch: cycles {min(its)}..{max(its)}, max relres {max(rels):.2e}")
    for k, (S, b) in enumerate(zip(Ss, bs)):
        pre, post = orders[k]
        h = dmg.Hierarchy(S, coarse_gemv=0, pre_order=pre, post_order=post)
        u1, k1, _, _ = h.solve(b, rtol=1e-10)
        assert k1 == its[k] and torch.equal(us[k], u1), (k, sizes[k])
        h.close()
    for n, (k, jac_h, K_h, b_h) in sorted(first.items()):
        pre, post = orders[k]
        orc = cycle.Oracle(boxmg.build_hierarchy(fem.assemble_stencil(jac_h, K_h, n, n)),
                           pre=pre, post=post)
        uo, ko, _, _ = cycle.solve(orc, b_h, 1e-10, max_iters=300)
        assert its[k] == ko, (k, n, its[k], ko)
        used = assert_iterate(f"batch instance {k} ({n}x{n}) vs oracle", host(us[k]), uo,
                              floor_ulps=grid_floor_ulps(n))
        _say(f"batch instance {k} ({n}x{n}): {ko} cycles, worst excess {used:.1f} eps max|u|")
    bt.close()


def test_gradient_bench_config_2049(dmg):
    """The differentiable solve bench.py times: the 2049^2 star (root seed 4), J(u) = 1/2 ||u - u_t||^2
    over the interior, with bench.py's tolerance (1e-10) for the forward and the adjoint solve.  Both
    sides take the same cycle counts, so u and lambda are the same iterates (parity to rounding, not
    to the solve tolerance).  DiffSolve's dJ/dK (per cell) is compared with the oracle's adjoint
    gradient of the same arrays within 1e-9 of sum_ab |lam_a G_e[a,b] u_b|, and dJ/db (= lambda)
    entry by entry within 1e-9."""
    import problems as pb

    n = 2049
    prob = pb.star(n, seed=4, device="cuda")
    as_dev = lambda x: torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()
    jac = as_dev(prob.jac)
    K = as_dev(prob.K).requires_grad_(True)
    b = as_dev(prob.b).requires_grad_(True)
    t = as_dev(prob.target)
    u = dmg.DiffSolve.apply(K, b, jac, 1e-10)
    d = (u - t)[1:-1, 1:-1]
    (0.5 * (d * d).sum()).backward()
    gK, gb = host(K.grad), host(b.grad)
    kf, ka = dmg.DiffSolve.last["forward"][0], dmg.DiffSolve.last["adjoint"][0]
    dmg.DiffSolve.clear_cache()
    del jac, K, b, t, u, d
    torch.cuda.empty_cache()
    S_or = fem.assemble_stencil(prob.jac, prob.K, n, n)
    orc = cycle.Oracle(boxmg.build_hierarchy(S_or))
    uo, ko, _, _ = cycle.solve(orc, prob.b, 1e-10)
    lo, kl, _, _ = cycle.solve(orc, adjoint.objective_grad_u(uo, prob.target), 1e-10)
    assert (kf, ka) == (ko, kl), ((kf, ka), (ko, kl))
    gKo = adjoint.grad_K(prob.jac, lo, uo, n, n)
    G = fem.element_matrices(prob.jac, n, n)
    scale = np.einsum("jia,jiab,jib->ji", np.abs(adjoint.local_values(lo)), np.abs(G),
                      np.abs(adjoint.local_values(uo)))
    assert_entrywise("2049x2049 dJ/dK", gK, gKo, scale, 1e-9)
    assert_iterate("2049x2049 dJ/db", gb, lo, rtol=1e-9, floor_ulps=int(1e-12 / EPS64))
    rel = float(np.linalg.norm(gK - gKo) / np.linalg.norm(gKo))
    _say(f"gradient 2049: oracle {ko} + {kl} cycles; ||dK - dK_oracle|| / ||dK_oracle|| = {rel:.2e}")
