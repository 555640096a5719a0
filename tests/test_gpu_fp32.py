"""Float32 V-cycles inside float64 iterative refinement (DMG_FP32_IR) against the oracle's
refinement (cycle.solve_ir): r = b - A x in float64, s = ||r||, r32 = fl32(r / s), e = 0, m
float32 V-cycles on (e, r32) with float32 roundings of the float64 Galerkin hierarchy (the
coarsest solve in float64), x += s e.

Bounds (entry by entry, tests/entrywise.py): one float32 cycle agrees with the oracle's float32
cycle to 1e-5 |ref| + FP32_FLOOR eps32 max|ref| (the two sum in different orders in float32,
and the library applies the levels below 33 x 33 as their float64 dense operator rounded to
float32); every refined iterate agrees with the oracle's to the same bound; the outer step
counts are equal.  The same holds with zebra line relaxation, whose float32 line solves (Thomas
recurrences here, LU in the oracle) differ by rounding."""
import numpy as np
import pytest
import torch

import problems as pb
from entrywise import EPS32, EPS64, assert_iterate
from oracle import boxmg, cycle, fem

pytestmark = pytest.mark.gpu
FP32_FLOOR = 64


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


LINE = {1: "xline", 2: "yline", 3: "alt"}


def _setup(prob, smoother=0):
    S_or = fem.assemble_stencil(prob.jac, prob.K, prob.nx, prob.ny)
    levels = boxmg.build_hierarchy(S_or)
    sm = LINE.get(smoother, "point")
    return (S_or, levels, cycle.Oracle(levels, smoother=sm),
            cycle.Oracle(levels, np.float32, smoother=sm))


def _check_fp32(name, got, ref):
    used = assert_iterate(name, got, ref, rtol=1e-5, eps=EPS32, floor_ulps=FP32_FLOOR)
    print(f"[fp32] {name}: worst excess {used:.2f} eps32 max|x|")
    return used


@pytest.mark.parametrize("wave", [0, 1])
@pytest.mark.parametrize("n", [257, 513])
def test_fp32_vcycle_matches_oracle_float32_cycle(dmg, n, wave):
    """One refinement step from x = 0 is x_1 = s V32(fl32(b / s)) with s = ||b||: the library's
    float32 V-cycle against the oracle's, entry by entry, in both strip-kernel families."""
    prob = pb.star(n, seed=11)
    S_or, levels, o64, o32 = _setup(prob)
    h = dmg.Hierarchy(dev(S_or), precision=dmg.DMG_FP32_IR, inner_cycles=1, strip_kernel=wave,
                      tile_rows=8)
    x1, k, _, _ = h.solve(dev(prob.b), rtol=1e-10, max_iters=1, raise_on_fail=False)
    assert k == 1
    xo, ko, _, _ = cycle.solve_ir(o64, o32, prob.b, 1e-10, inner=1, max_iters=1)
    _check_fp32(f"{n}x{n} float32 V-cycle (wave={wave})", host(x1), xo)
    h.close()


@pytest.mark.parametrize("inner", [1, 2])
@pytest.mark.parametrize("name", ["star257", "star97x65"])
def test_fp32_refinement_steps_match_oracle(dmg, name, inner):
    """Every outer refinement step's x against cycle.solve_ir's, the same step count, and the
    final solution against the float64 oracle solution."""
    prob = {"star257": lambda: pb.star(257, seed=2), "star97x65": lambda: pb.star(97, seed=1, ny=65)}[name]()
    S_or, levels, o64, o32 = _setup(prob)
    xo, ko, histo, its = cycle.solve_ir(o64, o32, prob.b, 1e-10, inner=inner, keep_iterates=True)
    h = dmg.Hierarchy(dev(S_or), precision=dmg.DMG_FP32_IR, inner_cycles=inner)
    b = dev(prob.b)
    x, k, rel, hist = h.solve(b, rtol=1e-10)
    assert rel <= 1e-10 and k == ko, (k, ko)
    assert np.allclose(hist, histo, rtol=1e-3)
    for step in range(1, ko + 1):
        xs, ks, _, _ = h.solve(b, rtol=1e-10, max_iters=step, raise_on_fail=False)
        assert ks == step
        _check_fp32(f"{name} m={inner} outer step {step}", host(xs), its[step - 1])
    # the refined solution and the float64 oracle solution: both reach 1e-10, so they differ by
    # at most about cond(A) 1e-10 relative; both are printed
    u64, _, _, _ = cycle.solve(o64, prob.b, 1e-10)
    err = float(np.linalg.norm(host(x) - u64) / np.linalg.norm(u64))
    print(f"[fp32] {name} m={inner}: {k} steps, ||x - x_64,oracle|| / ||x_64,oracle|| = {err:.2e}")
    assert err < 1e-7
    h.close()


def test_fp32_refinement_is_scale_invariant(dmg):
    """The residual is divided by its norm before rounding to float32, so the refinement works
    for right-hand sides far outside float32's range and commutes with scaling: b 2^-100 and
    b 2^100 (exact scalings) give x 2^-+100 bit for bit; b 1e-30 and b 1e30 the same steps and x
    to rounding."""
    prob = pb.star(129, seed=3)
    S_or, levels, o64, o32 = _setup(prob)
    h = dmg.Hierarchy(dev(S_or), precision=dmg.DMG_FP32_IR)
    b = dev(prob.b)
    x, k, rel, _ = h.solve(b, rtol=1e-10)
    x = x.clone()
    for e in (-100, 100):
        a = 2.0 ** e
        xa, ka, rela, _ = h.solve(b * a, rtol=1e-10)
        assert ka == k and rela <= 1e-10
        assert torch.equal(xa / a, x), e
    for a in (1e-30, 1e30):
        xa, ka, rela, _ = h.solve(b * a, rtol=1e-10)
        assert ka == k and rela <= 1e-10
        assert_iterate(f"b * {a:g}", host(xa / a), host(x), rtol=1e-10,
                       floor_ulps=int(1e-10 / EPS64))
    # the oracle's refinement on the scaled system takes the same steps
    _, ko, _, _ = cycle.solve_ir(o64, o32, prob.b * 1e-30, 1e-10)
    assert ko == k
    h.close()


@pytest.mark.parametrize("name,smoother", [("annulus65", 1), ("annulus65", 2), ("annulus65", 3),
                                           ("annulus129x97", 1), ("annulus129x97", 3),
                                           ("star97x65", 2), ("star97x65", 3)])
def test_fp32_refinement_with_line_relaxation_matches_oracle(dmg, name, smoother):
    """Float32 inner cycles with zebra line relaxation (x-lines, y-lines, alternating) inside
    float64 refinement: every outer step's x against the oracle's refinement with the same
    smoother in float32, the same step count, and the solution against the float64 line-smoothed
    oracle solution."""
    prob = {"annulus65": lambda: pb.quarter_annulus(65),
            "annulus129x97": lambda: pb.quarter_annulus(129, ny=97),
            "star97x65": lambda: pb.star(97, seed=1, ny=65)}[name]()
    S_or, levels, o64, o32 = _setup(prob, smoother)
    xo, ko, histo, its = cycle.solve_ir(o64, o32, prob.b, 1e-10, inner=1, keep_iterates=True)
    h = dmg.Hierarchy(dev(S_or), precision=dmg.DMG_FP32_IR, smoother=smoother, inner_cycles=1)
    b = dev(prob.b)
    x, k, rel, hist = h.solve(b, rtol=1e-10, max_iters=300)
    assert rel <= 1e-10 and k == ko, (k, ko)
    assert np.allclose(hist, histo, rtol=1e-3)
    worst = 0.0
    for step in range(1, min(ko, 6) + 1):
        xs, ks, _, _ = h.solve(b, rtol=1e-10, max_iters=step, raise_on_fail=False)
        assert ks == step
        worst = max(worst, _check_fp32(f"{name} smoother={smoother} outer step {step}", host(xs),
                                       its[step - 1]))
    u64, k64, _, _ = cycle.solve(o64, prob.b, 1e-10, max_iters=300)
    err = float(np.linalg.norm(host(x) - u64) / np.linalg.norm(u64))
    print(f"[fp32] {name} line smoother {smoother}: {k} steps (float64 line solve {k64} cycles), "
          f"error vs float64 oracle solution {err:.2e}")
    assert err < 1e-7
    h.close()
