"""The allocation-free residual norm (dmg_residual_norm_noalloc, its partials in a static device
array) against dmg_residual_norm on a hierarchy of the same stencil: bit for bit, on two calls
in a row, the second on a smaller grid (the array keeps the first call's contents)."""
import numpy as np
import pytest
import torch

import problems as pb

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dmg():
    import paper_2509_08109_amd as m
    m.lib()
    return m


def test_noalloc_residual_norm_matches_hierarchy_norm(dmg):
    for n, seed in ((257, 31), (65, 32)):
        print(f"[no-alloc] {n}x{n} seed {seed}", flush=True)
        p = pb.star(n, seed=seed)
        dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")
        S = dmg.assemble_stencil(dev(p.jac), dev(p.K))
        b = dev(p.b)
        u = dev(np.random.default_rng(seed).uniform(-1, 1, (n, n)))
        h = dmg.Hierarchy(S)
        ref = h.residual_norm(u, b)
        h.close()
        got = dmg.residual_norm_noalloc(S, u, b).cpu().numpy()
        assert got[1] == ref, (n, got[1], ref)
        assert got[0] == ref * ref or abs(got[0] - ref * ref) <= 4e-16 * ref * ref
        # the oracle's definition: ||b - A u|| over interior vertices
        from oracle import fem
        A = fem.stencil_to_matrix(S.cpu().numpy())
        r = (p.b.ravel() - A @ u.cpu().numpy().ravel()).reshape(n, n)[1:-1, 1:-1]
        assert abs(got[1] - np.linalg.norm(r)) <= 1e-13 * np.linalg.norm(r)


def test_noalloc_rejects_bad_arguments(dmg):
    S = torch.zeros((5, 2, 9), dtype=torch.float64, device="cuda")
    u = torch.zeros((2, 9), dtype=torch.float64, device="cuda")
    with pytest.raises(dmg.DmgError) as ei:
        dmg.residual_norm_noalloc(S, u, u)
    assert ei.value.code == 2
