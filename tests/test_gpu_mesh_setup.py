"""The device assembly of the coupled mass C (and C^T): bit-for-bit equal to the host assembly,
and equal to the oracle's C (exact overlap integral, and the rasterised rule of Sec. 2.3.1) with
the same sparsity, entry by entry to 1e-12 of its row's sum (an entry integrates the product of
two non-negative basis functions over one vertex's support, so its rounding is bounded by that
of the row's total, the integral of the vertex's hat function); a two-level cycle built on
either gives the same iterates."""
import numpy as np
import pytest
import scipy.sparse as spx
import torch

import problems as pb
from oracle import transfer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_2509_08109_amd as m
    m.lib()
    return m


def _csr(T, nv, ng):
    rp, ci, v = T.copy_C()
    return spx.csr_matrix((v, ci, rp), shape=(nv, ng))


@pytest.mark.parametrize("n,nq", [(33, 0), (65, 0), (33, 4)])
def test_device_C_equals_host_C_and_oracle(lib, n, nq):
    P = pb.star_dmg(n, seed=3, lognormal=False)
    m = P.mesh
    Td = lib.Transfer(m.xy_c, m.xy_p, m.tris, m.dof, n, n, nq=nq)
    Th = lib.Transfer(m.xy_c, m.xy_p, m.tris, m.dof, n, n, nq=nq, host_setup=True)
    rd, cd, vd = Td.copy_C()
    rh, ch, vh = Th.copy_C()
    assert np.array_equal(rd, rh) and np.array_equal(cd, ch) and np.array_equal(vd, vh)
    # the transfers built on either apply identically
    g = np.random.Generator(np.random.PCG64(2))
    uc = torch.as_tensor(np.pad(g.uniform(-1, 1, (n - 2, n - 2)), 1), dtype=torch.float64, device="cuda")
    assert torch.equal(Td.from_grid(uc), Th.from_grid(uc))
    Co = transfer.coupled_mass(m.xy_c, m.xy_p, m.tris, m.dof, n, n, nq=nq).tocsr()
    Cd = _csr(Td, m.nv, n * n)
    Co.sort_indices()
    assert np.array_equal(Cd.indptr, Co.indptr) and np.array_equal(Cd.indices, Co.indices)
    assert np.all(Co.data >= 0)
    rowsum = np.repeat(np.asarray(Co.sum(axis=1)).ravel(), np.diff(Co.indptr))
    d = np.abs(Cd.data - Co.data)
    worst = float(np.max(d / rowsum)) if d.size else 0.0
    print(f"[mesh C] n={n} nq={nq}: worst |C - C_oracle| / row sum {worst:.2e}, worst relative "
          f"{float(np.max(d / np.maximum(Co.data, 1e-300))):.2e}")
    assert worst <= 1e-12


def test_twolevel_on_device_or_host_C_cycles_identically(lib):
    n = 33
    P = pb.star_dmg(n, seed=1)
    m = P.mesh
    H = lib.Hierarchy(lib.assemble_stencil(torch.as_tensor(P.grid.jac, device="cuda"),
                                           torch.as_tensor(P.grid.K, device="cuda")))
    a = lib.TwoLevel(H, m.xy_c, m.xy_p, m.tris, m.dof, K_t=P.K_t)
    b = lib.TwoLevel(H, m.xy_c, m.xy_p, m.tris, m.dof, K_t=P.K_t, host_setup=True)
    f = torch.as_tensor(P.f, device="cuda")
    ua = torch.zeros(m.nv, dtype=torch.float64, device="cuda")
    ub = ua.clone()
    for _ in range(3):
        a.cycle(ua, f)
        b.cycle(ub, f)
    assert torch.equal(ua, ub)
