"""The star batch of ``problems.batch`` generated on a torch device.

The conformal square->disk part of every star map is the same for all instances, so it is
evaluated once per grid size on the host (``conformal_square_to_disk``); each instance's radial
deformation, the chain rule for its Jacobian, its log-normal coefficient and its right-hand side
follow on the device from the same random streams as ``problems.batch``.  Input generation only:
no solver arithmetic.
"""
from __future__ import annotations

import math

import numpy as np

from .fields import GAUSS_OFFSETS, grid_coords, uniform_rhs
from .maps import Star, conformal_square_to_disk


def _phi_tables(n: int, device, row_block: int = 64):
    """w and dw/dz of the conformal map at the 2x2 Gauss points ([4][n-1][n-1]) and w at the
    cell centres ([n-1][n-1]), as complex128 tensors on ``device`` (row blocks on a thread
    pool: the special functions release the GIL)."""
    import concurrent.futures as cf
    import os

    import torch

    xi, eta = grid_coords(n, n)
    h = xi[1] - xi[0]
    w = np.empty((4, n - 1, n - 1), dtype=np.complex128)
    dw = np.empty((4, n - 1, n - 1), dtype=np.complex128)
    wc = np.empty((n - 1, n - 1), dtype=np.complex128)

    def block(j0):
        j1 = min(n - 1, j0 + row_block)
        for q in range(4):
            qx, qy = q & 1, q >> 1
            XX, YY = np.meshgrid(xi[:-1] + h * GAUSS_OFFSETS[qx], eta[j0:j1] + h * GAUSS_OFFSETS[qy])
            w[q, j0:j1], dw[q, j0:j1] = conformal_square_to_disk(XX, YY)
        XC, YC = np.meshgrid(0.5 * (xi[:-1] + xi[1:]), 0.5 * (eta[j0:j1] + eta[j0 + 1:j1 + 1]))
        wc[j0:j1], _ = conformal_square_to_disk(XC, YC)

    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(block, range(0, n - 1, row_block)))
    t = lambda a: torch.as_tensor(a, dtype=torch.complex128, device=device)
    return t(w), t(dw), t(wc)


def _h_torch(mp: Star, w):
    """h(w) and dh/dw of the radial deformation (same recurrence as Star._h)."""
    import torch

    h = torch.zeros(w.shape, dtype=torch.float64, device=w.device)
    hw = torch.zeros_like(w)
    wk = torch.ones_like(w)
    for idx in range(len(mp.a)):
        k = idx + 1
        e = complex(math.cos(mp.phi[idx]), math.sin(mp.phi[idx]))
        hw = hw + (mp.a[idx] * e * k) * wk
        wk = wk * w
        h = h + mp.a[idx] * (e * wk).real
    return h, hw


def _jacobian_torch(mp: Star, w, dw):
    """dX/d(xi,eta) of X = R o Phi at the points of w, as in Star.jacobian: 4 float64 tensors."""
    h, hw = _h_torch(mp, w)
    hx, hy = hw.real, -hw.imag
    u, v = w.real, w.imag
    R11 = 1.0 + h + u * hx
    R12 = u * hy
    R21 = v * hx
    R22 = 1.0 + h + v * hy
    P11, P12, P21, P22 = dw.real, -dw.imag, dw.imag, dw.real
    return (R11 * P11 + R12 * P21, R11 * P12 + R12 * P22,
            R21 * P11 + R22 * P21, R21 * P12 + R22 * P22)


def _lognormal_torch(mp: Star, wc, rng: np.random.Generator, sigma: float = 1.0, ell: float = 0.1,
                     n_features: int = 1024):
    """K at the physical cell centres, drawing the random features exactly as lognormal_K."""
    import torch

    omega = rng.normal(0.0, 1.0 / ell, size=(n_features, 2))
    phase = rng.uniform(0.0, 2 * math.pi, size=n_features)
    h, _ = _h_torch(mp, wc)
    p = (1.0 + h) * wc
    dev = wc.device
    om = torch.as_tensor(omega, dtype=torch.float64, device=dev)
    ph = torch.as_tensor(phase, dtype=torch.float64, device=dev)
    pts = torch.stack([p.real.reshape(-1), p.imag.reshape(-1)], dim=1)
    g = torch.empty(pts.shape[0], dtype=torch.float64, device=dev)
    chunk = 1 << 16
    scale = sigma * math.sqrt(2.0 / n_features)
    for s in range(0, pts.shape[0], chunk):
        g[s:s + chunk] = scale * torch.cos(pts[s:s + chunk] @ om.T + ph).sum(dim=1)
    return torch.exp(g).reshape(wc.shape)


def star_batch_device(count: int, choices=(129, 257, 513, 1025), seed: int = 3, device="cuda"):
    """Yields (n, jac [16][n-1][n-1], K [n-1][n-1], b [n][n]) per instance, float64 tensors on
    ``device``: the instances of ``problems.batch(count, choices, seed)``."""
    import torch

    from . import batch_sizes

    sizes = batch_sizes(count, choices, seed)
    kids = np.random.SeedSequence(seed).spawn(count + 1)
    tables = {}
    for k, n in enumerate(sizes):
        if n not in tables:
            tables[n] = _phi_tables(n, device)
        w, dw, wc = tables[n]
        g_map, g_k, g_b, _, _ = [np.random.Generator(np.random.PCG64(s)) for s in kids[k].spawn(5)]
        mp = Star.random(g_map)
        K = _lognormal_torch(mp, wc, g_k)
        J = _jacobian_torch(mp, w, dw)                  # 4 x [4][n-1][n-1]
        jac = torch.stack([J[e][q] for q in range(4) for e in range(4)])
        b = torch.as_tensor(uniform_rhs(n, n, g_b), dtype=torch.float64, device=device)
        yield n, jac.contiguous(), K.contiguous(), b


def star_device(n: int, seed: int = 1, device="cuda"):
    """(jac [16][n-1][n-1], K [n-1][n-1], b [n][n]) of ``problems.star(n, seed)`` as float64
    tensors on ``device``."""
    import torch

    from . import streams

    g_map, g_k, g_b, _, _ = streams(seed)
    mp = Star.random(g_map)
    w, dw, wc = _phi_tables(n, device)
    K = _lognormal_torch(mp, wc, g_k)
    J = _jacobian_torch(mp, w, dw)
    jac = torch.stack([J[e][q] for q in range(4) for e in range(4)])
    b = torch.as_tensor(uniform_rhs(n, n, g_b), dtype=torch.float64, device=device)
    return jac.contiguous(), K.contiguous(), b


def lognormal_at_device(x, y, omega, phase, device, sigma: float = 1.0) -> np.ndarray:
    """``fields.lognormal_at`` evaluated with torch on ``device`` (host arrays in and out)."""
    import torch

    om = torch.as_tensor(omega, dtype=torch.float64, device=device)
    ph = torch.as_tensor(phase, dtype=torch.float64, device=device)
    pts = torch.as_tensor(np.stack([np.ravel(x), np.ravel(y)], axis=1), dtype=torch.float64,
                          device=device)
    g = torch.empty(pts.shape[0], dtype=torch.float64, device=device)
    chunk = 1 << 16
    scale = sigma * math.sqrt(2.0 / omega.shape[0])
    for s in range(0, pts.shape[0], chunk):
        g[s:s + chunk] = scale * torch.cos(pts[s:s + chunk] @ om.T + ph).sum(dim=1)
    return torch.exp(g).cpu().numpy().reshape(np.shape(x))


def star_dmg_device(n: int, seed: int = 1, device="cuda"):
    """The inputs of ``problems.star_dmg(n, seed)`` with the coefficient fields evaluated on
    ``device``: (jac [16][n-1][n-1], K [n-1][n-1]) as float64 tensors there, and the mesh, the
    per-triangle K_t and the right-hand side f on the host."""
    from . import lognormal_features, mesh_points_for_grid, lattice_mesh, streams

    jac, K, _ = star_device(n, seed, device)
    g = streams(seed, 7)
    mp = Star.random(streams(seed)[0])
    mesh = lattice_mesh(mp, mesh_points_for_grid(n), g[5])
    cen = mesh.xy_p[mesh.tris].mean(axis=1)
    omega, phase = lognormal_features(streams(seed)[1])
    K_t = lognormal_at_device(cen[:, 0], cen[:, 1], omega, phase, device)
    f = np.where(mesh.dof, g[6].uniform(-1.0, 1.0, size=mesh.dof.shape[0]), 0.0)
    return jac, K, mesh, K_t, f
