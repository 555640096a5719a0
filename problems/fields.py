"""Seeded synthetic inputs on a logically structured nx-by-ny vertex grid over (-1,1)^2.

Layout conventions shared by the library's boundary and the oracle (plain data, no method
arithmetic):

* vertex arrays  : float64 [ny][nx], i (the xi index) fastest, boundary ring included;
* cell arrays    : float64 [ny-1][nx-1], cell (i,j) spans [xi_i, xi_{i+1}] x [eta_j, eta_{j+1}];
* map Jacobian   : float64 [16][ny-1][nx-1]; plane 4*q + e holds entry e of dX/d(xi,eta)
                   (e = 0: dx/dxi, 1: dx/deta, 2: dy/dxi, 3: dy/deta) at the 2x2 Gauss point
                   q = qx + 2*qy of each cell, local offsets s_0 = 1/2 - 1/(2 sqrt 3) and
                   s_1 = 1/2 + 1/(2 sqrt 3) times the cell width.
"""
from __future__ import annotations

import math

import numpy as np

GAUSS_OFFSETS = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))


def grid_coords(nx: int, ny: int):
    """Vertex coordinates xi_i = -1 + 2 i/(nx-1), eta_j = -1 + 2 j/(ny-1)."""
    return np.linspace(-1.0, 1.0, nx), np.linspace(-1.0, 1.0, ny)


def sample_jacobian(mp, nx: int, ny: int, row_block: int = 128) -> np.ndarray:
    """dX/d(xi,eta) of the map at the 2x2 Gauss points of every cell: [16][ny-1][nx-1].
    Row blocks are evaluated on a thread pool (NumPy/SciPy ufuncs release the GIL)."""
    import concurrent.futures as cf
    import os

    xi, eta = grid_coords(nx, ny)
    hx, hy = xi[1] - xi[0], eta[1] - eta[0]
    out = np.empty((16, ny - 1, nx - 1))

    def block(j0):
        j1 = min(ny - 1, j0 + row_block)
        for q in range(4):
            qx, qy = q & 1, q >> 1
            X = xi[:-1] + hx * GAUSS_OFFSETS[qx]
            Y = eta[j0:j1] + hy * GAUSS_OFFSETS[qy]
            XX, YY = np.meshgrid(X, Y)
            J = mp.jacobian(XX, YY)
            for e in range(4):
                out[4 * q + e, j0:j1] = J[e]

    workers = min(16, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(block, range(0, ny - 1, row_block)))
    return out


def cell_centres_physical(mp, nx: int, ny: int):
    xi, eta = grid_coords(nx, ny)
    XX, YY = np.meshgrid(0.5 * (xi[:-1] + xi[1:]), 0.5 * (eta[:-1] + eta[1:]))
    return mp(XX, YY)


def lognormal_K(mp, nx: int, ny: int, rng: np.random.Generator, sigma: float = 1.0,
                ell: float = 0.1, n_features: int = 1024, device: str | None = None) -> np.ndarray:
    """K_e = exp(g(x_e)) at the physical centroid image of each cell, where g is a zero-mean
    Gaussian field with squared-exponential covariance (std sigma, length ell) drawn with
    random Fourier features: g = sigma sqrt(2/M) sum_m cos(omega_m . x + b_m),
    omega ~ N(0, ell^-2 I), b ~ U(0, 2 pi)."""
    import torch

    omega = rng.normal(0.0, 1.0 / ell, size=(n_features, 2))
    phase = rng.uniform(0.0, 2 * math.pi, size=n_features)
    x, y = cell_centres_physical(mp, nx, ny)
    dev = torch.device(device or "cpu")
    om = torch.as_tensor(omega, dtype=torch.float64, device=dev)
    ph = torch.as_tensor(phase, dtype=torch.float64, device=dev)
    pts = torch.as_tensor(np.stack([x.ravel(), y.ravel()], axis=1), dtype=torch.float64, device=dev)
    g = torch.empty(pts.shape[0], dtype=torch.float64, device=dev)
    chunk = 1 << 16
    scale = sigma * math.sqrt(2.0 / n_features)
    for s in range(0, pts.shape[0], chunk):
        g[s:s + chunk] = scale * torch.cos(pts[s:s + chunk] @ om.T + ph).sum(dim=1)
    return torch.exp(g).cpu().numpy().reshape(ny - 1, nx - 1)


def interior_mask(nx: int, ny: int) -> np.ndarray:
    m = np.zeros((ny, nx), dtype=bool)
    m[1:-1, 1:-1] = True
    return m


def uniform_rhs(nx: int, ny: int, rng: np.random.Generator) -> np.ndarray:
    """b_i ~ U(-1, 1) on interior vertices; 0 on the boundary ring."""
    b = np.zeros((ny, nx))
    b[1:-1, 1:-1] = rng.uniform(-1.0, 1.0, size=(ny - 2, nx - 2))
    return b


def smooth_target(nx: int, ny: int, rng: np.random.Generator, modes: int = 8) -> np.ndarray:
    """u_t = sum_{k,l<=modes} c_kl sin(k pi (xi+1)/2) sin(l pi (eta+1)/2), c_kl ~ N(0,1)/(k^2+l^2).
    Vanishes on the boundary ring."""
    xi, eta = grid_coords(nx, ny)
    k = np.arange(1, modes + 1)
    c = rng.normal(size=(modes, modes)) / (k[:, None] ** 2 + k[None, :] ** 2)
    sx = np.sin(np.outer(k, np.pi * (xi + 1) / 2))    # [k][nx]
    sy = np.sin(np.outer(k, np.pi * (eta + 1) / 2))   # [l][ny]
    u = sy.T @ c.T @ sx                                 # [ny][nx]: sum_{k,l} c_kl sy_l(j) sx_k(i)
    u[0, :] = u[-1, :] = 0.0
    u[:, 0] = u[:, -1] = 0.0
    return u


def sample_jacobian_patch(mp, n: int, i0: int, j0: int, m: int) -> np.ndarray:
    """The [16][m][m] block of ``sample_jacobian(mp, n, n)`` for cells [i0, i0+m) x [j0, j0+m)."""
    xi, eta = grid_coords(n, n)
    hx, hy = xi[1] - xi[0], eta[1] - eta[0]
    out = np.empty((16, m, m))
    for q in range(4):
        qx, qy = q & 1, q >> 1
        XX, YY = np.meshgrid(xi[i0:i0 + m] + hx * GAUSS_OFFSETS[qx], eta[j0:j0 + m] + hy * GAUSS_OFFSETS[qy])
        J = mp.jacobian(XX, YY)
        for e in range(4):
            out[4 * q + e] = J[e]
    return out


def lognormal_K_patch(mp, n: int, i0: int, j0: int, m: int, rng: np.random.Generator,
                      sigma: float = 1.0, ell: float = 0.1, n_features: int = 1024) -> np.ndarray:
    """The [m][m] block of ``lognormal_K(mp, n, n, rng)`` for cells [i0, i0+m) x [j0, j0+m),
    drawing the same random features from ``rng`` (evaluated with NumPy)."""
    omega = rng.normal(0.0, 1.0 / ell, size=(n_features, 2))
    phase = rng.uniform(0.0, 2 * math.pi, size=n_features)
    xi, eta = grid_coords(n, n)
    XX, YY = np.meshgrid(0.5 * (xi[i0:i0 + m] + xi[i0 + 1:i0 + m + 1]),
                         0.5 * (eta[j0:j0 + m] + eta[j0 + 1:j0 + m + 1]))
    x, y = mp(XX, YY)
    pts = np.stack([np.ravel(x), np.ravel(y)], axis=1)
    g = sigma * math.sqrt(2.0 / n_features) * np.cos(pts @ omega.T + phase).sum(axis=1)
    return np.exp(g).reshape(m, m)


def lognormal_features(rng: np.random.Generator, ell: float = 0.1, n_features: int = 1024):
    """The random Fourier features lognormal_K draws from ``rng`` (same order)."""
    omega = rng.normal(0.0, 1.0 / ell, size=(n_features, 2))
    phase = rng.uniform(0.0, 2 * math.pi, size=n_features)
    return omega, phase


def lognormal_at(x: np.ndarray, y: np.ndarray, omega: np.ndarray, phase: np.ndarray,
                 sigma: float = 1.0) -> np.ndarray:
    """exp(g) of the log-normal field with features (omega, phase) at physical points (x, y)."""
    pts = np.stack([np.ravel(x), np.ravel(y)], axis=1)
    g = np.empty(pts.shape[0])
    scale = sigma * math.sqrt(2.0 / omega.shape[0])
    for s in range(0, pts.shape[0], 1 << 15):
        g[s:s + (1 << 15)] = scale * np.cos(pts[s:s + (1 << 15)] @ omega.T + phase).sum(axis=1)
    return np.exp(g).reshape(np.shape(x))
