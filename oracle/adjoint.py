"""Adjoint gradients of a solve (oracle; test infrastructure only).

Objective J(u) = 1/2 sum_{interior v} (u_v - t_v)^2 with A(K) u = b and A(K) = sum_e K_e A_e
(A_e the Dirichlet-reduced element contribution of cell e, Sec. 2.1 assembly).  Since A is
symmetric, the adjoint state solves A lam = u - t, and
    dJ/db   = lam,
    dJ/dK_e = -lam^T A_e u = -lam_e^T G_e u_e   (local 4-vectors on the cell's vertices).
The paper does not discuss derivatives; this is the standard discrete adjoint of the linear
solve, pinned by central finite differences in tests/test_oracle_adjoint.py.
"""
from __future__ import annotations

import numpy as np

from .fem import _NODE_OFF, element_matrices


def local_values(v: np.ndarray):
    """[ny][nx] vertex array -> [ny-1][nx-1][4] values at each cell's SW, SE, NW, NE vertices."""
    ny, nx = v.shape
    out = np.empty((ny - 1, nx - 1, 4))
    for a, (di, dj) in enumerate(_NODE_OFF):
        out[..., a] = v[dj:ny - 1 + dj, di:nx - 1 + di]
    return out


def grad_K(jac: np.ndarray, lam: np.ndarray, u: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """dJ/dK_e = -lam_e^T G_e u_e; lam and u vanish on the boundary ring."""
    G = element_matrices(jac, nx, ny)
    le = local_values(lam)
    ue = local_values(u)
    return -np.einsum("jia,jiab,jib->ji", le, G, ue)


def objective(u: np.ndarray, target: np.ndarray) -> float:
    d = (u - target)[1:-1, 1:-1]
    return 0.5 * float(np.sum(d * d))


def objective_grad_u(u: np.ndarray, target: np.ndarray) -> np.ndarray:
    g = u - target
    g[0, :] = g[-1, :] = 0.0
    g[:, 0] = g[:, -1] = 0.0
    return g
