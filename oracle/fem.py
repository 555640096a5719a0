"""Q1 discretisation of the pulled-back diffusion problem (oracle; test infrastructure only).

Paper Sec. 2: the weak form on the physical domain is pulled back to Omega_c = (-1,1)^2
(eq. weak_computational); Sec. 2.1 gives the effective tensor
    D_c = J_T (D o T^{-1}) J_T^T |J_T^{-1}|.
With X = T^{-1} and J = dX/d(xi,eta) we have J_T = J^{-1} and |J_T^{-1}| = det J, so for a scalar
coefficient K the tensor is D_c = K * det(J) J^{-1} J^{-T}.  The integrals are evaluated with the
2x2 Gauss rule on every cell (the paper leaves the rule open, Sec. 2.1 "Discretization").

Storage (Sec. 4.1, remark on symmetric storage: five values per degree of freedom):
    S[0]=C (diagonal), S[1]=W (to (i-1,j)), S[2]=S (to (i,j-1)), S[3]=SW (to (i-1,j-1)),
    S[4]=SE (to (i+1,j-1)), all [ny][nx].  Dirichlet rows and couplings into the boundary are 0.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as spx

_G = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))
# local node order on a cell: 0 = SW (0,0), 1 = SE (1,0), 2 = NW (0,1), 3 = NE (1,1)
_NODE_OFF = ((0, 0), (1, 0), (0, 1), (1, 1))


def _grad_ref(s, t):
    """Gradients of the bilinear shape functions on [0,1]^2 at (s,t): array [4][2]."""
    return np.array([[-(1 - t), -(1 - s)],
                     [(1 - t), -s],
                     [-t, (1 - s)],
                     [t, s]])


def metric_tensor(J11, J12, J21, J22):
    """M = det(J) J^{-1} J^{-T} (the effective tensor of Sec. 2.1 with D = I), as (M11, M12, M22)."""
    det = J11 * J22 - J12 * J21
    Jinv = np.empty(np.shape(J11) + (2, 2))
    Jinv[..., 0, 0] = J22 / det
    Jinv[..., 0, 1] = -J12 / det
    Jinv[..., 1, 0] = -J21 / det
    Jinv[..., 1, 1] = J11 / det
    M = det[..., None, None] * np.einsum("...ik,...jk->...ij", Jinv, Jinv)
    return M[..., 0, 0], M[..., 0, 1], M[..., 1, 1]


def element_matrices(jac: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """Per-cell Q1 stiffness matrices G_e[a,b] = int_cell grad phi_a . M grad phi_b dxi for the
    metric M = det J J^{-1} J^{-T}, 2x2 Gauss rule.  Returns [ny-1][nx-1][4][4].

    On the reference cell [0,1]^2 with widths hx, hy: grad_xi = (d_s / hx, d_t / hy) and
    dxi = hx hy ds dt, so the xx term carries hy/hx and the yy term hx/hy."""
    hx, hy = 2.0 / (nx - 1), 2.0 / (ny - 1)
    G = np.zeros((ny - 1, nx - 1, 4, 4))
    for q in range(4):
        s, t = _G[q & 1], _G[q >> 1]
        d = _grad_ref(s, t)                                  # [4][2] in (s,t)
        gx, gy = d[:, 0] / hx, d[:, 1] / hy                  # d/dxi, d/deta
        M11, M12, M22 = metric_tensor(*(jac[4 * q + e] for e in range(4)))
        w = 0.25 * hx * hy
        G += w * (M11[..., None, None] * np.outer(gx, gx)
                  + M12[..., None, None] * (np.outer(gx, gy) + np.outer(gy, gx))
                  + M22[..., None, None] * np.outer(gy, gy))
    return G


def assemble_matrix(G: np.ndarray, K: np.ndarray, nx: int, ny: int) -> spx.csr_matrix:
    """Standard finite-element assembly A = sum_e K_e G_e over all vertices (row-major index
    j*nx + i), followed by Dirichlet elimination: rows and columns of boundary vertices are zeroed
    (the boundary values are lifted out of the system by the caller)."""
    rows, cols, vals = [], [], []
    jj, ii = np.meshgrid(np.arange(ny - 1), np.arange(nx - 1), indexing="ij")
    for a in range(4):
        for b in range(4):
            ia = (jj + _NODE_OFF[a][1]) * nx + ii + _NODE_OFF[a][0]
            ib = (jj + _NODE_OFF[b][1]) * nx + ii + _NODE_OFF[b][0]
            rows.append(ia.ravel())
            cols.append(ib.ravel())
            vals.append((K * G[..., a, b]).ravel())
    N = nx * ny
    A = spx.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(N, N)).tocsr()
    keep = np.zeros((ny, nx))
    keep[1:-1, 1:-1] = 1.0
    D = spx.diags(keep.ravel())
    A = (D @ A @ D).tocsr()
    A.eliminate_zeros()
    return A


def matrix_to_stencil(A: spx.spmatrix, nx: int, ny: int) -> np.ndarray:
    """Read the five stored couplings (C, W, S, SW, SE) of every vertex out of a 9-point matrix."""
    A = A.tocsr()
    S = np.zeros((5, ny, nx))
    offs = ((0, 0), (-1, 0), (0, -1), (-1, -1), (1, -1))
    for k, (di, dj) in enumerate(offs):
        for j in range(ny):
            for i in range(nx):
                i2, j2 = i + di, j + dj
                if 0 <= i2 < nx and 0 <= j2 < ny:
                    S[k, j, i] = A[j * nx + i, j2 * nx + i2]
    return S


def matrix_to_stencil_fast(A: spx.spmatrix, nx: int, ny: int) -> np.ndarray:
    """Same as matrix_to_stencil, vectorised (used at large sizes)."""
    A = A.tocoo()
    S = np.zeros((5, ny, nx))
    r, c, v = A.row, A.col, A.data
    jr, ir = np.divmod(r, nx)
    jc, ic = np.divmod(c, nx)
    di, dj = ic - ir, jc - jr
    for k, (ddi, ddj) in enumerate(((0, 0), (-1, 0), (0, -1), (-1, -1), (1, -1))):
        m = (di == ddi) & (dj == ddj)
        np.add.at(S[k], (jr[m], ir[m]), v[m])
    return S


def stencil_to_matrix(S: np.ndarray) -> spx.csr_matrix:
    """Full 9-point matrix from the symmetric 5-value storage: the E, N, NE, NW couplings of a
    vertex are the W, S, SW, SE values stored at the neighbour on the other end of the edge."""
    _, ny, nx = S.shape
    N = nx * ny
    idx = np.arange(N).reshape(ny, nx)
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [S[0].ravel()]
    for k, (di, dj) in ((1, (-1, 0)), (2, (0, -1)), (3, (-1, -1)), (4, (1, -1))):
        j0, j1 = max(0, -dj), ny - max(0, dj)
        i0, i1 = max(0, -di), nx - max(0, di)
        src = idx[j0:j1, i0:i1].ravel()
        dst = idx[j0 + dj:j1 + dj, i0 + di:i1 + di].ravel()
        v = S[k, j0:j1, i0:i1].ravel()
        rows += [src, dst]
        cols += [dst, src]
        vals += [v, v]
    A = spx.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(N, N)).tocsr()
    A.eliminate_zeros()
    return A


def assemble_stencil(jac: np.ndarray, K: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """The mapped Q1 operator A_c of Sec. 2.1 in 5-plane symmetric storage [5][ny][nx]."""
    G = element_matrices(jac, nx, ny)
    A = assemble_matrix(G, K, nx, ny)
    return matrix_to_stencil_fast(A, nx, ny)
