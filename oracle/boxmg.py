"""BoxMG hierarchy ingredients (oracle; test infrastructure only).

Paper Sec. 2.2 ("Multigrid Solver"): the structured solver coarsens geometrically by a factor of
two in each direction, uses operator-induced interpolation (Dendy's black-box multigrid, the
work cited as DendyBoxMG1982) and Galerkin coarse operators P^T A P, which stay 9-point in 2D
(Sec. 4.1, discussion of operator complexity).

Interpolation (written out from the operator-induced construction; the paper itself prints no
formula).  Coarse point (I,J) sits at fine (2I,2J).  All stencil values below are the couplings
of the fine point being interpolated (C, W, E, S, N, SW, SE, NW, NE):
  * coarse points: injection (weight 1);
  * x-line points (odd i, even j): collapse the stencil onto the line,
        w_W = -(W + NW + SW) / (C + N + S),   w_E = -(E + NE + SE) / (C + N + S);
  * y-line points (even i, odd j):
        w_S = -(S + SW + SE) / (C + W + E),   w_N = -(N + NW + NE) / (C + W + E);
  * centre points (odd, odd): solve the point's own equation with its four line neighbours
    replaced by their interpolants, e.g.
        P_SW = -(SW + W * w_S[W nbr] + S * w_W[S nbr]) / C, and likewise for SE, NW, NE;
  * boundary fine points interpolate to zero (their rows of A are zero).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as spx

from .fem import matrix_to_stencil_fast, stencil_to_matrix


def full_stencil(S: np.ndarray):
    """All nine couplings of every vertex as a dict of [ny][nx] arrays (zero outside the grid)."""
    _, ny, nx = S.shape
    C, W, So, SW, SE = S
    E = np.zeros_like(C)
    N = np.zeros_like(C)
    NE = np.zeros_like(C)
    NW = np.zeros_like(C)
    E[:, :-1] = W[:, 1:]            # E(i,j) = W(i+1,j)
    N[:-1, :] = So[1:, :]           # N(i,j) = S(i,j+1)
    NE[:-1, :-1] = SW[1:, 1:]       # NE(i,j) = SW(i+1,j+1)
    NW[:-1, 1:] = SE[1:, :-1]       # NW(i,j) = SE(i-1,j+1)
    return dict(C=C, W=W, E=E, S=So, N=N, SW=SW, SE=SE, NW=NW, NE=NE)


def coarse_dims(nx: int, ny: int):
    if (nx - 1) % 2 or (ny - 1) % 2:
        raise ValueError("grid dims must be odd to coarsen by two")
    return (nx + 1) // 2, (ny + 1) // 2


def interpolation(S: np.ndarray) -> spx.csr_matrix:
    """Operator-induced interpolation P (fine vertices x coarse vertices), sparse."""
    _, ny, nx = S.shape
    ncx, ncy = coarse_dims(nx, ny)
    st = full_stencil(S)
    fid = np.arange(nx * ny).reshape(ny, nx)
    cid = np.arange(ncx * ncy).reshape(ncy, ncx)
    rows, cols, vals = [], [], []

    def emit(f, c, v):
        rows.append(f.ravel()); cols.append(c.ravel()); vals.append(np.broadcast_to(v, f.shape).ravel())

    # interior fine points of each kind, as (row-slice, col-slice) pairs
    xl = (slice(2, ny - 1, 2), slice(1, nx - 1, 2))     # x-line: even j, odd i
    yl = (slice(1, ny - 1, 2), slice(2, nx - 1, 2))     # y-line: odd j, even i
    ce = (slice(1, ny - 1, 2), slice(1, nx - 1, 2))     # centre: odd j, odd i
    cp = (slice(2, ny - 1, 2), slice(2, nx - 1, 2))     # coarse points in the interior

    g = st
    wW = np.zeros((ny, nx)); wE = np.zeros((ny, nx))
    wS = np.zeros((ny, nx)); wN = np.zeros((ny, nx))
    d = g["C"][xl] + g["N"][xl] + g["S"][xl]
    wW[xl] = -(g["W"][xl] + g["NW"][xl] + g["SW"][xl]) / d
    wE[xl] = -(g["E"][xl] + g["NE"][xl] + g["SE"][xl]) / d
    d = g["C"][yl] + g["W"][yl] + g["E"][yl]
    wS[yl] = -(g["S"][yl] + g["SW"][yl] + g["SE"][yl]) / d
    wN[yl] = -(g["N"][yl] + g["NW"][yl] + g["NE"][yl]) / d

    # coarse points: injection
    emit(fid[cp], cid[1:ncy - 1, 1:ncx - 1], 1.0)
    # x-line points (2I+1, 2J): coarse (I, J) and (I+1, J)
    emit(fid[xl], cid[1:ncy - 1, 0:ncx - 1], wW[xl])
    emit(fid[xl], cid[1:ncy - 1, 1:ncx], wE[xl])
    # y-line points (2I, 2J+1): coarse (I, J) and (I, J+1)
    emit(fid[yl], cid[0:ncy - 1, 1:ncx - 1], wS[yl])
    emit(fid[yl], cid[1:ncy, 1:ncx - 1], wN[yl])
    # centre points (2I+1, 2J+1); W/E neighbours are y-line points, S/N neighbours x-line points
    j, i = np.meshgrid(np.arange(1, ny - 1, 2), np.arange(1, nx - 1, 2), indexing="ij")
    C = g["C"][j, i]
    W, E, So, N = g["W"][j, i], g["E"][j, i], g["S"][j, i], g["N"][j, i]
    pSW = -(g["SW"][j, i] + W * wS[j, i - 1] + So * wW[j - 1, i]) / C
    pSE = -(g["SE"][j, i] + E * wS[j, i + 1] + So * wE[j - 1, i]) / C
    pNW = -(g["NW"][j, i] + W * wN[j, i - 1] + N * wW[j + 1, i]) / C
    pNE = -(g["NE"][j, i] + E * wN[j, i + 1] + N * wE[j + 1, i]) / C
    f = fid[ce]
    emit(f, cid[0:ncy - 1, 0:ncx - 1], pSW)
    emit(f, cid[0:ncy - 1, 1:ncx], pSE)
    emit(f, cid[1:ncy, 0:ncx - 1], pNW)
    emit(f, cid[1:ncy, 1:ncx], pNE)
    P = spx.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(nx * ny, ncx * ncy)).tocsr()
    P.eliminate_zeros()
    return P


def galerkin(S: np.ndarray, P: spx.spmatrix) -> np.ndarray:
    """Coarse operator A_H = P^T A_h P in 5-plane storage; checks it is 9-point and symmetric."""
    _, ny, nx = S.shape
    ncx, ncy = coarse_dims(nx, ny)
    A = stencil_to_matrix(S)
    AH = (P.T @ A @ P).tocoo()
    jr, ir = np.divmod(AH.row, ncx)
    jc, ic = np.divmod(AH.col, ncx)
    nz = AH.data != 0
    if np.any((np.abs(ic - ir) > 1)[nz] | (np.abs(jc - jr) > 1)[nz]):
        raise AssertionError("Galerkin operator is not 9-point")
    asym = abs(AH - AH.T).max() if AH.nnz else 0.0
    scale = abs(AH).max() if AH.nnz else 1.0
    if asym > 1e-12 * scale:
        raise AssertionError(f"Galerkin operator not symmetric ({asym})")
    return matrix_to_stencil_fast(AH, ncx, ncy)


class Level:
    def __init__(self, S: np.ndarray):
        self.S = S
        self.ny, self.nx = S.shape[1:]
        self.A = stencil_to_matrix(S)
        self.P = None


def build_hierarchy(S: np.ndarray, coarsest_n: int = 3):
    """Levels from the fine stencil down to the first grid with min(nx, ny) <= coarsest_n, or
    with an even dimension (coarsening by two keeps the boundary on a coarse line only for odd
    dims), which is solved directly."""
    levels = [Level(np.array(S, dtype=np.float64))]
    while (min(levels[-1].nx, levels[-1].ny) > coarsest_n
           and levels[-1].nx % 2 == 1 and levels[-1].ny % 2 == 1):
        L = levels[-1]
        L.P = interpolation(L.S)
        levels.append(Level(galerkin(L.S, L.P)))
    return levels


def complexities(levels):
    """Grid complexity sum N_l / N_1 and operator complexity sum nnz_l / nnz_1 (Sec. 4,
    definitions of GC and OC), counting interior unknowns and stored matrix nonzeros."""
    N = [(L.nx - 2) * (L.ny - 2) for L in levels]
    nnz = [L.A.count_nonzero() for L in levels]
    return sum(N) / N[0], sum(nnz) / nnz[0]
