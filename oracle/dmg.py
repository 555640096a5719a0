"""The two-level diffeomorphic multigrid cycle (oracle; test infrastructure only).

Sec. 2.2 (solution phase): stationary iterations of a two-level cycle on the physical P1 system
A_p u_p = f_p:
  1. pre-relaxation of u_p,
  2. restriction of the residual to the grid, r_c = P^T (f_p - A_p u_p),
  3. one grid (BoxMG) V-cycle on A_c u_c = r_c from u_c = 0,
  4. interpolation of the correction, u_p += P u_c,
  5. post-relaxation.
P = M_p^{-1} C with the mass solve replaced by two CG iterations (Sec. 2.3), so P^T r is the
to_grid transfer and P u_c the from_grid transfer of oracle.transfer; A_p is the P1 stiffness
matrix of the physical mesh (the physical-grid discretisation of Sec. 4: piecewise-linear
elements on triangles).

Readings where the paper is silent or where its choice fails on these inputs:
  * mass solves: the paper applies M_p^{-1} with two unpreconditioned CG iterations and names mass
    lumping as a possible improvement.  On the synthetic meshes here the cycle with two CG
    iterations diverges as the mesh grows (convergence factor above 1 from 33^2 grids on), while
    lumped mass (M_p replaced by its row sums) converges at a size-independent rate; lumping is
    the default, CG-k is kept as an option;
  * coupled mass C with an 8 x 8 Gauss rule per grid cell: the physical triangles are several
    times smaller than a grid cell, and a 4 x 4 rule leaves some triangles without quadrature
    points, which slows the cycle as the mesh grows;
  * relaxation S: symmetric multicolour Gauss-Seidel -- a forward sweep over colours 0..C-1 then
    a backward sweep C-1..0, each colour updated at once (vertices of one colour are not
    coupled); colours from a greedy pass over the vertices in smallest-last order (Matula and
    Beck: vertices are taken out one at a time, each of least degree in the graph that remains,
    the smallest index among equals, and coloured in the reverse order), each vertex taking the
    smallest colour not used by an already coloured neighbour in the mesh graph (two unknowns
    are neighbours when they share a triangle; Dirichlet vertices have none).  The paper does not
    say how the colours are formed; this order needs 4 colours on the synthetic meshes, where
    the vertex index order needs 7, and each colour is one sequential pass.  The mesh graph
    holds the pattern of A_p, and unlike the numerical pattern it does not depend on whether a
    coupling cancels to exactly zero (right angles opposite an edge do that);
  * stopping test: ||f - A u||_2 <= rtol ||f - A u_0||_2 (the paper runs f = 0 from a random
    initial guess, so the test is relative to the initial residual);
  * coarse-grid scaling (Sec. 2.4): u_p += gamma P u_c with gamma = 1 unless set; gamma is
    estimated as the mean of the Ritz values of k steps of the generalized Lanczos recurrence
    for P^T A_p P x = lambda A_c x (the paper's k = 12), which is trace(T_k) / k, from a
    caller-supplied start vector on the interior grid points.
Dirichlet vertices carry identity rows, so they keep u = f (= 0).
"""
from __future__ import annotations

import heapq

import numpy as np
import scipy.sparse as spx
import scipy.sparse.linalg as spl

from . import transfer


def p1_element_stiffness(xy: np.ndarray) -> np.ndarray:
    """int_t grad phi_a . grad phi_b over the triangle with vertex coordinates xy [3][2]."""
    (xa, ya), (xb, yb), (xc, yc) = xy
    det = (xb - xa) * (yc - ya) - (xc - xa) * (yb - ya)
    area = 0.5 * abs(det)
    # gradients of the barycentric coordinates: grad l_a = (y_b - y_c, x_c - x_b) / det, ...
    g = np.array([[yb - yc, xc - xb], [yc - ya, xa - xc], [ya - yb, xb - xa]]) / det
    return area * (g @ g.T)


def p1_stiffness(xy_p: np.ndarray, tris: np.ndarray, dof: np.ndarray,
                 K_t: np.ndarray | None = None) -> spx.csr_matrix:
    """A_p = sum_t K_t G_t (G_t the element stiffness); rows and columns of non-dof vertices
    replaced by the identity."""
    nv = xy_p.shape[0]
    K_t = np.ones(tris.shape[0]) if K_t is None else np.asarray(K_t, dtype=np.float64)
    rows, cols, vals = [], [], []
    for t, tv in enumerate(tris):
        G = K_t[t] * p1_element_stiffness(xy_p[tv])
        for a in range(3):
            for b in range(3):
                rows.append(tv[a])
                cols.append(tv[b])
                vals.append(G[a, b])
    A = spx.coo_matrix((vals, (rows, cols)), shape=(nv, nv)).tocsr()
    d = spx.diags(dof.astype(np.float64))
    A = (d @ A @ d + spx.diags((~dof).astype(np.float64))).tocsr()
    A.eliminate_zeros()
    return A


def mesh_graph(tris: np.ndarray, dof: np.ndarray) -> spx.csr_matrix:
    """Pattern of the unknowns' couplings: v ~ w when v != w share a triangle and both are
    unknowns (dof); Dirichlet vertices are isolated."""
    nv = dof.shape[0]
    rows, cols = [], []
    for tv in tris:
        for a in range(3):
            for b in range(3):
                if a != b and dof[tv[a]] and dof[tv[b]]:
                    rows.append(tv[a])
                    cols.append(tv[b])
    G = spx.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(nv, nv)).tocsr()
    G.sum_duplicates()
    return G


def mesh_colouring(tris: np.ndarray, dof: np.ndarray) -> np.ndarray:
    """The relaxation's colours: greedy colouring of the mesh graph in smallest-last order."""
    G = mesh_graph(tris, dof)
    return greedy_colouring(G, smallest_last_order(G))


def smallest_last_order(A: spx.spmatrix) -> np.ndarray:
    """Smallest-last order of the graph with the off-diagonal pattern of A: vertices are taken
    out one at a time, each of least degree among those left (counting only neighbours that are
    left; the smallest index among equals), and the order is the reverse of the removals."""
    A = spx.csr_matrix(A)
    n = A.shape[0]
    nbrs = [[int(w) for w in A.indices[A.indptr[v]:A.indptr[v + 1]] if w != v] for v in range(n)]
    deg = [len(x) for x in nbrs]
    heap = [(deg[v], v) for v in range(n)]
    heapq.heapify(heap)
    gone = [False] * n
    removed = []
    while heap:
        d, v = heapq.heappop(heap)
        if gone[v] or d != deg[v]:  # an entry from before a neighbour left
            continue
        gone[v] = True
        removed.append(v)
        for w in nbrs[v]:
            if not gone[w]:
                deg[w] -= 1
                heapq.heappush(heap, (deg[w], w))
    return np.array(removed[::-1], dtype=np.int64)


def greedy_colouring(A: spx.spmatrix, order=None) -> np.ndarray:
    """Colour of each vertex: vertices in ``order`` (index order when None), each the smallest
    colour unused by its already coloured neighbours (off-diagonal entries of the pattern of A)."""
    A = spx.csr_matrix(A)
    n = A.shape[0]
    colour = -np.ones(n, dtype=np.int64)
    for v in (range(n) if order is None else order):
        v = int(v)
        nb = A.indices[A.indptr[v]:A.indptr[v + 1]]
        used = {int(colour[w]) for w in nb if w != v and colour[w] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[v] = c
    return colour


def sgs(A: spx.csr_matrix, u: np.ndarray, f: np.ndarray, colour: np.ndarray) -> np.ndarray:
    """One symmetric multicolour Gauss-Seidel step (forward then backward over the colours),
    in place."""
    diag = A.diagonal()
    ncol = int(colour.max()) + 1
    for c in list(range(ncol)) + list(range(ncol - 1, -1, -1)):
        idx = np.nonzero(colour == c)[0]
        Au = A[idx] @ u
        u[idx] = (f[idx] - (Au - diag[idx] * u[idx])) / diag[idx]
    return u


def lumped(M: spx.spmatrix) -> np.ndarray:
    """Row sums of the mass matrix (1 on the identity rows of Dirichlet vertices)."""
    return np.asarray(M.sum(axis=1)).ravel()


class TwoLevel:
    """The two-level cycle of Sec. 2.2 on (A_p, M_p, C) with the grid V-cycle of ``grid``;
    colour: the relaxation colours (mesh_colouring of the mesh); mass = "lumped" (default) or an
    int k for k CG iterations (the paper's k = 2)."""

    def __init__(self, A_p, M_p, C, grid, nx: int, ny: int, colour, mass="lumped"):
        self.A, self.M, self.C = spx.csr_matrix(A_p), M_p, spx.csr_matrix(C)
        self.grid, self.nx, self.ny = grid, nx, ny
        self.colour = np.asarray(colour)
        self.mass = mass
        self.ML = lumped(M_p)
        self.gamma = 1.0

    def _minv(self, y):
        if self.mass == "lumped":
            return y / self.ML
        return transfer.cg2(self.M, y, int(self.mass))

    def cycle(self, u: np.ndarray, f: np.ndarray) -> np.ndarray:
        sgs(self.A, u, f, self.colour)
        r = f - self.A @ u
        rc = self.C.T @ self._minv(r)                      # P^T r
        ec = np.zeros(self.nx * self.ny)
        self.grid.vcycle(ec, rc)
        u += self.gamma * self._minv(self.C @ ec)          # gamma P e_c
        sgs(self.A, u, f, self.colour)
        return u


def lanczos_mean(apply_G, solve_A, apply_A, v0: np.ndarray, k: int):
    """k steps of the Lanczos recurrence for the pencil G x = lambda A x (A SPD, G symmetric) in
    the A-inner product, from v0:
        v_1 = v0 / |v0|_A;  w = A^{-1} G v_j;  alpha_j = (G v_j) . v_j;
        w -= alpha_j v_j + beta_{j-1} v_{j-1};  beta_j = |w|_A;  v_{j+1} = w / beta_j.
    The recurrence stops early when the Krylov space is invariant (beta_j <= 1e-13 |alpha_j|):
    the Ritz values found are then eigenvalues of the pencil.  Returns (mean of the Ritz values =
    trace(T_m) / m, the m x m tridiagonal T_m), m <= k the steps taken."""
    v = np.asarray(v0, dtype=np.float64).copy()
    Av = apply_A(v)
    nrm = np.sqrt(float(v @ Av))
    v, Av = v / nrm, Av / nrm
    v_prev, Av_prev, beta = np.zeros_like(v), np.zeros_like(v), 0.0
    alphas, betas = [], []
    for j in range(k):
        g = apply_G(v)
        alpha = float(g @ v)
        w = solve_A(g) - alpha * v - beta * v_prev
        Aw = g - alpha * Av - beta * Av_prev                # = A w for the exact solve
        alphas.append(alpha)
        if j + 1 == k:
            break
        beta = np.sqrt(max(float(w @ Aw), 0.0))
        if not beta > 1e-13 * abs(alpha):
            break
        betas.append(beta)
        v_prev, Av_prev = v, Av
        v, Av = w / beta, Aw / beta
    T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
    return float(np.mean(alphas)), T


def coarse_scaling(tl: TwoLevel, v0: np.ndarray, k: int = 12):
    """Sec. 2.4's gamma for the lumped-mass cycle: the generalized Lanczos mean of
    P^T A_p P x = lambda A_c x over the interior grid unknowns (A_c the grid operator, solved
    exactly), from v0 (a grid vector; its boundary ring is ignored).  Returns (gamma, T_k)."""
    if tl.mass != "lumped":
        raise ValueError("the scaling estimate is defined for the linear (lumped) transfer")
    nx, ny = tl.nx, tl.ny
    inner = np.zeros((ny, nx), dtype=bool)
    inner[1:-1, 1:-1] = True
    ii = np.nonzero(inner.ravel())[0]
    Ac = spx.csr_matrix(tl.grid.levels[0].A)[ii][:, ii].tocsc()
    lu = spl.splu(Ac)
    P = (spx.diags(1.0 / tl.ML) @ tl.C).tocsr()[:, ii]     # lumped P restricted to the unknowns
    G = (P.T @ tl.A @ P).tocsr()
    return lanczos_mean(lambda x: G @ x, lu.solve, lambda x: Ac @ x,
                        np.asarray(v0, dtype=np.float64).ravel()[ii], k)


def solve(tl: TwoLevel, f: np.ndarray, u0: np.ndarray | None = None, rtol: float = 1e-10,
          max_iters: int = 200, keep_iterates: bool = False):
    """Stationary two-level iterations until ||f - A u|| <= rtol ||f - A u_0||.
    Returns (u, cycles, relative residual history, iterates)."""
    f = np.asarray(f, dtype=np.float64)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64)
    r0 = float(np.linalg.norm(f - tl.A @ u))
    hist, its = [], []
    k = 0
    if r0 == 0.0:
        return u, 0, [0.0], ([] if keep_iterates else None)
    while k < max_iters:
        tl.cycle(u, f)
        k += 1
        rr = float(np.linalg.norm(f - tl.A @ u)) / r0
        hist.append(rr)
        if keep_iterates:
            its.append(u.copy())
        if rr <= rtol:
            break
    return u, k, hist, (its if keep_iterates else None)
