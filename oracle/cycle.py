"""Smoother, V-cycle and solve drivers (oracle; test infrastructure only).

Paper Sec. 2.2: the structured hierarchy is solved with BoxMG V-cycles; the stopping rule of
Sec. 4 is a Euclidean residual norm below 1e-10 (read here as relative to ||b||_2, starting from
u_0 = 0).  The paper does not name the smoother; this library fixes four-colour Gauss-Seidel:
colour(i,j) = (i mod 2) + 2 (j mod 2); points of one colour are never coupled by a 9-point
stencil, so each colour step updates all its points from
    u_p <- (b_p - sum_{q != p} A_pq u_q) / A_pp.
Pre-smoothing visits colours 0,1,2,3 and post-smoothing 3,2,1,0, which makes the V-cycle a
symmetric operator.  For anisotropic operators (BoxMG's robustness for them is what the paper
relies on for its computational solve) the smoother may instead be zebra line Gauss-Seidel:
each interior line of one parity solves its own equations exactly with the other unknowns
held, x-lines (rows), y-lines (columns) or both alternately, even lines first, reversed in the
post-smoothing sweep.

Every routine takes a ``dtype`` so the same definitions run in float64 or float32; the float32
V-cycle keeps the coarsest solve in float64 (upcast, solve, round back).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as spx

PRE_ORDER = (0, 1, 2, 3)
POST_ORDER = (3, 2, 1, 0)
# Line relaxation (zebra line Gauss-Seidel): the pre-smoothing sweeps as (direction, parity),
# even lines first; the post-smoothing sweep runs them in reverse, which keeps the V-cycle
# symmetric.  "alt" alternates x-lines (rows) and y-lines (columns).
LINE_SWEEPS = {
    "xline": (("x", 0), ("x", 1)),
    "yline": (("y", 0), ("y", 1)),
    "alt": (("x", 0), ("x", 1), ("y", 0), ("y", 1)),
}


def colour_masks(nx: int, ny: int):
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    inner = (i > 0) & (i < nx - 1) & (j > 0) & (j < ny - 1)
    col = (i & 1) + 2 * (j & 1)
    return [(inner & (col == c)).ravel() for c in range(4)]


class OracleLevel:
    """One level in a given precision: off-diagonal part, diagonal, colour masks, P."""

    def __init__(self, lvl, dtype):
        self.nx, self.ny = lvl.nx, lvl.ny
        A = lvl.A.astype(dtype).tocsr()
        self.A = A
        self.diag = A.diagonal().astype(dtype)
        self.off = (A - spx.diags(A.diagonal())).tocsr().astype(dtype)
        self.off.eliminate_zeros()
        self.masks = colour_masks(self.nx, self.ny)
        self.P = None if lvl.P is None else lvl.P.astype(dtype).tocsr()
        self.PT = None if lvl.P is None else lvl.P.T.astype(dtype).tocsr()
        self.dtype = dtype


class Oracle:
    """A hierarchy prepared for cycling in ``dtype``; the coarsest interior system is factored
    once by dense Cholesky in float64.  ``pre``/``post`` are the colour orders of one pre/post
    sweep and ``nu_pre``/``nu_post`` the sweep counts of a V(nu_pre, nu_post) cycle."""

    def __init__(self, levels, dtype=np.float64, pre=None, post=None, nu_pre=1, nu_post=1,
                 smoother="point"):
        self.dtype = np.dtype(dtype)
        self.pre = tuple(PRE_ORDER if pre is None else pre)
        self.post = tuple(POST_ORDER if post is None else post)
        self.nu_pre, self.nu_post = nu_pre, nu_post
        if smoother not in LINE_SWEEPS and smoother != "point":
            raise ValueError(f"unknown smoother {smoother!r}")
        self.smoother = smoother
        self.levels = [OracleLevel(L, self.dtype) for L in levels]
        last = levels[-1]
        inner = colour_masks(last.nx, last.ny)
        self.coarse_idx = np.flatnonzero(inner[0] | inner[1] | inner[2] | inner[3])
        Ad = last.A.toarray()[np.ix_(self.coarse_idx, self.coarse_idx)]
        self.chol = sla.cho_factor(Ad, lower=True) if len(self.coarse_idx) else None

    # -- building blocks ------------------------------------------------------------------
    def smooth(self, l: int, u: np.ndarray, b: np.ndarray, order) -> np.ndarray:
        L = self.levels[l]
        for c in order:
            m = L.masks[c]
            t = b - L.off @ u
            u[m] = t[m] / L.diag[m]
        return u

    def line_smooth(self, l: int, u: np.ndarray, b: np.ndarray, direction: str,
                    parity: int) -> np.ndarray:
        """Line Gauss-Seidel on the interior lines of one parity: x-lines are rows j, y-lines are
        columns i, with index % 2 == parity.  Each line solves its own equations exactly for its
        own unknowns, the other unknowns held at their current values; lines of one parity are
        not coupled by a 9-point stencil, so their order does not matter."""
        L = self.levels[l]
        nx, ny = L.nx, L.ny
        A = L.A.tocsr()
        count = ny if direction == "x" else nx
        for k in range(1, count - 1):
            if k % 2 != parity:
                continue
            if direction == "x":
                I = k * nx + np.arange(1, nx - 1)
            else:
                I = np.arange(1, ny - 1) * nx + k
            AI = A[I]
            AII = AI[:, I].toarray()
            rhs = b[I] - (AI @ u - AII @ u[I])
            u[I] = np.linalg.solve(AII, rhs)
        return u

    def _sweep(self, l: int, u: np.ndarray, b: np.ndarray, pre: bool) -> np.ndarray:
        if self.smoother == "point":
            return self.smooth(l, u, b, self.pre if pre else self.post)
        seq = LINE_SWEEPS[self.smoother]
        for direction, parity in (seq if pre else seq[::-1]):
            self.line_smooth(l, u, b, direction, parity)
        return u

    def residual(self, l: int, u: np.ndarray, b: np.ndarray) -> np.ndarray:
        L = self.levels[l]
        r = b - L.A @ u
        # Dirichlet vertices carry no equation
        r[~(L.masks[0] | L.masks[1] | L.masks[2] | L.masks[3])] = 0
        return r

    def restrict(self, l: int, r: np.ndarray) -> np.ndarray:
        return self.levels[l].PT @ r

    def prolong(self, l: int, e: np.ndarray) -> np.ndarray:
        return self.levels[l].P @ e

    def coarse_solve(self, b: np.ndarray) -> np.ndarray:
        u = np.zeros_like(b)
        if self.chol is not None:
            x = sla.cho_solve(self.chol, b[self.coarse_idx].astype(np.float64))
            u[self.coarse_idx] = x.astype(self.dtype)
        return u

    # -- cycles ---------------------------------------------------------------------------
    def vcycle(self, u: np.ndarray, b: np.ndarray, l: int = 0) -> np.ndarray:
        """One V(1,1) cycle on level l, updating u in place (flattened [ny*nx] vectors)."""
        if l == len(self.levels) - 1:
            u[:] = self.coarse_solve(b)
            return u
        for _ in range(self.nu_pre):
            self._sweep(l, u, b, True)
        r = self.residual(l, u, b)
        bc = self.restrict(l, r)
        ec = np.zeros_like(bc)
        self.vcycle(ec, bc, l + 1)
        u += self.prolong(l, ec)
        for _ in range(self.nu_post):
            self._sweep(l, u, b, False)
        return u


def _flat(x, dtype):
    return np.array(x, dtype=dtype).ravel()


def residual_norm(orc: Oracle, u, b) -> float:
    return float(np.linalg.norm(orc.residual(0, _flat(u, np.float64), _flat(b, np.float64))))


def solve(orc: Oracle, b: np.ndarray, rtol: float = 1e-10, max_iters: int = 200, u0=None,
          keep_iterates: bool = False):
    """Stationary V(1,1) iteration from u0 (default 0) until ||b - A u||_2 <= rtol ||b||_2.
    Returns (u [ny][nx], iterations, relative residual history, iterates or None)."""
    L0 = orc.levels[0]
    shape = (L0.ny, L0.nx)
    bf = _flat(b, np.float64)
    bf[~(L0.masks[0] | L0.masks[1] | L0.masks[2] | L0.masks[3])] = 0.0
    u = np.zeros_like(bf) if u0 is None else _flat(u0, np.float64)
    bn = np.linalg.norm(bf)
    hist, its = [], []
    if bn == 0.0:
        return u.reshape(shape) * 0.0, 0, [0.0], ([] if keep_iterates else None)
    rel = np.linalg.norm(orc.residual(0, u, bf)) / bn
    k = 0
    while rel > rtol and k < max_iters:
        orc.vcycle(u, bf)
        k += 1
        rel = np.linalg.norm(orc.residual(0, u, bf)) / bn
        hist.append(rel)
        if keep_iterates:
            its.append(u.reshape(shape).copy())
    return u.reshape(shape), k, hist, (its if keep_iterates else None)


def solve_ir(orc64: Oracle, orc32: Oracle, b: np.ndarray, rtol: float = 1e-10, inner: int = 1,
             max_iters: int = 200, keep_iterates: bool = False):
    """Float32 V-cycles as the preconditioner inside float64 iterative refinement:
        r = b - A x (float64); s = ||r||; r32 = fl32(r / s); e = 0;
        inner x V-cycle in float32 on (e, r32); x += s * e.
    Stops on the float64 relative residual.  Returns (x, outer steps, history, iterates)."""
    L0 = orc64.levels[0]
    shape = (L0.ny, L0.nx)
    bf = _flat(b, np.float64)
    bf[~(L0.masks[0] | L0.masks[1] | L0.masks[2] | L0.masks[3])] = 0.0
    x = np.zeros_like(bf)
    bn = np.linalg.norm(bf)
    hist, its = [], []
    if bn == 0.0:
        return x.reshape(shape), 0, [0.0], ([] if keep_iterates else None)
    r = orc64.residual(0, x, bf)
    s = np.linalg.norm(r)
    k = 0
    while s > rtol * bn and k < max_iters:
        r32 = (r / s).astype(np.float32)
        e = np.zeros_like(r32)
        for _ in range(inner):
            orc32.vcycle(e, r32)
        x += s * e.astype(np.float64)
        k += 1
        r = orc64.residual(0, x, bf)
        s = np.linalg.norm(r)
        hist.append(s / bn)
        if keep_iterates:
            its.append(x.reshape(shape).copy())
    return x.reshape(shape), k, hist, (its if keep_iterates else None)


def convergence_factor(hist, skip: int = 2) -> float:
    """Geometric-mean residual reduction per cycle after the first ``skip`` cycles."""
    h = [v for v in hist if v > 0]
    if len(h) <= skip + 1:
        return float("nan")
    return (h[-1] / h[skip]) ** (1.0 / (len(h) - 1 - skip))
