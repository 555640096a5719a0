"""Entry-by-entry comparison of library arrays with the oracle's.

Every check has the form |got - ref| <= rtol * scale, entry by entry, where `scale` >= |ref| is
the magnitude of the terms that were summed to form that entry.  A sum of terms t_k computed in
two different orders differs by at most a few units of roundoff times sum |t_k|, so this is the
quantity against which a rounding-order difference is measured; where the terms do not cancel,
scale equals |ref| and the check is purely relative.  Boundary entries that are exactly zero in
the reference have scale zero there, so they must be exactly zero in the library too.

  * stencils (5-plane, any level): the coupling a_vn of an SPD matrix obeys
    |a_vn| <= sqrt(a_vv a_nn), and the element sums that form it are bounded the same way
    (Cauchy-Schwarz over the cells), so scale = sqrt(C_v C_n), the diagonal of the point itself
    for plane 0;
  * Galerkin stencils additionally: scale = (|P|^T |A| |P|)_IJ, the sum of the magnitudes of the
    triple-product terms;
  * interpolation weights: numerator and denominator term magnitudes of the collapsed
    equations, propagated through the centre-point formula;
  * iterates of V-cycles and solves: |got - ref| <= rtol |ref| + floor eps max|ref|.  Every cycle
    computes its correction from r = b - A u, whose rounding (eps |A| |u| per entry) the cycle
    maps through an approximate inverse of A; the smooth part of that rounding is amplified by
    up to cond(A) ~ h^-2, and the coarse-grid correction spreads it over every point.  The
    difference between two correctly rounded implementations is therefore a multiple of
    eps max|u| at any point, independent of |u_i|, growing with the grid: measured worst
    11, 43, 86, 81 and 1108 eps max|u| at 65^2, 129^2, 257^2, 1025^2 and 4097^2.  The floor is
    FLOOR_ULPS = 256 eps max|u| up to 1025^2 and grows as (n - 1)^2 beyond (grid_floor_ulps);
    at points where the solution crosses zero only such a floor can bound the difference, and
    elsewhere the check is relative (at 1025^2 the floor equals 1e-12 |u_i| at
    |u_i| = 0.057 max|u|).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as spx

EPS64 = float(np.finfo(np.float64).eps)
EPS32 = float(np.finfo(np.float32).eps)
FLOOR_ULPS = 256

# neighbour offsets (di, dj) of the five stored planes: C, W, S, SW, SE
PLANE_OFFSETS = ((0, 0), (-1, 0), (0, -1), (-1, -1), (1, -1))


def _shift(a: np.ndarray, di: int, dj: int) -> np.ndarray:
    """out[j, i] = a[j + dj, i + di] (zero outside the grid)."""
    ny, nx = a.shape
    out = np.zeros_like(a)
    js = slice(max(0, -dj), min(ny, ny - dj))
    is_ = slice(max(0, -di), min(nx, nx - di))
    jd = slice(max(0, dj), min(ny, ny + dj))
    id_ = slice(max(0, di), min(nx, nx + di))
    out[js, is_] = a[jd, id_]
    return out


def stencil_scale(S: np.ndarray) -> np.ndarray:
    """sqrt(C_v C_n) per stored coupling of a 5-plane stencil [5][ny][nx]."""
    C = np.abs(S[0])
    out = np.empty_like(S)
    for p, (di, dj) in enumerate(PLANE_OFFSETS):
        out[p] = np.sqrt(C * _shift(C, di, dj))
    return out


def matrix_planes(M: spx.spmatrix, nx: int, ny: int) -> np.ndarray:
    """The five stored planes of a 9-point matrix M on an nx x ny grid (entry (v, neighbour))."""
    M = M.tocsr()
    out = np.zeros((5, ny, nx))
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    v = (j * nx + i).ravel()
    for p, (di, dj) in enumerate(PLANE_OFFSETS):
        ii, jj = i.ravel() + di, j.ravel() + dj
        ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny)
        vals = np.zeros(v.size)
        vals[ok] = np.asarray(M[v[ok], jj[ok] * nx + ii[ok]]).ravel()
        out[p] = vals.reshape(ny, nx)
    return out


def galerkin_scale(A_fine: spx.spmatrix, P: spx.spmatrix, ncx: int, ncy: int,
                   S_coarse: np.ndarray) -> np.ndarray:
    """max(sqrt(C_I C_J), (|P|^T |A| |P|)_IJ) per stored coupling of the coarse stencil."""
    Pa = abs(P).tocsr()
    T = (Pa.T @ abs(A_fine).tocsr() @ Pa).tocsr()
    return np.maximum(stencil_scale(S_coarse), matrix_planes(T, ncx, ncy))


def interp_scale(S: np.ndarray, Pp: np.ndarray) -> np.ndarray:
    """Rounding magnitude of each interpolation weight in the library's 8-plane layout
    [8][ncy][ncx] (planes: w_W, w_E of the x-line point (2I+1, 2J); w_S, w_N of the y-line point
    (2I, 2J+1); the four weights of the centre point (2I+1, 2J+1)), from the reference fine
    stencil S and reference weights Pp.  A ratio -n/d of sums n, d has rounding bounded by
    eps (sum|n terms| + |n/d| sum|d terms|) / |d|; the centre formula adds the magnitudes
    carried by the neighbouring line weights it uses."""
    _, ny, nx = S.shape
    C, W, So, SW, SE = (S[k] for k in range(5))
    E = _shift(W, 1, 0)
    N = _shift(So, 0, 1)
    NE = _shift(SW, 1, 1)
    NW = _shift(SE, -1, 1)
    a = np.abs
    ncy, ncx = Pp.shape[1:]
    out = np.zeros_like(Pp)

    def at(arr, di, dj):
        """arr at fine (2I + di, 2J + dj) for every coarse (I, J) (zero off the grid)."""
        res = np.zeros((ncy, ncx))
        jj = 2 * np.arange(ncy)[:, None] + dj
        ii = 2 * np.arange(ncx)[None, :] + di
        ok = (jj >= 0) & (jj < ny) & (ii >= 0) & (ii < nx)
        jc = np.clip(jj, 0, ny - 1)
        ic = np.clip(ii, 0, nx - 1)
        res[:] = np.where(ok, arr[jc, ic], 0.0)
        return res

    def ratio_scale(num_terms, den_terms, w):
        d = np.abs(sum(den_terms))
        n = sum(a(t) for t in num_terms)
        dd = sum(a(t) for t in den_terms)
        with np.errstate(divide="ignore", invalid="ignore"):
            s = np.where(d > 0, (n + np.abs(w) * dd) / np.where(d > 0, d, 1.0), 0.0)
        return s

    # x-line point (2I+1, 2J)
    g = {k: at(v, 1, 0) for k, v in dict(C=C, N=N, S=So, W=W, NW=NW, SW=SW, E=E, NE=NE, SE=SE).items()}
    out[0] = ratio_scale([g["W"], g["NW"], g["SW"]], [g["C"], g["N"], g["S"]], Pp[0])
    out[1] = ratio_scale([g["E"], g["NE"], g["SE"]], [g["C"], g["N"], g["S"]], Pp[1])
    # y-line point (2I, 2J+1)
    g = {k: at(v, 0, 1) for k, v in dict(C=C, W=W, E=E, S=So, SW=SW, SE=SE, N=N, NW=NW, NE=NE).items()}
    out[2] = ratio_scale([g["S"], g["SW"], g["SE"]], [g["C"], g["W"], g["E"]], Pp[2])
    out[3] = ratio_scale([g["N"], g["NW"], g["NE"]], [g["C"], g["W"], g["E"]], Pp[3])
    # centre point (2I+1, 2J+1): P_SW = -(SW + W wS[W nb] + S wW[S nb]) / C, etc.
    g = {k: at(v, 1, 1) for k, v in dict(C=C, W=W, E=E, S=So, N=N, SW=SW, SE=SE, NW=NW, NE=NE).items()}

    def nb(plane, dI, dJ, arr):
        res = np.zeros((ncy, ncx))
        js = slice(max(0, -dJ), min(ncy, ncy - dJ))
        is_ = slice(max(0, -dI), min(ncx, ncx - dI))
        jd = slice(max(0, dJ), min(ncy, ncy + dJ))
        id_ = slice(max(0, dI), min(ncx, ncx + dI))
        res[js, is_] = arr[plane][jd, id_]
        return res

    def centre(corner, side1, w1, s1, side2, w2, s2, w):
        Cc = g["C"]
        num = a(g[corner]) + a(g[side1]) * (a(w1) + s1) + a(g[side2]) * (a(w2) + s2)
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(Cc > 0, num / np.where(Cc > 0, Cc, 1.0) + np.abs(w), 0.0)

    out[4] = centre("SW", "W", nb(2, 0, 0, Pp), nb(2, 0, 0, out), "S", nb(0, 0, 0, Pp), nb(0, 0, 0, out), Pp[4])
    out[5] = centre("SE", "E", nb(2, 1, 0, Pp), nb(2, 1, 0, out), "S", nb(1, 0, 0, Pp), nb(1, 0, 0, out), Pp[5])
    out[6] = centre("NW", "W", nb(3, 0, 0, Pp), nb(3, 0, 0, out), "N", nb(0, 0, 1, Pp), nb(0, 0, 1, out), Pp[6])
    out[7] = centre("NE", "E", nb(3, 1, 0, Pp), nb(3, 1, 0, out), "N", nb(1, 0, 1, Pp), nb(1, 0, 1, out), Pp[7])
    return np.maximum(out, np.abs(Pp))


def worst_ratio(got: np.ndarray, ref: np.ndarray, scale: np.ndarray):
    """(max over entries of |got - ref| / scale, index of the worst entry); entries with scale 0
    must match exactly (inf otherwise)."""
    d = np.abs(np.asarray(got, dtype=np.float64) - np.asarray(ref, dtype=np.float64))
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(scale > 0, d / np.where(scale > 0, scale, 1.0), np.where(d > 0, np.inf, 0.0))
    k = int(np.argmax(r))
    return float(r.ravel()[k]), np.unravel_index(k, r.shape)


def assert_entrywise(name: str, got, ref, scale, rtol: float):
    r, idx = worst_ratio(got, ref, scale)
    assert r <= rtol, (f"{name}: |got - ref| / scale = {r:.3e} > {rtol:.1e} at {idx} "
                       f"(got {np.asarray(got)[idx]!r}, ref {np.asarray(ref)[idx]!r}, "
                       f"scale {np.asarray(scale)[idx]!r})")
    return r


def p_planes(P: spx.spmatrix, nx: int, ny: int) -> np.ndarray:
    """A sparse interpolation matrix P (fine x coarse) in the library's 8-plane layout
    [8][ncy][ncx]: entry (I, J) of plane p is the weight of fine point f_p(I, J) to coarse point
    c_p(I, J) (planes 0, 1: x-line point (2I+1, 2J) to (I, J), (I+1, J); 2, 3: y-line point
    (2I, 2J+1) to (I, J), (I, J+1); 4..7: centre point (2I+1, 2J+1) to (I, J), (I+1, J),
    (I, J+1), (I+1, J+1)); zero where either point is off the grid."""
    P = P.tocsr()
    ncx, ncy = (nx + 1) // 2, (ny + 1) // 2
    J, I = np.meshgrid(np.arange(ncy), np.arange(ncx), indexing="ij")
    spec = [((1, 0), (0, 0)), ((1, 0), (1, 0)), ((0, 1), (0, 0)), ((0, 1), (0, 1)),
            ((1, 1), (0, 0)), ((1, 1), (1, 0)), ((1, 1), (0, 1)), ((1, 1), (1, 1))]
    out = np.zeros((8, ncy, ncx))
    for p, ((fi, fj), (ci, cj)) in enumerate(spec):
        i, j = 2 * I + fi, 2 * J + fj
        a, b = I + ci, J + cj
        ok = (i < nx) & (j < ny) & (a < ncx) & (b < ncy)
        vals = np.zeros(I.size)
        okf = ok.ravel()
        if okf.any():
            vals[okf] = np.asarray(P[(j * nx + i).ravel()[okf], (b * ncx + a).ravel()[okf]]).ravel()
        out[p] = vals.reshape(ncy, ncx)
    return out


def grid_floor_ulps(nx: int, ny: int | None = None) -> int:
    """The iterate floor for an nx x ny grid: FLOOR_ULPS up to 1025^2, then growing as the
    conditioning of A, (n - 1)^2."""
    n = max(nx, ny or nx)
    return int(FLOOR_ULPS * max(1.0, ((n - 1) / 1024.0) ** 2))


def assert_iterate(name: str, got, ref, rtol: float = 1e-12, eps: float = EPS64,
                   floor_ulps: int = FLOOR_ULPS):
    """Iterate check: |got - ref| <= rtol |ref| + floor_ulps eps max|ref| at every entry.
    Returns the worst (|got - ref| - rtol |ref|) / (eps max|ref|), the floor actually used."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    m = float(np.abs(ref).max()) if ref.size else 0.0
    d = np.abs(got - ref)
    excess = d - rtol * np.abs(ref)
    k = int(np.argmax(excess)) if ref.size else 0
    used = float(excess.ravel()[k]) / (eps * m) if m > 0 else float(d.max(initial=0.0))
    if m == 0.0:
        assert not np.any(d), f"{name}: reference is zero, got max |got| = {d.max()}"
        return 0.0
    idx = np.unravel_index(k, ref.shape)
    assert used <= floor_ulps, (f"{name}: |got - ref| = {d[idx]:.3e} at {idx} exceeds {rtol:.0e} |ref| "
                                f"({rtol * abs(ref[idx]):.3e}) by {used:.1f} eps max|ref| "
                                f"(> {floor_ulps}); ref {ref[idx]!r}, got {got[idx]!r}")
    return used


def assert_stencil(name: str, got, ref_S):
    """A 5-plane stencil entry by entry at 1e-12 of sqrt(C_v C_n)."""
    return assert_entrywise(name, got, ref_S, stencil_scale(ref_S), 1e-12)


def assert_hierarchy(name: str, levels_got, levels_ref, galerkin: bool = True):
    """Every level's stencil (sqrt(C_v C_n) scale; Galerkin levels also against the triple-product
    scale) and interpolation weights (their rounding scale), entry by entry at 1e-12.
    levels_got: [(S [5][ny][nx], P [8][ncy][ncx] or None)] as host arrays."""
    worst = 0.0
    for l, ((S, P), L) in enumerate(zip(levels_got, levels_ref)):
        worst = max(worst, assert_stencil(f"{name}: stencil level {l}", S, L.S))
        if l > 0 and galerkin:
            Lf = levels_ref[l - 1]
            worst = max(worst, assert_entrywise(f"{name}: Galerkin level {l}", S, L.S,
                                                galerkin_scale(Lf.A, Lf.P, L.nx, L.ny, L.S), 1e-12))
        if L.P is not None:
            Pp = p_planes(L.P, L.nx, L.ny)
            worst = max(worst, assert_entrywise(f"{name}: P level {l}", P, Pp,
                                                interp_scale(L.S, Pp), 1e-12))
    return worst
