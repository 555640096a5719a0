"""L2-projection transfers between a P1 triangle mesh and the structured grid
(oracle; test infrastructure only).

Paper Sec. 2.3 (Interpolation): u_p = argmin ||u_p - u_c o T||_{L2(Omega_p)} gives
M_p u_p = C u_c (eqs. physical_mass, coupled_mass), so P = M_p^{-1} C, and the Riesz-map argument
gives the restriction R = P^T = C^T M_p^{-1} (eq. restriction_fn and what follows).  M_p^{-1} is
applied approximately by two iterations of unpreconditioned CG (end of the interpolation
subsection; repeated in the timing discussion of Sec. 4.3).

Sec. 2.3.1 (Coupled Mass Evaluation) evaluates C in the computational domain
(eq. coupled_mass_comp): each physical triangle's vertices are mapped through T giving a straight
triangle tt in Omega_c; the grid cells overlapping tt are found (rasterisation); a tensor Gauss
rule on each such cell is evaluated, quadrature points outside tt count as zero, and points
inside evaluate the P1 basis through tt's barycentric coordinates.  Reading taken here: with only
the vertices mapped, T is affine on each triangle, so the Jacobian factor |J_T^{-1}| is the
constant area(tau_p) / area(tt).

Vertex sets: physical vertices flagged as Dirichlet, and grid boundary vertices, carry no degree
of freedom; their rows / columns are absent (C) or decoupled identity rows (M_p), which leaves CG
on the reduced system unchanged.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as spx


def p1_mass(xy_p: np.ndarray, tris: np.ndarray, dof: np.ndarray) -> spx.csr_matrix:
    """P1 mass matrix: element matrix (area/12) [[2,1,1],[1,2,1],[1,1,2]]; rows/columns of
    non-dof vertices replaced by the identity."""
    nv = xy_p.shape[0]
    p = xy_p[tris]                                   # [nt][3][2]
    area = 0.5 * np.abs((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                        - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    loc = np.array([[2.0, 1.0, 1.0], [1.0, 2.0, 1.0], [1.0, 1.0, 2.0]]) / 12.0
    rows = np.repeat(tris, 3, axis=1).ravel()
    cols = np.tile(tris, (1, 3)).ravel()
    vals = (area[:, None, None] * loc[None]).ravel()
    M = spx.coo_matrix((vals, (rows, cols)), shape=(nv, nv)).tocsr()
    d = spx.diags(dof.astype(np.float64))
    M = (d @ M @ d + spx.diags((~dof).astype(np.float64))).tocsr()
    M.eliminate_zeros()
    return M


def gauss_legendre_01(nq: int):
    x, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * (x + 1.0), 0.5 * w


def coupled_mass(xy_c: np.ndarray, xy_p: np.ndarray, tris: np.ndarray, dof: np.ndarray,
                 nx: int, ny: int, nq: int = 4, drop_grid_boundary: bool = True) -> spx.csr_matrix:
    """C[i, g] = int_{Omega_p} phi_p^i (phi_c^g o T) dx evaluated as in Sec. 2.3.1:
    rows = physical vertices (0 for Dirichlet vertices), columns = grid vertices j*nx + i
    (0 for boundary grid vertices unless ``drop_grid_boundary`` is False).  nq = 0 selects the
    exact overlap integral (``coupled_mass_exact``)."""
    if nq == 0:
        return coupled_mass_exact(xy_c, xy_p, tris, dof, nx, ny, drop_grid_boundary)
    hx, hy = 2.0 / (nx - 1), 2.0 / (ny - 1)
    qs, qw = gauss_legendre_01(nq)
    rows, cols, vals = [], [], []
    grid_dof = np.zeros((ny, nx), dtype=bool)
    grid_dof[1:-1, 1:-1] = True
    if not drop_grid_boundary:
        grid_dof[:] = True
    grid_dof = grid_dof.ravel()
    for t in range(tris.shape[0]):
        v = tris[t]
        c = xy_c[v]                                   # mapped vertices: triangle tt in Omega_c
        p = xy_p[v]
        area_c = 0.5 * ((c[1, 0] - c[0, 0]) * (c[2, 1] - c[0, 1]) - (c[2, 0] - c[0, 0]) * (c[1, 1] - c[0, 1]))
        area_p = 0.5 * abs((p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[2, 0] - p[0, 0]) * (p[1, 1] - p[0, 1]))
        jac = area_p / abs(area_c)
        # rasterise: every cell meeting the bounding box of tt
        i0 = int(np.clip(np.floor((c[:, 0].min() + 1.0) / hx), 0, nx - 2))
        i1 = int(np.clip(np.floor((c[:, 0].max() + 1.0) / hx), 0, nx - 2))
        j0 = int(np.clip(np.floor((c[:, 1].min() + 1.0) / hy), 0, ny - 2))
        j1 = int(np.clip(np.floor((c[:, 1].max() + 1.0) / hy), 0, ny - 2))
        for cj in range(j0, j1 + 1):
            for ci in range(i0, i1 + 1):
                for qy in range(nq):
                    for qx in range(nq):
                        s, tt = qs[qx], qs[qy]
                        X = -1.0 + (ci + s) * hx
                        Y = -1.0 + (cj + tt) * hy
                        # barycentric coordinates of (X, Y) in the mapped triangle
                        l1 = ((c[2, 1] - c[0, 1]) * (X - c[0, 0]) - (c[2, 0] - c[0, 0]) * (Y - c[0, 1])) / (2 * area_c)
                        l2 = (-(c[1, 1] - c[0, 1]) * (X - c[0, 0]) + (c[1, 0] - c[0, 0]) * (Y - c[0, 1])) / (2 * area_c)
                        l0 = 1.0 - l1 - l2
                        lam = (l0, l1, l2)
                        if min(lam) < 0.0:
                            continue                  # outside the mapped element: evaluates as 0
                        w = qw[qx] * qw[qy] * hx * hy * jac
                        phic = ((1 - s) * (1 - tt), s * (1 - tt), (1 - s) * tt, s * tt)
                        gidx = (cj * nx + ci, cj * nx + ci + 1, (cj + 1) * nx + ci, (cj + 1) * nx + ci + 1)
                        for a in range(3):
                            for g in range(4):
                                rows.append(v[a]); cols.append(gidx[g]); vals.append(w * lam[a] * phic[g])
    C = spx.coo_matrix((vals, (rows, cols)), shape=(xy_p.shape[0], nx * ny)).tocsr()
    C = (spx.diags(dof.astype(np.float64)) @ C @ spx.diags(grid_dof.astype(np.float64))).tocsr()
    C.eliminate_zeros()
    return C


def clip_to_box(poly: list, x0: float, x1: float, y0: float, y1: float) -> list:
    """Sutherland-Hodgman: the part of the convex polygon ``poly`` (list of (x, y)) inside the
    box [x0, x1] x [y0, y1]."""
    def clip(pts, inside, cross):
        out = []
        for k in range(len(pts)):
            a, b = pts[k - 1], pts[k]
            ia, ib = inside(a), inside(b)
            if ib:
                if not ia:
                    out.append(cross(a, b))
                out.append(b)
            elif ia:
                out.append(cross(a, b))
        return out

    def at_x(xc):
        return lambda a, b: (xc, a[1] + (b[1] - a[1]) * (xc - a[0]) / (b[0] - a[0]))

    def at_y(yc):
        return lambda a, b: (a[0] + (b[0] - a[0]) * (yc - a[1]) / (b[1] - a[1]), yc)

    pts = list(poly)
    for inside, cross in ((lambda p: p[0] >= x0, at_x(x0)), (lambda p: p[0] <= x1, at_x(x1)),
                          (lambda p: p[1] >= y0, at_y(y0)), (lambda p: p[1] <= y1, at_y(y1))):
        if not pts:
            break
        pts = clip(pts, inside, cross)
    return pts


def collapsed_rule(A, B, Cv, order: int = 3):
    """Points and weights of a rule on triangle (A, B, C) from Gauss-Legendre on the unit square
    through the collapsed map (xi, eta) -> (1 - xi) A + xi (1 - eta) B + xi eta C, whose Jacobian
    is 2 |T| xi; with 3 x 3 points it integrates polynomials of degree <= 4 exactly."""
    g, w = gauss_legendre_01(order)
    A, B, Cv = (np.asarray(v, dtype=np.float64) for v in (A, B, Cv))
    area2 = abs((B[0] - A[0]) * (Cv[1] - A[1]) - (Cv[0] - A[0]) * (B[1] - A[1]))
    pts, wts = [], []
    for a in range(order):
        for b in range(order):
            xi, eta = g[a], g[b]
            pts.append((1 - xi) * A + xi * (1 - eta) * B + xi * eta * Cv)
            wts.append(w[a] * w[b] * area2 * xi)
    return np.array(pts), np.array(wts)


def coupled_mass_exact(xy_c: np.ndarray, xy_p: np.ndarray, tris: np.ndarray, dof: np.ndarray,
                       nx: int, ny: int, drop_grid_boundary: bool = True) -> spx.csr_matrix:
    """C of Sec. 2.3.1 integrated exactly (up to rounding) in the computational domain: every
    mapped triangle is clipped against every grid cell it meets; on the overlap polygon the
    integrand lambda_a * phi_c^g (linear times bilinear, degree 3) is integrated by a fan of
    triangles with the collapsed 3 x 3 Gauss rule; the Jacobian factor is area(tau_p) /
    area(mapped tau).  The limit of the rasterised rule of ``coupled_mass`` as nq grows."""
    hx, hy = 2.0 / (nx - 1), 2.0 / (ny - 1)
    rows, cols, vals = [], [], []
    grid_dof = np.zeros((ny, nx), dtype=bool)
    grid_dof[1:-1, 1:-1] = True
    if not drop_grid_boundary:
        grid_dof[:] = True
    grid_dof = grid_dof.ravel()
    for t in range(tris.shape[0]):
        v = tris[t]
        c = xy_c[v]
        p = xy_p[v]
        det_c = (c[1, 0] - c[0, 0]) * (c[2, 1] - c[0, 1]) - (c[2, 0] - c[0, 0]) * (c[1, 1] - c[0, 1])
        det_p = (p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[2, 0] - p[0, 0]) * (p[1, 1] - p[0, 1])
        jac = abs(det_p) / abs(det_c)
        i0 = int(np.clip(np.floor((c[:, 0].min() + 1.0) / hx), 0, nx - 2))
        i1 = int(np.clip(np.floor((c[:, 0].max() + 1.0) / hx), 0, nx - 2))
        j0 = int(np.clip(np.floor((c[:, 1].min() + 1.0) / hy), 0, ny - 2))
        j1 = int(np.clip(np.floor((c[:, 1].max() + 1.0) / hy), 0, ny - 2))
        tri = [tuple(c[0]), tuple(c[1]), tuple(c[2])]
        for cj in range(j0, j1 + 1):
            for ci in range(i0, i1 + 1):
                X0, Y0 = -1.0 + ci * hx, -1.0 + cj * hy
                poly = clip_to_box(tri, X0, X0 + hx, Y0, Y0 + hy)
                if len(poly) < 3:
                    continue
                gidx = (cj * nx + ci, cj * nx + ci + 1, (cj + 1) * nx + ci, (cj + 1) * nx + ci + 1)
                acc = np.zeros((3, 4))
                for k in range(1, len(poly) - 1):
                    pts, wts = collapsed_rule(poly[0], poly[k], poly[k + 1])
                    X, Y = pts[:, 0], pts[:, 1]
                    l1 = ((c[2, 1] - c[0, 1]) * (X - c[0, 0]) - (c[2, 0] - c[0, 0]) * (Y - c[0, 1])) / det_c
                    l2 = (-(c[1, 1] - c[0, 1]) * (X - c[0, 0]) + (c[1, 0] - c[0, 0]) * (Y - c[0, 1])) / det_c
                    lam = (1.0 - l1 - l2, l1, l2)
                    s, tt = (X - X0) / hx, (Y - Y0) / hy
                    phic = ((1 - s) * (1 - tt), s * (1 - tt), (1 - s) * tt, s * tt)
                    for a in range(3):
                        for g in range(4):
                            acc[a, g] += float(np.sum(wts * lam[a] * phic[g]))
                for a in range(3):
                    for g in range(4):
                        rows.append(v[a]); cols.append(gidx[g]); vals.append(jac * acc[a, g])
    C = spx.coo_matrix((vals, (rows, cols)), shape=(xy_p.shape[0], nx * ny)).tocsr()
    C = (spx.diags(dof.astype(np.float64)) @ C @ spx.diags(grid_dof.astype(np.float64))).tocsr()
    C.eliminate_zeros()
    return C


def cg2(M: spx.spmatrix, y: np.ndarray, iters: int = 2) -> np.ndarray:
    """``iters`` iterations of textbook unpreconditioned CG for M x = y from x_0 = 0."""
    x = np.zeros_like(y)
    r = y.copy()
    p = r.copy()
    rr = float(r @ r)
    for _ in range(iters):
        if rr == 0.0:
            break
        q = M @ p
        alpha = rr / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


def from_grid(M, C, u_c: np.ndarray, iters: int = 2) -> np.ndarray:
    """Interpolation u_p = M_p^{-1} C u_c with M_p^{-1} replaced by two CG iterations."""
    return cg2(M, C @ np.asarray(u_c, dtype=np.float64).ravel(), iters)


def to_grid(M, C, r_p: np.ndarray, nx: int, ny: int, iters: int = 2) -> np.ndarray:
    """Restriction r_c = C^T M_p^{-1} r_p with the same approximate mass solve."""
    return (C.T @ cg2(M, np.asarray(r_p, dtype=np.float64), iters)).reshape(ny, nx)
