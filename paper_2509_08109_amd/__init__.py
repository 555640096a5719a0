"""MI355X (gfx950) structured multigrid for remapped elliptic problems.

Python binding over the C ABI of libdmg.so (include/dmg.h).  Every numerical step runs in the
library's HIP kernels; this module only checks tensor shapes/dtypes/devices, allocates device
memory through PyTorch and passes pointers and the current HIP stream.

    S = assemble_stencil(jac, K)              # [5][ny][nx] mapped Q1 stencil
    h = Hierarchy(S)                          # operator-induced interpolation + Galerkin levels
    u, iters, relres, hist = h.solve(b, rtol=1e-10)
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import DMG_FP32_IR, DMG_FP64, DMG_MESH_HOST_SETUP, DMG_MESH_MATRIX_FREE, DmgError, Options, default_options

__all__ = ["Hierarchy", "assemble_stencil", "grad_K", "Transfer", "TwoLevel", "BatchSolver", "DiffSolve",
           "default_options", "Options", "DmgError", "DMG_FP64", "DMG_FP32_IR", "lib", "version"]


def lib():
    return _lib.load()


def version() -> str:
    return lib().dmg_version().decode()


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev(t: torch.Tensor, shape, name: str, dtype=torch.float64) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


def assemble_stencil(jac: torch.Tensor, K: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Mapped Q1 stencil from map Jacobians at the 2x2 Gauss points ([16][ny-1][nx-1]) and a
    per-cell coefficient ([ny-1][nx-1]); returns [5][ny][nx] float64."""
    ny, nx = K.shape[0] + 1, K.shape[1] + 1
    pj = _dev(jac, (16, ny - 1, nx - 1), "jac")
    pk = _dev(K, (ny - 1, nx - 1), "K")
    if out is None:
        out = torch.empty((5, ny, nx), dtype=torch.float64, device=K.device)
    ps = _dev(out, (5, ny, nx), "out")
    _lib.check(lib().dmg_assemble_stencil(pj, pk, nx, ny, ps, _stream(K.device)))
    return out


def residual_norm_noalloc(S: torch.Tensor, u: torch.Tensor, b: torch.Tensor,
                          out: torch.Tensor | None = None) -> torch.Tensor:
    """(||b - A u||^2, ||b - A u||) of the stencil S [5][ny][nx] into a device tensor of 2, with
    no workspace and no device allocation inside the library (asynchronous on the current
    stream)."""
    _, ny, nx = S.shape
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=S.device)
    _lib.check(lib().dmg_residual_norm_noalloc(_dev(S, (5, ny, nx), "S"), _dev(u, (ny, nx), "u"),
                                               _dev(b, (ny, nx), "b"), nx, ny, _dev(out, (2,), "out"),
                                               _stream(S.device)))
    return out


def grad_K(jac: torch.Tensor, lam: torch.Tensor, u: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """dK_e = -lam_e^T G_e u_e per cell ([ny-1][nx-1])."""
    ny, nx = u.shape
    pj = _dev(jac, (16, ny - 1, nx - 1), "jac")
    pl = _dev(lam, (ny, nx), "lam")
    pu = _dev(u, (ny, nx), "u")
    if out is None:
        out = torch.empty((ny - 1, nx - 1), dtype=torch.float64, device=u.device)
    po = _dev(out, (ny - 1, nx - 1), "out")
    _lib.check(lib().dmg_grad_K(pj, pl, pu, nx, ny, po, _stream(u.device)))
    return out


class Hierarchy:
    """BoxMG hierarchy of a fine stencil S [5][ny][nx] (float64, on a GPU)."""

    def __init__(self, S: torch.Tensor, opts: Options | None = None, **kw):
        _, ny, nx = S.shape
        self.nx, self.ny, self.device = nx, ny, S.device
        self.opts = opts if opts is not None else default_options(**kw)
        nbytes = C.c_size_t()
        _lib.check(lib().dmg_workspace_bytes(nx, ny, C.byref(self.opts), C.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=S.device)
        base = self.workspace.data_ptr()
        self._off = (-base) % 256
        self._ws_ptr = base + self._off
        h = C.c_void_p()
        _lib.check(lib().dmg_setup(_dev(S, (5, ny, nx), "S"), nx, ny, C.byref(self.opts),
                                   self._ws_ptr, int(nbytes.value), _stream(S.device), C.byref(h)))
        self._h = h

    # -- inspection --------------------------------------------------------------------
    def _view(self, ptr: int, count: int) -> torch.Tensor:
        off = ptr - self.workspace.data_ptr()
        if off % 8 or off < 0 or off + 8 * count > self.workspace.numel():
            raise RuntimeError("pointer outside the workspace")
        return self.workspace[off:off + 8 * count].view(torch.float64)

    def stats(self):
        lv, gc, oc = C.c_int32(), C.c_double(), C.c_double()
        _lib.check(lib().dmg_stats(self._h, C.byref(lv), C.byref(gc), C.byref(oc)))
        return int(lv.value), float(gc.value), float(oc.value)

    @property
    def num_levels(self) -> int:
        return self.stats()[0]

    def level(self, l: int):
        """(S_l [5][ny][nx], P_l [8][nyc][nxc] or None) as views into the workspace."""
        nx, ny, ps, pp = C.c_int32(), C.c_int32(), C.c_void_p(), C.c_void_p()
        _lib.check(lib().dmg_hier_level(self._h, l, C.byref(nx), C.byref(ny), C.byref(ps), C.byref(pp)))
        nx, ny = nx.value, ny.value
        S = self._view(ps.value, 5 * nx * ny).view(5, ny, nx)
        P = None
        if pp.value:
            ncx, ncy = (nx + 1) // 2, (ny + 1) // 2
            P = self._view(pp.value, 8 * ncx * ncy).view(8, ncy, ncx)
        return S, P

    def refresh(self, S: torch.Tensor) -> None:
        """Recompute the hierarchy in place from a new fine stencil of the same dims (enqueued
        on the current stream without waiting; a non-SPD coarsest grid is reported by the next
        solve)."""
        _lib.check(lib().dmg_refresh(self._h, _dev(S, (5, self.ny, self.nx), "S"), _stream(self.device)))

    def refresh_assembled(self, jac: torch.Tensor, K: torch.Tensor) -> None:
        """assemble_stencil(jac, K) followed by refresh(), with the fine stencil assembled straight
        into the hierarchy (no stencil array of the caller's); the same bits."""
        pj = _dev(jac, (16, self.ny - 1, self.nx - 1), "jac")
        pk = _dev(K, (self.ny - 1, self.nx - 1), "K")
        _lib.check(lib().dmg_refresh_assembled(self._h, pj, pk, _stream(self.device)))

    @property
    def strip_levels(self) -> int:
        """Levels handled by the fused strip kernels (the rest run in the coarse-tail kernel)."""
        n = 0
        for l in range(self.num_levels):
            S, _ = self.level(l)
            if max(S.shape[1], S.shape[2]) > 65:
                n += 1
        return n

    def sweep(self, level: int, kind: int, u: torch.Tensor, b: torch.Tensor) -> None:
        """One fused sweep kernel on a level (kind 0: pre + restriction, 1: prolongation + post)."""
        S, _ = self.level(level)
        shp = (S.shape[1], S.shape[2])
        _lib.check(lib().dmg_sweep(self._h, level, kind, _dev(u, shp, "u"), _dev(b, shp, "b"),
                                   _stream(self.device)))

    def autotune(self, b: torch.Tensor, tiles: bool = True, colour_order: bool = False, reps: int = 10,
                 inner_cycles: bool = False):
        """Pick launch shapes per level (and optionally the colour order, and for float32
        refinement the float32 cycles per step) by timing on this hierarchy; returns config()."""
        u = torch.zeros((self.ny, self.nx), dtype=torch.float64, device=self.device)
        flags = (1 if tiles else 0) | (2 if colour_order else 0) | (4 if inner_cycles else 0)
        _lib.check(lib().dmg_autotune(self._h, _dev(u, (self.ny, self.nx), "u"),
                                      _dev(b, (self.ny, self.nx), "b"), flags, reps, _stream(self.device)))
        return self.config()

    def config(self):
        """{'levels': [(bw, seg_h) of the pre sweep per level], 'post_levels': [the same for the
        post sweep], 'pre_order': [...], 'post_order': [...]}"""
        out, post_out = [], []
        pre, post = (C.c_int32 * 4)(), (C.c_int32 * 4)()
        for l in range(self.num_levels):
            bw, sh = C.c_int32(), C.c_int32()
            _lib.check(lib().dmg_hier_config(self._h, l, C.byref(bw), C.byref(sh), pre, post))
            out.append((int(bw.value), int(sh.value)))
            _lib.check(lib().dmg_hier_sweep_config(self._h, l, 1, C.byref(bw), C.byref(sh)))
            post_out.append((int(bw.value), int(sh.value)))
        inner = C.c_int32()
        _lib.check(lib().dmg_hier_inner_cycles(self._h, C.byref(inner)))
        return {"levels": out, "post_levels": post_out, "pre_order": list(pre),
                "post_order": list(post), "inner_cycles": int(inner.value)}

    # -- cycles and solves ---------------------------------------------------------------
    def vcycle(self, u: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
        shp = (self.ny, self.nx)
        _lib.check(lib().dmg_vcycle(self._h, _dev(u, shp, "u"), _dev(b, shp, "b"), _stream(self.device)))
        return u

    def residual_norm(self, u: torch.Tensor, b: torch.Tensor) -> float:
        shp = (self.ny, self.nx)
        out = C.c_double()
        _lib.check(lib().dmg_residual_norm(self._h, _dev(u, shp, "u"), _dev(b, shp, "b"), C.byref(out),
                                           _stream(self.device)))
        return float(out.value)

    def solve(self, b: torch.Tensor, u: torch.Tensor | None = None, rtol: float = 1e-10,
              max_iters: int = 200, raise_on_fail: bool = True):
        """Solve A u = b from u (default zeros); returns (u, iterations, relres, history)."""
        shp = (self.ny, self.nx)
        if u is None:
            u = torch.zeros(shp, dtype=torch.float64, device=self.device)
        hist = (C.c_double * max(1, max_iters))()
        it, rr = C.c_int32(), C.c_double()
        st = lib().dmg_solve(self._h, _dev(u, shp, "u"), _dev(b, shp, "b"), float(rtol), int(max_iters),
                             C.byref(it), C.byref(rr), hist, _stream(self.device))
        if st != 0 and (raise_on_fail or st != 6):
            _lib.check(st)
        k = int(it.value)
        return u, k, float(rr.value), [hist[i] for i in range(k)]

    def close(self):
        if getattr(self, "_h", None):
            lib().dmg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _mesh_flags(host_setup: bool, matrix_free: bool) -> int:
    return (DMG_MESH_HOST_SETUP if host_setup else 0) | (DMG_MESH_MATRIX_FREE if matrix_free else 0)


class Transfer:
    """L2-projection transfers between a P1 mesh and the grid (host mesh arrays).  host_setup:
    assemble C on the host; matrix_free: store no C, recompute its action from the overlap sets
    on every apply."""

    def __init__(self, xy_c, xy_p, tris, dof, nx: int, ny: int, nq: int = 4, device="cuda",
                 host_setup: bool = False, matrix_free: bool = False):
        self.xy_c = np.ascontiguousarray(xy_c, dtype=np.float64)
        self.xy_p = np.ascontiguousarray(xy_p, dtype=np.float64)
        self.tris = np.ascontiguousarray(tris, dtype=np.int32)
        self.dof = np.ascontiguousarray(dof, dtype=np.uint8)
        self.nv, self.nt = self.xy_c.shape[0], self.tris.shape[0]
        if self.xy_c.shape != (self.nv, 2) or self.xy_p.shape != (self.nv, 2) or self.tris.shape != (self.nt, 3) \
                or self.dof.shape != (self.nv,):
            raise ValueError("mesh arrays have inconsistent shapes")
        self.nx, self.ny = nx, ny
        self.device = torch.device(device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(lib().dmg_transfer_create_mesh(self.nv, self.nt, self.xy_c.ctypes.data,
                                                      self.xy_p.ctypes.data, self.tris.ctypes.data,
                                                      self.dof.ctypes.data, nx, ny, nq,
                                                      _mesh_flags(host_setup, matrix_free),
                                                      _stream(self.device), C.byref(h)))
        self._h = h

    @classmethod
    def from_csr(cls, C_mat, M_mat, nx: int, ny: int, device="cuda"):
        """A transfer over the caller's coupled mass C (Np x nx*ny) and mass matrix M_p (Np x Np),
        given as scipy CSR matrices (copied to the device and kept alive by the object, as is the
        workspace)."""
        self = cls.__new__(cls)
        self.device = torch.device(device)
        self.nx, self.ny = nx, ny
        C_mat, M_mat = C_mat.tocsr(), M_mat.tocsr()
        np_, nc = C_mat.shape
        if nc != nx * ny or M_mat.shape != (np_, np_):
            raise ValueError("C must be Np x nx*ny and M_p Np x Np")
        self.nv = np_
        as_dev = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=self.device)
        self._csr = [as_dev(C_mat.indptr, torch.int32), as_dev(C_mat.indices, torch.int32),
                     as_dev(C_mat.data, torch.float64), as_dev(M_mat.indptr, torch.int32),
                     as_dev(M_mat.indices, torch.int32), as_dev(M_mat.data, torch.float64)]
        nbytes = C.c_size_t()
        _lib.check(lib().dmg_transfer_workspace_bytes(np_, nc, int(C_mat.nnz), C.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        ws = base + (-base) % 256
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(lib().dmg_transfer_create(np_, nc, *(t.data_ptr() for t in self._csr), ws,
                                                 int(nbytes.value), _stream(self.device), C.byref(h)))
        self._h = h
        return self

    def copy_C(self):
        """C as (rp, ci, v) host arrays, rows in the caller's vertex order."""
        nnz = self.nnz()[0]
        rp = np.empty(self.nv + 1, dtype=np.int32)
        ci = np.empty(max(nnz, 1), dtype=np.int32)
        v = np.empty(max(nnz, 1), dtype=np.float64)
        _lib.check(lib().dmg_transfer_copy_C(self._h, rp.ctypes.data, ci.ctypes.data, v.ctypes.data))
        return rp, ci[:nnz], v[:nnz]

    def nnz(self):
        a, b = C.c_int64(), C.c_int64()
        _lib.check(lib().dmg_transfer_info(self._h, C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    def memory(self):
        """(device bytes holding C, triangle-cell pairs of the overlap sets or 0)."""
        a, b = C.c_size_t(), C.c_int64()
        _lib.check(lib().dmg_transfer_memory(self._h, C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    def from_grid(self, u_c: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.nv, dtype=torch.float64, device=self.device)
        _lib.check(lib().dmg_transfer_from_grid(self._h, _dev(u_c, (self.ny, self.nx), "u_c"),
                                                _dev(out, (self.nv,), "out"), _stream(self.device)))
        return out

    def to_grid(self, r_p: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        _lib.check(lib().dmg_transfer_to_grid(self._h, _dev(r_p, (self.nv,), "r_p"),
                                              _dev(out, (self.ny, self.nx), "out"), _stream(self.device)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().dmg_transfer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TwoLevel:
    """The two-level cycle on a physical P1 mesh (host mesh arrays) over the grid hierarchy
    ``grid`` (a Hierarchy on the grid that the mesh maps to; it must outlive this object).
    nq: 0 for the exact coupled mass (default) or the order of the rasterised rule;
    mass: "lumped" or "cg2"; host_setup: assemble C on the host (the default is the device);
    matrix_free: store no C (as for Transfer)."""

    def __init__(self, grid: Hierarchy, xy_c, xy_p, tris, dof, K_t=None, nq: int = 0, mass: str = "lumped",
                 host_setup: bool = False, matrix_free: bool = False):
        if mass not in ("lumped", "cg2"):
            raise ValueError("mass must be 'lumped' or 'cg2'")
        self.grid = grid
        self.device = grid.device
        xy_c = np.ascontiguousarray(xy_c, dtype=np.float64)
        xy_p = np.ascontiguousarray(xy_p, dtype=np.float64)
        tris = np.ascontiguousarray(tris, dtype=np.int32)
        dof = np.ascontiguousarray(dof, dtype=np.uint8)
        self.nv, self.nt = xy_c.shape[0], tris.shape[0]
        if xy_c.shape != (self.nv, 2) or xy_p.shape != (self.nv, 2) or tris.shape != (self.nt, 3) \
                or dof.shape != (self.nv,):
            raise ValueError("mesh arrays have inconsistent shapes")
        kt = None
        if K_t is not None:
            kt = np.ascontiguousarray(K_t, dtype=np.float64)
            if kt.shape != (self.nt,):
                raise ValueError("K_t must hold one value per triangle")
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(lib().dmg_twolevel_create(self.nv, self.nt, xy_c.ctypes.data, xy_p.ctypes.data,
                                                 tris.ctypes.data, dof.ctypes.data,
                                                 None if kt is None else kt.ctypes.data, grid._h, nq,
                                                 0 if mass == "lumped" else 2,
                                                 _mesh_flags(host_setup, matrix_free),
                                                 _stream(self.device), C.byref(h)))
        self._h = h

    def info(self):
        """(number of colours, stored entries of A_p, colour of each vertex)."""
        nc, nnz = C.c_int32(), C.c_int64()
        col = np.empty(self.nv, dtype=np.int32)
        _lib.check(lib().dmg_twolevel_info(self._h, C.byref(nc), C.byref(nnz), col.ctypes.data))
        return int(nc.value), int(nnz.value), col

    def set_scaling(self, gamma: float) -> None:
        """Coarse-grid scaling: later cycles add gamma P e_c."""
        _lib.check(lib().dmg_twolevel_set_scaling(self._h, float(gamma)))

    def estimate_scaling(self, v0: torch.Tensor, k: int = 12):
        """Generalized Lanczos estimate of gamma from the start vector v0 [ny][nx];
        returns (gamma, T) with T the tridiagonal of the steps taken."""
        shp = (self.grid.ny, self.grid.nx)
        T = np.zeros((k, k))
        gam, m = C.c_double(), C.c_int32()
        _lib.check(lib().dmg_twolevel_scaling(self._h, _dev(v0, shp, "v0"), int(k), C.byref(gam),
                                              T.ctypes.data, C.byref(m), _stream(self.device)))
        return float(gam.value), T[:m.value, :m.value].copy()

    def cycle(self, u: torch.Tensor, f: torch.Tensor) -> torch.Tensor:
        """One cycle on u (in place)."""
        _lib.check(lib().dmg_twolevel_cycle(self._h, _dev(u, (self.nv,), "u"), _dev(f, (self.nv,), "f"),
                                            _stream(self.device)))
        return u

    def solve(self, f: torch.Tensor, u: torch.Tensor | None = None, rtol: float = 1e-10,
              max_iters: int = 200, raise_on_fail: bool = True):
        """Cycles from u (default zeros) until ||f - A u|| <= rtol ||f - A u_0||;
        returns (u, cycles, relres, history)."""
        if u is None:
            u = torch.zeros(self.nv, dtype=torch.float64, device=self.device)
        hist = (C.c_double * max(1, max_iters))()
        it, rr = C.c_int32(), C.c_double()
        st = lib().dmg_twolevel_solve(self._h, _dev(u, (self.nv,), "u"), _dev(f, (self.nv,), "f"), float(rtol),
                                      int(max_iters), C.byref(it), C.byref(rr), hist, _stream(self.device))
        if st != 0 and (raise_on_fail or st != 6):
            _lib.check(st)
        k = int(it.value)
        return u, k, float(rr.value), [hist[i] for i in range(k)]

    def close(self):
        if getattr(self, "_h", None):
            lib().dmg_twolevel_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver:
    """Independent instances (stencils S_k [5][ny_k][nx_k]) solved together."""

    def __init__(self, stencils, opts: Options | None = None, **kw):
        self.count = len(stencils)
        self.dims = [(int(S.shape[2]), int(S.shape[1])) for S in stencils]
        self.device = stencils[0].device
        self.opts = opts if opts is not None else default_options(**kw)
        self._nx = (C.c_int32 * self.count)(*[d[0] for d in self.dims])
        self._ny = (C.c_int32 * self.count)(*[d[1] for d in self.dims])
        nbytes = C.c_size_t()
        _lib.check(lib().dmg_batch_workspace_bytes(self.count, self._nx, self._ny, C.byref(self.opts),
                                                   C.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        ws = self.workspace.data_ptr()
        ws += (-ws) % 256
        ptrs = (C.c_void_p * self.count)(*[_dev(S, (5, ny, nx), f"S[{k}]")
                                           for k, (S, (nx, ny)) in enumerate(zip(stencils, self.dims))])
        h = C.c_void_p()
        _lib.check(lib().dmg_batch_setup(self.count, self._nx, self._ny, ptrs, C.byref(self.opts), ws,
                                         int(nbytes.value), _stream(self.device), C.byref(h)))
        self._h = h

    def _ptrs(self, arrays, name):
        return (C.c_void_p * self.count)(*[_dev(a, (ny, nx), name) for a, (nx, ny) in zip(arrays, self.dims)])

    def autotune(self, bs, reps: int = 3, tiles: bool = True, colour_order: bool = False):
        """Pick per-size launch shapes and the tail workgroup size by timing batched steps (tiles),
        and/or the colour-order pair of each size class by timing whole batched solves
        (colour_order, which changes the iterates); returns config()."""
        us = [torch.zeros((ny, nx), dtype=torch.float64, device=self.device) for nx, ny in self.dims]
        flags = (1 if tiles else 0) | (2 if colour_order else 0)
        _lib.check(lib().dmg_batch_autotune(self._h, self._ptrs(us, "u"), self._ptrs(bs, "b"), flags,
                                            int(reps), _stream(self.device)))
        return self.config()

    def config(self):
        """{'pre_order': [...], 'post_order': [...] (instance 0's), 'tail_threads': n,
        'orders': [(pre, post) of each instance]}"""
        pre, post, tt = (C.c_int32 * 4)(), (C.c_int32 * 4)(), C.c_int32()
        _lib.check(lib().dmg_batch_config(self._h, pre, post, C.byref(tt)))
        orders = []
        for k in range(self.count):
            p, q = (C.c_int32 * 4)(), (C.c_int32 * 4)()
            _lib.check(lib().dmg_batch_instance_orders(self._h, k, p, q))
            orders.append((tuple(p), tuple(q)))
        return {"pre_order": list(pre), "post_order": list(post), "tail_threads": int(tt.value),
                "orders": orders}

    def solve(self, bs, us=None, rtol: float = 1e-10, max_iters: int = 200, raise_on_fail: bool = True):
        if us is None:
            us = [torch.zeros((ny, nx), dtype=torch.float64, device=self.device) for nx, ny in self.dims]
        up = self._ptrs(us, "u")
        bp = self._ptrs(bs, "b")
        it = (C.c_int32 * self.count)()
        rr = (C.c_double * self.count)()
        st = lib().dmg_batch_solve(self._h, up, bp, float(rtol), int(max_iters), it, rr, _stream(self.device))
        if st != 0 and (raise_on_fail or st != 6):
            _lib.check(st)
        return us, list(it), list(rr)

    def close(self):
        if getattr(self, "_h", None):
            lib().dmg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _interior(x: torch.Tensor) -> torch.Tensor:
    y = x.clone()
    y[0, :] = 0
    y[-1, :] = 0
    y[:, 0] = 0
    y[:, -1] = 0
    return y


class _DiffSolver:
    """The hierarchy and buffers that DiffSolve reuses for one (device, grid, options): each
    solve copies K into the same array and refreshes the hierarchy from (jac, K), the stencil
    assembled straight into it (so the hierarchy is recomputed, never kept from an earlier call;
    from the second refresh with the same jac on, the setup runs as a replayed graph), then
    solves in the same two buffers, whose captured solve graphs are replayed instead of captured
    anew."""

    _cache: dict = {}

    @classmethod
    def solve(cls, jac: torch.Tensor, K: torch.Tensor, rhs: torch.Tensor, opts: Options | None,
              rtol: float, max_iters: int):
        o = opts if opts is not None else default_options()
        shp = (K.shape[0] + 1, K.shape[1] + 1)
        if tuple(rhs.shape) != shp or rhs.dtype != torch.float64 or rhs.device != K.device:
            raise ValueError(f"right-hand side must be float64 {shp} on {K.device}")
        key = (K.device, shp, bytes(o))
        ent = cls._cache.get(key)
        if ent is None:
            ent = cls._cache[key] = cls()
            ent.h = Hierarchy(assemble_stencil(jac, K), o)
            ent.K = K.detach().to(torch.float64).contiguous().clone()
            ent.u = torch.empty(shp, dtype=torch.float64, device=K.device)
            ent.b = torch.empty(shp, dtype=torch.float64, device=K.device)
        else:
            ent.K.copy_(K)
            ent.h.refresh_assembled(jac, ent.K)
        ent.b.copy_(rhs)
        ent.u.zero_()
        _, its, rr, _ = ent.h.solve(ent.b, u=ent.u, rtol=rtol, max_iters=max_iters,
                                    raise_on_fail=False)
        return ent.u.clone(), its, rr


class DiffSolve(torch.autograd.Function):
    last = None
    """u = A(K)^{-1} b with A the mapped Q1 operator; gradients w.r.t. K (per cell) and b.

    Forward saves only (K, b, u); backward recomputes the stencil and hierarchy, solves the
    adjoint system A lam = du (A is symmetric, so the same V-cycle serves), and returns
    dK = -lam_e^T G_e u_e and db = lam.  Calls on one device share one hierarchy and its
    buffers per grid size and options (DiffSolve.clear_cache() frees them), so they must not
    run concurrently on different streams.
    """

    @staticmethod
    def _check(which: str, its: int, rr: float, rtol: float, strict: bool) -> None:
        if strict and not rr <= rtol:
            raise DmgError(6, f"{which} solve stopped at relative residual {rr:.3e} after {its} "
                              f"cycles, above rtol {rtol:.1e} (pass strict=False to accept it)")

    @staticmethod
    def forward(ctx, K, b, jac, rtol=1e-12, max_iters=200, opts=None, strict=True):
        """strict (default): raise DmgError (DMG_ERR_NO_CONVERGENCE) when the forward solve, or
        later the adjoint solve, ends above rtol; strict=False returns the last iterate (its
        cycles and relative residual are in DiffSolve.last)."""
        u, its, rr = _DiffSolver.solve(jac, K.detach().contiguous(), b.detach(), opts, rtol,
                                       max_iters)
        DiffSolve.last = {"forward": (its, rr)}
        DiffSolve._check("forward", its, rr, rtol, strict)
        ctx.save_for_backward(K, b, u)
        ctx.jac, ctx.rtol, ctx.max_iters, ctx.opts, ctx.strict = jac, rtol, max_iters, opts, strict
        return u

    @staticmethod
    def backward(ctx, gu):
        K, b, u = ctx.saved_tensors
        lam, its, rr = _DiffSolver.solve(ctx.jac, K.detach().contiguous(),
                                         _interior(gu.contiguous().to(torch.float64)), ctx.opts,
                                         ctx.rtol, ctx.max_iters)
        DiffSolve.last = dict(DiffSolve.last or {}, adjoint=(its, rr))
        DiffSolve._check("adjoint", its, rr, ctx.rtol, ctx.strict)
        dK = grad_K(ctx.jac, lam, u) if ctx.needs_input_grad[0] else None
        db = lam if ctx.needs_input_grad[1] else None
        return dK, db, None, None, None, None, None

    @staticmethod
    def clear_cache() -> None:
        for ent in _DiffSolver._cache.values():
            ent.h.close()
        _DiffSolver._cache.clear()
