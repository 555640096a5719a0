"""The C-ABI library loads, exports every function include/dmg.h declares, and rejects bad
arguments on the host before touching a GPU (no compute calls here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmg.h")


@pytest.fixture(scope="module")
def dmg():
    import paper_2509_08109_amd as m
    if not os.path.exists(m._lib.LIB_PATH):
        from paper_2509_08109_amd.build import build
        build()
    return m


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dmg_[A-Za-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dmg_assemble_stencil", "dmg_setup", "dmg_vcycle", "dmg_solve",
                     "dmg_transfer_to_grid", "dmg_transfer_from_grid", "dmg_grad_K",
                     "dmg_batch_solve", "dmg_twolevel_create", "dmg_twolevel_cycle",
                     "dmg_twolevel_solve", "dmg_twolevel_scaling", "dmg_twolevel_set_scaling"):
        assert required in names


def test_library_exports_every_declared_symbol(dmg):
    lib = dmg.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(declared_functions()) <= set(dmg._lib.SIGNATURES)


def test_default_options(dmg):
    o = dmg.default_options()
    assert (o.nu_pre, o.nu_post, o.coarsest_n, o.precision, o.inner_cycles) == (1, 1, 3, 0, 1)
    assert list(o.pre_order) == [0, 1, 2, 3] and list(o.post_order) == [3, 2, 1, 0]
    assert C.sizeof(dmg.Options) == 4 * (2 + 4 + 4 + 6 + 6)
    assert o.strip_kernel == 1 and o.use_graph == 1
    assert dmg.version().startswith("dmg")


@pytest.mark.parametrize("nx,ny", [(64, 65), (65, 64), (2, 3), (1, 1), (66, 66), (0, 5)])
def test_workspace_rejects_bad_dims(dmg, nx, ny):
    lib = dmg.lib()
    nbytes = C.c_size_t()
    st = lib.dmg_workspace_bytes(nx, ny, C.byref(dmg.default_options()), C.byref(nbytes))
    assert st == 2
    assert "odd" in lib.dmg_last_error().decode()


@pytest.mark.parametrize("nx,ny", [(33, 49), (97, 65), (45, 67), (25, 25)])
def test_workspace_accepts_odd_dims(dmg, nx, ny):
    """Odd dims that are not 2^k + 1 coarsen until a dim turns even (33 x 49 -> ... -> 3 x 4)."""
    nbytes = C.c_size_t()
    assert dmg.lib().dmg_workspace_bytes(nx, ny, C.byref(dmg.default_options()), C.byref(nbytes)) == 0
    assert nbytes.value > 8 * 10 * nx * ny


def test_workspace_rejects_a_wide_coarsest_grid(dmg):
    """131 = 2 * 65 + 1 stops at 66 points a side, more than the coarse kernel holds."""
    lib = dmg.lib()
    nbytes = C.c_size_t()
    assert lib.dmg_workspace_bytes(131, 131, C.byref(dmg.default_options()), C.byref(nbytes)) == 2
    assert "coarsest grid" in lib.dmg_last_error().decode()


def test_workspace_sizes_scale_with_grid(dmg):
    lib = dmg.lib()
    sizes = []
    for n in (257, 513, 1025):
        nb = C.c_size_t()
        assert lib.dmg_workspace_bytes(n, n, C.byref(dmg.default_options()), C.byref(nb)) == 0
        sizes.append(nb.value)
    # ~ (5 S + 5 point-major S + 2 P + u, t, b, r) words per fine point, times 4/3 for the
    # coarse levels, plus a fixed part (the dense coarse operator: up to 2 x 961^2 words)
    assert 8 * 10 * 1025 * 1025 < sizes[2] < 8 * 22 * 1025 * 1025 + 2 * 8 * 961 * 961
    assert 3.5 < (sizes[2] - sizes[1]) / (sizes[1] - sizes[0]) < 4.5
    nb32 = C.c_size_t()
    o = dmg.default_options(precision=dmg.DMG_FP32_IR)
    assert lib.dmg_workspace_bytes(257, 257, C.byref(o), C.byref(nb32)) == 0
    assert nb32.value > sizes[0]


@pytest.mark.parametrize("field,value", [("nu_pre", -1), ("coarsest_n", 2), ("precision", 7),
                                         ("inner_cycles", 0), ("pre_order", [0, 0, 1, 2]),
                                         ("strip_kernel", 2), ("coarse_gemv", 2)])
def test_options_validation(dmg, field, value):
    lib = dmg.lib()
    o = dmg.default_options(**{field: value})
    nb = C.c_size_t()
    assert lib.dmg_workspace_bytes(65, 65, C.byref(o), C.byref(nb)) == 1


def test_null_and_small_workspace_rejected_on_host(dmg):
    lib = dmg.lib()
    h = C.c_void_p()
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    o = dmg.default_options()
    assert lib.dmg_setup(None, 65, 65, C.byref(o), fake, 1 << 20, None, C.byref(h)) == 1
    assert lib.dmg_setup(fake, 64, 65, C.byref(o), fake, 1 << 20, None, C.byref(h)) == 2
    assert lib.dmg_setup(fake, 65, 65, C.byref(o), None, 1 << 20, None, C.byref(h)) == 3
    assert lib.dmg_setup(fake, 65, 65, C.byref(o), C.c_void_p(0x1001), 1 << 30, None, C.byref(h)) == 3
    assert lib.dmg_setup(fake, 65, 65, C.byref(o), fake, 16, None, C.byref(h)) == 3
    assert "too small" in lib.dmg_last_error().decode()
    assert lib.dmg_assemble_stencil(None, fake, 9, 9, fake, None) == 1
    assert lib.dmg_assemble_stencil(fake, fake, 2, 9, fake, None) == 2
    assert lib.dmg_grad_K(fake, fake, None, 9, 9, fake, None) == 1
    assert lib.dmg_solve(None, fake, fake, 1e-10, 10, None, None, None, None) == 1


def test_transfer_validation_on_host(dmg):
    import numpy as np
    lib = dmg.lib()
    h = C.c_void_p()
    xy = np.zeros((3, 2))
    tris = np.array([[0, 1, 5]], dtype=np.int32)       # index out of range
    dof = np.ones(3, dtype=np.uint8)
    st = lib.dmg_transfer_create_mesh(3, 1, xy.ctypes.data, xy.ctypes.data, tris.ctypes.data, dof.ctypes.data,
                                 9, 9, 4, 0, None, C.byref(h))
    assert st == 1 and "out of range" in lib.dmg_last_error().decode()
    assert lib.dmg_transfer_create_mesh(3, 1, xy.ctypes.data, xy.ctypes.data, tris.ctypes.data, dof.ctypes.data,
                                   9, 9, -1, 0, None, C.byref(h)) == 1
    assert "nq" in lib.dmg_last_error().decode()
    # the matrix-free flag goes through the same checks before any device work
    assert lib.dmg_transfer_create_mesh(3, 1, xy.ctypes.data, xy.ctypes.data, tris.ctypes.data, dof.ctypes.data,
                                   9, 9, 4, dmg.DMG_MESH_MATRIX_FREE, None, C.byref(h)) == 1
    assert "out of range" in lib.dmg_last_error().decode()
    nb, pairs = C.c_size_t(), C.c_int64()
    assert lib.dmg_transfer_memory(None, C.byref(nb), C.byref(pairs)) == 1


def test_refresh_assembled_validation_on_host(dmg):
    lib = dmg.lib()
    fake = C.c_void_p(0x1000)
    assert lib.dmg_refresh_assembled(None, fake, fake, None) == 1
    assert lib.dmg_refresh_assembled(fake, None, fake, None) == 1
    assert lib.dmg_refresh_assembled(fake, fake, None, None) == 1
    assert "null" in lib.dmg_last_error().decode()


def test_transfer_csr_validation_on_host(dmg):
    """The CSR form's size query and the checks made before any device access."""
    lib = dmg.lib()
    nb = C.c_size_t()
    assert lib.dmg_transfer_workspace_bytes(100, 81, 900, C.byref(nb)) == 0
    # C^T (82 row pointers, 900 entries), four CG vectors, partials and scalars, transpose scratch
    assert nb.value >= 4 * 82 + 12 * 900 + 4 * 8 * 100
    assert lib.dmg_transfer_workspace_bytes(0, 81, 900, C.byref(nb)) == 1
    assert lib.dmg_transfer_workspace_bytes(100, 81, -1, C.byref(nb)) == 1
    h = C.c_void_p()
    fake = C.c_void_p(0x1000)
    assert lib.dmg_transfer_create(0, 81, fake, fake, fake, fake, fake, fake, fake, 1 << 20, None,
                                   C.byref(h)) == 1
    assert lib.dmg_transfer_create(100, 81, None, fake, fake, fake, fake, fake, fake, 1 << 20, None,
                                   C.byref(h)) == 1
    assert lib.dmg_transfer_create(100, 81, fake, fake, fake, fake, fake, fake, C.c_void_p(0x1008),
                                   1 << 20, None, C.byref(h)) == 3
    assert "aligned" in lib.dmg_last_error().decode()


def test_twolevel_validation_on_host(dmg):
    """Argument checks that return before any device work (the grid handle is not read)."""
    import numpy as np
    lib = dmg.lib()
    h = C.c_void_p()
    fake = C.c_void_p(0x1000)
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    tris = np.array([[0, 1, 2]], dtype=np.int32)
    dof = np.ones(3, dtype=np.uint8)
    args = lambda tr, xyp: (3, 1, xy.ctypes.data, xyp.ctypes.data, tr.ctypes.data, dof.ctypes.data)
    assert lib.dmg_twolevel_create(*args(tris, xy), None, None, 8, 0, 0, None, C.byref(h)) == 1
    assert lib.dmg_twolevel_create(*args(tris, xy), None, fake, 8, 3, 0, None, C.byref(h)) == 1
    assert "mass" in lib.dmg_last_error().decode()
    assert lib.dmg_twolevel_create(*args(tris, xy), None, fake, -1, 0, 0, None, C.byref(h)) == 1
    bad = np.array([[0, 1, 7]], dtype=np.int32)
    assert lib.dmg_twolevel_create(*args(bad, xy), None, fake, 8, 0, 0, None, C.byref(h)) == 1
    assert "out of range" in lib.dmg_last_error().decode()
    flat = np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0]])
    assert lib.dmg_twolevel_create(*args(tris, flat), None, fake, 8, 0, 0, None, C.byref(h)) == 1
    assert "degenerate" in lib.dmg_last_error().decode()
    assert lib.dmg_twolevel_solve(None, fake, fake, 1e-10, 10, None, None, None, None) == 1
    assert lib.dmg_twolevel_cycle(None, fake, fake, None) == 1


def test_batch_validation_on_host(dmg):
    lib = dmg.lib()
    nx = (C.c_int32 * 2)(65, 64)
    nb = C.c_size_t()
    assert lib.dmg_batch_workspace_bytes(2, nx, nx, C.byref(dmg.default_options()), C.byref(nb)) == 2
    assert lib.dmg_batch_workspace_bytes(0, nx, nx, C.byref(dmg.default_options()), C.byref(nb)) == 1


def test_product_package_does_not_import_oracle():
    """The product path never touches the oracle (checked on the source text)."""
    pkg = os.path.join(ROOT, "paper_2509_08109_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.replace("the oracle", ""), f
