"""Host-side checks of the C ABI (no GPU needed): the in-tree library loads, exports every
function include/ppmpm.h declares, and sizes workspaces / rejects invalid problems without
touching a device."""
import ctypes
import os

import pytest

from paper_1905_00671_amd import binding as B
from paper_1905_00671_amd import workloads as W

needs_lib = pytest.mark.skipif(not os.path.exists(B.LIB_PATH), reason="libppmpm.so not built")


@needs_lib
def test_library_exports_every_declared_symbol():
    L = B.lib()
    syms = B.header_symbols()
    assert len(syms) >= 11
    for s in syms:
        assert hasattr(L, s), s


@needs_lib
def test_workspace_bytes_and_validation():
    L = B.lib()
    w = W.config(1)
    g = B.make_grid(w.grid)
    o = B.make_options(w.options)
    n64 = L.ppmpm_workspace_bytes(ctypes.byref(g), w.particles.n, ctypes.byref(o))
    o32 = B.make_options(w.options, precision=B.MIXED)
    n32 = L.ppmpm_workspace_bytes(ctypes.byref(g), w.particles.n, ctypes.byref(o32))
    assert n64 > 0 and 0 < n32 < n64
    # GIMP in 3D and a zero particle count are rejected
    w3 = W.footing3d(n=4, nsteps=1)
    g3 = B.make_grid(w3.grid)
    o3 = B.make_options(w3.options, shape=W.GIMP)
    assert L.ppmpm_workspace_bytes(ctypes.byref(g3), w3.particles.n, ctypes.byref(o3)) == 0
    assert L.ppmpm_workspace_bytes(ctypes.byref(g), 0, ctypes.byref(o)) == 0


@needs_lib
def test_workspace_grows_with_problem_size():
    L = B.lib()
    sizes = []
    for n in (16, 32, 64):
        w = W.consolidation2d(n, 1e-12)
        g = B.make_grid(w.grid)
        o = B.make_options(w.options)
        sizes.append(L.ppmpm_workspace_bytes(ctypes.byref(g), w.particles.n, ctypes.byref(o)))
    assert sizes[0] < sizes[1] < sizes[2]
    # roughly proportional to the particle count for large grids
    assert 3.0 < sizes[2] / sizes[1] < 5.0
