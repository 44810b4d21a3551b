"""The C ABI on the CPU: the built library loads, exports every function the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_0810_2273_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_0810_2273_amd import build_ext

        build_ext.build()
    return _lib


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "vdwdf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\([^;{]*\)\s*;", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ("build_phi_table", "compute_q0", "enl_energy", "enl_potential", "enl_potential_batched",
              "enl_workspace_size", "vdw_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    lib = L.lib()
    for n in _declared_functions():
        assert hasattr(lib, n), n
    assert set(L.EXPORTS) <= set(_declared_functions())
    assert b"gfx950" in lib.vdw_version()


def test_host_side_validation(L):
    lib = L.lib()
    g = L.VdwGrid()
    for a in range(3):
        g.n[a] = 8
        g.cell[a][a] = 4.0
    assert lib.compute_q0(None, 1e-5, None, None, None, None, None, None) == L.VDW_EINVAL
    assert lib.compute_q0(ct.byref(g), 1e-5, None, None, None, None, None, None) == L.VDW_EINVAL
    assert b"NULL" in lib.vdw_last_error()
    skew = L.VdwGrid.from_buffer_copy(g)
    skew.cell[0][1] = 0.5
    dummy = ct.c_void_p(16)
    assert lib.compute_q0(ct.byref(skew), 1e-5, dummy, None, dummy, None, None, None) == L.VDW_EUNSUPPORTED
    small = L.VdwGrid.from_buffer_copy(g)
    small.n[2] = 2
    assert lib.compute_q0(ct.byref(small), 1e-5, dummy, None, dummy, None, None, None) == L.VDW_EINVAL
    assert lib.compute_q0(ct.byref(g), 0.0, dummy, None, dummy, None, None, None) == L.VDW_EINVAL
    tp = L.VdwTableParams(2, 16, 48.0, 8, 12, 4.0, 64.0)
    assert lib.build_phi_table(ct.byref(tp), dummy, None, None) == L.VDW_EINVAL
    tp = L.VdwTableParams(64, 16, -1.0, 8, 12, 4.0, 64.0)
    assert lib.build_phi_table(ct.byref(tp), dummy, None, None) == L.VDW_EINVAL
    tp = L.VdwTableParams(64, 16, 12.0, 40, 12, 4.0, 64.0)
    assert lib.build_phi_table(ct.byref(tp), dummy, None, None) == L.VDW_EINVAL
    tp = L.VdwTableParams(64, 16, 12.0, 8, 12, 4.0, 64.0)
    o = L.VdwOpts()
    o.n_cut = 1e-5
    o.precision = 1
    o.self_term = 1
    o.table_lds_rows = -1
    E = (ct.c_double * 3)()
    # FP32C without an FP32 table
    assert lib.enl_energy(ct.byref(g), dummy, dummy, dummy, None, ct.byref(tp), ct.byref(o), dummy, 1 << 20, E,
                          None) == L.VDW_EINVAL
    o.precision = 7
    assert lib.enl_energy(ct.byref(g), dummy, dummy, dummy, dummy, ct.byref(tp), ct.byref(o), dummy, 1 << 20, E,
                          None) == L.VDW_EINVAL
    assert lib.enl_workspace_size(ct.byref(g), ct.byref(tp), ct.byref(o)) == 0
    o.precision = 0
    o.n_cut = float("nan")
    assert lib.enl_energy(ct.byref(g), dummy, dummy, dummy, None, ct.byref(tp), ct.byref(o), dummy, 1 << 20, E,
                          None) == L.VDW_EINVAL
    o.n_cut = 1e-5
    assert lib.enl_workspace_size(ct.byref(g), ct.byref(tp), ct.byref(o)) > 0
    o.j_chunks = 99
    assert lib.enl_workspace_size(ct.byref(g), ct.byref(tp), ct.byref(o)) == 0


def test_batch_plan_host_validation(L):
    """The plan entry points reject NULL handles and arguments on the host."""
    lib = L.lib()
    dummy = ct.c_void_p(16)
    h = ct.c_void_p()
    g = L.VdwGrid()
    for a in range(3):
        g.n[a] = 8
        g.cell[a][a] = 4.0
    tp = L.VdwTableParams(64, 16, 12.0, 8, 12, 4.0, 64.0)
    o = L.VdwOpts()
    o.n_cut = 1e-5
    o.precision = 1
    offs = (ct.c_int64 * 2)(0, 512)
    assert lib.enl_batch_plan_create(1, ct.byref(g), offs, ct.byref(tp), ct.byref(o), 1, dummy, 1 << 20, None,
                                     None) == L.VDW_EINVAL
    assert lib.enl_batch_plan_create(1, ct.byref(g), None, ct.byref(tp), ct.byref(o), 1, dummy, 1 << 20,
                                     ct.byref(h), None) == L.VDW_EINVAL
    assert h.value is None
    assert lib.enl_batch_plan_create(1, ct.byref(g), offs, ct.byref(tp), ct.byref(o), 2, dummy, 1 << 20,
                                     ct.byref(h), None) == L.VDW_EINVAL
    o.precision = 7
    assert lib.enl_batch_plan_create(1, ct.byref(g), offs, ct.byref(tp), ct.byref(o), 1, dummy, 1 << 20,
                                     ct.byref(h), None) == L.VDW_EINVAL
    assert h.value is None
    assert lib.enl_batch_plan_execute(None, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy,
                                      None) == L.VDW_EINVAL
    assert lib.enl_batch_plan_capture(None, dummy, dummy, dummy, dummy, dummy, dummy, dummy, dummy,
                                      dummy) == L.VDW_EINVAL
    assert lib.enl_batch_plan_replay(None, None) == L.VDW_EINVAL
    assert lib.enl_batch_plan_destroy(None) == L.VDW_OK
