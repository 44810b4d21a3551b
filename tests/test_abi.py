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
    # a skew cell whose lattice vectors are linearly dependent
    flat = L.VdwGrid.from_buffer_copy(g)
    flat.cell[1][0], flat.cell[1][1] = 4.0, 0.0
    dummy = ct.c_void_p(16)  # never dereferenced: every call below fails validation first
    assert lib.compute_q0(ct.byref(flat), 1e-5, dummy, None, dummy, None, None, None) == L.VDW_EINVAL
    assert b"degenerate" in lib.vdw_last_error()
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
    # skew cells are planned (general-metric kernels), Kahan runs included
    o.j_chunks = 0
    skew = L.VdwGrid.from_buffer_copy(g)
    skew.cell[1][0] = 1.5
    assert lib.enl_workspace_size(ct.byref(skew), ct.byref(tp), ct.byref(o)) > 0
    o.kahan = 1
    o.precision = 1
    assert lib.enl_workspace_size(ct.byref(skew), ct.byref(tp), ct.byref(o)) > 0


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


def test_xc_host_side(L, oracle):
    """xc_energies rejects bad arguments before any device work; its
    workspace grows with the grid up to a fixed number of block partials;
    vdw_recombine (host arithmetic) is Eq. (3), checked against the oracle on
    the paper's sample-run energies."""
    import math

    lib = L.lib()
    g = L.VdwGrid()
    g.n[:] = (8, 8, 8)
    for a in range(3):
        g.cell[a][a] = 8 * 0.4
    small = lib.xc_workspace_size(ct.byref(g))
    assert small > 0
    g2 = L.VdwGrid()
    g2.n[:] = (96, 96, 96)
    for a in range(3):
        g2.cell[a][a] = 96 * 0.25
    big = lib.xc_workspace_size(ct.byref(g2))
    assert small < big <= (5 * 2048 + 6) * 8
    E = (ct.c_double * 5)()
    ws = ct.c_void_p(16)  # never dereferenced: validation fails first
    assert lib.xc_energies(ct.byref(g), None, 1e-12, ws, big, E, None) == L.VDW_EINVAL
    assert lib.xc_energies(ct.byref(g), ws, -1.0, ws, big, E, None) == L.VDW_EINVAL
    assert lib.xc_energies(ct.byref(g), ws, float("nan"), ws, big, E, None) == L.VDW_EINVAL
    assert lib.xc_energies(ct.byref(g), ws, 1e-12, ws, small - 8, E, None) == L.VDW_EWORKSPACE
    bad = L.VdwGrid()
    bad.n[:] = (2, 8, 8)
    assert lib.xc_workspace_size(ct.byref(bad)) == 0
    # Eq. (3) on the sample run's printed energies (eV; only the differences matter)
    ex_lda, ec_lda, ex_pbe, ec_pbe, ex_rev = -783.10552037, -59.77262220, -810.50311278, -42.20550892, -811.6072505786024
    e_nl = 6.16752468
    xc = (ct.c_double * 5)(ex_lda, ec_lda, ex_pbe, ec_pbe, ex_rev)
    assert lib.vdw_recombine(xc, e_nl, 0.0, 0) == pytest.approx(oracle.recombine(e_nl, ec_lda, ec_pbe), abs=1e-12)
    assert lib.vdw_recombine(xc, e_nl, -1234.5, 1) == pytest.approx(
        oracle.recombine(e_nl, ec_lda, ec_pbe, Ex_pbe=ex_pbe, Ex_new=ex_rev, E_dft=-1234.5), abs=1e-9)
    assert math.isnan(lib.vdw_recombine(xc, e_nl, 0.0, 2))
    assert math.isnan(lib.vdw_recombine(None, e_nl, 0.0, 0))


def test_spectral_gradient_host_validation(L):
    """The gradient selector is validated and the spectral form needs the
    gradient planes and a periodic axis of at most 4096 points, before any
    device work; the batched calls size a workspace for it (no call here
    reaches the device)."""
    lib = L.lib()
    dummy = ct.c_void_p(16)  # never dereferenced
    g = L.VdwGrid()
    for a in range(3):
        g.n[a] = 8
        g.cell[a][a] = 4.0
        g.periodic[a] = 1
    g.gradient = 2
    assert lib.compute_q0(ct.byref(g), 1e-5, dummy, dummy, dummy, None, None, None) == L.VDW_EINVAL
    g.gradient = 1
    assert lib.compute_q0(ct.byref(g), 1e-5, dummy, None, dummy, None, None, None) == L.VDW_EINVAL
    assert b"grad_d" in lib.vdw_last_error()
    long = L.VdwGrid.from_buffer_copy(g)
    long.n[0] = 5000
    assert lib.compute_q0(ct.byref(long), 1e-5, dummy, dummy, dummy, None, None, None) == L.VDW_EINVAL
    tp = L.VdwTableParams(64, 16, 12.0, 8, 12, 4.0, 64.0)
    o = L.VdwOpts()
    o.n_cut = 1e-5
    o.self_term = 1
    o.table_lds_rows = -1
    fd = L.VdwGrid.from_buffer_copy(g)
    fd.gradient = 0
    lib.enl_batched_workspace_size.restype = ct.c_size_t
    both = (L.VdwGrid * 2)(g, fd)
    assert lib.enl_batched_workspace_size(2, both, ct.byref(tp), ct.byref(o)) > 0
    assert lib.xc_workspace_size(ct.byref(g)) > 3 * 512 * 8


def test_cubic_interpolant_host_validation(L):
    """interp must be 0 or 1, and the cubic form is refused for Kahan runs
    before any device work."""
    lib = L.lib()
    dummy = ct.c_void_p(16)  # never dereferenced
    g = L.VdwGrid()
    for a in range(3):
        g.n[a] = 8
        g.cell[a][a] = 4.0
    o = L.VdwOpts()
    o.n_cut = 1e-5
    o.self_term = 1
    o.table_lds_rows = -1
    o.precision = 1
    o.kahan = 1
    E = (ct.c_double * 3)()
    tp = L.VdwTableParams(64, 16, 12.0, 8, 12, 4.0, 64.0, 2)
    assert lib.build_phi_table(ct.byref(tp), dummy, None, None) == L.VDW_EINVAL
    tp = L.VdwTableParams(64, 16, 12.0, 8, 12, 4.0, 64.0, 1)
    assert lib.enl_energy(ct.byref(g), dummy, dummy, dummy, dummy, ct.byref(tp), ct.byref(o), dummy, 1 << 30, E,
                          None) == L.VDW_EUNSUPPORTED
    assert b"Kahan" in lib.vdw_last_error()


def test_far_shell_host_validation(L):
    """far_max: >= 0, no distance cut, >= image_max on periodic axes, a
    bounded shell; the workspace grows by the table of T over the grid
    displacements and two row arrays per density.  Sizes only: no call here
    reaches the device."""
    lib = L.lib()
    lib.enl_workspace_size.restype = ct.c_size_t
    lib.enl_batched_workspace_size.restype = ct.c_size_t
    g = L.VdwGrid()
    for a, (n, per) in enumerate(((8, 1), (6, 1), (10, 0))):
        g.n[a] = n
        g.cell[a][a] = 0.5 * n
        g.periodic[a] = per
    tp = L.VdwTableParams(64, 16, 12.0, 8, 12, 4.0, 64.0)

    def opts(**kw):
        o = L.VdwOpts()
        o.n_cut = 1e-5
        o.self_term = 1
        o.table_lds_rows = -1
        for k, v in kw.items():
            if k in ("image_max", "far_max"):
                for a in range(3):
                    getattr(o, k)[a] = v[a]
            else:
                setattr(o, k, v)
        return o

    def size(o, B=1):
        arr = (L.VdwGrid * B)(*([g] * B))
        return lib.enl_batched_workspace_size(B, arr, ct.byref(tp), ct.byref(o))

    base = size(opts(image_max=(1, 1, 0)))
    far = size(opts(image_max=(1, 1, 0), far_max=(4, 3, 0)))
    assert base > 0 and far > 0
    ne = (2 * 8 - 1) * (2 * 6 - 1) * (2 * 10 - 1)
    assert far - base >= 8 * ne + 2 * 8 * (8 * 6 * 10)
    # far_max on a non-periodic axis alone selects nothing
    assert size(opts(image_max=(1, 1, 0), far_max=(0, 0, 7))) == base
    assert size(opts(far_max=(-1, 0, 0))) == 0
    assert b"far_max" in lib.vdw_last_error()
    assert size(opts(image_max=(2, 1, 0), far_max=(1, 3, 0))) == 0
    assert b"below image_max" in lib.vdw_last_error()
    assert size(opts(r_cut=10.0, far_max=(3, 3, 0))) == 0
    assert b"distance cut" in lib.vdw_last_error()
    assert size(opts(far_max=(3000, 3000, 0))) == 0
    assert b"lattice vectors" in lib.vdw_last_error()
    # a batch: one table and one set of row partials per density
    one = size(opts(far_max=(3, 3, 0)))
    assert size(opts(far_max=(3, 3, 0)), B=2) > one
