"""The boundary from plain C (CPU side): vdwdf.h compiles as strict C99 on
its own, and the C caller in tests/c_abi (built by the package build with
gcc -std=c99 -Wall -Wextra -Werror against the header and libvdwdf.so)
loads and exports its entry points.  Nothing here reaches the device."""
import ctypes as ct
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEMO = os.path.join(ROOT, "tests", "c_abi", "libenl_from_c.so")


def test_header_is_strict_c99(tmp_path):
    src = tmp_path / "use_header.c"
    src.write_text('#include "vdwdf.h"\n'
                   "int main(void) {\n"
                   "    vdw_grid g; vdw_opts o; vdw_table_params t; vdw_stats s;\n"
                   "    (void)g; (void)o; (void)t; (void)s;\n"
                   "    return VDW_OK + VDW_FP64 + VDW_GRAD_FD + VDW_INTERP_BILINEAR;\n"
                   "}\n")
    r = subprocess.run(["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", "-fsyntax-only",
                        "-I" + os.path.join(ROOT, "include"), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


class TableParams(ct.Structure):
    _fields_ = [("n_D", ct.c_int32), ("n_sigma", ct.c_int32), ("D_max", ct.c_double), ("gl_points", ct.c_int32),
                ("graded_levels", ct.c_int32), ("kappa", ct.c_double), ("A0", ct.c_double), ("interp", ct.c_int32)]


def test_c_caller_loads_and_exports():
    assert os.path.exists(DEMO), "build the package first (__graft_entry__.build)"
    lib = ct.CDLL(DEMO)
    assert hasattr(lib, "vdw_c_demo") and hasattr(lib, "vdw_c_demo_table")
    tp = TableParams()
    lib.vdw_c_demo_table(ct.byref(tp))  # host only
    assert (tp.n_D, tp.n_sigma, tp.D_max, tp.gl_points, tp.graded_levels, tp.kappa, tp.A0, tp.interp) == \
        (256, 16, 16.0, 6, 8, 2.0, 20.0, 0)
