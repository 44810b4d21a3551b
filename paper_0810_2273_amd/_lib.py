"""ctypes view of libvdwdf.so (the C ABI declared in include/vdwdf.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvdwdf.so")

VDW_OK = 0
VDW_EINVAL = -1
VDW_ENOMEM = -2
VDW_EHIP = -3
VDW_EUNSUPPORTED = -4
VDW_EWORKSPACE = -5
VDW_ENONFINITE = -6
VDW_FP64 = 0
VDW_FP32C = 1

EXPORTS = (
    "vdw_last_error", "vdw_version", "build_phi_table", "compute_q0", "enl_workspace_size", "enl_energy",
    "enl_potential", "enl_batched_workspace_size", "enl_potential_batched", "vdw_last_stats", "vdw_set_timing",
    "enl_batch_plan_create", "enl_batch_plan_execute", "enl_batch_plan_capture", "enl_batch_plan_replay",
    "enl_batch_plan_destroy", "xc_workspace_size", "xc_energies", "vdw_recombine", "enl_potential_noalloc",
    "vdw_image_window",
)


class VdwGrid(ct.Structure):
    _fields_ = [("n", ct.c_int32 * 3), ("cell", (ct.c_double * 3) * 3), ("periodic", ct.c_int32 * 3),
                ("gradient", ct.c_int32)]


class VdwTableParams(ct.Structure):
    _fields_ = [
        ("n_D", ct.c_int32), ("n_sigma", ct.c_int32), ("D_max", ct.c_double),
        ("gl_points", ct.c_int32), ("graded_levels", ct.c_int32), ("kappa", ct.c_double), ("A0", ct.c_double),
        ("interp", ct.c_int32),
    ]


class VdwOpts(ct.Structure):
    _fields_ = [
        ("n_cut", ct.c_double), ("r_cut", ct.c_double), ("image_max", ct.c_int32 * 3),
        ("precision", ct.c_int32), ("self_term", ct.c_int32), ("table_lds_rows", ct.c_int32),
        ("block_threads", ct.c_int32), ("j_chunks", ct.c_int32), ("grid_blocks", ct.c_int32), ("kahan", ct.c_int32),
        ("far_max", ct.c_int32 * 3),
    ]


class VdwStats(ct.Structure):
    _fields_ = [
        ("retained", ct.c_int64), ("pairs", ct.c_double), ("pair_kernel_ms", ct.c_float),
        ("lds_rows", ct.c_int32), ("block_threads", ct.c_int32), ("j_chunks", ct.c_int32), ("grid_blocks", ct.c_int32),
        ("diag_items", ct.c_int32), ("far_pairs", ct.c_double), ("far_kernel_ms", ct.c_float),
        ("image_reach", ct.c_double), ("image_cut_covered", ct.c_int32), ("q0_min", ct.c_double),
        ("far_D_min", ct.c_double),
    ]


class VdwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libvdwdf error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no fallback path")
    L = ct.CDLL(LIB_PATH)
    P, vp, d, i32, sz = ct.POINTER, ct.c_void_p, ct.c_double, ct.c_int32, ct.c_size_t
    L.vdw_last_error.restype = ct.c_char_p
    L.vdw_version.restype = ct.c_char_p
    L.build_phi_table.restype = ct.c_int
    L.build_phi_table.argtypes = [P(VdwTableParams), vp, vp, vp]
    L.compute_q0.restype = ct.c_int
    L.compute_q0.argtypes = [P(VdwGrid), d, vp, vp, vp, vp, vp, vp]
    L.enl_workspace_size.restype = sz
    L.enl_workspace_size.argtypes = [P(VdwGrid), P(VdwTableParams), P(VdwOpts)]
    L.enl_batched_workspace_size.restype = sz
    L.enl_batched_workspace_size.argtypes = [i32, P(VdwGrid), P(VdwTableParams), P(VdwOpts)]
    L.enl_energy.restype = ct.c_int
    L.enl_energy.argtypes = [P(VdwGrid), vp, vp, vp, vp, P(VdwTableParams), P(VdwOpts), vp, sz, P(d), vp]
    L.enl_potential.restype = ct.c_int
    L.enl_potential.argtypes = [P(VdwGrid), vp, vp, vp, vp, vp, vp, vp, P(VdwTableParams), P(VdwOpts), vp, sz,
                                vp, P(d), vp]
    L.vdw_image_window.restype = ct.c_int
    L.vdw_image_window.argtypes = [P(VdwGrid), P(VdwOpts), P(d), P(i32)]
    L.enl_potential_noalloc.restype = ct.c_int
    L.enl_potential_noalloc.argtypes = [P(VdwGrid), vp, vp, vp, vp, vp, vp, vp, P(VdwTableParams), P(VdwOpts),
                                        vp, P(d), vp]
    L.enl_potential_batched.restype = ct.c_int
    L.enl_potential_batched.argtypes = [i32, P(VdwGrid), P(ct.c_int64), vp, vp, vp, vp, vp, vp, vp,
                                        P(VdwTableParams), P(VdwOpts), vp, sz, vp, P(d), vp]
    L.enl_batch_plan_create.restype = ct.c_int
    L.enl_batch_plan_create.argtypes = [i32, P(VdwGrid), P(ct.c_int64), P(VdwTableParams), P(VdwOpts), i32, vp, sz,
                                        P(vp), vp]
    L.enl_batch_plan_execute.restype = ct.c_int
    L.enl_batch_plan_execute.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.enl_batch_plan_capture.restype = ct.c_int
    L.enl_batch_plan_capture.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.enl_batch_plan_replay.restype = ct.c_int
    L.enl_batch_plan_replay.argtypes = [vp, vp]
    L.enl_batch_plan_destroy.restype = ct.c_int
    L.enl_batch_plan_destroy.argtypes = [vp]
    L.vdw_last_stats.restype = ct.c_int
    L.vdw_last_stats.argtypes = [P(VdwStats)]
    L.vdw_set_timing.restype = None
    L.vdw_set_timing.argtypes = [i32]
    L.xc_workspace_size.restype = sz
    L.xc_workspace_size.argtypes = [P(VdwGrid)]
    L.xc_energies.restype = ct.c_int
    L.xc_energies.argtypes = [P(VdwGrid), vp, d, vp, sz, P(d), vp]
    L.vdw_recombine.restype = d
    L.vdw_recombine.argtypes = [P(d), d, d, i32]
    _lib = L
    return L


def check(rc):
    if rc != VDW_OK:
        raise VdwError(rc, lib().vdw_last_error().decode())
    return rc
