"""MI355X (gfx950) implementation of the vdW-DF nonlocal correlation energy
E_c^nl and its potential (Lazic et al., arXiv:0810.2273, Sec. 2-3): a C-ABI
HIP library (include/vdwdf.h) and this thin binding."""
from .api import (  # noqa: F401
    BatchPlan, EnlFunction, Grid, Opts, Table, TableParams, build_phi_table, compute_q0, compute_q0_batched, energy,
    enl_energy, enl_potential, enl_potential_batched, enl_potential_noalloc, enl_workspace_size, image_window,
    last_stats, pack_batch, recombine, release_workspaces, set_timing, version, xc_energies, xc_workspace_size,
)
from ._lib import VDW_FP32C, VDW_FP64, VdwError  # noqa: F401
