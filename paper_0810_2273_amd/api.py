"""Python binding of libvdwdf.so with the C ABI's names.

PyTorch supplies device memory and streams; each function marshals
arguments and calls the library, which runs every step on the GPU.  There
is no CPU fallback: without the built library, or without a GPU, these
functions raise.
"""
from __future__ import annotations

import ctypes as ct
from dataclasses import dataclass, field

import torch

from . import _lib as L

DEFAULT_RULE = dict(gl_points=8, graded_levels=12, kappa=4.0, A0=64.0)


@dataclass
class TableParams:
    """Kernel table over D in [0, D_max] x sigma = delta^2 in [0, 1] and the quadrature rule."""

    n_D: int = 2048
    n_sigma: int = 64
    D_max: float = 48.0
    gl_points: int = 8
    graded_levels: int = 12
    kappa: float = 4.0
    A0: float = 64.0

    def c(self) -> L.VdwTableParams:
        return L.VdwTableParams(self.n_D, self.n_sigma, self.D_max, self.gl_points, self.graded_levels,
                                self.kappa, self.A0)


@dataclass
class Grid:
    """Orthorhombic equidistant grid: n points per axis, spacing h (bohr); x fastest."""

    n: tuple
    h: tuple
    periodic: tuple = (0, 0, 0)

    @property
    def G(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def dV(self) -> float:
        return float(self.h[0]) * float(self.h[1]) * float(self.h[2])

    def c(self) -> L.VdwGrid:
        g = L.VdwGrid()
        for a in range(3):
            g.n[a] = int(self.n[a])
            g.periodic[a] = int(self.periodic[a])
            for b in range(3):
                g.cell[a][b] = float(self.n[a] * self.h[a]) if a == b else 0.0
        return g


@dataclass
class Opts:
    n_cut: float = 1e-5
    r_cut: float = 0.0
    image_max: tuple = (0, 0, 0)
    precision: int = L.VDW_FP32C
    self_term: int = 1
    table_lds_rows: int = -1
    block_threads: int = 0
    j_chunks: int = 0
    grid_blocks: int = 0
    kahan: int = 0

    def c(self) -> L.VdwOpts:
        o = L.VdwOpts()
        o.n_cut = self.n_cut
        o.r_cut = self.r_cut
        for a in range(3):
            o.image_max[a] = int(self.image_max[a])
        o.precision = self.precision
        o.self_term = self.self_term
        o.table_lds_rows = self.table_lds_rows
        o.block_threads = self.block_threads
        o.j_chunks = self.j_chunks
        o.grid_blocks = self.grid_blocks
        o.kahan = self.kahan
        return o


@dataclass
class Table:
    params: TableParams
    phi64: torch.Tensor
    phi32: torch.Tensor | None = None


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors passed to libvdwdf must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors passed to libvdwdf must be contiguous")
    return ct.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def _f64(t, name):
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    return t


def version() -> str:
    return L.lib().vdw_version().decode()


def build_phi_table(params: TableParams | None = None, device="cuda", fp32: bool = True, stream=None) -> Table:
    """Fill the kernel table on the GPU (FP64, plus an FP32 copy)."""
    params = params or TableParams()
    phi64 = torch.empty((params.n_D, params.n_sigma), dtype=torch.float64, device=device)
    phi32 = torch.empty((params.n_D, params.n_sigma), dtype=torch.float32, device=device) if fp32 else None
    tp = params.c()
    L.check(L.lib().build_phi_table(ct.byref(tp), _ptr(phi64), _ptr(phi32), _stream(stream)))
    return Table(params, phi64, phi32)


def compute_q0(grid: Grid, n: torch.Tensor, n_cut: float, derivatives: bool = True, stream=None) -> dict:
    """Gradient (3 planes), q0, dq0/dn and dq0/d|grad n|^2 on every grid point."""
    _f64(n, "n")
    G = grid.G
    if n.numel() != G:
        raise ValueError("n does not match the grid")
    dev = n.device
    q0 = torch.empty(G, dtype=torch.float64, device=dev)
    grad = torch.empty(3 * G, dtype=torch.float64, device=dev) if derivatives else None
    dqdn = torch.empty(G, dtype=torch.float64, device=dev) if derivatives else None
    dqdg = torch.empty(G, dtype=torch.float64, device=dev) if derivatives else None
    g = grid.c()
    L.check(L.lib().compute_q0(ct.byref(g), float(n_cut), _ptr(n), _ptr(grad), _ptr(q0), _ptr(dqdn), _ptr(dqdg),
                               _stream(stream)))
    return dict(q0=q0, grad=grad, dq_dn=dqdn, dq_dg=dqdg)


_WS = {}


def _workspace(nbytes: int, device) -> torch.Tensor:
    key = (str(device),)
    ws = _WS.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _WS[key] = ws
    return ws


def enl_workspace_size(grid: Grid, table: Table | TableParams, opts: Opts) -> int:
    tp = (table.params if isinstance(table, Table) else table).c()
    g, o = grid.c(), opts.c()
    return int(L.lib().enl_workspace_size(ct.byref(g), ct.byref(tp), ct.byref(o)))


def enl_energy(grid: Grid, n: torch.Tensor, q0: torch.Tensor, table: Table, opts: Opts, stream=None):
    """(E_pair0, E_pairL, E_self) in Hartree."""
    _f64(n, "n")
    _f64(q0, "q0")
    tp, g, o = table.params.c(), grid.c(), opts.c()
    nbytes = int(L.lib().enl_workspace_size(ct.byref(g), ct.byref(tp), ct.byref(o)))
    if nbytes == 0:
        raise L.VdwError(L.VDW_EINVAL, "invalid arguments for enl_workspace_size")
    ws = _workspace(nbytes, n.device)
    E = (ct.c_double * 3)()
    L.check(L.lib().enl_energy(ct.byref(g), _ptr(n), _ptr(q0), _ptr(table.phi64), _ptr(table.phi32),
                               ct.byref(tp), ct.byref(o), _ptr(ws), ws.numel(), E, _stream(stream)))
    return float(E[0]), float(E[1]), float(E[2])


def enl_potential(grid: Grid, n: torch.Tensor, qd: dict, table: Table, opts: Opts, stream=None):
    """Energies and dE/dn on every grid point (the potential is dE/dn / dV)."""
    _f64(n, "n")
    tp, g, o = table.params.c(), grid.c(), opts.c()
    nbytes = int(L.lib().enl_workspace_size(ct.byref(g), ct.byref(tp), ct.byref(o)))
    if nbytes == 0:
        raise L.VdwError(L.VDW_EINVAL, "invalid arguments for enl_workspace_size")
    ws = _workspace(nbytes, n.device)
    dEdn = torch.empty(grid.G, dtype=torch.float64, device=n.device)
    E = (ct.c_double * 3)()
    L.check(L.lib().enl_potential(ct.byref(g), _ptr(n), _ptr(qd["q0"]), _ptr(qd["grad"]), _ptr(qd["dq_dn"]),
                                  _ptr(qd["dq_dg"]), _ptr(table.phi64), _ptr(table.phi32), ct.byref(tp),
                                  ct.byref(o), _ptr(ws), ws.numel(), _ptr(dEdn), E, _stream(stream)))
    return (float(E[0]), float(E[1]), float(E[2])), dEdn


def pack_batch(grids, ns):
    """Concatenate densities into one packed array with the offsets the batched call takes."""
    offs = [0]
    for g in grids:
        offs.append(offs[-1] + g.G)
    n = torch.cat([x.reshape(-1) for x in ns])
    return n, offs


def compute_q0_batched(grids, n_packed: torch.Tensor, offs, n_cut: float, stream=None) -> dict:
    """compute_q0 on every density of a packed batch (one launch per density)."""
    Gt = offs[-1]
    dev = n_packed.device
    out = dict(q0=torch.empty(Gt, dtype=torch.float64, device=dev),
               grad=torch.empty(3 * Gt, dtype=torch.float64, device=dev),
               dq_dn=torch.empty(Gt, dtype=torch.float64, device=dev),
               dq_dg=torch.empty(Gt, dtype=torch.float64, device=dev))
    for b, gr in enumerate(grids):
        a, e = offs[b], offs[b + 1]
        g = gr.c()
        L.check(L.lib().compute_q0(ct.byref(g), float(n_cut), _ptr(n_packed[a:e]), _ptr(out["grad"][3 * a:3 * e]),
                                   _ptr(out["q0"][a:e]), _ptr(out["dq_dn"][a:e]), _ptr(out["dq_dg"][a:e]),
                                   _stream(stream)))
    return out


def enl_potential_batched(grids, n_packed: torch.Tensor, offs, qd: dict, table: Table, opts: Opts, stream=None):
    """enl_potential for a packed batch in one pass; returns ([(E0, EL, Es)] per density, dEdn packed)."""
    B = len(grids)
    garr = (L.VdwGrid * B)(*[g.c() for g in grids])
    off = (ct.c_int64 * (B + 1))(*offs)
    tp, o = table.params.c(), opts.c()
    nbytes = int(L.lib().enl_batched_workspace_size(B, garr, ct.byref(tp), ct.byref(o)))
    if nbytes == 0:
        raise L.VdwError(L.VDW_EINVAL, "invalid arguments for enl_batched_workspace_size")
    ws = _workspace(nbytes, n_packed.device)
    dEdn = torch.empty(offs[-1], dtype=torch.float64, device=n_packed.device)
    E = (ct.c_double * (3 * B))()
    L.check(L.lib().enl_potential_batched(B, garr, off, _ptr(n_packed), _ptr(qd["q0"]), _ptr(qd["grad"]),
                                          _ptr(qd["dq_dn"]), _ptr(qd["dq_dg"]), _ptr(table.phi64),
                                          _ptr(table.phi32), ct.byref(tp), ct.byref(o), _ptr(ws), ws.numel(),
                                          _ptr(dEdn), E, _stream(stream)))
    return [(float(E[3 * b]), float(E[3 * b + 1]), float(E[3 * b + 2])) for b in range(B)], dEdn


def last_stats() -> dict:
    s = L.VdwStats()
    L.check(L.lib().vdw_last_stats(ct.byref(s)))
    return dict(retained=s.retained, pairs=s.pairs, pair_kernel_ms=s.pair_kernel_ms, lds_rows=s.lds_rows,
                block_threads=s.block_threads, j_chunks=s.j_chunks, grid_blocks=s.grid_blocks)


def set_timing(on: bool):
    L.lib().vdw_set_timing(1 if on else 0)


class EnlFunction(torch.autograd.Function):
    """E_c^nl(n) with backward dE/dn from enl_potential (through q0 and the
    finite-difference gradient)."""

    @staticmethod
    def forward(ctx, n, grid: Grid, table: Table, opts: Opts):
        flat = n.detach().reshape(-1).contiguous()
        qd = compute_q0(grid, flat, opts.n_cut, derivatives=True)
        E, dEdn = enl_potential(grid, flat, qd, table, opts)
        ctx.save_for_backward(dEdn)
        ctx.shape = n.shape
        return n.new_tensor(E[0] + E[1] + E[2])

    @staticmethod
    def backward(ctx, gout):
        (dEdn,) = ctx.saved_tensors
        return (gout * dEdn).reshape(ctx.shape), None, None, None


def energy(n: torch.Tensor, grid: Grid, table: Table, opts: Opts) -> torch.Tensor:
    """Differentiable E_c^nl of a density on the GPU."""
    return EnlFunction.apply(n, grid, table, opts)
