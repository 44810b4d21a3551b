"""Python binding of libvdwdf.so with the C ABI's names.

PyTorch supplies device memory and streams; each function marshals
arguments and calls the library, which runs every step on the GPU.  There
is no CPU fallback: without the built library, or without a GPU, these
functions raise.
"""
from __future__ import annotations

import ctypes as ct
import threading
from dataclasses import dataclass, field

import torch

from . import _lib as L

DEFAULT_RULE = dict(gl_points=8, graded_levels=12, kappa=16.0, A0=512.0)


@dataclass
class TableParams:
    """Kernel table over D in [0, D_max] x sigma = delta^2 in [0, 1] and the quadrature rule."""

    n_D: int = 2048
    n_sigma: int = 64
    D_max: float = 48.0
    gl_points: int = 8
    graded_levels: int = 12
    kappa: float = 16.0
    A0: float = 512.0
    interp: int = 0  # 0 bilinear, 1 cubic (C1) in D and linear in sigma

    def c(self) -> L.VdwTableParams:
        return L.VdwTableParams(self.n_D, self.n_sigma, self.D_max, self.gl_points, self.graded_levels,
                                self.kappa, self.A0, self.interp)


@dataclass
class Grid:
    """Equidistant grid, n points per axis, x fastest.  Orthorhombic with
    spacing h (bohr), or, with `cell` (rows: lattice vectors a, b, c in bohr),
    any (skew) cell divided into n[0] x n[1] x n[2] steps (h is then unused).
    gradient="spectral" takes the Fourier derivative on periodic axes."""

    n: tuple
    h: tuple = (0.0, 0.0, 0.0)
    periodic: tuple = (0, 0, 0)
    cell: tuple | None = None
    gradient: str = "fd"  # "fd" or "spectral" (Fourier derivative on periodic axes)

    @property
    def G(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def dV(self) -> float:
        if self.cell is not None:
            import numpy as np

            return abs(float(np.linalg.det(np.asarray(self.cell, dtype=np.float64)))) / self.G
        return float(self.h[0]) * float(self.h[1]) * float(self.h[2])

    def c(self) -> L.VdwGrid:
        g = L.VdwGrid()
        if self.gradient not in ("fd", "spectral"):
            raise ValueError("gradient must be 'fd' or 'spectral'")
        g.gradient = 1 if self.gradient == "spectral" else 0
        for a in range(3):
            g.n[a] = int(self.n[a])
            g.periodic[a] = int(self.periodic[a])
            for b in range(3):
                if self.cell is not None:
                    g.cell[a][b] = float(self.cell[a][b])
                else:
                    g.cell[a][b] = float(self.n[a] * self.h[a]) if a == b else 0.0
        return g


@dataclass
class Opts:
    """vdw_opts: density cut-off, distance cut and near images (image_max,
    summed with the table), precision (FP32C or FP64), on-site term, tile
    shape, Kahan runs, and the far image shell (far_max: the cells beyond
    image_max up to far_max with the kernel's large-D asymptote, no r_cut)."""

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
    far_max: tuple = (0, 0, 0)

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
        for a in range(3):
            o.far_max[a] = int(self.far_max[a])
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
    # the spectral gradient stages its Fourier derivatives in the gradient planes
    grad = torch.empty(3 * G, dtype=torch.float64, device=dev) if derivatives or grid.gradient == "spectral" else None
    dqdn = torch.empty(G, dtype=torch.float64, device=dev) if derivatives else None
    dqdg = torch.empty(G, dtype=torch.float64, device=dev) if derivatives else None
    g = grid.c()
    L.check(L.lib().compute_q0(ct.byref(g), float(n_cut), _ptr(n), _ptr(grad), _ptr(q0), _ptr(dqdn), _ptr(dqdg),
                               _stream(stream)))
    return dict(q0=q0, grad=grad, dq_dn=dqdn, dq_dg=dqdg)


_WS = {}
_WS_LOCK = threading.Lock()


def _workspace(nbytes: int, device, stream=None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """The device workspace of one call: the caller's `ws` if given (checked
    for size), else a cached buffer per (device, stream).  Calls on different
    streams then never share scratch (the C ABI requires that); calls on one
    stream are ordered by it, and a buffer replaced by a larger one is freed
    through torch's stream-ordered allocator."""
    if ws is not None:
        if ws.dtype != torch.uint8 or not ws.is_contiguous() or ws.device != torch.device(device):
            raise TypeError("ws must be a contiguous uint8 tensor on the density's device")
        if ws.numel() < nbytes:
            raise L.VdwError(L.VDW_EWORKSPACE, f"workspace has {ws.numel()} bytes, needs {nbytes}")
        return ws
    s = stream if stream is not None else torch.cuda.current_stream(device)
    key = (str(torch.device(device)), int(s.cuda_stream))
    with _WS_LOCK:
        buf = _WS.get(key)
        if buf is None or buf.numel() < nbytes:
            with torch.cuda.stream(s):
                buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
            _WS[key] = buf
    return buf


def release_workspaces():
    """Drop the cached per-(device, stream) workspaces (they keep the largest
    size any call needed, e.g. during a tile-shape sweep) and return the
    memory to the device.  Calls still running on other streams keep theirs
    until they finish (torch's stream-ordered allocator)."""
    with _WS_LOCK:
        _WS.clear()
    torch.cuda.empty_cache()


def enl_workspace_size(grid: Grid, table: Table | TableParams, opts: Opts) -> int:
    tp = (table.params if isinstance(table, Table) else table).c()
    g, o = grid.c(), opts.c()
    return int(L.lib().enl_workspace_size(ct.byref(g), ct.byref(tp), ct.byref(o)))


def enl_energy(grid: Grid, n: torch.Tensor, q0: torch.Tensor, table: Table, opts: Opts, stream=None, ws=None):
    """(E_pair0, E_pairL, E_self) in Hartree.  `ws`: an optional caller-owned
    uint8 workspace of at least enl_workspace_size bytes."""
    _f64(n, "n")
    _f64(q0, "q0")
    tp, g, o = table.params.c(), grid.c(), opts.c()
    nbytes = int(L.lib().enl_workspace_size(ct.byref(g), ct.byref(tp), ct.byref(o)))
    if nbytes == 0:
        raise L.VdwError(L.VDW_EINVAL, "invalid arguments for enl_workspace_size")
    ws = _workspace(nbytes, n.device, stream, ws)
    E = (ct.c_double * 3)()
    L.check(L.lib().enl_energy(ct.byref(g), _ptr(n), _ptr(q0), _ptr(table.phi64), _ptr(table.phi32),
                               ct.byref(tp), ct.byref(o), _ptr(ws), ws.numel(), E, _stream(stream)))
    return float(E[0]), float(E[1]), float(E[2])


def enl_potential(grid: Grid, n: torch.Tensor, qd: dict, table: Table, opts: Opts, stream=None, ws=None):
    """Energies and dE/dn on every grid point (the potential is dE/dn / dV).
    `ws`: an optional caller-owned uint8 workspace (enl_workspace_size bytes)."""
    _f64(n, "n")
    tp, g, o = table.params.c(), grid.c(), opts.c()
    nbytes = int(L.lib().enl_workspace_size(ct.byref(g), ct.byref(tp), ct.byref(o)))
    if nbytes == 0:
        raise L.VdwError(L.VDW_EINVAL, "invalid arguments for enl_workspace_size")
    ws = _workspace(nbytes, n.device, stream, ws)
    dEdn = torch.empty(grid.G, dtype=torch.float64, device=n.device)
    E = (ct.c_double * 3)()
    L.check(L.lib().enl_potential(ct.byref(g), _ptr(n), _ptr(qd["q0"]), _ptr(qd["grad"]), _ptr(qd["dq_dn"]),
                                  _ptr(qd["dq_dg"]), _ptr(table.phi64), _ptr(table.phi32), ct.byref(tp),
                                  ct.byref(o), _ptr(ws), ws.numel(), _ptr(dEdn), E, _stream(stream)))
    return (float(E[0]), float(E[1]), float(E[2])), dEdn


def enl_potential_noalloc(grid: Grid, n: torch.Tensor, qd: dict, table: Table, opts: Opts, stream=None):
    """enl_potential on the library's static device scratch (no workspace is
    allocated; grids up to the scratch size, calls on one GPU serialised by
    the caller).  The dE/dn output is allocated here by torch; a caller that
    cannot allocate passes its own buffer through the C ABI."""
    _f64(n, "n")
    tp, g, o = table.params.c(), grid.c(), opts.c()
    dEdn = torch.empty(grid.G, dtype=torch.float64, device=n.device)
    E = (ct.c_double * 3)()
    L.check(L.lib().enl_potential_noalloc(ct.byref(g), _ptr(n), _ptr(qd["q0"]), _ptr(qd["grad"]),
                                          _ptr(qd["dq_dn"]), _ptr(qd["dq_dg"]), _ptr(table.phi64),
                                          _ptr(table.phi32), ct.byref(tp), ct.byref(o), _ptr(dEdn), E,
                                          _stream(stream)))
    return (float(E[0]), float(E[1]), float(E[2])), dEdn


XC_TERMS = ("Ex_lda", "Ec_lda", "Ex_pbe", "Ec_pbe", "Ex_revpbe")


def xc_workspace_size(grid: Grid) -> int:
    g = grid.c()
    return int(L.lib().xc_workspace_size(ct.byref(g)))


def xc_energies(grid: Grid, n: torch.Tensor, n_floor: float = 1e-12, stream=None) -> dict:
    """E_x^LDA, E_c^LDA, E_x^PBE, E_c^PBE and E_x^revPBE (Hartree) of the
    density, over the grid points with n > n_floor."""
    _f64(n, "n")
    g = grid.c()
    nbytes = int(L.lib().xc_workspace_size(ct.byref(g)))
    if nbytes == 0:
        raise L.VdwError(L.VDW_EINVAL, "invalid grid for xc_workspace_size")
    ws = _workspace(nbytes, n.device, stream)
    E = (ct.c_double * 5)()
    L.check(L.lib().xc_energies(ct.byref(g), _ptr(n), float(n_floor), _ptr(ws), ws.numel(), E, _stream(stream)))
    return dict(zip(XC_TERMS, (float(x) for x in E)))


def recombine(xc: dict, E_nl: float, E_dft: float = 0.0, exchange: str = "pbe") -> float:
    """Eq. (3): E_dft - E_x^PBE - E_c^PBE + (E_x + E_c^LDA + E_nl), E_x the
    PBE or revPBE exchange of `xc` (from xc_energies)."""
    if exchange not in ("pbe", "revpbe"):
        raise ValueError("exchange must be 'pbe' or 'revpbe'")
    E = (ct.c_double * 5)(*(xc[k] for k in XC_TERMS))
    return float(L.lib().vdw_recombine(E, float(E_nl), float(E_dft), 1 if exchange == "revpbe" else 0))


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


def enl_potential_batched(grids, n_packed: torch.Tensor, offs, qd: dict, table: Table, opts: Opts, stream=None,
                          ws=None):
    """enl_potential for a packed batch in one pass; returns ([(E0, EL, Es)] per density, dEdn packed)."""
    B = len(grids)
    garr = (L.VdwGrid * B)(*[g.c() for g in grids])
    off = (ct.c_int64 * (B + 1))(*offs)
    tp, o = table.params.c(), opts.c()
    nbytes = int(L.lib().enl_batched_workspace_size(B, garr, ct.byref(tp), ct.byref(o)))
    if nbytes == 0:
        raise L.VdwError(L.VDW_EINVAL, "invalid arguments for enl_batched_workspace_size")
    ws = _workspace(nbytes, n_packed.device, stream, ws)
    dEdn = torch.empty(offs[-1], dtype=torch.float64, device=n_packed.device)
    E = (ct.c_double * (3 * B))()
    L.check(L.lib().enl_potential_batched(B, garr, off, _ptr(n_packed), _ptr(qd["q0"]), _ptr(qd["grad"]),
                                          _ptr(qd["dq_dn"]), _ptr(qd["dq_dg"]), _ptr(table.phi64),
                                          _ptr(table.phi32), ct.byref(tp), ct.byref(o), _ptr(ws), ws.numel(),
                                          _ptr(dEdn), E, _stream(stream)))
    return [(float(E[3 * b]), float(E[3 * b + 1]), float(E[3 * b + 2])) for b in range(B)], dEdn


class BatchPlan:
    """A batch plan (enl_batch_plan_*): the descriptors of B densities are
    uploaded once; each ``execute`` then enqueues a whole evaluation (q0 of
    every density, compaction, the persistent pair kernel, reductions, the
    adjoint) as kernel launches only, which ``capture`` records into a HIP
    graph that ``replay`` relaunches.  The plan owns its workspace and the
    per-point buffers (grad, q0, dq_dn, dq_dg, dEdn) and ``E`` (4B+1 doubles:
    3 energies per density, B retained counts, the non-finite flag)."""

    def __init__(self, grids, offs, table: Table, opts: Opts, potential: bool = True, device="cuda", stream=None):
        self._h = None
        B = len(grids)
        self.B, self.offs, self.table, self.potential = B, list(offs), table, bool(potential)
        garr = (L.VdwGrid * B)(*[g.c() for g in grids])
        off = (ct.c_int64 * (B + 1))(*offs)
        tp, o = table.params.c(), opts.c()
        nbytes = int(L.lib().enl_batched_workspace_size(B, garr, ct.byref(tp), ct.byref(o)))
        if nbytes == 0:
            raise L.VdwError(L.VDW_EINVAL, "invalid arguments for enl_batched_workspace_size")
        Gt = offs[-1]
        f64 = dict(dtype=torch.float64, device=device)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.q0 = torch.empty(Gt, **f64)
        # the spectral gradient is staged in grad, so such plans keep it also for the energy only
        spectral = any(g.gradient == "spectral" for g in grids)
        self.grad = torch.empty(3 * Gt, **f64) if (potential or spectral) else None
        self.dq_dn = torch.empty(Gt, **f64) if potential else None
        self.dq_dg = torch.empty(Gt, **f64) if potential else None
        self.dEdn = torch.empty(Gt, **f64) if potential else None
        self.E = torch.empty(4 * B + 1, **f64)
        h = ct.c_void_p()
        L.check(L.lib().enl_batch_plan_create(B, garr, off, ct.byref(tp), ct.byref(o), 1 if potential else 0,
                                              _ptr(self.ws), self.ws.numel(), ct.byref(h), _stream(stream)))
        self._h = h
        self._bound = None

    def _args(self, n):
        _f64(n, "n")
        if n.numel() != self.offs[-1]:
            raise ValueError("n does not match the plan's grids")
        return (_ptr(n), _ptr(self.grad), _ptr(self.q0), _ptr(self.dq_dn), _ptr(self.dq_dg), _ptr(self.table.phi64),
                _ptr(self.table.phi32), _ptr(self.dEdn), _ptr(self.E))

    def execute(self, n: torch.Tensor, stream=None):
        L.check(L.lib().enl_batch_plan_execute(self._h, *self._args(n), _stream(stream)))

    def capture(self, n: torch.Tensor):
        """Record one evaluation on ``n`` (its buffer is read at every replay)."""
        L.check(L.lib().enl_batch_plan_capture(self._h, *self._args(n)))
        self._bound = n

    def replay(self, stream=None):
        L.check(L.lib().enl_batch_plan_replay(self._h, _stream(stream)))

    def energies(self):
        """[(E_pair0, E_pairL, E_self)] per density after the last evaluation
        (waits for it); raises for a density that held NaN or Inf."""
        e = self.E.cpu().tolist()
        if e[4 * self.B] != 0.0:
            raise L.VdwError(L.VDW_ENONFINITE, "the density holds NaN or Inf values")
        return [(e[3 * b], e[3 * b + 1], e[3 * b + 2]) for b in range(self.B)]

    def retained(self):
        return [int(x) for x in self.E[3 * self.B:4 * self.B].cpu().tolist()]

    def close(self):
        if self._h is not None and self._h.value:
            L.check(L.lib().enl_batch_plan_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def last_stats() -> dict:
    s = L.VdwStats()
    L.check(L.lib().vdw_last_stats(ct.byref(s)))
    return dict(retained=s.retained, pairs=s.pairs, pair_kernel_ms=s.pair_kernel_ms, lds_rows=s.lds_rows,
                block_threads=s.block_threads, j_chunks=s.j_chunks, grid_blocks=s.grid_blocks,
                diag_items=s.diag_items, far_pairs=s.far_pairs, far_kernel_ms=s.far_kernel_ms,
                image_reach=s.image_reach, image_cut_covered=s.image_cut_covered, q0_min=s.q0_min,
                far_D_min=s.far_D_min)


def image_window(grid: Grid, opts: Opts):
    """(reach in bohr, covers) of the near image window (vdw_image_window):
    every pair closer than reach is summed; covers is 1 when reach > r_cut,
    0 when the window leaves out pairs inside the cut (or there is no cut),
    -1 without periodic axes.  Host only."""
    g, o = grid.c(), opts.c()
    reach = ct.c_double()
    covers = ct.c_int32()
    L.check(L.lib().vdw_image_window(ct.byref(g), ct.byref(o), ct.byref(reach), ct.byref(covers)))
    return float(reach.value), int(covers.value)


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
