"""TEST ORACLE for the vdW-DF nonlocal-correlation path (test infrastructure).

Plain FP64 CPU reference of everything the GPU library computes.  It is
written from the mathematics of Lazic et al. (arXiv:0810.2273), Sec. 2
(Eqs. 1-2, the kernel of Dion et al. and its large-D asymptote), Sec. 3
(gradient, density cut-off, 0th cell plus periodic repetition), Sec. 7
(the large-D form of the kernel for the far repeated cells), and from the
published ingredients that paper builds on: the Dion et al. q0 (LDA
exchange-correlation plus gradient term), the Perdew-Wang 1992 LDA
correlation, and the PBE and revPBE exchange and PBE correlation energies
that enter the recombination of Eq. (3).  The heavy loops (quadrature of
the kernel, the double sum) live in vdw_oracle.c; the O(grid) steps are
numpy/scipy here.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may use
this module.  It shares no code with the HIP library and does not import
it.  Every function is pinned by tests/test_oracle_*.py.

Units: Hartree atomic units (bohr, Hartree, electrons / bohr^3).
"""
from __future__ import annotations

import ctypes as ct
import math
import os
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None


class TableParams(ct.Structure):
    """Table layout and quadrature rule (mirrors vo_table_params)."""

    _fields_ = [
        ("n_D", ct.c_int32),
        ("n_sigma", ct.c_int32),
        ("D_max", ct.c_double),
        ("gl_points", ct.c_int32),
        ("graded_levels", ct.c_int32),
        ("kappa", ct.c_double),
        ("A0", ct.c_double),
        ("interp", ct.c_int32),
    ]


def table_params(n_D=1024, n_sigma=32, D_max=48.0, gl_points=8, graded_levels=12, kappa=16.0, A0=512.0, interp=0):
    """interp: 0 bilinear, 1 cubic (C1) in D and linear in sigma."""
    return TableParams(n_D, n_sigma, D_max, gl_points, graded_levels, kappa, A0, interp)


def lib():
    """Load liboracle.so, building it with gcc if it is not there yet."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b

        _b.build()
    L = ct.CDLL(_LIB_PATH)
    d, i32, i64, P = ct.c_double, ct.c_int32, ct.c_int64, ct.POINTER
    dp = P(d)
    L.vo_asym_C.restype = d
    L.vo_gauss_legendre.argtypes = [ct.c_int, dp, dp]
    L.vo_U.restype = d
    L.vo_U.argtypes = [d]
    for f in (L.vo_W2, L.vo_W_literal, L.vo_nu):
        f.restype = d
        f.argtypes = [d, d]
    L.vo_T.restype = d
    L.vo_T.argtypes = [d, d, d, d]
    L.vo_rule_nodes.restype = ct.c_int
    L.vo_rule_nodes.argtypes = [d, d, P(TableParams), dp, dp, ct.c_int]
    L.vo_dion_phi.restype = d
    L.vo_dion_phi.argtypes = [d, d, P(TableParams)]
    L.vo_phi_Dsigma.restype = d
    L.vo_phi_Dsigma.argtypes = [d, d, P(TableParams)]
    L.vo_build_table.restype = ct.c_int
    L.vo_build_table.argtypes = [P(TableParams), dp]
    L.vo_table_nodes.restype = ct.c_int
    L.vo_phi_many.restype = ct.c_int
    L.vo_phi_many.argtypes = [ct.c_long, dp, dp, P(TableParams), dp]
    L.vo_table_nodes.argtypes = [P(TableParams), ct.c_long, P(i32), P(i32), dp]
    L.vo_table_interp.restype = d
    L.vo_table_interp.argtypes = [dp, P(TableParams), d, d, dp, dp]
    L.vo_pair_phi.restype = d
    L.vo_pair_phi.argtypes = [d, d, d, dp, P(TableParams), dp]
    L.vo_self_phi.restype = d
    L.vo_self_phi.argtypes = [d, d, dp, P(TableParams), dp]
    L.vo_self_voxel.restype = d
    L.vo_self_voxel.argtypes = [d, dp, ct.c_int, dp, P(TableParams), dp]
    L.vo_self_voxel_many.restype = ct.c_int
    L.vo_self_voxel_many.argtypes = [ct.c_long, dp, dp, ct.c_int, dp, P(TableParams), dp, dp]
    L.vo_pair_rows.restype = ct.c_int
    L.vo_pair_rows.argtypes = [
        ct.c_long, P(i32), P(i32), P(i32), dp, dp,
        dp, P(i32), P(i32), P(i32), d,
        dp, P(TableParams), ct.c_long, P(i64), dp, dp, dp,
    ]
    L.vo_image_pair_sum.restype = d
    L.vo_image_pair_sum.argtypes = [
        ct.c_long, P(i32), P(i32), P(i32), dp, dp,
        dp, P(i32), P(i32), d, dp, P(TableParams),
    ]
    L.vo_block_sum.restype = d
    L.vo_block_sum.argtypes = [
        ct.c_long, P(i32), ct.c_long, P(i32),
        P(i32), P(i32), P(i32), dp, dp,
        dp, P(i32), P(i32), P(i32), d, dp, P(TableParams),
    ]
    L.vo_pair_rows_cell.restype = ct.c_int
    L.vo_pair_rows_cell.argtypes = L.vo_pair_rows.argtypes
    L.vo_block_sum_cell.restype = d
    L.vo_block_sum_cell.argtypes = L.vo_block_sum.argtypes
    L.vo_far_T.restype = d
    L.vo_far_T.argtypes = [dp, P(i32), P(i32), P(i32), P(i32), d, d, d]
    L.vo_far_rows.restype = ct.c_int
    L.vo_far_rows.argtypes = [
        ct.c_long, P(i32), P(i32), P(i32), dp, dp,
        dp, P(i32), P(i32), P(i32), P(i32), ct.c_long, P(i64), dp, dp,
    ]
    L.vo_num_threads.restype = ct.c_int
    _lib = L
    return L


def _p(a, ctype):
    return a.ctypes.data_as(ct.POINTER(ctype))


def num_threads() -> int:
    return int(lib().vo_num_threads())


# --------------------------------------------------------------------------
# Kernel phi and its table (Sec. 2: phi by the double integral of Dion et al.;
# Sec. 7: table limits and node counts fixed by refinement checks).
# --------------------------------------------------------------------------

def asym_C() -> float:
    return float(lib().vo_asym_C())


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().vo_gauss_legendre(n, _p(x, ct.c_double), _p(w, ct.c_double))
    return x, w


def U(x):
    return float(lib().vo_U(float(x)))


def W2(a, b):
    """a^2 b^2 W(a, b) in the cancellation-free grouping."""
    return float(lib().vo_W2(float(a), float(b)))


def W_literal(a, b):
    return float(lib().vo_W_literal(float(a), float(b)))


def T(w, x, y, z):
    return float(lib().vo_T(w, x, y, z))


def nu(y, d):
    return float(lib().vo_nu(float(y), float(d)))


def rule_nodes(d1, d2, tp):
    n = lib().vo_rule_nodes(d1, d2, ct.byref(tp), None, None, 0)
    a = np.zeros(n)
    w = np.zeros(n)
    lib().vo_rule_nodes(d1, d2, ct.byref(tp), _p(a, ct.c_double), _p(w, ct.c_double), n)
    return a, w


def dion_phi(d1, d2, tp) -> float:
    return float(lib().vo_dion_phi(float(d1), float(d2), ct.byref(tp)))


def phi_Dsigma(D, sigma, tp) -> float:
    return float(lib().vo_phi_Dsigma(float(D), float(sigma), ct.byref(tp)))


def phi_many(D, sigma, tp) -> np.ndarray:
    """phi(D_t, sigma_t) for arrays of points (threads over the points)."""
    D = np.ascontiguousarray(D, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    out = np.zeros(D.shape)
    lib().vo_phi_many(D.size, _p(D, ct.c_double), _p(sigma, ct.c_double), ct.byref(tp), _p(out, ct.c_double))
    return out


def build_table(tp) -> np.ndarray:
    """phi(D_k, sigma_l), shape (n_D, n_sigma); row 0 linearly extrapolated."""
    out = np.zeros((tp.n_D, tp.n_sigma))
    rc = lib().vo_build_table(ct.byref(tp), _p(out, ct.c_double))
    if rc != 0:
        raise ValueError("bad table parameters")
    return out


def table_nodes(tp, k, l) -> np.ndarray:
    k = np.ascontiguousarray(k, dtype=np.int32)
    l = np.ascontiguousarray(l, dtype=np.int32)
    out = np.zeros(len(k))
    lib().vo_table_nodes(ct.byref(tp), len(k), _p(k, ct.c_int32), _p(l, ct.c_int32), _p(out, ct.c_double))
    return out


def table_interp(tab, tp, D, sigma):
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    dD = ct.c_double()
    dS = ct.c_double()
    v = lib().vo_table_interp(_p(tab, ct.c_double), ct.byref(tp), float(D), float(sigma), ct.byref(dD), ct.byref(dS))
    return float(v), dD.value, dS.value


def pair_phi(qi, qj, r, tab, tp):
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    dq = ct.c_double()
    v = lib().vo_pair_phi(float(qi), float(qj), float(r), _p(tab, ct.c_double), ct.byref(tp), ct.byref(dq))
    return float(v), dq.value


def self_phi(q, rho_s, tab, tp):
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    dq = ct.c_double()
    v = lib().vo_self_phi(float(q), float(rho_s), _p(tab, ct.c_double), ct.byref(tp), ct.byref(dq))
    return float(v), dq.value


VOXEL_GL_POINTS = 8  # Gauss-Legendre points per octant axis of the voxel rule


def self_voxel(q, steps, tab, tp, g=VOXEL_GL_POINTS):
    """The voxel double average Phi_V(q) of phi~(., 0) over the grid cell
    spanned by the step vectors (rows of `steps`) and d Phi_V / d q."""
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    E = np.ascontiguousarray(np.asarray(steps, dtype=np.float64).reshape(9))
    dq = ct.c_double()
    v = lib().vo_self_voxel(float(q), _p(E, ct.c_double), int(g), _p(tab, ct.c_double), ct.byref(tp), ct.byref(dq))
    return float(v), dq.value


def self_voxel_many(q, steps, tab, tp, g=VOXEL_GL_POINTS):
    """self_voxel at every value of the array q: (Phi_V, dPhi_V/dq)."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    E = np.ascontiguousarray(np.asarray(steps, dtype=np.float64).reshape(9))
    phi = np.zeros(len(q))
    dphi = np.zeros(len(q))
    lib().vo_self_voxel_many(len(q), _p(q, ct.c_double), _p(E, ct.c_double), int(g), _p(tab, ct.c_double),
                             ct.byref(tp), _p(phi, ct.c_double), _p(dphi, ct.c_double))
    return phi, dphi


# Phi_V(q) tabulated over ln q (the on-site term self_term = 2): nodes
# ln q_k = VOXEL_LNQ_LO + k * dlnq, k = 0 .. VOXEL_TABLE_NODES - 1, spanning
# q in [2^-6, 2^7], each node by the voxel rule; between nodes the Catmull-Rom
# cubic in ln q (rows beyond the ends extrapolated linearly); q outside the
# range takes the rule directly.
VOXEL_TABLE_NODES = 4096
VOXEL_LNQ_LO = -6.0 * math.log(2.0)
VOXEL_LNQ_HI = 7.0 * math.log(2.0)


_VOXEL_TABLES = {}


def voxel_table(steps, tab, tp):
    """Phi_V at the ln q nodes, for the grid cell spanned by `steps` (kept
    for the last few (cell, table) pairs)."""
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    key = (tuple(np.asarray(steps, dtype=np.float64).ravel()), tab.shape, hash(tab.tobytes()),
           tuple(getattr(tp, f) for f, _ in tp._fields_))
    if key not in _VOXEL_TABLES:
        if len(_VOXEL_TABLES) >= 4:
            _VOXEL_TABLES.pop(next(iter(_VOXEL_TABLES)))
        x = VOXEL_LNQ_LO + np.arange(VOXEL_TABLE_NODES) * ((VOXEL_LNQ_HI - VOXEL_LNQ_LO) / (VOXEL_TABLE_NODES - 1))
        _VOXEL_TABLES[key] = self_voxel_many(np.exp(x), steps, tab, tp)[0]
    return _VOXEL_TABLES[key]


def voxel_interp(vt, q, steps, tab, tp):
    """(Phi_V, dPhi_V/dq) at the array q from the node values vt: the
    Catmull-Rom cubic in ln q, its derivative divided by q; outside the
    node range the voxel rule itself."""
    q = np.atleast_1d(np.asarray(q, dtype=np.float64))
    n = len(vt)
    dx = (VOXEL_LNQ_HI - VOXEL_LNQ_LO) / (n - 1)
    f = np.concatenate([[2 * vt[0] - vt[1]], vt, [2 * vt[-1] - vt[-2]]])  # f[k + 1] = node k
    phi = np.zeros(len(q))
    dphi = np.zeros(len(q))
    inside = (q >= math.exp(VOXEL_LNQ_LO)) & (q <= math.exp(VOXEL_LNQ_HI))
    xs = (np.log(q[inside]) - VOXEL_LNQ_LO) / dx
    k = np.clip(np.floor(xs).astype(np.int64), 0, n - 2)
    t = xs - k
    f0, f1, f2, f3 = f[k], f[k + 1], f[k + 2], f[k + 3]
    m1, m2 = 0.5 * (f2 - f0), 0.5 * (f3 - f1)
    t2, t3 = t * t, t * t * t
    phi[inside] = (2 * t3 - 3 * t2 + 1) * f1 + (t3 - 2 * t2 + t) * m1 + (-2 * t3 + 3 * t2) * f2 + (t3 - t2) * m2
    dt = (6 * t2 - 6 * t) * (f1 - f2) + (3 * t2 - 4 * t + 1) * m1 + (3 * t2 - 2 * t) * m2
    dphi[inside] = dt / (dx * q[inside])
    if (~inside).any():
        phi[~inside], dphi[~inside] = self_voxel_many(q[~inside], steps, tab, tp)
    return phi, dphi


def onsite_phi(grid, q, tab, tp, self_term):
    """The on-site value and its q-derivative: self_term 1 (or True) takes
    phi~(q rho_s, 0) with the sphere radius of self_radius, 2 the voxel
    double average through its table over ln q, 0 (or False) nothing."""
    if self_term is True or self_term == 1:
        return self_phi(q, self_radius(grid.dV), tab, tp)
    if self_term == 2:
        vt = voxel_table(grid.steps, tab, tp)
        p, d = voxel_interp(vt, [q], grid.steps, tab, tp)
        return float(p[0]), float(d[0])
    return 0.0, 0.0


# --------------------------------------------------------------------------
# Grid (Sec. 2: the density on an equidistant grid of the unit cell; the
# sample run of App. A has a hexagonal, i.e. skew, cell).
# --------------------------------------------------------------------------


@dataclass
class Grid:
    """Equidistant grid; point (ix, iy, iz) = ix e_x + iy e_y + iz e_z with the
    step vectors e_a = (lattice vector a) / n_a.  Without `cell` the cell is
    orthorhombic with e_a = h_a along axis a; with `cell` (rows: the lattice
    vectors a, b, c in bohr) it may be skew, and `h` is not used.

    Arrays are (nz, ny, nx) in C order, so x is the fastest index.
    """

    n: tuple  # (nx, ny, nz)
    h: tuple  # (hx, hy, hz) bohr
    periodic: tuple = (0, 0, 0)
    cell: tuple | None = None
    gradient: str = "fd"  # "fd", or "spectral": Fourier derivative on periodic axes (FD on the others)

    @property
    def G(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def skew(self) -> bool:
        if self.cell is None:
            return False
        c = np.asarray(self.cell, dtype=np.float64)
        return bool(np.any(c[~np.eye(3, dtype=bool)] != 0.0))

    @property
    def steps(self) -> np.ndarray:
        """3 x 3, row a = the step vector e_a."""
        if self.cell is None:
            return np.diag(np.asarray(self.h, dtype=np.float64))
        c = np.asarray(self.cell, dtype=np.float64).reshape(3, 3)
        return c / np.asarray(self.n, dtype=np.float64)[:, None]

    @property
    def dV(self) -> float:
        if self.skew:
            return abs(float(np.linalg.det(self.steps)))
        return float(self.h[0] * self.h[1] * self.h[2])


def grid_of_cell(n, cell, periodic=(0, 0, 0), gradient="fd") -> Grid:
    """Grid of an n[0] x n[1] x n[2] division of the cell (rows a, b, c); a
    diagonal cell gives the orthorhombic form."""
    c = np.asarray(cell, dtype=np.float64).reshape(3, 3)
    h = tuple(float(np.linalg.norm(c[a]) / n[a]) for a in range(3))
    g = Grid(tuple(n), h, tuple(periodic), tuple(map(tuple, c)), gradient)
    if not g.skew:
        return Grid(tuple(n), tuple(float(c[a, a] / n[a]) for a in range(3)), tuple(periodic), None, gradient)
    return g


def cell_volume_element(cell, n) -> float:
    """dV = |det(cell)| / (n0 n1 n2) for a general (possibly skew) cell."""
    c = np.asarray(cell, dtype=np.float64).reshape(3, 3)
    return abs(float(np.linalg.det(c))) / float(n[0] * n[1] * n[2])


def diff_matrix_1d(N: int, h: float, periodic: bool) -> sp.csr_matrix:
    """Second-order finite-difference d/dx on N equidistant points.

    Central (f[i+1] - f[i-1]) / 2h inside; periodic wrap on periodic axes;
    one-sided (-3 f0 + 4 f1 - f2) / 2h and (3 f[N-1] - 4 f[N-2] + f[N-3]) / 2h
    at the two faces of a non-periodic axis.
    """
    if N < 3:
        raise ValueError("need at least 3 points per axis")
    rows, cols, vals = [], [], []
    c = 1.0 / (2.0 * h)
    for i in range(N):
        if periodic:
            rows += [i, i]
            cols += [(i + 1) % N, (i - 1) % N]
            vals += [c, -c]
        elif i == 0:
            rows += [0, 0, 0]
            cols += [0, 1, 2]
            vals += [-3 * c, 4 * c, -c]
        elif i == N - 1:
            rows += [i, i, i]
            cols += [N - 3, N - 2, N - 1]
            vals += [c, -4 * c, 3 * c]
        else:
            rows += [i, i]
            cols += [i + 1, i - 1]
            vals += [c, -c]
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def fourier_wavenumbers(N: int, h: float) -> np.ndarray:
    """2 pi m / (N h) for the DFT frequencies m = 0, 1, .., -1, with the
    unpaired Nyquist frequency of an even N set to zero (its derivative is
    not a real periodic function)."""
    k = np.fft.fftfreq(N) * N * (2.0 * math.pi / (N * h))
    if N % 2 == 0:
        k[N // 2] = 0.0
    return k


def spectral_matrix_1d(N: int, h: float) -> sp.csr_matrix:
    """The Fourier derivative on N periodic points of spacing h as a dense
    N x N operator: column j is the derivative of the j-th unit vector,
    computed by FFT (multiply by i k, transform back)."""
    k = fourier_wavenumbers(N, h)
    D = np.real(np.fft.ifft(1j * k[:, None] * np.fft.fft(np.eye(N), axis=0), axis=0))
    return sp.csr_matrix(D)


def _axis_op(grid: Grid, a: int, step: float):
    N = grid.n[a]
    if grid.gradient == "spectral" and grid.periodic[a]:
        return spectral_matrix_1d(N, step)
    return diff_matrix_1d(N, step, bool(grid.periodic[a]))


def gradient_operators(grid: Grid):
    """Sparse G x G operators (Gx, Gy, Gz) on the flattened (x fastest) grid.
    On a skew grid the differences along the grid axes give d_a = e_a . grad n
    (per grid step), and grad n = E^-1 d with E the matrix of step vectors.
    With grid.gradient == "spectral" the periodic axes take the Fourier
    derivative instead of finite differences."""
    nx, ny, nz = grid.n
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    if grid.skew:
        D = (sp.kron(Iz, sp.kron(Iy, _axis_op(grid, 0, 1.0))).tocsr(),
             sp.kron(Iz, sp.kron(_axis_op(grid, 1, 1.0), Ix)).tocsr(),
             sp.kron(_axis_op(grid, 2, 1.0), sp.kron(Iy, Ix)).tocsr())
        Einv = np.linalg.inv(grid.steps)
        return tuple((Einv[c, 0] * D[0] + Einv[c, 1] * D[1] + Einv[c, 2] * D[2]).tocsr() for c in range(3))
    Dx = _axis_op(grid, 0, grid.h[0])
    Dy = _axis_op(grid, 1, grid.h[1])
    Dz = _axis_op(grid, 2, grid.h[2])
    Gx = sp.kron(Iz, sp.kron(Iy, Dx)).tocsr()
    Gy = sp.kron(Iz, sp.kron(Dy, Ix)).tocsr()
    Gz = sp.kron(Dz, sp.kron(Iy, Ix)).tocsr()
    return Gx, Gy, Gz


def gradient(grid: Grid, rho: np.ndarray):
    """(dn/dx, dn/dy, dn/dz) on the flattened grid.  Fourier derivatives
    (grid.gradient == "spectral", periodic axes) are taken by FFT along the
    axis; the result equals gradient_operators(grid) applied to rho."""
    r = np.asarray(rho, dtype=np.float64).reshape(-1)
    if grid.gradient != "spectral" or not any(grid.periodic):
        return tuple(G @ r for G in gradient_operators(grid))
    nx, ny, nz = grid.n
    f = r.reshape(nz, ny, nx)
    steps = (1.0, 1.0, 1.0) if grid.skew else tuple(grid.h)
    I = (sp.identity(nx), sp.identity(ny), sp.identity(nz))
    d = []
    for a in range(3):
        if grid.periodic[a]:
            ax = 2 - a
            shape = [1, 1, 1]
            shape[ax] = grid.n[a]
            k = fourier_wavenumbers(grid.n[a], steps[a]).reshape(shape)
            d.append(np.real(np.fft.ifft(1j * k * np.fft.fft(f, axis=ax), axis=ax)).reshape(-1))
        else:
            D1 = diff_matrix_1d(grid.n[a], steps[a], False)
            op = (sp.kron(I[2], sp.kron(I[1], D1)), sp.kron(I[2], sp.kron(D1, I[0])), sp.kron(D1, sp.kron(I[1], I[0])))[a]
            d.append(op.tocsr() @ r)
    if not grid.skew:
        return tuple(d)
    Einv = np.linalg.inv(grid.steps)
    return tuple(Einv[c, 0] * d[0] + Einv[c, 1] * d[1] + Einv[c, 2] * d[2] for c in range(3))


# --------------------------------------------------------------------------
# LDA correlation (Perdew-Wang 1992, unpolarised) and q0 (Dion et al.).
# --------------------------------------------------------------------------

PW92_A = 0.031091
PW92_ALPHA1 = 0.21370
PW92_BETA = (7.5957, 3.5876, 1.6382, 0.49294)
Z_AB = -0.8491


def pw92_ec(rs):
    """eps_c(r_s) = -2A (1 + a1 rs) ln(1 + 1/Q), Q = 2A(b1 rs^1/2 + b2 rs + b3 rs^3/2 + b4 rs^2),
    and its derivative in r_s.  The logarithm is taken as log1p(1/Q)."""
    rs = np.asarray(rs, dtype=np.float64)
    b1, b2, b3, b4 = PW92_BETA
    A, a1 = PW92_A, PW92_ALPHA1
    s = np.sqrt(rs)
    Q = 2.0 * A * (b1 * s + b2 * rs + b3 * rs * s + b4 * rs * rs)
    L = np.log1p(1.0 / Q)
    ec = -2.0 * A * (1.0 + a1 * rs) * L
    dQ = 2.0 * A * (0.5 * b1 / s + b2 + 1.5 * b3 * s + 2.0 * b4 * rs)
    dec = -2.0 * A * a1 * L + 2.0 * A * (1.0 + a1 * rs) * dQ / (Q * (Q + 1.0))
    return ec, dec


def q0_of(n, g):
    """q0 = -(4 pi / 3) eps_xc^0 with eps_xc^0 = eps_x^LDA + eps_c^LDA - eps_x^LDA (Z_ab / 9) s^2,
    s = |grad n| / (2 k_F n).  Equivalent form used here:
        q0 = k_F - (4 pi / 3) eps_c(r_s) - (Z_ab / 36) g / (k_F n^2),  g = |grad n|^2.
    Returns (q0, dq0/dn at fixed g, dq0/dg)."""
    n = np.asarray(n, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    kF = np.cbrt(3.0 * math.pi ** 2 * n)
    rs = np.cbrt(3.0 / (4.0 * math.pi * n))
    ec, dec = pw92_ec(rs)
    q = kF - (4.0 * math.pi / 3.0) * ec - (Z_AB / 36.0) * g / (kF * n * n)
    dq_dn = kF / (3.0 * n) + (4.0 * math.pi / 3.0) * dec * rs / (3.0 * n) + 7.0 * Z_AB * g / (108.0 * kF * n ** 3)
    dq_dg = -Z_AB / (36.0 * kF * n * n)
    return q, dq_dn, dq_dg


def compute_q0(grid: Grid, rho, n_cut):
    """Gradient, then q0 and its derivatives on the retained points n >= n_cut (0 elsewhere)."""
    r = np.asarray(rho, dtype=np.float64).reshape(-1)
    gx, gy, gz = gradient(grid, r)
    g = gx * gx + gy * gy + gz * gz
    keep = r >= n_cut
    q = np.zeros_like(r)
    dqdn = np.zeros_like(r)
    dqdg = np.zeros_like(r)
    qq, a, b = q0_of(r[keep], g[keep])
    q[keep], dqdn[keep], dqdg[keep] = qq, a, b
    return dict(gx=gx, gy=gy, gz=gz, g=g, q0=q, dq_dn=dqdn, dq_dg=dqdg, keep=keep)


# --------------------------------------------------------------------------
# Local and semilocal exchange-correlation energies and the recombination of
# Eq. (3).  The paper's code evaluates these from the same density (Sec. 3,
# the list of steps; Sec. 5 sample output), with the PBE and revPBE forms of
# the works it cites.  Spin-unpolarised, Hartree units.
# --------------------------------------------------------------------------

PBE_KAPPA = 0.804        # PBE exchange: upper bound of the enhancement is 1 + kappa
REVPBE_KAPPA = 1.245     # revPBE (Zhang and Yang): the same form with a larger kappa
PBE_BETA = 0.06672455060314922                   # gradient-expansion coefficient of correlation
PBE_MU = PBE_BETA * math.pi ** 2 / 3.0           # exchange coefficient that cancels it at small s
PBE_GAMMA = (1.0 - math.log(2.0)) / math.pi ** 2


def lda_eps_x(n):
    """Exchange energy per electron of the uniform gas: -3 k_F / (4 pi)."""
    kF = np.cbrt(3.0 * math.pi ** 2 * np.asarray(n, dtype=np.float64))
    return -3.0 * kF / (4.0 * math.pi)


def pbe_fx(s2, kappa=PBE_KAPPA):
    """Exchange enhancement F_x(s) = 1 + kappa - kappa / (1 + mu s^2 / kappa)."""
    s2 = np.asarray(s2, dtype=np.float64)
    return 1.0 + kappa - kappa / (1.0 + PBE_MU * s2 / kappa)


def pbe_h(rs, t2):
    """Gradient correction H(r_s, t) of PBE correlation (unpolarised):
    H = gamma ln(1 + (beta/gamma) t^2 (1 + A t^2) / (1 + A t^2 + A^2 t^4)),
    A = (beta/gamma) / (exp(-eps_c/gamma) - 1)."""
    rs = np.asarray(rs, dtype=np.float64)
    t2 = np.asarray(t2, dtype=np.float64)
    ec, _ = pw92_ec(rs)
    A = (PBE_BETA / PBE_GAMMA) / np.expm1(-ec / PBE_GAMMA)
    y = A * t2
    return PBE_GAMMA * np.log1p((PBE_BETA / PBE_GAMMA) * t2 * (1.0 + y) / (1.0 + y + y * y))


def xc_energies(grid: Grid, rho, n_floor: float):
    """E_x^LDA, E_c^LDA (PW92), E_x^PBE, E_c^PBE, E_x^revPBE: dV times the sum
    over grid points with n > n_floor of n eps(n, |grad n|), the gradient by
    the finite differences of Sec. 3.  s = |grad n| / (2 k_F n), t = |grad n|
    / (2 k_s n), k_s = sqrt(4 k_F / pi)."""
    r = np.asarray(rho, dtype=np.float64).reshape(-1)
    gx, gy, gz = gradient(grid, r)
    keep = r > n_floor
    n = r[keep]
    g2 = (gx * gx + gy * gy + gz * gz)[keep]
    kF = np.cbrt(3.0 * math.pi ** 2 * n)
    rs = np.cbrt(3.0 / (4.0 * math.pi * n))
    ks2 = 4.0 * kF / math.pi
    ex = lda_eps_x(n)
    ec, _ = pw92_ec(rs)
    s2 = g2 / (2.0 * kF * n) ** 2
    t2 = g2 / (4.0 * ks2 * n * n)
    dV = grid.dV
    return dict(Ex_lda=dV * np.sum(n * ex), Ec_lda=dV * np.sum(n * ec),
                Ex_pbe=dV * np.sum(n * ex * pbe_fx(s2, PBE_KAPPA)), Ec_pbe=dV * np.sum(n * (ec + pbe_h(rs, t2))),
                Ex_revpbe=dV * np.sum(n * ex * pbe_fx(s2, REVPBE_KAPPA)))


def recombine(E_nl, Ec_lda, Ec_pbe, Ex_pbe=None, Ex_new=None, E_dft=None):
    """Eq. (3): E_tot^NL = E_tot^DFT - E_x^PBE - E_c^PBE + (E_x + E_c^LDA + E_c^NL),
    E_x being E_x^PBE or E_x^revPBE (Ex_new).  Without E_tot^DFT, the part
    that does not need it, -E_c^PBE + E_c^LDA + E_c^NL (+ E_x^new - E_x^PBE
    when an exchange is given), the sum the sample output prints."""
    delta = -Ec_pbe + Ec_lda + E_nl
    if Ex_new is not None:
        delta += Ex_new - Ex_pbe
    return delta if E_dft is None else E_dft + delta


# --------------------------------------------------------------------------
# The double sum of Eq. (2) with the self term, and its derivative.
# --------------------------------------------------------------------------


def self_radius(dV: float) -> float:
    """rho_s = (3 dV / 4 pi)^(1/3) e^(-1/3): for phi = c - b ln D the mean of
    phi(q r) over a ball of volume dV equals phi(q rho_s)."""
    return (3.0 * dV / (4.0 * math.pi)) ** (1.0 / 3.0) * math.exp(-1.0 / 3.0)


def _points(grid: Grid, keep):
    idx = np.flatnonzero(keep)
    nx, ny, _ = grid.n
    ix = (idx % nx).astype(np.int32)
    iy = ((idx // nx) % ny).astype(np.int32)
    iz = (idx // (nx * ny)).astype(np.int32)
    return idx, ix, iy, iz


def pair_rows(grid: Grid, ix, iy, iz, n, q, tab, tp, image_max=(0, 0, 0), r_cut=0.0, rows=None):
    """Per-row sums S0 (0th cell), S0 (images), Sq over all j and images."""
    ix = np.ascontiguousarray(ix, dtype=np.int32)
    iy = np.ascontiguousarray(iy, dtype=np.int32)
    iz = np.ascontiguousarray(iz, dtype=np.int32)
    n = np.ascontiguousarray(n, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    h = np.asarray(grid.h, dtype=np.float64)
    gd = np.asarray(grid.n, dtype=np.int32)
    per = np.asarray(grid.periodic, dtype=np.int32)
    im = np.asarray(image_max, dtype=np.int32)
    if rows is None:
        nrows = len(n)
        rows_p = None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        nrows = len(rows)
        rows_p = _p(rows, ct.c_int64)
    S0c = np.zeros(nrows)
    S0i = np.zeros(nrows)
    Sq = np.zeros(nrows)
    if grid.skew:
        h = np.ascontiguousarray(grid.steps.ravel())
    (lib().vo_pair_rows_cell if grid.skew else lib().vo_pair_rows)(
        len(n), _p(ix, ct.c_int32), _p(iy, ct.c_int32), _p(iz, ct.c_int32), _p(n, ct.c_double), _p(q, ct.c_double),
        _p(h, ct.c_double), _p(gd, ct.c_int32), _p(per, ct.c_int32), _p(im, ct.c_int32), float(r_cut),
        _p(tab, ct.c_double), ct.byref(tp), nrows, rows_p, _p(S0c, ct.c_double), _p(S0i, ct.c_double), _p(Sq, ct.c_double),
    )
    return S0c, S0i, Sq


def image_pair_sum(grid: Grid, ix, iy, iz, n, q, tab, tp, m, r_cut=0.0) -> float:
    """sum_i n_i sum_j n_j phi~ over the pairs of the single image shift m
    (integer cell multiples; (i, i) skipped for m = 0), with the distance cut.
    Orthorhombic grids only."""
    if grid.skew:
        raise ValueError("image_pair_sum: orthorhombic grids only")
    ix = np.ascontiguousarray(ix, dtype=np.int32)
    iy = np.ascontiguousarray(iy, dtype=np.int32)
    iz = np.ascontiguousarray(iz, dtype=np.int32)
    n = np.ascontiguousarray(n, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    h = np.asarray(grid.h, dtype=np.float64)
    gd = np.asarray(grid.n, dtype=np.int32)
    mm = np.asarray(m, dtype=np.int32)
    return float(lib().vo_image_pair_sum(
        len(n), _p(ix, ct.c_int32), _p(iy, ct.c_int32), _p(iz, ct.c_int32), _p(n, ct.c_double), _p(q, ct.c_double),
        _p(h, ct.c_double), _p(gd, ct.c_int32), _p(mm, ct.c_int32), float(r_cut), _p(tab, ct.c_double),
        ct.byref(tp)))


def half_image_shifts(grid: Grid, image_max):
    """One of each pair (m, -m) of the nonzero image shifts |m_a| <= image_max[a]
    on periodic axes: the shifts whose first nonzero component is positive."""
    lim = [int(image_max[a]) if grid.periodic[a] else 0 for a in range(3)]
    out = []
    for a in range(-lim[0], lim[0] + 1):
        for b in range(-lim[1], lim[1] + 1):
            for c in range(-lim[2], lim[2] + 1):
                first = next((v for v in (a, b, c) if v != 0), 0)
                if first > 0:
                    out.append((a, b, c))
    return out


def block_sum(grid: Grid, A, B, ix, iy, iz, n, q, tab, tp, image_max=(0, 0, 0), r_cut=0.0):
    """sum_{a in A, b in B} n_a n_b phi~_ab over images, skipping (a, a, 0)."""
    A = np.ascontiguousarray(A, dtype=np.int32)
    B = np.ascontiguousarray(B, dtype=np.int32)
    ix = np.ascontiguousarray(ix, dtype=np.int32)
    iy = np.ascontiguousarray(iy, dtype=np.int32)
    iz = np.ascontiguousarray(iz, dtype=np.int32)
    n = np.ascontiguousarray(n, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    h = np.asarray(grid.h, dtype=np.float64)
    gd = np.asarray(grid.n, dtype=np.int32)
    per = np.asarray(grid.periodic, dtype=np.int32)
    im = np.asarray(image_max, dtype=np.int32)
    if grid.skew:
        h = np.ascontiguousarray(grid.steps.ravel())
    return float((lib().vo_block_sum_cell if grid.skew else lib().vo_block_sum)(
        len(A), _p(A, ct.c_int32), len(B), _p(B, ct.c_int32),
        _p(ix, ct.c_int32), _p(iy, ct.c_int32), _p(iz, ct.c_int32), _p(n, ct.c_double), _p(q, ct.c_double),
        _p(h, ct.c_double), _p(gd, ct.c_int32), _p(per, ct.c_int32), _p(im, ct.c_int32), float(r_cut),
        _p(tab, ct.c_double), ct.byref(tp)))


def far_on(grid: Grid, far_max) -> bool:
    """True when far_max selects a far image shell on some periodic axis."""
    return far_max is not None and any(p and f > 0 for p, f in zip(grid.periodic, far_max))


def check_far(grid: Grid, image_max, far_max, r_cut):
    """The far shell needs no distance cut and far_max >= image_max on every
    periodic axis."""
    if not far_on(grid, far_max):
        return
    if r_cut > 0.0:
        raise ValueError("the far image shell is defined without a distance cut")
    for p, m, f in zip(grid.periodic, image_max, far_max):
        if p and f < m:
            raise ValueError("far_max must be >= image_max on every periodic axis")


def far_T(grid: Grid, image_max, far_max, d):
    """T(d) = sum over the far shell of |d - L|^-6 (bohr^-6) for grid
    displacements d (rows of integer steps along the three axes)."""
    E = np.ascontiguousarray(grid.steps.ravel())
    gd = np.asarray(grid.n, dtype=np.int32)
    per = np.asarray(grid.periodic, dtype=np.int32)
    im = np.asarray(image_max, dtype=np.int32)
    fm = np.asarray(far_max, dtype=np.int32)
    d = np.atleast_2d(np.asarray(d, dtype=np.float64))
    return np.array([lib().vo_far_T(_p(E, ct.c_double), _p(gd, ct.c_int32), _p(per, ct.c_int32),
                                    _p(im, ct.c_int32), _p(fm, ct.c_int32), *map(float, row)) for row in d])


def far_rows(grid: Grid, ix, iy, iz, n, q, image_max, far_max, rows=None):
    """Per-row sums of the far image shell (the kernel's large-D asymptote
    summed over the images beyond image_max up to far_max, the pair i = j
    included): F0_i = sum_j n_j phi_far(i, j), Fq_i = sum_j n_j d phi_far / d q_i."""
    ix = np.ascontiguousarray(ix, dtype=np.int32)
    iy = np.ascontiguousarray(iy, dtype=np.int32)
    iz = np.ascontiguousarray(iz, dtype=np.int32)
    n = np.ascontiguousarray(n, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    E = np.ascontiguousarray(grid.steps.ravel())
    gd = np.asarray(grid.n, dtype=np.int32)
    per = np.asarray(grid.periodic, dtype=np.int32)
    im = np.asarray(image_max, dtype=np.int32)
    fm = np.asarray(far_max, dtype=np.int32)
    if rows is None:
        nrows, rows_p = len(n), None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        nrows, rows_p = len(rows), _p(rows, ct.c_int64)
    F0 = np.zeros(nrows)
    Fq = np.zeros(nrows)
    rc = lib().vo_far_rows(len(n), _p(ix, ct.c_int32), _p(iy, ct.c_int32), _p(iz, ct.c_int32), _p(n, ct.c_double),
                           _p(q, ct.c_double), _p(E, ct.c_double), _p(gd, ct.c_int32), _p(per, ct.c_int32),
                           _p(im, ct.c_int32), _p(fm, ct.c_int32), nrows, rows_p, _p(F0, ct.c_double),
                           _p(Fq, ct.c_double))
    if rc:
        raise MemoryError("far_rows: table allocation failed")
    return F0, Fq


@dataclass
class Result:
    E_pair0: float
    E_pairL: float
    E_self: float
    dEdn: np.ndarray | None = None
    S0: np.ndarray | None = None
    Sq: np.ndarray | None = None
    q0: dict | None = None

    @property
    def E(self) -> float:
        return self.E_pair0 + self.E_pairL + self.E_self


def evaluate(grid: Grid, rho, tab, tp, n_cut, image_max=(0, 0, 0), r_cut=0.0, self_term=True, potential=False,
             far_max=None):
    """E_c^nl = 1/2 dV^2 sum_{(i,j,L) != (i,i,0)} n_i n_j phi~ (Eq. 2 with the volume
    element written out) + E_self, and optionally dE/dn at every grid point.
    With far_max the far image shell (see far_rows) joins the image sums."""
    check_far(grid, image_max, far_max, r_cut)
    r = np.asarray(rho, dtype=np.float64).reshape(-1)
    qd = compute_q0(grid, r, n_cut)
    keep = qd["keep"]
    idx, ix, iy, iz = _points(grid, keep)
    nS = r[idx]
    qS = qd["q0"][idx]
    dV = grid.dV
    S0c, S0i, Sq = pair_rows(grid, ix, iy, iz, nS, qS, tab, tp, image_max, r_cut)
    if far_on(grid, far_max):
        F0, Fq = far_rows(grid, ix, iy, iz, nS, qS, image_max, far_max)
        S0i = S0i + F0
        Sq = Sq + Fq
    E0 = 0.5 * dV * dV * float(np.sum(nS * S0c))
    EL = 0.5 * dV * dV * float(np.sum(nS * S0i))
    Phi = np.zeros(len(nS))
    dPhi = np.zeros(len(nS))
    if self_term == 2:
        Phi, dPhi = voxel_interp(voxel_table(grid.steps, tab, tp), qS, grid.steps, tab, tp)
    elif self_term:
        for t in range(len(nS)):
            Phi[t], dPhi[t] = onsite_phi(grid, qS[t], tab, tp, self_term)
    Es = 0.5 * dV * dV * float(np.sum(nS * nS * Phi))
    res = Result(E0, EL, Es, S0=S0c + S0i, Sq=Sq, q0=qd)
    if potential:
        res.dEdn = adjoint(grid, r, qd, idx, nS, S0c + S0i, Sq, Phi, dPhi)
    return res


def adjoint(grid: Grid, rho, qd, idx, nS, S0, Sq, Phi, dPhi):
    """dE/dn_k on the whole grid.

    For k retained:  dE/dn_k|_q = dV^2 (S0_k + n_k Phi_k),
                     dE/dq_k    = dV^2 n_k (Sq_k + 1/2 n_k dPhi_k),
    and q_k depends on n_k directly and on g = |grad n|^2 of the
    finite-difference gradient, so
       v = [k in S](dE/dn|_q + dE/dq dq/dn) + sum_a G_a^T B_a,
       B_a = [i in S] dE/dq_i dq/dg_i 2 (d_a n)_i,
    with G_a the gradient operators (the transpose makes dropped points
    that feed a retained point's stencil pick up their share)."""
    dV = grid.dV
    G = grid.G
    dEdn_q = dV * dV * (S0 + nS * Phi)
    dEdq = dV * dV * nS * (Sq + 0.5 * nS * dPhi)
    v = np.zeros(G)
    v[idx] = dEdn_q + dEdq * qd["dq_dn"][idx]
    ops = gradient_operators(grid)
    for Ga, comp in zip(ops, ("gx", "gy", "gz")):
        B = np.zeros(G)
        B[idx] = dEdq * qd["dq_dg"][idx] * 2.0 * qd[comp][idx]
        v += Ga.T @ B
    return v


def local_energy_change(grid: Grid, rho, k, eps, tab, tp, n_cut, image_max=(0, 0, 0), r_cut=0.0, self_term=True,
                        ops=None):
    """E(n + eps e_k) - E(n - eps e_k), recomputing only the rows whose n or
    q change (k and its finite-difference neighbours).  With P that set:
      sum over all pairs = (pairs outside P) + 2 R(P) - PP,
      R(P) = sum_{i in P, j} n_i n_j phi~_ij,  PP = sum_{i, j in P}.
    `ops` may pass gradient_operators(grid) in, for repeated calls."""
    r0 = np.asarray(rho, dtype=np.float64).reshape(-1).copy()
    ops = gradient_operators(grid) if ops is None else ops
    touched = set([int(k)])
    for Ga in ops:
        col = Ga.getcol(int(k)).tocoo()
        touched.update(int(i) for i in col.row)
    keep = r0 >= n_cut
    idx, ix, iy, iz = _points(grid, keep)
    pos = {int(g): t for t, g in enumerate(idx)}
    P = np.array(sorted(pos[g] for g in touched if g in pos), dtype=np.int32)
    allS = np.arange(len(idx), dtype=np.int32)
    dV = grid.dV

    def part(rr):
        gx, gy, gz = (Ga @ rr for Ga in ops)
        g = gx * gx + gy * gy + gz * gz
        q = np.zeros_like(rr)
        q[keep] = q0_of(rr[keep], g[keep])[0]
        nS, qS = rr[idx], q[idx]
        R = block_sum(grid, P, allS, ix, iy, iz, nS, qS, tab, tp, image_max, r_cut)
        PP = block_sum(grid, P, P, ix, iy, iz, nS, qS, tab, tp, image_max, r_cut)
        e = 0.5 * dV * dV * (2.0 * R - PP)
        if self_term:
            for t in P:
                e += 0.5 * dV * dV * nS[t] * nS[t] * onsite_phi(grid, qS[t], tab, tp, self_term)[0]
        return e

    rp = r0.copy()
    rp[k] += eps
    rm = r0.copy()
    rm[k] -= eps
    if not (np.array_equal(rp >= n_cut, keep) and np.array_equal(rm >= n_cut, keep)):
        raise ValueError("perturbation changes the retained set")
    return part(rp) - part(rm)


def potential_at(grid: Grid, rho, ks, tab, tp, n_cut, image_max=(0, 0, 0), r_cut=0.0, self_term=True,
                 far_max=None):
    """dE/dn_k at the grid points ks only: the rows of the double sum that
    the formula of `adjoint` needs at k (k itself and the kept points whose
    gradient stencil contains k) are summed over every j, nothing else.
    Same arithmetic as `evaluate(..., potential=True)` restricted to ks."""
    check_far(grid, image_max, far_max, r_cut)
    r = np.asarray(rho, dtype=np.float64).reshape(-1)
    qd = compute_q0(grid, r, n_cut)
    keep = qd["keep"]
    idx, ix, iy, iz = _points(grid, keep)
    pos = {int(g): t for t, g in enumerate(idx)}
    ops = gradient_operators(grid)
    cols = [Ga.tocsc() for Ga in ops]
    need = set()
    for k in ks:
        k = int(k)
        if keep[k]:
            need.add(k)
        for Gc in cols:
            need.update(int(i) for i in Gc.getcol(k).indices if keep[int(i)])
    gl = np.array(sorted(need), dtype=np.int64)
    rows = np.array([pos[int(g)] for g in gl], dtype=np.int64)
    nS, qS = r[idx], qd["q0"][idx]
    if len(rows):
        S0c, S0i, Sq = pair_rows(grid, ix, iy, iz, nS, qS, tab, tp, image_max, r_cut, rows=rows)
        if far_on(grid, far_max):
            F0, Fq = far_rows(grid, ix, iy, iz, nS, qS, image_max, far_max, rows=rows)
            S0i = S0i + F0
            Sq = Sq + Fq
    else:
        S0c = S0i = Sq = np.zeros(0)
    dV = grid.dV
    dEdn_q = {}
    dEdq = {}
    for t, g in enumerate(gl):
        n = r[g]
        Phi, dPhi = onsite_phi(grid, qS[rows[t]], tab, tp, self_term)
        dEdn_q[int(g)] = dV * dV * (S0c[t] + S0i[t] + n * Phi)
        dEdq[int(g)] = dV * dV * n * (Sq[t] + 0.5 * n * dPhi)
    out = np.zeros(len(ks))
    comps = (qd["gx"], qd["gy"], qd["gz"])
    for s, k in enumerate(ks):
        k = int(k)
        v = 0.0
        if keep[k]:
            v += dEdn_q[k] + dEdq[k] * qd["dq_dn"][k]
        for Gc, ga in zip(cols, comps):
            col = Gc.getcol(k)
            for i, c in zip(col.indices, col.data):
                i = int(i)
                if keep[i]:
                    v += c * dEdq[i] * qd["dq_dg"][i] * 2.0 * ga[i]
        out[s] = v
    return out
