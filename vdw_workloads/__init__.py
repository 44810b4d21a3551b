"""Seeded synthetic densities for the vdW-DF nonlocal-correlation path.

Input generators only: nothing here computes any part of the method.  Both
the test oracle and the GPU path take their inputs from this module.

The paper's own examples (a Kr dimer and a Xe monolayer, Sec. 6) use DFT
densities that are not available here; these generators stand in for them
with atoms made of exponential shells,
    n_atom(r) = sum_k A_k exp(-alpha_k |r - R|),   A_k = f_k Z alpha_k^3 / (8 pi),
so that every shell integrates to f_k Z electrons (int A e^{-a r} d^3r = 8 pi A / a^3),
with shell fractions f_k = w_k / sum w, w_k ~ U(0.2, 1) from the seed.

Units: bohr and electrons / bohr^3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    n: tuple  # (nx, ny, nz)
    h: tuple  # (hx, hy, hz)
    periodic: tuple
    rho: np.ndarray  # (nz, ny, nx) float64, x fastest
    n_cut: float
    image_max: tuple = (0, 0, 0)
    r_cut: float = 0.0
    table: dict = field(default_factory=lambda: dict(n_D=2048, n_sigma=64, D_max=48.0))
    meta: dict = field(default_factory=dict)
    cell: tuple | None = None  # rows: lattice vectors a, b, c (bohr) of a skew cell; None: orthorhombic from h

    @property
    def G(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def dV(self) -> float:
        if self.cell is not None:
            return abs(float(np.linalg.det(np.asarray(self.cell, dtype=np.float64)))) / self.G
        return float(self.h[0] * self.h[1] * self.h[2])

    def electrons(self) -> float:
        return float(self.rho.sum() * self.dV)


def shell_weights(rng: np.random.Generator, nshell: int) -> np.ndarray:
    w = rng.uniform(0.2, 1.0, size=nshell)
    return w / w.sum()


def _coords(n, h):
    nx, ny, nz = n
    z = np.arange(nz, dtype=np.float64) * h[2]
    y = np.arange(ny, dtype=np.float64) * h[1]
    x = np.arange(nx, dtype=np.float64) * h[0]
    return z[:, None, None], y[None, :, None], x[None, None, :]


def atom_density(n, h, center, Z, alphas, fracs, lateral_images=0, cell=None) -> np.ndarray:
    """Exponential-shell atom on the grid; with lateral_images > 0 the atom is
    repeated over (m, p) cells |m|, |p| <= lateral_images along x and y."""
    Zc, Yc, Xc = _coords(n, h)
    out = np.zeros((n[2], n[1], n[0]))
    amps = [f * Z * a ** 3 / (8.0 * math.pi) for f, a in zip(fracs, alphas)]
    shifts = [(0.0, 0.0)]
    if lateral_images:
        shifts = [(m * cell[0], p * cell[1]) for m in range(-lateral_images, lateral_images + 1)
                  for p in range(-lateral_images, lateral_images + 1)]
    for sx, sy in shifts:
        dz2 = (Zc - center[2]) ** 2
        dy2 = (Yc - center[1] - sy) ** 2
        dx2 = (Xc - center[0] - sx) ** 2
        r = np.sqrt(dz2 + dy2 + dx2)
        for A, a in zip(amps, alphas):
            out += A * np.exp(-a * r)
    return out


def cell_points(n, cell) -> np.ndarray:
    """Cartesian positions (nz, ny, nx, 3) of the grid points
    i0 e_0 + i1 e_1 + i2 e_2, e_a = cell[a] / n[a]."""
    E = np.asarray(cell, dtype=np.float64) / np.asarray(n, dtype=np.float64)[:, None]
    u2, u1, u0 = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    return u0[..., None] * E[0] + u1[..., None] * E[1] + u2[..., None] * E[2]


def cell_atom_density(n, cell, center, Z, alphas, fracs, periodic=(0, 0, 0), images=0) -> np.ndarray:
    """Exponential-shell atom on the grid of a (possibly skew) cell, repeated
    over the lattice translations sum_a m_a cell[a] with |m_a| <= images on
    periodic axes."""
    P = cell_points(n, cell)
    C = np.asarray(cell, dtype=np.float64)
    out = np.zeros(P.shape[:3])
    amps = [f * Z * a ** 3 / (8.0 * math.pi) for f, a in zip(fracs, alphas)]
    rng_ = [range(-images, images + 1) if periodic[a] else range(0, 1) for a in range(3)]
    for m0 in rng_[0]:
        for m1 in rng_[1]:
            for m2 in rng_[2]:
                shift = m0 * C[0] + m1 * C[1] + m2 * C[2]
                r = np.linalg.norm(P - (np.asarray(center) + shift), axis=-1)
                for A, a in zip(amps, alphas):
                    out += A * np.exp(-a * r)
    return out


# ---------------------------------------------------------------------------
# Named workloads.
# ---------------------------------------------------------------------------


def dimer_small(seed: int = 1) -> Workload:
    """Tiny dimer: 12 bohr cube, 24^3 nodes at i * 0.5, two identical 8-electron
    atoms (alpha = 8.0, 2.5, 0.9) at (6 -+ 1.8, 6, 6), n_cut = 1e-6, table
    1024 x 32 on D in [0, 48]; energy in plain FP64."""
    rng = np.random.default_rng(seed)
    f = shell_weights(rng, 3)
    n, h = (24, 24, 24), (0.5, 0.5, 0.5)
    alphas = (8.0, 2.5, 0.9)
    rho = atom_density(n, h, (6.0 - 1.8, 6.0, 6.0), 8.0, alphas, f) + atom_density(n, h, (6.0 + 1.8, 6.0, 6.0), 8.0, alphas, f)
    return Workload("dimer-24^3-h0.5", n, h, (0, 0, 0), rho, 1e-6, table=dict(n_D=1024, n_sigma=32, D_max=48.0),
                    meta=dict(seed=seed, fracs=f.tolist()))


KR_ALPHAS = (30.0, 8.0, 2.5, 0.8)
KR_SEPARATIONS = (6.0, 7.0, 8.0, 10.0, 14.0)


def kr_dimer(R: float = 7.0, seed: int = 2, which: str = "both") -> Workload:
    """Kr2-like dimer: 24 bohr cube, 96^3 nodes (h = 0.25), two 36-electron atoms
    (alpha = 30, 8, 2.5, 0.8; one shell draw shared by every R) at (12 -+ R/2, 12, 12),
    n_cut = 1e-5, table 2048 x 64.  which = 'A' or 'B' gives one atom alone at
    the same position (for E(inf) = E(A) + E(B))."""
    rng = np.random.default_rng(seed)
    f = shell_weights(rng, 4)
    n, h = (96, 96, 96), (0.25, 0.25, 0.25)
    rho = np.zeros((96, 96, 96))
    if which in ("both", "A"):
        rho += atom_density(n, h, (12.0 - R / 2, 12.0, 12.0), 36.0, KR_ALPHAS, f)
    if which in ("both", "B"):
        rho += atom_density(n, h, (12.0 + R / 2, 12.0, 12.0), 36.0, KR_ALPHAS, f)
    return Workload(f"kr-dimer-96^3-R{R:g}-{which}", n, h, (0, 0, 0), rho, 1e-5,
                    table=dict(n_D=2048, n_sigma=64, D_max=48.0), meta=dict(seed=seed, R=R, fracs=f.tolist()))


def xe_slab(seed: int = 3, nxy: int = 48, nz: int = 224) -> Workload:
    """Xe-monolayer-like slab: orthorhombic 8.6 x 8.6 x 40 bohr cell, 48 x 48 x 224
    grid, periodic in x and y, one 54-electron atom (alpha = 30, 8, 2.5, 0.8) at
    (4.3, 4.3, 20), density periodised over |m|, |p| <= 4 atom images; n_cut = 1e-5;
    images |m|, |p| <= 3 with |r - r'| <= 30 bohr."""
    rng = np.random.default_rng(seed)
    f = shell_weights(rng, 4)
    cell = (8.6, 8.6, 40.0)
    n = (nxy, nxy, nz)
    h = (cell[0] / n[0], cell[1] / n[1], cell[2] / n[2])
    rho = atom_density(n, h, (4.3, 4.3, 20.0), 54.0, KR_ALPHAS, f, lateral_images=4, cell=cell)
    return Workload(f"xe-slab-{nxy}x{nxy}x{nz}", n, h, (1, 1, 0), rho, 1e-5, image_max=(3, 3, 0), r_cut=30.0,
                    table=dict(n_D=2048, n_sigma=64, D_max=48.0), meta=dict(seed=seed, fracs=f.tolist(), cell=cell))


HEX_CELL_XE = ((8.6, 0.0, 0.0), (4.3, 8.6 * math.sqrt(3.0) / 2.0, 0.0), (0.0, 0.0, 40.0))


def xe_hex_slab(seed: int = 3, nxy: int = 48, nz: int = 224) -> Workload:
    """The Xe-slab workload on the hexagonal cell of a close-packed monolayer
    (the geometry of the paper's sample run, App. A): a = (8.6, 0, 0),
    b = (4.3, 7.45, 0), c = (0, 0, 40) bohr, nxy x nxy x nz grid, periodic in
    a and b, one 54-electron atom (alpha = 30, 8, 2.5, 0.8) at the cell centre
    in the plane z = 20, periodised over |m|, |p| <= 4 cells; n_cut = 1e-5;
    images |m|, |p| <= 4 with |r - r'| <= 30 bohr (the cell is thinner across
    its short diagonal, so one more image ring than the square cell)."""
    rng = np.random.default_rng(seed)
    f = shell_weights(rng, 4)
    n = (nxy, nxy, nz)
    C = np.asarray(HEX_CELL_XE)
    center = tuple(0.5 * C[0] + 0.5 * C[1] + np.array([0.0, 0.0, 20.0]))
    rho = cell_atom_density(n, C, center, 54.0, KR_ALPHAS, f, periodic=(1, 1, 0), images=4)
    h = tuple(float(np.linalg.norm(C[a]) / n[a]) for a in range(3))
    return Workload(f"xe-hex-slab-{nxy}x{nxy}x{nz}", n, h, (1, 1, 0), rho, 1e-5, image_max=(4, 4, 0), r_cut=30.0,
                    table=dict(n_D=2048, n_sigma=64, D_max=48.0), meta=dict(seed=seed, fracs=f.tolist()),
                    cell=tuple(map(tuple, C)))


def random_skew(n=(7, 6, 5), cell=((2.8, 0.0, 0.0), (1.1, 2.6, 0.0), (0.4, -0.3, 2.9)), periodic=(0, 0, 0),
                seed: int = 0, n_cut: float = 1e-3, image_max=(0, 0, 0), r_cut: float = 0.0, table=None) -> Workload:
    """A smooth random density on a small skew grid (three exponential blobs
    at random fractional positions, repeated over one ring of cells on
    periodic axes, plus a floor), for oracle pins and GPU parity."""
    rng = np.random.default_rng(seed)
    C = np.asarray(cell, dtype=np.float64)
    rho = np.full((n[2], n[1], n[0]), 2e-3)
    for _ in range(3):
        frac = rng.uniform(0.2, 0.8, size=3)
        Z = rng.uniform(0.5, 3.0)
        a = rng.uniform(0.8, 3.0)
        rho += cell_atom_density(n, C, tuple(frac @ C), Z, (a,), (1.0,), periodic=periodic, images=1)
    rho *= rng.uniform(0.9, 1.1, size=rho.shape)
    h = tuple(float(np.linalg.norm(C[a]) / n[a]) for a in range(3))
    return Workload(f"skew-{n[0]}x{n[1]}x{n[2]}-s{seed}", tuple(n), h, tuple(periodic), rho, n_cut,
                    image_max=tuple(image_max), r_cut=r_cut, table=table or dict(n_D=256, n_sigma=16, D_max=24.0),
                    meta=dict(seed=seed), cell=tuple(map(tuple, C)))


def molecule_batch(count: int = 64, seed: int = 5, min_edge: int = 16, max_edge: int = 64) -> list:
    """Batch of molecule-like densities: cubic boxes of U{min_edge..max_edge}
    nodes at h = 0.3, U{2..12} atoms placed uniformly at >= 4 bohr from each
    other (an atom is dropped after 10^4 failed placements, never below 2),
    Z ~ U{1..36}, three sorted alpha ~ U(0.7, 10); n_cut = 1e-5."""
    rng = np.random.default_rng(seed)
    out = []
    h = 0.3
    for m in range(count):
        edge = int(rng.integers(min_edge, max_edge + 1))
        L = edge * h
        natoms = int(rng.integers(2, 13))
        pos = []
        fails = 0
        while len(pos) < natoms:
            p = rng.uniform(0.0, L, size=3)
            if all(np.linalg.norm(p - q) >= 4.0 for q in pos):
                pos.append(p)
                fails = 0
            else:
                fails += 1
                if fails >= 10000:
                    natoms = max(2, natoms - 1)
                    fails = 0
                    if len(pos) >= natoms:
                        break
        if len(pos) < 2:
            # a box too small for two atoms 4 bohr apart: put them on the diagonal
            pos = [np.array([0.5, 0.5, 0.5]), np.array([L - 0.5, L - 0.5, L - 0.5])]
        rho = np.zeros((edge, edge, edge))
        atoms = []
        for p in pos:
            Z = float(rng.integers(1, 37))
            alphas = np.sort(rng.uniform(0.7, 10.0, size=3))
            f = shell_weights(rng, 3)
            rho += atom_density((edge, edge, edge), (h, h, h), tuple(p), Z, tuple(alphas), f)
            atoms.append(dict(pos=p.tolist(), Z=Z, alphas=alphas.tolist()))
        out.append(Workload(f"mol{m}-{edge}^3", (edge,) * 3, (h, h, h), (0, 0, 0), rho, 1e-5,
                            table=dict(n_D=2048, n_sigma=64, D_max=48.0), meta=dict(seed=seed, atoms=atoms)))
    return out


def random_small(n=(6, 5, 7), h=(0.4, 0.45, 0.5), periodic=(0, 0, 0), seed: int = 0, n_cut: float = 1e-3,
                 image_max=(0, 0, 0), r_cut: float = 0.0, table=None) -> Workload:
    """A smooth random density on a small grid (two or three exponential blobs
    plus a floor), for brute-force and derivative checks."""
    rng = np.random.default_rng(seed)
    rho = np.full((n[2], n[1], n[0]), 2e-3)
    L = [n[a] * h[a] for a in range(3)]
    for _ in range(3):
        c = rng.uniform(0.2, 0.8, size=3) * np.array(L)
        Z = rng.uniform(0.5, 3.0)
        a = rng.uniform(0.8, 3.0)
        rho += atom_density(n, h, tuple(c), Z, (a,), (1.0,))
    rho *= rng.uniform(0.9, 1.1, size=rho.shape)
    return Workload(f"random-{n[0]}x{n[1]}x{n[2]}-s{seed}", tuple(n), tuple(h), tuple(periodic), rho, n_cut,
                    image_max=tuple(image_max), r_cut=r_cut,
                    table=table or dict(n_D=256, n_sigma=16, D_max=24.0), meta=dict(seed=seed))


def scaled_dimer(edge: int = 32, h: float = 0.4, R: float = 5.0, seed: int = 2, Z: float = 10.0,
                 alphas=(12.0, 4.0, 1.6, 0.8), n_cut: float = 1e-5) -> Workload:
    """A dimer on a mid-size grid (a few 1e3-1e4 retained points), for parity
    checks that the oracle finishes in seconds while spanning many tiles."""
    rng = np.random.default_rng(seed)
    f = shell_weights(rng, len(alphas))
    n = (edge, edge, edge)
    c = edge * h / 2
    rho = atom_density(n, (h, h, h), (c - R / 2, c, c), Z, alphas, f) + atom_density(n, (h, h, h), (c + R / 2, c, c), Z, alphas, f)
    return Workload(f"dimer-{edge}^3-h{h:g}", n, (h, h, h), (0, 0, 0), rho, n_cut,
                    table=dict(n_D=2048, n_sigma=64, D_max=48.0), meta=dict(seed=seed))


def scaled_slab(nxy: int = 12, nz: int = 40, seed: int = 3, image_max=(3, 3, 0), r_cut: float = 30.0) -> Workload:
    """Xe-slab shape on a coarse grid (same cell, atom and images) for parity."""
    w = xe_slab(seed=seed, nxy=nxy, nz=nz)
    w.image_max = tuple(image_max)
    w.r_cut = r_cut
    w.name = f"xe-slab-{nxy}x{nxy}x{nz}"
    return w
