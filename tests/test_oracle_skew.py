"""Pins of the oracle on skew (non-orthogonal) cells, the geometry of the
paper's sample run (a hexagonal cell, App. A): the finite-difference
gradient mapped through the step vectors is exact on quadratics and on
lattice plane waves; a sheared description of an orthorhombic crystal gives
the same pair sums point by point; rigid rotations of the cell change
nothing; the adjoint equals central differences for a kink-free kernel;
dV and the exchange-correlation energies of a uniform density."""
import math

import numpy as np
import pytest

import vdw_workloads as W

CELL = ((2.8, 0.0, 0.0), (1.1, 2.6, 0.0), (0.4, -0.3, 2.9))
DIRAC = 0.7385587663820224


def _bilinear_table(oracle, nD=9, nS=5, Dmax=8.0, c=(0.3, -0.7, 1.9, 0.45)):
    tp = oracle.table_params(n_D=nD, n_sigma=nS, D_max=Dmax)
    Dk = np.arange(nD) * Dmax / (nD - 1)
    sl = np.arange(nS) / (nS - 1)
    return tp, c[0] + c[1] * Dk[:, None] + c[2] * sl[None, :] + c[3] * Dk[:, None] * sl[None, :]


def test_grid_of_cell(oracle):
    g = oracle.grid_of_cell((7, 6, 5), CELL)
    assert g.skew
    assert g.dV == pytest.approx(abs(np.linalg.det(np.asarray(CELL))) / (7 * 6 * 5), rel=1e-14)
    assert np.allclose(g.steps * np.array([[7], [6], [5]]), np.asarray(CELL), atol=1e-15)
    ortho = oracle.grid_of_cell((4, 5, 6), ((2.0, 0, 0), (0, 2.5, 0), (0, 0, 3.0)))
    assert not ortho.skew and ortho.cell is None and ortho.h == (0.5, 0.5, 0.5)


def test_skew_gradient_exact_on_quadratics(oracle):
    """f(r) = c0 + c.r + r^T A r is quadratic in the grid indices too, so the
    second-order differences along the grid axes are exact, and E^-1 maps
    them to the Cartesian gradient c + 2 A r (a transposed map fails)."""
    n = (7, 6, 5)
    g = oracle.grid_of_cell(n, CELL)
    P = W.cell_points(n, CELL).reshape(-1, 3)
    c = np.array([0.3, -1.2, 0.7])
    A = np.array([[0.9, 0.2, -0.4], [0.2, -0.5, 0.3], [-0.4, 0.3, 1.1]])
    f = 1.5 + P @ c + np.einsum("pi,ij,pj->p", P, A, P)
    gx, gy, gz = oracle.gradient(g, f)
    exp = c[None, :] + 2.0 * P @ A
    assert np.abs(np.stack([gx, gy, gz], 1) - exp).max() < 1e-11


def test_skew_gradient_periodic_plane_wave(oracle):
    """On a fully periodic skew cell, f = sin(k.r) with k a reciprocal-lattice
    vector is periodic; the central difference along e_a is exactly
    cos(k.r) sin(k.e_a), so the mapped gradient is E^-1 of those."""
    n = (9, 8, 7)
    g = oracle.grid_of_cell(n, CELL, (1, 1, 1))
    C = np.asarray(CELL)
    B = 2 * math.pi * np.linalg.inv(C).T  # rows: reciprocal vectors, b_i . a_j = 2 pi delta_ij
    k = 1 * B[0] - 2 * B[1] + 1 * B[2]
    P = W.cell_points(n, CELL).reshape(-1, 3)
    f = np.sin(P @ k)
    grad = np.stack(oracle.gradient(g, f), 1)
    E = g.steps
    d = np.cos(P @ k)[:, None] * np.sin(E @ k)[None, :]
    exp = d @ np.linalg.inv(E).T
    assert np.abs(grad - exp).max() < 1e-12
    # and it approaches the exact gradient cos(k.r) k as the grid is refined
    assert np.abs(grad - np.cos(P @ k)[:, None] * k[None, :]).max() < 0.5 * np.abs(k).max()


def test_sheared_description_of_an_orthorhombic_crystal(oracle):
    """An orthorhombic grid periodic in x and y, and the same points described
    by the skew cell a' = a, b' = a + b (grid point (i, j) of the skew cell is
    point ((i + j) mod nx, j) of the orthorhombic one): with image ranges that
    cover r_cut in both descriptions, every point has the same pair sums."""
    nx, ny, nz = 8, 8, 4
    h = (0.5, 0.6, 0.7)
    tp, tab = _bilinear_table(oracle, nD=17, nS=5, Dmax=40.0, c=(0.3, -0.004, 0.5, 0.001))
    go = oracle.Grid((nx, ny, nz), h, (1, 1, 0))
    cell = ((nx * h[0], 0.0, 0.0), (nx * h[0], ny * h[1], 0.0), (0.0, 0.0, nz * h[2]))
    gs = oracle.grid_of_cell((nx, ny, nz), cell, (1, 1, 0))
    assert gs.skew and gs.dV == pytest.approx(go.dV, rel=1e-14)
    rng = np.random.default_rng(4)
    n_o = rng.uniform(0.01, 1.0, size=(nz, ny, nx))
    q_o = rng.uniform(0.5, 3.0, size=(nz, ny, nx))
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    n_s = n_o[k, j, (i + j) % nx]
    q_s = q_o[k, j, (i + j) % nx]
    r_cut = 4.5

    def sums(g, nn, qq, im):
        idx, ix, iy, iz = oracle._points(g, np.ones(g.G, bool))
        S0c, S0i, Sq = oracle.pair_rows(g, ix, iy, iz, nn.ravel(), qq.ravel(), tab, tp, im, r_cut)
        return (S0c + S0i).reshape(nz, ny, nx), Sq.reshape(nz, ny, nx), S0c.reshape(nz, ny, nx)

    So, Sqo, So_home = sums(go, n_o, q_o, (2, 2, 0))
    Ss, Sqs, Ss_home = sums(gs, n_s, q_s, (4, 2, 0))
    assert np.allclose(Ss, So[k, j, (i + j) % nx], rtol=1e-12, atol=0)
    assert np.allclose(Sqs, Sqo[k, j, (i + j) % nx], rtol=1e-12, atol=0)
    # the split into the home cell and its images does depend on the description
    assert not np.allclose(Ss_home, So_home[k, j, (i + j) % nx], rtol=1e-6)


@pytest.mark.parametrize("periodic,image_max,r_cut", [((0, 0, 0), (0, 0, 0), 0.0), ((1, 1, 0), (1, 1, 0), 4.0)])
def test_skew_rotation_invariance(oracle, table_cache, periodic, image_max, r_cut):
    """Rotating the whole cell moves no distance and no |grad n|: energies and
    dE/dn are unchanged."""
    tp, tab = table_cache(n_D=256, n_sigma=16, D_max=12.0, gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)
    wl = W.random_skew(periodic=periodic, seed=9, image_max=image_max, r_cut=r_cut)
    th, ph = 0.7, -1.1
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, math.cos(ph), -math.sin(ph)], [0, math.sin(ph), math.cos(ph)]])
    R = Rx @ Rz
    g0 = oracle.grid_of_cell(wl.n, wl.cell, periodic)
    g1 = oracle.grid_of_cell(wl.n, np.asarray(wl.cell) @ R.T, periodic)
    e0 = oracle.evaluate(g0, wl.rho, tab, tp, wl.n_cut, image_max, r_cut, potential=True)
    e1 = oracle.evaluate(g1, wl.rho, tab, tp, wl.n_cut, image_max, r_cut, potential=True)
    for a, b in ((e0.E_pair0, e1.E_pair0), (e0.E_pairL, e1.E_pairL), (e0.E_self, e1.E_self)):
        assert a == pytest.approx(b, rel=1e-11, abs=1e-300)
    assert np.abs(e0.dEdn - e1.dEdn).max() <= 1e-10 * np.abs(e0.dEdn).max()
    if any(image_max):
        assert e0.E_pairL != 0.0


@pytest.mark.parametrize("periodic,image_max,r_cut", [((0, 0, 0), (0, 0, 0), 0.0), ((1, 0, 1), (2, 0, 1), 3.5)])
def test_skew_adjoint_exact_for_kink_free_kernel(oracle, periodic, image_max, r_cut):
    """dE/dn from the adjoint (the transposed skew gradient included) equals
    central differences of E for a table bilinear in (D, sigma)."""
    tp, tab = _bilinear_table(oracle, nD=9, nS=5, Dmax=400.0, c=(0.3, -0.1 * 2.5 / 400.0, 1.9, 0.05 * 2.5 / 400.0))
    wl = W.random_skew(periodic=periodic, seed=5, n_cut=4e-3, image_max=image_max, r_cut=r_cut)
    g = oracle.grid_of_cell(wl.n, wl.cell, periodic)
    rho = wl.rho.reshape(-1).copy()
    dropped = g.n[0] * 2 + 3
    rho[dropped] = 0.5 * wl.n_cut
    res = oracle.evaluate(g, rho, tab, tp, wl.n_cut, image_max, r_cut, potential=True)
    rng = np.random.default_rng(2)
    for kk in list(rng.choice(np.flatnonzero(rho >= 2 * wl.n_cut), 8, replace=False)) + [dropped]:
        eps = 2e-5 * rho[kk]
        fd = oracle.local_energy_change(g, rho, kk, eps, tab, tp, wl.n_cut, image_max, r_cut) / (2 * eps)
        assert fd == pytest.approx(res.dEdn[kk], rel=1e-5, abs=1e-10 * np.abs(res.dEdn).max()), kk
    assert res.dEdn[dropped] != 0.0


def test_skew_uniform_density_xc_and_volume(oracle):
    """A uniform density on a periodic skew cell: Dirac exchange with the cell
    volume |det(a, b, c)|, and no gradient terms."""
    n = (6, 5, 4)
    g = oracle.grid_of_cell(n, CELL, (1, 1, 1))
    n0 = 0.07
    E = oracle.xc_energies(g, np.full(g.G, n0), 1e-12)
    V = abs(np.linalg.det(np.asarray(CELL)))
    assert E["Ex_lda"] == pytest.approx(-DIRAC * n0 ** (4 / 3) * V, rel=1e-13)
    assert E["Ex_pbe"] == pytest.approx(E["Ex_lda"], rel=1e-15) and E["Ec_pbe"] == pytest.approx(E["Ec_lda"], rel=1e-15)
