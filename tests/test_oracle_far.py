"""Pins of the oracle's far image shell: the images beyond image_max (up to
far_max) enter with the kernel's large-D asymptote (Dion et al., Eq. 17 of
their paper; the sums over repeated cells of Sec. 7), folded into the
lattice sum T(d) = sum_L |d - L|^-6 per pair.

* T against a plain loop over explicit Cartesian lattice vectors;
* the shell identity: when every pair of the images beyond image_max has
  D >= D_max, the table-and-asymptote sum over images up to far_max equals
  the sum up to image_max plus the far shell, for the energies and for
  dE/dn (the far terms' q-derivatives and their path through the adjoint),
  on orthorhombic and skew cells, periodic in one, two or three axes;
* dE/dn against central differences of the energy (kink-free table);
* the r^-6 tail: the shell beyond far_max shrinks like far_max^-4 on a
  two-dimensional lattice;
* argument checks (no distance cut, far_max >= image_max)."""
import itertools
import math

import numpy as np
import pytest

import vdw_workloads as W

CELL = ((2.8, 0.0, 0.0), (1.1, 2.6, 0.0), (0.4, -0.3, 2.9))


def _bilinear_table(oracle, nD, nS, Dmax, c):
    tp = oracle.table_params(n_D=nD, n_sigma=nS, D_max=Dmax)
    Dk = np.arange(nD) * Dmax / (nD - 1)
    sl = np.arange(nS) / (nS - 1)
    return tp, c[0] + c[1] * Dk[:, None] + c[2] * sl[None, :] + c[3] * Dk[:, None] * sl[None, :]


def _grid(oracle, wl):
    if wl.cell is not None:
        return oracle.grid_of_cell(wl.n, wl.cell, wl.periodic)
    return oracle.Grid(wl.n, wl.h, wl.periodic)


@pytest.mark.parametrize("periodic,image_max,far_max", [((1, 1, 0), (1, 1, 0), (3, 4, 0)),
                                                        ((1, 0, 1), (0, 0, 1), (2, 0, 2)),
                                                        ((1, 1, 1), (1, 0, 1), (2, 1, 2))])
def test_far_T_against_explicit_lattice(oracle, periodic, image_max, far_max):
    """T(d) equals a plain loop over the Cartesian vectors of the shell."""
    g = oracle.grid_of_cell((5, 4, 3), CELL, periodic)
    C = np.asarray(CELL)  # rows: lattice vectors (n_a steps each)
    rng = np.random.default_rng(1)
    ds = rng.integers(-4, 5, size=(6, 3)) % np.array([5, 4, 3])
    ds = np.vstack([ds, [[0, 0, 0]], [[-4, 3, -2]]])
    got = oracle.far_T(g, image_max, far_max, ds)
    rng_a = [range(-far_max[a], far_max[a] + 1) if periodic[a] else range(1) for a in range(3)]
    for d, t in zip(ds, got):
        r0 = d @ g.steps
        s = 0.0
        for m in itertools.product(*rng_a):
            if all(abs(m[a]) <= (image_max[a] if periodic[a] else 0) for a in range(3)):
                continue
            L = np.asarray(m, dtype=float) @ C
            s += 1.0 / np.linalg.norm(r0 - L) ** 6
        assert t == pytest.approx(s, rel=1e-13)


CASES = [
    # (periodic, cell, near image_max, far image_max)
    ((1, 1, 0), None, (1, 1, 0), (3, 3, 0)),
    ((1, 0, 0), None, (0, 0, 0), (4, 0, 0)),
    ((1, 1, 1), CELL, (1, 1, 1), (2, 2, 2)),
    ((1, 1, 0), CELL, (0, 1, 0), (2, 3, 0)),
]


def _workload(case, seed):
    periodic, cell, _, _ = case
    if cell is None:
        return W.random_small(n=(5, 4, 6), h=(0.5, 0.6, 0.45), periodic=periodic, seed=seed, n_cut=1e-4)
    return W.random_skew(n=(5, 4, 3), cell=cell, periodic=periodic, seed=seed, n_cut=1e-4)


def _min_far_D(oracle, g, wl, image_max, far_max):
    """Smallest D over the pairs of the images beyond image_max (up to far_max)."""
    qd = oracle.compute_q0(g, wl.rho, wl.n_cut)
    idx, ix, iy, iz = oracle._points(g, qd["keep"])
    q = qd["q0"][idx]
    P = np.stack([ix, iy, iz], 1).astype(float)
    rng_a = [range(-far_max[a], far_max[a] + 1) if g.periodic[a] else range(1) for a in range(3)]
    dmin = np.inf
    for m in itertools.product(*rng_a):
        if all(abs(m[a]) <= (image_max[a] if g.periodic[a] else 0) for a in range(3)):
            continue
        sh = np.asarray(m) * np.asarray(g.n)
        d = (P[:, None, :] - P[None, :, :] - sh) @ g.steps
        r = np.linalg.norm(d, axis=2)
        dmin = min(dmin, float(np.min(0.5 * (q[:, None] + q[None, :]) * r)))
    return dmin


@pytest.mark.parametrize("c", range(len(CASES)))
def test_shell_identity(oracle, c):
    """With D_max below every D of the shell, the near sum up to far_max is
    the near sum up to image_max plus the far shell: energies and dE/dn."""
    periodic, cell, near, far = CASES[c]
    wl = _workload(CASES[c], 30 + c)
    g = _grid(oracle, wl)
    # D_max below every D of the shell (the premise), 1 or less
    Dmax = min(1.0, 0.9 * _min_far_D(oracle, g, wl, near, far))
    tp, tab = _bilinear_table(oracle, 9, 5, Dmax, (0.3, -0.2, 0.9, 0.1))
    full = oracle.evaluate(g, wl.rho, tab, tp, wl.n_cut, far, potential=True)
    split = oracle.evaluate(g, wl.rho, tab, tp, wl.n_cut, near, potential=True, far_max=far)
    assert split.E_pair0 == pytest.approx(full.E_pair0, rel=1e-14)
    assert split.E_self == pytest.approx(full.E_self, rel=1e-14)
    assert split.E_pairL == pytest.approx(full.E_pairL, rel=1e-12)
    assert np.abs(split.dEdn - full.dEdn).max() <= 1e-11 * np.abs(full.dEdn).max()
    # the far shell is not negligible here (the identity is not vacuous)
    base = oracle.evaluate(g, wl.rho, tab, tp, wl.n_cut, near)
    assert abs(split.E_pairL - base.E_pairL) > 1e-3 * abs(full.E_pairL)


def test_shell_identity_between_two_near_ranges(oracle):
    """near(M1) + far(M1 -> F) = near(M2) + far(M2 -> F) for M1 < M2 < F."""
    case = CASES[0]
    wl = _workload(case, 41)
    g = _grid(oracle, wl)
    tp, tab = _bilinear_table(oracle, 9, 5, 1.0, (0.3, -0.2, 0.9, 0.1))
    assert _min_far_D(oracle, g, wl, (1, 1, 0), (4, 4, 0)) >= 1.0 + 1e-9
    a = oracle.evaluate(g, wl.rho, tab, tp, wl.n_cut, (1, 1, 0), potential=True, far_max=(4, 4, 0))
    b = oracle.evaluate(g, wl.rho, tab, tp, wl.n_cut, (2, 3, 0), potential=True, far_max=(4, 4, 0))
    assert a.E == pytest.approx(b.E, rel=1e-13)
    assert np.abs(a.dEdn - b.dEdn).max() <= 1e-11 * np.abs(a.dEdn).max()


@pytest.mark.parametrize("c", [0, 2])
def test_far_adjoint_against_central_differences(oracle, c):
    """dE/dn with the far shell (kink-free table, no pair reaches D_max in
    the near images) equals central differences of the energy."""
    periodic, cell, near, far = CASES[c]
    wl = _workload(CASES[c], 50 + c)
    g = _grid(oracle, wl)
    tp, tab = _bilinear_table(oracle, 9, 5, 400.0, (0.3, -0.1 * 2.5 / 400.0, 1.9, 0.05 * 2.5 / 400.0))
    rho = wl.rho.reshape(-1).copy()
    res = oracle.evaluate(g, rho, tab, tp, wl.n_cut, near, potential=True, far_max=far)
    rng = np.random.default_rng(3)
    for k in rng.choice(np.flatnonzero(rho >= 2 * wl.n_cut), 5, replace=False):
        eps = 2e-5 * rho[k]
        rp = rho.copy()
        rp[k] += eps
        rm = rho.copy()
        rm[k] -= eps
        ep = oracle.evaluate(g, rp, tab, tp, wl.n_cut, near, far_max=far).E
        em = oracle.evaluate(g, rm, tab, tp, wl.n_cut, near, far_max=far).E
        assert (ep - em) / (2 * eps) == pytest.approx(res.dEdn[k], rel=2e-6), k


def test_far_shell_tail_decay(oracle):
    """On a two-dimensional lattice the shell beyond F holds about 1/F^4 of
    the r^-6 sum: doubling F cuts the remainder by about 16."""
    wl = _workload(CASES[0], 60)
    g = _grid(oracle, wl)
    tp, tab = _bilinear_table(oracle, 9, 5, 1.0, (0.3, -0.2, 0.9, 0.1))
    E = {F: oracle.evaluate(g, wl.rho, tab, tp, wl.n_cut, (1, 1, 0), far_max=(F, F, 0)).E_pairL for F in (4, 8, 16)}
    r = (E[4] - E[8]) / (E[8] - E[16])
    assert 10.0 < r < 24.0
    assert E[4] > E[8] > E[16]  # every far term is negative (-C / ...)


def test_far_arguments(oracle):
    wl = _workload(CASES[0], 70)
    g = _grid(oracle, wl)
    tp, tab = _bilinear_table(oracle, 9, 5, 1.0, (0.3, -0.2, 0.9, 0.1))
    with pytest.raises(ValueError):
        oracle.evaluate(g, wl.rho, tab, tp, wl.n_cut, (1, 1, 0), r_cut=5.0, far_max=(3, 3, 0))
    with pytest.raises(ValueError):
        oracle.evaluate(g, wl.rho, tab, tp, wl.n_cut, (2, 1, 0), far_max=(1, 3, 0))
    # far_max on a non-periodic axis alone selects nothing
    a = oracle.evaluate(g, wl.rho, tab, tp, wl.n_cut, (1, 1, 0), far_max=(0, 0, 5))
    b = oracle.evaluate(g, wl.rho, tab, tp, wl.n_cut, (1, 1, 0))
    assert a.E == b.E
    assert math.isfinite(a.E)


def test_far_T_square_lattice_closed_form(oracle):
    """A point and all its images on a square lattice of side L: the r^-6
    lattice sum is 4 zeta(3) beta(3) / L^6 (zeta(3) Apery's constant,
    beta(3) = pi^3 / 32); the shell out to 100 rings misses less than 1e-8
    of it.  On a rectangular lattice of sides L, 2L the sum splits into the
    two axes' closed forms (2 zeta(6) / L^6 + 2 zeta(6) / (2L)^6) plus the
    off-axis terms, checked here only for its axis part being a lower
    bound."""
    g = oracle.Grid((4, 4, 3), (0.5, 0.5, 0.5), (1, 1, 0))
    L = 2.0
    zeta3 = 1.2020569031595942
    beta3 = math.pi ** 3 / 32.0
    T0 = float(oracle.far_T(g, (0, 0, 0), (100, 100, 0), [[0, 0, 0]])[0])
    assert T0 == pytest.approx(4.0 * zeta3 * beta3 / L ** 6, rel=1e-8)
    rect = oracle.Grid((4, 8, 3), (0.5, 0.5, 0.5), (1, 1, 0))
    zeta6 = math.pi ** 6 / 945.0
    T1 = float(oracle.far_T(rect, (0, 0, 0), (100, 100, 0), [[0, 0, 0]])[0])
    assert T1 > 2.0 * zeta6 / L ** 6 + 2.0 * zeta6 / (2 * L) ** 6
    # one axis only: the chain sum 2 zeta(6) / L^6
    chain = oracle.Grid((4, 4, 3), (0.5, 0.5, 0.5), (1, 0, 0))
    T2 = float(oracle.far_T(chain, (0, 0, 0), (2000, 0, 0), [[0, 0, 0]])[0])
    assert T2 == pytest.approx(2.0 * zeta6 / L ** 6, rel=1e-12)
