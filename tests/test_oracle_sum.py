"""Pins of the oracle's interpolated kernel, the double sum of Eq. (2)
(0th cell and periodic images, Sec. 3) and its derivative."""
import math

import numpy as np
import pytest

import vdw_workloads as W
from oracle import brute

C_ASYM = 12.0 * (4.0 * math.pi / 9.0) ** 3
CHEAP_RULE = dict(gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)


def _bilinear_table(oracle, nD=9, nS=5, Dmax=8.0, c=(0.3, -0.7, 1.9, 0.45)):
    tp = oracle.table_params(n_D=nD, n_sigma=nS, D_max=Dmax)
    Dk = np.arange(nD) * Dmax / (nD - 1)
    sl = np.arange(nS) / (nS - 1)
    tab = c[0] + c[1] * Dk[:, None] + c[2] * sl[None, :] + c[3] * Dk[:, None] * sl[None, :]
    return tp, tab


def test_interp_exact_for_bilinear_functions(oracle):
    c = (0.3, -0.7, 1.9, 0.45)
    tp, tab = _bilinear_table(oracle, c=c)
    rng = np.random.default_rng(0)
    for D, s in zip(rng.uniform(0, 7.999, 50), rng.uniform(0, 1, 50)):
        v, dD, dS = oracle.table_interp(tab, tp, D, s)
        assert v == pytest.approx(c[0] + c[1] * D + c[2] * s + c[3] * D * s, abs=1e-13)
        assert dD == pytest.approx(c[1] + c[3] * s, abs=1e-12)
        assert dS == pytest.approx(c[2] + c[3] * D, abs=1e-12)
    # nodes and the sigma = 1 edge
    assert oracle.table_interp(tab, tp, 3.0, 0.5)[0] == pytest.approx(tab[3, 2], abs=1e-14)
    assert oracle.table_interp(tab, tp, 2.0, 1.0)[0] == pytest.approx(tab[2, 4], abs=1e-14)


def test_pair_phi_branches_and_q_derivative(oracle, table_cache):
    tp, tab = table_cache(n_D=128, n_sigma=16, D_max=12.0, **CHEAP_RULE)
    # asymptote branch
    qi, qj, r = 2.0, 0.7, 9.5  # D = 12.825 >= 12
    v, _ = oracle.pair_phi(qi, qj, r, tab, tp)
    d1, d2 = qi * r, qj * r
    assert v == pytest.approx(-C_ASYM / (d1 ** 2 * d2 ** 2 * (d1 ** 2 + d2 ** 2)), rel=1e-14)
    # table branch reproduces the interpolant at (D, delta^2)
    qi, qj, r = 1.3, 0.4, 3.1
    D = 0.5 * (qi + qj) * r
    s = ((qi - qj) / (qi + qj)) ** 2
    assert oracle.pair_phi(qi, qj, r, tab, tp)[0] == pytest.approx(oracle.table_interp(tab, tp, D, s)[0], rel=1e-15)
    # d phi~ / d q_i by central differences, both branches, away from nodes
    for qi, qj, r in [(1.3, 0.4, 3.1), (0.55, 0.9, 1.7), (2.0, 0.7, 9.5), (0.8, 0.8001, 2.2)]:
        e = 1e-7
        fp = oracle.pair_phi(qi + e, qj, r, tab, tp)[0]
        fm = oracle.pair_phi(qi - e, qj, r, tab, tp)[0]
        assert (fp - fm) / (2 * e) == pytest.approx(oracle.pair_phi(qi, qj, r, tab, tp)[1], rel=1e-6, abs=1e-9)
    # symmetric in (q_i, q_j)
    assert oracle.pair_phi(1.3, 0.4, 3.1, tab, tp)[0] == oracle.pair_phi(0.4, 1.3, 3.1, tab, tp)[0]


def _points(oracle, wl):
    g = oracle.Grid(wl.n, wl.h, wl.periodic)
    qd = oracle.compute_q0(g, wl.rho, wl.n_cut)
    idx, ix, iy, iz = oracle._points(g, qd["keep"])
    r = wl.rho.reshape(-1)
    return g, qd, idx, ix, iy, iz, r[idx], qd["q0"][idx]


@pytest.mark.parametrize("periodic,image_max,r_cut", [((0, 0, 0), (0, 0, 0), 0.0),
                                                      ((1, 1, 0), (1, 1, 0), 3.23),
                                                      ((0, 1, 1), (0, 2, 1), 0.0)])
def test_pair_sum_matches_pure_python_brute_force(oracle, table_cache, periodic, image_max, r_cut):
    tp, tab = table_cache(n_D=64, n_sigma=8, D_max=6.0, **CHEAP_RULE)
    wl = W.random_small(n=(6, 5, 4), h=(0.4, 0.45, 0.5), periodic=periodic, seed=7,
                        image_max=image_max, r_cut=r_cut)
    wl.n_cut = float(np.quantile(wl.rho, 0.3))  # drop about 30 % of the points
    g, qd, idx, ix, iy, iz, nS, qS = _points(oracle, wl)
    assert 20 < len(idx) < g.G
    S0c, S0i, _ = oracle.pair_rows(g, ix, iy, iz, nS, qS, tab, tp, image_max, r_cut)
    dV = g.dV
    e0 = 0.5 * dV * dV * float(np.sum(nS * S0c))
    eL = 0.5 * dV * dV * float(np.sum(nS * S0i))
    pts = list(zip(ix.tolist(), iy.tolist(), iz.tolist(), nS.tolist(), qS.tolist()))
    b0, bL = brute.pair_energy(pts, g.h, g.n, periodic, image_max, r_cut, tab.tolist(), tp.D_max, dV)
    assert e0 == pytest.approx(b0, rel=1e-13)
    assert eL == pytest.approx(bL, rel=1e-13, abs=1e-300)
    if any(image_max):
        assert abs(bL) > 0
    # the same energies one image shift at a time: the 0th cell, and the images
    # as twice the sum over one of each pair (m, -m)
    h0 = 0.5 * dV * dV * oracle.image_pair_sum(g, ix, iy, iz, nS, qS, tab, tp, (0, 0, 0), r_cut)
    half = oracle.half_image_shifts(g, image_max)
    full = [m for m in np.ndindex(*(2 * np.asarray(image_max) * np.asarray(periodic) + 1))]
    assert 2 * len(half) + 1 == len(full)
    hL = dV * dV * sum(oracle.image_pair_sum(g, ix, iy, iz, nS, qS, tab, tp, m, r_cut) for m in half)
    assert h0 == pytest.approx(b0, rel=1e-13)
    assert hL == pytest.approx(bL, rel=1e-13, abs=1e-300)


def test_pair_sum_constant_table_closed_form(oracle):
    """phi~ = c on every node: E_pair = 1/2 dV^2 c sum_{i != j} n_i n_j while all D < D_max."""
    tp = oracle.table_params(n_D=4, n_sigma=3, D_max=1e4)
    tab = np.full((4, 3), 0.37)
    wl = W.random_small(seed=3)
    res = oracle.evaluate(oracle.Grid(wl.n, wl.h, wl.periodic), wl.rho, tab, tp, wl.n_cut, self_term=False)
    n = wl.rho.reshape(-1)
    n = n[n >= wl.n_cut]
    ref = 0.5 * wl.dV ** 2 * 0.37 * (n.sum() ** 2 - (n * n).sum())
    assert res.E_pair0 == pytest.approx(ref, rel=1e-13)


def test_translation_invariance_isolated(oracle, table_cache):
    tp, tab = table_cache(n_D=128, n_sigma=16, D_max=12.0, **CHEAP_RULE)
    n, h = (22, 20, 22), (0.4, 0.4, 0.4)

    def dens(shift):
        c = np.array([2.8, 2.8, 2.8]) + np.array(shift) * 0.4
        return (W.atom_density(n, h, tuple(c), 3.0, (1.5, 3.0), (0.6, 0.4))
                + W.atom_density(n, h, tuple(c + [1.6, 0.8, 0.4]), 2.0, (2.0,), (1.0,)))

    cut = 5e-2
    e = []
    for s in [(0, 0, 0), (3, 2, 4)]:
        rho = dens(s)
        keep = rho >= cut
        zz, yy, xx = np.nonzero(keep)
        assert xx.min() >= 2 and yy.min() >= 2 and zz.min() >= 2
        assert xx.max() <= n[0] - 3 and yy.max() <= n[1] - 3 and zz.max() <= n[2] - 3
        e.append(oracle.evaluate(oracle.Grid(n, h), rho, tab, tp, cut).E)
    assert e[0] == pytest.approx(e[1], rel=1e-12)


def test_translation_invariance_slab(oracle, table_cache):
    """Periodic in x and y: an in-plane grid shift with wrap-around leaves E
    unchanged when the image set holds every L within r_cut of any pair."""
    tp, tab = table_cache(n_D=128, n_sigma=16, D_max=12.0, **CHEAP_RULE)
    n, h = (6, 6, 10), (0.5, 0.5, 0.5)
    rng = np.random.default_rng(11)
    base = 0.05 + rng.uniform(0, 0.02, size=(n[2], n[1], n[0]))
    base *= np.exp(-((np.arange(n[2]) - 4.5) * 0.5) ** 2)[:, None, None]
    cut = 1e-3
    Lmax = (n[0] - 1) * h[0]
    r_cut = 4.0
    m = math.ceil((r_cut + Lmax) / (n[0] * h[0]))
    e = []
    for sx, sy in [(0, 0), (2, 5)]:
        rho = np.roll(np.roll(base, sx, axis=2), sy, axis=1)
        g = oracle.Grid(n, h, (1, 1, 0))
        e.append(oracle.evaluate(g, rho, tab, tp, cut, image_max=(m, m, 0), r_cut=r_cut).E)
    assert e[0] == pytest.approx(e[1], rel=1e-12)


def test_c6_identity_far_apart(oracle, table_cache):
    """Two densities whose every cross pair has D >= D_max interact only through
    the asymptote: E(A+B) - E(A) - E(B) = -C dV^2 sum_{A x B} n_i n_j /
    (r^6 q_i^2 q_j^2 (q_i^2 + q_j^2))."""
    tp, tab = table_cache(n_D=64, n_sigma=8, D_max=4.0, **CHEAP_RULE)
    n, h = (30, 10, 10), (0.5, 0.5, 0.5)
    Z, Y, X = np.meshgrid(np.arange(10) * 0.5, np.arange(10) * 0.5, np.arange(30) * 0.5, indexing="ij")

    def blob(cx, Zc):
        r = np.sqrt((X - cx) ** 2 + (Y - 2.25) ** 2 + (Z - 2.25) ** 2)
        return np.where(r < 1.6, Zc * np.exp(-1.2 * r), 0.0)

    A, B = blob(2.25, 2.0), blob(12.25, 1.5)
    cut = 0.05
    g = oracle.Grid(n, h)
    eA = oracle.evaluate(g, A, tab, tp, cut)
    eB = oracle.evaluate(g, B, tab, tp, cut)
    eAB = oracle.evaluate(g, A + B, tab, tp, cut)
    qa, qb = eA.q0["q0"], eB.q0["q0"]
    ia = np.flatnonzero(A.ravel() >= cut)
    ib = np.flatnonzero(B.ravel() >= cut)

    def xyz(i):
        return np.stack([(i % 30) * 0.5, (i // 30 % 10) * 0.5, (i // 300) * 0.5], 1)

    rr = np.linalg.norm(xyz(ia)[:, None, :] - xyz(ib)[None, :, :], axis=2)
    Qa, Qb = qa[ia][:, None], qb[ib][None, :]
    assert (0.5 * (Qa + Qb) * rr).min() >= tp.D_max
    cross = -C_ASYM * (A.ravel()[ia][:, None] * B.ravel()[ib][None, :]
                       / (rr ** 6 * Qa ** 2 * Qb ** 2 * (Qa ** 2 + Qb ** 2))).sum() * g.dV ** 2
    assert eAB.E - eA.E - eB.E == pytest.approx(cross, rel=1e-10)
    assert cross < 0


ADJ_CASES = [((0, 0, 0), (0, 0, 0), 0.0), ((1, 0, 1), (2, 0, 1), 3.0), ((1, 1, 0), (1, 1, 0), 0.0)]


def _adjoint_case(oracle, tab, tp, periodic, image_max, r_cut, eps_rel, tol):
    wl = W.random_small(n=(6, 6, 5), h=(0.4, 0.4, 0.45), periodic=periodic, seed=5, n_cut=4e-3,
                        image_max=image_max, r_cut=r_cut)
    g = oracle.Grid(wl.n, wl.h, wl.periodic)
    rho = wl.rho.reshape(-1).copy()
    dropped = g.n[0] * 2 + 3
    rho[dropped] = 0.5 * wl.n_cut  # dropped, but inside a retained point's stencil
    res = oracle.evaluate(g, rho, tab, tp, wl.n_cut, image_max, r_cut, potential=True)
    rng = np.random.default_rng(1)
    ks = list(rng.choice(np.flatnonzero(rho >= 2 * wl.n_cut), 10, replace=False)) + [dropped]
    for k in ks:
        eps = eps_rel * rho[k]
        fd = oracle.local_energy_change(g, rho, k, eps, tab, tp, wl.n_cut, image_max, r_cut) / (2 * eps)
        assert fd == pytest.approx(res.dEdn[k], rel=tol, abs=1e-10 * np.abs(res.dEdn).max()), k
    assert res.dEdn[dropped] != 0.0


@pytest.mark.parametrize("Dmax", [400.0, 1e-3])
@pytest.mark.parametrize("periodic,image_max,r_cut", ADJ_CASES)
def test_adjoint_exact_for_kink_free_kernel(oracle, periodic, image_max, r_cut, Dmax):
    """With a table bilinear in (D, sigma) the interpolant has no kinks, so
    dE/dn_k from the adjoint formulas must equal central differences of E
    (recomputed over the rows the perturbation touches) to rounding.  D_max =
    400 keeps every pair on the table branch, D_max = 1e-3 puts every pair on
    the (smooth) asymptote branch; the jump between the two at D_max is a true
    discontinuity of the kernel and is left out."""
    tp, tab = _bilinear_table(oracle, nD=9, nS=5, Dmax=Dmax, c=(0.3, -0.1 * 2.5 / Dmax, 1.9, 0.05 * 2.5 / Dmax))
    _adjoint_case(oracle, tab, tp, periodic, image_max, r_cut, 2e-5, 1e-5)


@pytest.mark.parametrize("periodic,image_max,r_cut", ADJ_CASES)
def test_adjoint_matches_local_difference_physical_table(oracle, table_cache, periodic, image_max, r_cut):
    """Same with the Dion table: central differences straddle bilinear kinks of
    the interpolant, which bounds the agreement (here 2e-4 relative)."""
    tp, tab = table_cache(n_D=256, n_sigma=16, D_max=12.0, **CHEAP_RULE)
    _adjoint_case(oracle, tab, tp, periodic, image_max, r_cut, 1e-6, 2e-4)


def test_self_term_sphere_average(oracle):
    """For phi = c - b ln D the mean of phi(q r) over a ball of volume dV is
    phi(q rho_s): check rho_s by integrating ln r over the ball."""
    dV = 0.37
    R = (3 * dV / (4 * math.pi)) ** (1 / 3)
    from scipy.integrate import quad

    mean_ln = quad(lambda r: 3 * r * r / R ** 3 * math.log(r), 0.0, R, epsabs=1e-15, epsrel=1e-14)[0]
    assert math.log(oracle.self_radius(dV)) == pytest.approx(mean_ln, rel=1e-12)


def test_cutoff_convergence(oracle, table_cache):
    """E converges as the density cut-off decreases (the cut-off 'does not
    reduce the accuracy', Sec. 3)."""
    tp, tab = table_cache(n_D=128, n_sigma=16, D_max=12.0, **CHEAP_RULE)
    wl = W.random_small(n=(8, 8, 8), h=(0.5, 0.5, 0.5), seed=2)
    g = oracle.Grid(wl.n, wl.h)
    rho = wl.rho * np.exp(-np.linspace(0, 6, 8))[None, None, :]
    E = [oracle.evaluate(g, rho, tab, tp, c).E for c in (1e-2, 1e-3, 1e-4, 1e-5)]
    d = np.abs(np.diff(E))
    assert d[1] < d[0] and d[2] < d[1]
