"""Pins of the C1 interpolant (interp = 1): cubic in D through the
Catmull-Rom form of each sigma column, linear in sigma.  It reproduces the
table at the nodes and quadratics in D exactly between interior nodes, its
D-derivative is continuous at the nodes (the bilinear one jumps), its
derivatives match central differences, and the kinks it removes tighten the
agreement of the adjoint with central differences of the energy on the Dion
table."""
import numpy as np
import pytest

import vdw_workloads as W

CHEAP_RULE = dict(gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)


def _quad_table(oracle, nD=12, nS=5, Dmax=11.0):
    tp = oracle.table_params(n_D=nD, n_sigma=nS, D_max=Dmax, interp=1)
    Dk = np.arange(nD) * Dmax / (nD - 1)
    sl = np.arange(nS) / (nS - 1)
    f = lambda D, s: 0.4 - 0.3 * D + 0.05 * D * D + s * (1.2 + 0.1 * D - 0.02 * D * D)  # noqa: E731
    return tp, f(Dk[:, None], sl[None, :]), f


def test_nodes_and_quadratics(oracle):
    tp, tab, f = _quad_table(oracle)
    dD = tp.D_max / (tp.n_D - 1)
    for k in range(tp.n_D - 1):
        for l in range(tp.n_sigma):
            v, _, _ = oracle.table_interp(tab, tp, k * dD, l / (tp.n_sigma - 1))
            assert v == pytest.approx(tab[k, l], abs=1e-13)
    rng = np.random.default_rng(0)
    for D, s in zip(rng.uniform(dD, tp.D_max - 2 * dD, 60), rng.uniform(0, 1, 60)):  # interior intervals
        v, gD, gS = oracle.table_interp(tab, tp, D, s)
        assert v == pytest.approx(f(D, s), abs=1e-12)
        assert gD == pytest.approx(-0.3 + 0.1 * D + s * (0.1 - 0.04 * D), abs=1e-11)
        assert gS == pytest.approx(1.2 + 0.1 * D - 0.02 * D * D, abs=1e-11)


def test_c1_in_D_and_derivatives(oracle, table_cache):
    tp0, tab = table_cache(n_D=256, n_sigma=16, D_max=12.0, **CHEAP_RULE)
    tp = oracle.table_params(n_D=256, n_sigma=16, D_max=12.0, interp=1, **CHEAP_RULE)
    dD = tp.D_max / (tp.n_D - 1)
    e = 1e-9
    for k in (1, 7, 40, 200):
        D = k * dD
        for s in (0.0, 0.37):
            _, gl, _ = oracle.table_interp(tab, tp, D - e, s)
            _, gr, _ = oracle.table_interp(tab, tp, D + e, s)
            assert gl == pytest.approx(gr, rel=1e-6, abs=1e-9)  # continuous
            _, bl, _ = oracle.table_interp(tab, tp0, D - e, s)
            _, br, _ = oracle.table_interp(tab, tp0, D + e, s)
            if k == 7:  # (rows 0, 1, 2 are collinear by construction, so node 1 has no kink)
                assert abs(bl - br) > 1e-3 * max(abs(bl), 1e-3)  # the bilinear slope jumps
    for D, s in ((0.33, 0.21), (5.01, 0.713), (11.3, 0.051)):  # off the sigma nodes (kinks in sigma remain)
        h = 1e-6
        vp, _, _ = oracle.table_interp(tab, tp, D + h, s)
        vm, _, _ = oracle.table_interp(tab, tp, D - h, s)
        _, gD, gS = oracle.table_interp(tab, tp, D, s)
        assert (vp - vm) / (2 * h) == pytest.approx(gD, rel=1e-6)
        sp, _, _ = oracle.table_interp(tab, tp, D, s + h)
        sm, _, _ = oracle.table_interp(tab, tp, D, s - h)
        assert (sp - sm) / (2 * h) == pytest.approx(gS, rel=1e-6)


def test_adjoint_closer_to_central_differences(oracle, table_cache):
    """Central differences of the energy with the step of the full-size
    check (1e-4 n_k) straddle kinks of the bilinear interpolant (reading
    R13: up to 1e-3 away from the exact adjoint here); without the D kinks
    they agree to 1e-7 (the sigma kinks remain)."""
    _, tab = table_cache(n_D=256, n_sigma=16, D_max=12.0, **CHEAP_RULE)
    wl = W.random_small(n=(6, 6, 5), h=(0.4, 0.4, 0.45), seed=5, n_cut=4e-3)
    g = oracle.Grid(wl.n, wl.h, wl.periodic)
    rho = wl.rho.reshape(-1)
    ks = np.random.default_rng(1).choice(np.flatnonzero(rho >= 2 * wl.n_cut), 12, replace=False)
    err = {}
    for interp in (0, 1):
        tp = oracle.table_params(n_D=256, n_sigma=16, D_max=12.0, interp=interp, **CHEAP_RULE)
        res = oracle.evaluate(g, rho, tab, tp, wl.n_cut, potential=True)
        worst = 0.0
        for k in ks:
            eps = 1e-4 * rho[k]
            fd = oracle.local_energy_change(g, rho, k, eps, tab, tp, wl.n_cut) / (2 * eps)
            worst = max(worst, abs(fd - res.dEdn[k]) / abs(res.dEdn[k]))
        err[interp] = worst
    assert err[0] > 1e-4 and err[1] < 1e-6
