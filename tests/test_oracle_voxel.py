"""Pins of the voxel on-site term (self_term = 2): the double average of the
kernel at delta = 0 over the grid cell, E_self = 1/2 dV^2 sum n_i^2
Phi_V(q_i), the finite-volume counterpart of the paper's unexplained phi0
step (App. A).  The rule's weights integrate the tent to one; a constant
kernel averages to itself; a kernel linear in D averages to the mean
distance of two points in the cell (Robbins' constant for a cube); the
q-derivative; the rule converges; rotations and a sheared description of the
same cell change nothing; and the adjoint with this term equals central
differences for a kink-free kernel."""
import math

import numpy as np
import pytest

import vdw_workloads as W

ROBBINS = 0.66170718226717623515  # mean distance of two uniform points in the unit cube


def _linear_table(oracle, a, b, Dmax=1e4, nD=9, nS=3):
    tp = oracle.table_params(n_D=nD, n_sigma=nS, D_max=Dmax)
    Dk = np.arange(nD) * Dmax / (nD - 1)
    return tp, np.repeat((a + b * Dk)[:, None], nS, axis=1)


def test_constant_kernel(oracle):
    tp, tab = _linear_table(oracle, 0.37, 0.0)
    E = np.diag([0.3, 0.45, 0.5])
    v, d = oracle.self_voxel(2.0, E, tab, tp)
    assert v == pytest.approx(0.37, rel=1e-14) and abs(d) < 1e-14


@pytest.mark.parametrize("g,tol", [(8, 2e-4), (24, 2e-6)])
def test_linear_kernel_gives_mean_distance(oracle, g, tol):
    """phi~ = a + b D: Phi_V(q) = a + b q <|r - r'|>, and for a cube of side h
    the mean distance is h times Robbins' constant; d Phi_V/dq = b <|r - r'|>."""
    a, b, h, q = 0.2, -0.03, 0.4, 1.7
    tp, tab = _linear_table(oracle, a, b)
    v, d = oracle.self_voxel(q, np.diag([h, h, h]), tab, tp, g=g)
    assert (v - a) / (b * q * h) == pytest.approx(ROBBINS, rel=tol)
    assert d / (b * h) == pytest.approx(ROBBINS, rel=tol)


def test_rule_converges_on_the_dion_table(oracle, table_cache):
    tp, tab = table_cache(n_D=256, n_sigma=16, D_max=12.0, gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)
    E = np.diag([0.25, 0.3, 0.35])
    for q in (0.3, 1.5, 6.0):
        v8, _ = oracle.self_voxel(q, E, tab, tp, g=8)
        v32, _ = oracle.self_voxel(q, E, tab, tp, g=32)
        assert v8 == pytest.approx(v32, rel=2e-3), q
    # q-derivative against central differences of the rule itself
    q, e = 1.3, 1e-6
    vp, _ = oracle.self_voxel(q + e, E, tab, tp)
    vm, _ = oracle.self_voxel(q - e, E, tab, tp)
    _, d = oracle.self_voxel(q, E, tab, tp)
    assert (vp - vm) / (2 * e) == pytest.approx(d, rel=1e-6)


def test_rotation_and_shear_invariance(oracle, table_cache):
    """Rotating the cell leaves Phi_V unchanged; so does an inversion (the
    octants are symmetric); a different but equal-shaped description of the
    same parallelepiped (e.g. permuted step vectors) too."""
    tp, tab = table_cache(n_D=256, n_sigma=16, D_max=12.0, gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)
    E = np.array([[0.3, 0.0, 0.0], [0.12, 0.28, 0.0], [0.05, -0.04, 0.33]])
    th = 0.9
    R = np.array([[math.cos(th), 0, math.sin(th)], [0, 1, 0], [-math.sin(th), 0, math.cos(th)]])
    v0, d0 = oracle.self_voxel(1.1, E, tab, tp)
    v1, d1 = oracle.self_voxel(1.1, E @ R.T, tab, tp)
    v2, _ = oracle.self_voxel(1.1, -E, tab, tp)
    v3, _ = oracle.self_voxel(1.1, E[[2, 0, 1]], tab, tp)
    assert v1 == pytest.approx(v0, rel=1e-13) and d1 == pytest.approx(d0, rel=1e-13)
    assert v2 == pytest.approx(v0, rel=1e-13) and v3 == pytest.approx(v0, rel=1e-13)


def test_adjoint_with_voxel_term(oracle):
    nD, nS, Dmax = 9, 5, 400.0
    tp = oracle.table_params(n_D=nD, n_sigma=nS, D_max=Dmax)
    Dk = np.arange(nD) * Dmax / (nD - 1)
    sl = np.arange(nS) / (nS - 1)
    c = (0.3, -0.1 * 2.5 / Dmax, 1.9, 0.05 * 2.5 / Dmax)
    tab = c[0] + c[1] * Dk[:, None] + c[2] * sl[None, :] + c[3] * Dk[:, None] * sl[None, :]
    wl = W.random_skew(periodic=(1, 0, 0), seed=6, n_cut=4e-3, image_max=(1, 0, 0))
    g = oracle.grid_of_cell(wl.n, wl.cell, wl.periodic)
    rho = wl.rho.reshape(-1).copy()
    res = oracle.evaluate(g, rho, tab, tp, wl.n_cut, wl.image_max, 0.0, self_term=2, potential=True)
    assert res.E_self != 0.0
    rng = np.random.default_rng(3)
    for k in rng.choice(np.flatnonzero(rho >= 2 * wl.n_cut), 6, replace=False):
        eps = 2e-5 * rho[k]
        fd = oracle.local_energy_change(g, rho, k, eps, tab, tp, wl.n_cut, wl.image_max, 0.0, self_term=2) / (2 * eps)
        assert fd == pytest.approx(res.dEdn[k], rel=1e-5, abs=1e-10 * np.abs(res.dEdn).max()), k


def test_voxel_table_against_the_rule(oracle, table_cache):
    """self_term = 2 reads Phi_V from its table over ln q (4096 nodes on
    q in [2^-6, 2^7]): the node values are the rule's, between nodes the
    Catmull-Rom cubic in ln q stays within 1e-5 of the largest |Phi_V| of the
    rule (the rule itself is good to ~1e-4, its kinks from the kernel table's
    bilinear form limiting the cubic's accuracy), q outside the range takes
    the rule itself, and dPhi_V/dq is the interpolant's own derivative."""
    tp, tab = table_cache(n_D=256, n_sigma=16, D_max=12.0, gl_points=6, graded_levels=8, kappa=2.0, A0=20.0)
    E = np.diag([0.25, 0.3, 0.35])
    vt = oracle.voxel_table(E, tab, tp)
    n = oracle.VOXEL_TABLE_NODES
    assert len(vt) == n
    xk = oracle.VOXEL_LNQ_LO + np.array([0, 1, 777, n - 2, n - 1]) * (
        (oracle.VOXEL_LNQ_HI - oracle.VOXEL_LNQ_LO) / (n - 1))
    qk = np.exp(xk)
    direct = oracle.self_voxel_many(qk, E, tab, tp)[0]
    assert np.allclose(oracle.voxel_interp(vt, qk, E, tab, tp)[0], direct, rtol=1e-12, atol=0)
    rng = np.random.default_rng(5)
    q = np.exp(rng.uniform(oracle.VOXEL_LNQ_LO, oracle.VOXEL_LNQ_HI, 200))
    got, dgot = oracle.voxel_interp(vt, q, E, tab, tp)
    ref = oracle.self_voxel_many(q, E, tab, tp)[0]
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    eps = 1e-7 * q
    fp = oracle.voxel_interp(vt, q + eps, E, tab, tp)[0]
    fm = oracle.voxel_interp(vt, q - eps, E, tab, tp)[0]
    assert np.allclose((fp - fm) / (2 * eps), dgot, rtol=1e-5, atol=1e-9 * np.abs(dgot).max())
    out = np.array([1e-3, 300.0])
    assert np.array_equal(oracle.voxel_interp(vt, out, E, tab, tp)[0], oracle.self_voxel_many(out, E, tab, tp)[0])
