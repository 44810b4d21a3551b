"""Pins of the oracle's O(grid) steps: finite-difference gradient (Sec. 3),
Perdew-Wang 1992 LDA correlation and q0 of Dion et al."""
import math

import numpy as np
import pytest


def test_gradient_exact_on_quadratics(oracle):
    """Second-order central and one-sided differences are exact on quadratics,
    interior and faces of non-periodic axes."""
    g = oracle.Grid((7, 5, 6), (0.3, 0.45, 0.2), (0, 0, 0))
    nx, ny, nz = g.n
    z, y, x = np.meshgrid(np.arange(nz) * g.h[2], np.arange(ny) * g.h[1], np.arange(nx) * g.h[0], indexing="ij")
    f = 1.5 + 0.3 * x - 2.0 * y + 0.7 * z + 0.9 * x * x - 0.4 * y * y + 1.1 * z * z + 0.5 * x * y - 0.8 * y * z + 0.25 * x * z
    gx, gy, gz = oracle.gradient(g, f)
    ex = 0.3 + 1.8 * x + 0.5 * y + 0.25 * z
    ey = -2.0 - 0.8 * y + 0.5 * x - 0.8 * z
    ez = 0.7 + 2.2 * z - 0.8 * y + 0.25 * x
    assert np.abs(gx - ex.ravel()).max() < 1e-12
    assert np.abs(gy - ey.ravel()).max() < 1e-12
    assert np.abs(gz - ez.ravel()).max() < 1e-12


def test_gradient_periodic_axis_closed_form(oracle):
    """On a periodic axis the central difference of sin(k x) is exactly
    sin(k h)/h cos(k x) (wrap-around included)."""
    n = (12, 4, 3)
    h = (0.5, 0.3, 0.4)
    g = oracle.Grid(n, h, (1, 0, 0))
    L = n[0] * h[0]
    k = 2 * math.pi * 2 / L
    x = np.arange(n[0]) * h[0]
    f = np.broadcast_to(np.sin(k * x)[None, None, :], (n[2], n[1], n[0]))
    gx, gy, gz = oracle.gradient(g, f)
    exp = np.broadcast_to((math.sin(k * h[0]) / h[0] * np.cos(k * x))[None, None, :], f.shape).ravel()
    assert np.abs(gx - exp).max() < 1e-13
    assert np.abs(gy).max() < 1e-13 and np.abs(gz).max() < 1e-13


def test_pw92_limits(oracle):
    """High density: eps_c - A ln r_s -> 2A ln(2 A beta1) = -0.046644 (the c1 of
    the PW92 fit); low density: r_s eps_c -> -alpha1 / beta4 = -0.43352."""
    A = 0.031091
    ec, _ = oracle.pw92_ec(np.array([1e-10]))
    assert ec[0] - A * math.log(1e-10) == pytest.approx(-0.046644, abs=2e-5)
    # (the next term is smaller by beta3 / (beta4 sqrt(r_s)))
    ec, _ = oracle.pw92_ec(np.array([1e12]))
    assert 1e12 * ec[0] == pytest.approx(-0.21370 / 0.49294, rel=1e-5)
    # the logarithm stays accurate at very low density (log1p, not log(1 + x))
    ec, _ = oracle.pw92_ec(np.array([1e8]))
    assert 1e8 * ec[0] == pytest.approx(-0.21370 / 0.49294, rel=1e-3)


def test_pw92_derivative_fd(oracle):
    for rs in (0.01, 0.3, 1.0, 4.0, 30.0, 500.0):
        e = 1e-6 * rs
        ep, _ = oracle.pw92_ec(np.array([rs + e]))
        em, _ = oracle.pw92_ec(np.array([rs - e]))
        _, d = oracle.pw92_ec(np.array([rs]))
        assert (ep[0] - em[0]) / (2 * e) == pytest.approx(d[0], rel=1e-7)


def test_q0_matches_definition_via_s(oracle):
    """The simplified q0 equals the definition -(4 pi/3) eps_xc^0 with
    eps_xc^0 = eps_x + eps_c - eps_x (Z_ab/9) s^2, eps_x = -3 k_F/(4 pi),
    s = |grad n| / (2 k_F n)."""
    n = np.array([1e-5, 3e-3, 0.2, 1.0, 40.0, 5e3])
    g = np.array([1e-9, 2e-5, 0.3, 0.0, 900.0, 1e8])
    q, _, _ = oracle.q0_of(n, g)
    kF = (3 * math.pi ** 2 * n) ** (1 / 3)
    rs = (3 / (4 * math.pi * n)) ** (1 / 3)
    ec, _ = oracle.pw92_ec(rs)
    ex = -3 * kF / (4 * math.pi)
    s2 = g / (2 * kF * n) ** 2
    ref = -(4 * math.pi / 3) * (ex + ec - ex * (-0.8491 / 9) * s2)
    assert np.allclose(q, ref, rtol=1e-13, atol=0)


def test_q0_derivatives_fd(oracle):
    n = np.array([2e-5, 1e-3, 0.05, 2.0, 300.0])
    g = np.array([1e-8, 1e-5, 0.02, 5.0, 1e5])
    _, dn, dg = oracle.q0_of(n, g)
    e = 1e-6
    qp, _, _ = oracle.q0_of(n * (1 + e), g)
    qm, _, _ = oracle.q0_of(n * (1 - e), g)
    assert np.allclose((qp - qm) / (2 * e * n), dn, rtol=1e-7)
    qp, _, _ = oracle.q0_of(n, g * (1 + e))
    qm, _, _ = oracle.q0_of(n, g * (1 - e))
    assert np.allclose((qp - qm) / (2 * e * g), dg, rtol=1e-7)


def test_compute_q0_zero_below_cut(oracle):
    g = oracle.Grid((4, 4, 4), (0.5, 0.5, 0.5))
    rho = np.full((4, 4, 4), 1e-3)
    rho[0, 0, 0] = 5e-6
    rho[1, 2, 3] = -1e-6
    out = oracle.compute_q0(g, rho, 1e-5)
    assert out["q0"][0] == 0 and out["dq_dn"][0] == 0 and out["dq_dg"][0] == 0
    assert out["q0"][3 + 4 * (2 + 4 * 1)] == 0
    assert out["keep"].sum() == 62
    assert np.all(out["q0"][out["keep"]] > 0)
