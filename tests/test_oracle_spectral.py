"""Pins of the oracle's Fourier-derivative gradient (the paper computes the
gradient by FFT, Sec. 3 and the sample run's timing, App. A): the operator
built by FFT equals the textbook closed form (cotangent for even, cosecant
for odd N), is antisymmetric and annihilates constants; trigonometric
polynomials below the Nyquist frequency are differentiated exactly; the
Nyquist mode of an even N has derivative zero; the FFT and operator forms
agree on mixed periodic / open and on skew grids; and the adjoint of the
whole energy equals central differences for a kink-free kernel."""
import math

import numpy as np
import pytest

import vdw_workloads as W


@pytest.mark.parametrize("N", [8, 9, 12, 15])
def test_operator_closed_form(oracle, N):
    h = 0.37
    D = oracle.spectral_matrix_1d(N, h).toarray()
    j = np.arange(N)
    m = j[:, None] - j[None, :]
    with np.errstate(divide="ignore"):
        x = m * math.pi / N
        if N % 2 == 0:
            ref = 0.5 * (-1.0) ** m / np.tan(x)
        else:
            ref = 0.5 * (-1.0) ** m / np.sin(x)
    ref[m == 0] = 0.0
    ref *= 2 * math.pi / (N * h)
    assert np.abs(D - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(D + D.T).max() < 1e-13 * np.abs(D).max()
    assert np.abs(D @ np.ones(N)).max() < 1e-12


def test_trig_polynomials_exact_and_nyquist(oracle):
    """Periodic x (N = 12, even) and y (N = 9, odd), open z: below the
    Nyquist frequency the derivative is exact; cos(pi x / h) on the even
    axis (the Nyquist mode) has derivative zero."""
    n, h = (12, 9, 7), (0.4, 0.5, 0.3)
    g = oracle.Grid(n, h, (1, 1, 0), gradient="spectral")
    L = [n[a] * h[a] for a in range(3)]
    z, y, x = np.meshgrid(np.arange(n[2]) * h[2], np.arange(n[1]) * h[1], np.arange(n[0]) * h[0], indexing="ij")
    kx, ky = 2 * math.pi * 5 / L[0], 2 * math.pi * 4 / L[1]
    f = np.sin(kx * x + 0.3) * np.cos(ky * y) + 0.5 * np.cos(2 * math.pi * x / L[0]) + z * z
    gx, gy, gz = oracle.gradient(g, f)
    ex = kx * np.cos(kx * x + 0.3) * np.cos(ky * y) - 0.5 * (2 * math.pi / L[0]) * np.sin(2 * math.pi * x / L[0])
    ey = -ky * np.sin(kx * x + 0.3) * np.sin(ky * y)
    assert np.abs(gx - ex.ravel()).max() < 1e-12
    assert np.abs(gy - ey.ravel()).max() < 1e-12
    assert np.abs(gz - 2 * z.ravel()).max() < 1e-12  # open axis: second-order differences, exact on z^2
    nyq = np.cos(math.pi * x / h[0])
    assert np.abs(oracle.gradient(g, nyq)[0]).max() < 1e-12


@pytest.mark.parametrize("skew", [False, True])
def test_fft_form_equals_operator_form(oracle, skew):
    if skew:
        wl = W.random_skew(n=(8, 7, 6), periodic=(1, 0, 1), seed=3)
        g = oracle.grid_of_cell(wl.n, wl.cell, wl.periodic, gradient="spectral")
    else:
        wl = W.random_small(n=(8, 7, 6), periodic=(1, 1, 0), seed=3)
        g = oracle.Grid(wl.n, wl.h, wl.periodic, gradient="spectral")
    r = wl.rho.reshape(-1)
    a = oracle.gradient(g, r)
    b = tuple(G @ r for G in oracle.gradient_operators(g))
    for u, v in zip(a, b):
        assert np.abs(u - v).max() < 1e-12 * np.abs(v).max()
    # and the finite-difference form differs (a different operator)
    gf = oracle.Grid(g.n, g.h, g.periodic, g.cell, "fd")
    assert np.abs(oracle.gradient(gf, r)[0] - a[0]).max() > 1e-6


def test_more_accurate_than_differences_on_smooth_periodic_density(oracle):
    n, h = (24, 6, 6), (0.25, 0.5, 0.5)
    L = n[0] * h[0]
    x = np.broadcast_to((np.arange(n[0]) * h[0])[None, None, :], (n[2], n[1], n[0]))
    f = np.exp(np.sin(2 * math.pi * x / L))
    exact = (2 * math.pi / L) * np.cos(2 * math.pi * x / L) * f
    es = np.abs(oracle.gradient(oracle.Grid(n, h, (1, 1, 1), gradient="spectral"), f)[0] - exact.ravel()).max()
    ef = np.abs(oracle.gradient(oracle.Grid(n, h, (1, 1, 1)), f)[0] - exact.ravel()).max()
    assert es < 1e-6 * ef


@pytest.mark.parametrize("periodic,image_max", [((1, 1, 1), (1, 0, 0)), ((1, 0, 1), (0, 0, 0))])
def test_adjoint_exact_for_kink_free_kernel(oracle, periodic, image_max):
    nD, nS, Dmax = 9, 5, 400.0
    tp = oracle.table_params(n_D=nD, n_sigma=nS, D_max=Dmax)
    Dk = np.arange(nD) * Dmax / (nD - 1)
    sl = np.arange(nS) / (nS - 1)
    c = (0.3, -0.1 * 2.5 / Dmax, 1.9, 0.05 * 2.5 / Dmax)
    tab = c[0] + c[1] * Dk[:, None] + c[2] * sl[None, :] + c[3] * Dk[:, None] * sl[None, :]
    wl = W.random_small(n=(6, 6, 5), h=(0.4, 0.4, 0.45), periodic=periodic, seed=5, n_cut=4e-3, image_max=image_max)
    g = oracle.Grid(wl.n, wl.h, wl.periodic, gradient="spectral")
    rho = wl.rho.reshape(-1).copy()
    res = oracle.evaluate(g, rho, tab, tp, wl.n_cut, image_max, 0.0, potential=True)
    rng = np.random.default_rng(4)
    ops = oracle.gradient_operators(g)
    for k in rng.choice(np.flatnonzero(rho >= 2 * wl.n_cut), 6, replace=False):
        eps = 2e-5 * rho[k]
        fd = oracle.local_energy_change(g, rho, k, eps, tab, tp, wl.n_cut, image_max, 0.0, ops=ops) / (2 * eps)
        assert fd == pytest.approx(res.dEdn[k], rel=1e-5, abs=1e-10 * np.abs(res.dEdn).max()), k
