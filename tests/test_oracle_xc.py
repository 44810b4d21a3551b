"""Pins of the oracle's exchange-correlation energies and of the Eq. (3)
recombination: closed forms (Dirac exchange of the uniform gas), the limits
that define the PBE forms (enhancement bound 1 + kappa, gradient-expansion
coefficients mu and beta, correlation vanishing for rapidly varying
densities), exact uniform-coordinate scaling of exchange, translation
invariance, and the paper's printed sample-run energies."""
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
DIRAC = 0.7385587663820224  # (3/4)(3/pi)^(1/3): E_x^LDA = -DIRAC * integral of n^(4/3)


def _periodic_grid(oracle, n=(12, 10, 8), h=(0.4, 0.35, 0.5)):
    return oracle.Grid(n, h, (1, 1, 1))


def _smooth_density(g, eps=0.3, n0=0.05):
    nx, ny, nz = g.n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    f = (1 + eps * np.sin(2 * math.pi * x / nx) * np.cos(2 * math.pi * y / ny)
         + 0.5 * eps * np.sin(2 * math.pi * (z / nz + 0.1)))
    return n0 * f.ravel()


def test_uniform_gas_is_dirac_exchange_and_pw92(oracle):
    """Constant density on a periodic grid: no gradient, so PBE and revPBE
    reduce to LDA, and E_x^LDA = -(3/4)(3/pi)^(1/3) n^(4/3) V."""
    g = _periodic_grid(oracle)
    for n0 in (1e-4, 0.03, 2.5):
        E = oracle.xc_energies(g, np.full(g.G, n0), 1e-12)
        V = g.G * g.dV
        assert E["Ex_lda"] == pytest.approx(-DIRAC * n0 ** (4 / 3) * V, rel=1e-13)
        rs = (3 / (4 * math.pi * n0)) ** (1 / 3)
        ec, _ = oracle.pw92_ec(np.array([rs]))
        assert E["Ec_lda"] == pytest.approx(n0 * ec[0] * V, rel=1e-13)
        assert E["Ex_pbe"] == E["Ex_lda"] and E["Ex_revpbe"] == E["Ex_lda"] and E["Ec_pbe"] == E["Ec_lda"]


def test_enhancement_factor_limits(oracle):
    """F_x(0) = 1, F_x -> 1 + kappa (0.804 PBE, 1.245 revPBE) for large s, and
    (F_x - 1)/s^2 -> mu = 0.21951 (the published PBE value) for small s."""
    for kappa in (oracle.PBE_KAPPA, oracle.REVPBE_KAPPA):
        assert oracle.pbe_fx(0.0, kappa) == 1.0
        assert oracle.pbe_fx(1e12, kappa) == pytest.approx(1 + kappa, rel=1e-10)
        s2 = 1e-8
        assert (oracle.pbe_fx(s2, kappa) - 1) / s2 == pytest.approx(0.21951, abs=1e-5)
    assert oracle.pbe_fx(1e12, oracle.PBE_KAPPA) == pytest.approx(1.804, abs=1e-9)
    assert oracle.pbe_fx(1e12, oracle.REVPBE_KAPPA) == pytest.approx(2.245, abs=1e-9)
    # monotone in s
    s2 = np.logspace(-4, 3, 50)
    assert np.all(np.diff(oracle.pbe_fx(s2)) > 0)


def test_correlation_gradient_limits(oracle):
    """H -> beta t^2 with beta = 0.066725 for slowly varying densities, and
    eps_c + H -> 0 for rapidly varying ones (PBE's design conditions); H >= 0.
    The next term of the small-t series is -beta^2 t^4 / (2 gamma), and gamma
    is the high-density coefficient of the uniform-gas correlation, i.e. the
    A = 0.031091 of the PW92 fit."""
    for rs in (0.1, 1.0, 3.0, 20.0):
        t2 = 1e-8
        assert oracle.pbe_h(rs, t2) / t2 == pytest.approx(0.066725, abs=2e-6)
        beta = oracle.pbe_h(rs, t2) / t2
        t2 = 1e-5
        assert (oracle.pbe_h(rs, t2) - 0.06672455060314922 * t2) / t2 ** 2 == pytest.approx(
            -0.06672455060314922 ** 2 / (2 * 0.031091), rel=1e-3)
        assert beta == pytest.approx(0.06672455060314922, rel=1e-6)
        ec, _ = oracle.pw92_ec(np.array([rs]))
        assert ec[0] + oracle.pbe_h(rs, 1e10) == pytest.approx(0.0, abs=1e-8 * abs(ec[0]))
        t2s = np.logspace(-3, 3, 40)
        h = oracle.pbe_h(rs, t2s)
        assert np.all(h > 0) and np.all(np.diff(h) > 0) and np.all(h < -ec[0])


def test_exchange_uniform_coordinate_scaling(oracle):
    """n_l(r) = l^3 n(l r) gives E_x[n_l] = l E_x[n] for LDA, PBE and revPBE
    exchange; on the grid the values scale by l^3 and the spacings by 1/l."""
    g = _periodic_grid(oracle)
    rho = _smooth_density(g)
    E1 = oracle.xc_energies(g, rho, 1e-12)
    for lam in (0.5, 1.7, 3.0):
        gl = oracle.Grid(g.n, tuple(h / lam for h in g.h), g.periodic)
        El = oracle.xc_energies(gl, lam ** 3 * rho, 1e-12)
        for k in ("Ex_lda", "Ex_pbe", "Ex_revpbe"):
            assert El[k] == pytest.approx(lam * E1[k], rel=1e-12), k
        # correlation does not scale that way (it is not homogeneous of degree 1)
        assert El["Ec_lda"] != pytest.approx(lam * E1["Ec_lda"], rel=1e-3)


def test_gradient_expansion_coefficients(oracle):
    """A density with small relative gradients: E_x^PBE - E_x^LDA approaches
    -DIRAC mu / (4 (3 pi^2)^(2/3)) * sum |grad n|^2 n^(-4/3) dV, and
    E_c^PBE - E_c^LDA approaches beta pi / 16 * sum |grad n|^2 / (k_F n) dV
    (the s^2 and t^2 terms written through |grad n|)."""
    g = _periodic_grid(oracle, n=(24, 20, 16), h=(0.5, 0.5, 0.5))
    rho = _smooth_density(g, eps=0.01, n0=0.2)
    E = oracle.xc_energies(g, rho, 1e-12)
    gx, gy, gz = oracle.gradient(g, rho)
    g2 = gx * gx + gy * gy + gz * gz
    mu, beta = 0.2195149727645171, 0.06672455060314922
    dx = -DIRAC * mu / (4 * (3 * math.pi ** 2) ** (2 / 3)) * np.sum(g2 * rho ** (-4 / 3)) * g.dV
    kF = (3 * math.pi ** 2 * rho) ** (1 / 3)
    dc = beta * math.pi / 16 * np.sum(g2 / (kF * rho)) * g.dV
    assert (E["Ex_pbe"] - E["Ex_lda"]) / dx == pytest.approx(1.0, abs=1e-4)
    assert (E["Ec_pbe"] - E["Ec_lda"]) / dc == pytest.approx(1.0, abs=1e-3)
    # revPBE has the same small-s coefficient
    assert (E["Ex_revpbe"] - E["Ex_lda"]) / dx == pytest.approx(1.0, abs=1e-4)


def test_translation_invariance_and_floor(oracle):
    """Shifting a periodic density by whole grid steps leaves the energies
    unchanged; points at or below the floor (negative densities included, as
    in the paper's sample run) add nothing and leave every energy finite."""
    g = _periodic_grid(oracle)
    rho = _smooth_density(g).reshape(g.n[2], g.n[1], g.n[0])
    E0 = oracle.xc_energies(g, rho, 1e-12)
    E1 = oracle.xc_energies(g, np.roll(rho, (2, -3, 5), axis=(0, 1, 2)), 1e-12)
    for k in E0:
        assert E1[k] == pytest.approx(E0[k], rel=1e-13)
    r2 = rho.copy().ravel()
    r2[::17] = -1e-6
    E2 = oracle.xc_energies(g, r2, 1e-12)
    assert all(math.isfinite(v) for v in E2.values())
    # LDA terms have no gradient: dropping points removes exactly their share
    keep = r2 > 1e-12
    assert E2["Ex_lda"] == pytest.approx(-DIRAC * np.sum(r2[keep] ** (4 / 3)) * g.dV, rel=1e-13)


def _golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "xe_layer_sample_run.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = [float(x) for x in v.split()]
    return vals


def test_recombination_reproduces_the_sample_run(oracle):
    """App. A sample run (eV): -E_c^PBE + E_c^LDA + E_c^NL is the printed
    'needed number'; Eq. (3) adds E_tot^DFT and, for revPBE exchange,
    E_x^revPBE - E_x^PBE."""
    g = _golden()
    ex_pbe, ec_pbe, _ = g["E_pbe"]
    ec_lda = g["E_lda"][1]
    e_nl = g["E_nl"][2]
    assert oracle.recombine(e_nl, ec_lda, ec_pbe) == pytest.approx(g["needed_number"][0], abs=2e-8)
    e_dft = -1234.5
    assert oracle.recombine(e_nl, ec_lda, ec_pbe, E_dft=e_dft) == pytest.approx(e_dft + g["needed_number"][0],
                                                                               abs=2e-8)
    ex_rev = -811.6072505786024  # the X_rev_PBE line of the same output
    tot = oracle.recombine(e_nl, ec_lda, ec_pbe, Ex_pbe=ex_pbe, Ex_new=ex_rev, E_dft=e_dft)
    # Eq. (3) term by term
    assert tot == pytest.approx(e_dft - ex_pbe - ec_pbe + (ex_rev + ec_lda + e_nl), abs=1e-9)
