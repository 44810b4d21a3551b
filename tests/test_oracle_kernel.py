"""Pins of the oracle's kernel phi(d1, d2) and its quadrature rule.

The kernel is the double integral of Dion et al. (their Eq. 14), which the
paper names in Sec. 2 as the way phi is calculated, with the large-D
asymptote of their Eq. 17 (also named in Sec. 2).  Each pin below checks
the oracle against something other than itself: a library routine, a
closed form, a property the kernel is built to have, or a different
quadrature of the same integral.
"""
import math

import numpy as np
import pytest

GAMMA = 4.0 * math.pi / 9.0
C_ASYM = 12.0 * GAMMA ** 3


def test_gauss_legendre_matches_library(oracle):
    for n in (1, 2, 5, 8, 16, 32):
        x, w = oracle.gauss_legendre(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        assert np.allclose(x, xr, atol=1e-15, rtol=0)
        assert np.allclose(w, wr, atol=1e-15, rtol=0)


def test_gauss_legendre_integrates_polynomials_exactly(oracle):
    n = 8
    x, w = oracle.gauss_legendre(n)
    for deg in range(2 * n):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.dot(w, x ** deg) - exact) < 1e-14


def test_U_series_and_direct_forms_agree(oracle):
    # U(x) = (sin x - x cos x)/x: series below 0.5, direct above; both forms
    # are accurate near the switch, and U ~ x^2/3 at small x.
    for x in (0.3, 0.45, 0.5, 0.55, 0.8):
        direct = (math.sin(x) - x * math.cos(x)) / x
        assert abs(oracle.U(x) - direct) < 1e-14
    for x in (1e-6, 1e-4, 1e-3):
        assert abs(oracle.U(x) / (x * x / 3.0) - 1.0) < x * x / 5 + 1e-15


def test_W_regrouping_and_origin_limit(oracle):
    # the cancellation-free grouping equals the literal formula ...
    for a, b in [(0.7, 1.3), (2.0, 5.5), (10.0, 0.9), (33.3, 17.1)]:
        lit = oracle.W_literal(a, b) * a * a * b * b
        assert abs(oracle.W2(a, b) - lit) <= 1e-12 * max(1.0, abs(lit))
    # ... and W(a, b) -> 2/3 at the origin (the bracket's series starts a^3 b^3 / 3)
    for a, b in [(1e-3, 2e-3), (1e-5, 1e-5), (3e-4, 1e-6)]:
        assert abs(oracle.W2(a, b) / (a * a * b * b) - 2.0 / 3.0) < 1e-5
    # W is symmetric
    assert oracle.W2(1.7, 0.4) == pytest.approx(oracle.W2(0.4, 1.7), rel=1e-15)


def test_T_and_nu_limits(oracle):
    # T(w,x,y,z) is invariant under (a <-> b) = (w,x,y,z) -> (x,w,z,y) and
    # under (d1 <-> d2) = (w,x,y,z) -> (y,z,w,x)
    w, x, y, z = 0.3, 1.7, 2.2, 0.05
    t = oracle.T(w, x, y, z)
    assert oracle.T(x, w, z, y) == pytest.approx(t, rel=1e-15)
    assert oracle.T(y, z, w, x) == pytest.approx(t, rel=1e-15)
    # nu(y) = y^2 / (2 h(y/d)) -> d^2/(2 gamma) for y << d and y^2/2 for y >> d
    d = 2.0
    assert oracle.nu(1e-5, d) == pytest.approx(d * d / (2 * GAMMA), rel=1e-9)
    assert oracle.nu(50.0, d) == pytest.approx(50.0 ** 2 / 2, rel=1e-15)
    assert oracle.nu(3.0, 0.0) == pytest.approx(4.5, rel=1e-15)


def test_asymptote_constant(oracle):
    assert oracle.asym_C() == pytest.approx(32.665048684, rel=1e-10)


def test_phi_symmetric_in_d1_d2(oracle):
    tp = oracle.table_params()
    for d1, d2 in [(0.3, 1.1), (2.0, 0.05), (5.0, 9.0), (0.0, 0.7)]:
        a = oracle.dion_phi(d1, d2, tp)
        b = oracle.dion_phi(d2, d1, tp)
        assert abs(a - b) <= 1e-13 * max(1e-6, abs(a))


def test_phi_large_D_asymptote(oracle):
    """phi -> -C / (d1^2 d2^2 (d1^2 + d2^2)) for large D (Dion et al. Eq. 17).

    The corrections to the asymptote come from h(y/d) = 1 - exp(-gamma y^2/d^2)
    and die off exponentially in the smaller of d1, d2: once both exceed 20 the
    kernel equals the asymptote to the accuracy of the quadrature rule (about
    1e-7), while at d2 ~ 8 it still differs by more than 1e-3."""
    tp = oracle.table_params()
    for D, delta in [(20.0, 0.0), (30.0, 0.0), (40.0, 0.0), (47.0, 0.0), (30.0, 0.3), (47.0, 0.5), (40.0, 0.5)]:
        d1, d2 = D * (1 + delta), D * (1 - delta)
        asym = -C_ASYM / (d1 ** 2 * d2 ** 2 * (d1 ** 2 + d2 ** 2))
        phi = oracle.phi_Dsigma(D, delta * delta, tp)
        assert abs(phi / asym - 1.0) < 2e-7, (D, delta, phi, asym)
    for D, delta in [(8.0, 0.0), (20.0, 0.8), (12.0, 0.5)]:
        d1, d2 = D * (1 + delta), D * (1 - delta)
        asym = -C_ASYM / (d1 ** 2 * d2 ** 2 * (d1 ** 2 + d2 ** 2))
        assert abs(oracle.phi_Dsigma(D, delta * delta, tp) / asym - 1.0) > 1e-3, (D, delta)
    # and it is not yet asymptotic at D = 2 (sign differs)
    assert oracle.phi_Dsigma(2.0, 0.0, tp) > 0


def test_phi_small_D_log_slope(oracle):
    """At D = 0 the integrand behaves like (4/3)/(a^2+b^2) + (16/3) a^2 b^2/(a^2+b^2)^3
    near the origin, so phi(D, 0) = const - (2/pi) ln D + o(1) as D -> 0."""
    tp = oracle.table_params()
    p1 = oracle.phi_Dsigma(2e-3, 0.0, tp)
    p2 = oracle.phi_Dsigma(1e-3, 0.0, tp)
    slope = (p2 - p1) / math.log(2.0)
    assert abs(slope - 2.0 / math.pi) < 0.01 * (2.0 / math.pi), slope


def test_phi_zero_integral_uniform_gas(oracle):
    """For a uniform density (constant q0, delta = 0) the nonlocal term must
    vanish (LDA correlation is exact there), i.e. int_0^inf D^2 phi(D, 0) dD = 0;
    Dion et al. build the kernel with this property.  With the converged rule
    the integral vanishes to a few 1e-10 of int D^2 |phi| (the D quadrature
    below and the asymptotic tail beyond D = 20 are exact to that level)."""
    tp = oracle.table_params()
    x, w = np.polynomial.legendre.leggauss(12)
    edges = [0.0, 0.05, 0.2, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 5.0, 6.5, 8.0, 10.0, 13.0, 16.0, 20.0]
    D, wt = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        D.extend(0.5 * (hi + lo) + 0.5 * (hi - lo) * x)
        wt.extend(0.5 * (hi - lo) * w)
    D, wt = np.array(D), np.array(wt)
    f = D * D * oracle.phi_many(D, np.zeros_like(D), tp)
    total = float(wt @ f)
    total_abs = float(wt @ np.abs(f))
    Dc = edges[-1]
    total += -C_ASYM / (2.0 * 3.0 * Dc ** 3)  # int_Dc^inf D^2 (-C / (2 D^6)) dD
    assert abs(total) < 5e-9 * total_abs, (total, total_abs)


def _literal_integrand(a, b, d1, d2):
    """a^2 b^2 W(a,b) T(nu(a), nu(b), nu'(a), nu'(b)) on a grid, literal W."""
    A, B = np.meshgrid(a, b, indexing="ij")
    sa, ca, sb, cb = np.sin(A), np.cos(A), np.sin(B), np.cos(B)
    W = 2 * ((3 - A * A) * B * cb * sa + (3 - B * B) * A * ca * sb + (A * A + B * B - 3) * sa * sb
             - 3 * A * B * ca * cb) / (A ** 3 * B ** 3)

    def nu(y, d):
        if d == 0:
            return y * y / 2
        return y * y / (2 * -np.expm1(-GAMMA * (y / d) ** 2))

    w, x = nu(A, d1), nu(B, d1)
    y, z = nu(A, d2), nu(B, d2)
    T = 0.5 * (1 / (w + x) + 1 / (y + z)) * (1 / ((w + y) * (x + z)) + 1 / ((w + z) * (y + x)))
    return A * A * B * B * W * T


def test_rule_against_different_quadrature(oracle):
    """Composite GL of another panel layout (factor-3 grading, unit-width panels,
    16 points) over the same [0, A]^2 agrees with the rule: the nodes, weights
    and symmetric summation of the rule are right.  (A short cut-off keeps the
    literal numpy integrand small.)"""
    tp = oracle.table_params(kappa=4.0, A0=64.0)
    x16, w16 = np.polynomial.legendre.leggauss(16)
    for D, delta in [(0.5, 0.0), (1.0, 0.6), (3.0, 0.0), (0.2, 0.9)]:
        d1, d2 = D * (1 + delta), D * (1 - delta)
        # the rule's cut-off: smallest odd multiple of pi/2 >= max(A0, kappa max(d1, d2))
        target = max(tp.A0, tp.kappa * max(d1, d2))
        m = 0
        while (2 * m + 1) * math.pi / 2 < target:
            m += 1
        A = (2 * m + 1) * math.pi / 2
        a_rule, _ = oracle.rule_nodes(d1, d2, tp)
        assert a_rule[-1] < A and a_rule[-1] > A - math.pi / 2
        edges = [0.0] + [3.0 ** (-k) for k in range(12, 0, -1)] + list(np.arange(1.0, A, 1.0)) + [A]
        nodes, wts = [], []
        for lo, hi in zip(edges[:-1], edges[1:]):
            nodes.append(0.5 * (hi + lo) + 0.5 * (hi - lo) * x16)
            wts.append(0.5 * (hi - lo) * w16)
        a = np.concatenate(nodes)
        wt = np.concatenate(wts)
        F = _literal_integrand(a, a, d1, d2)
        ref = 2 / math.pi ** 2 * float(wt @ F @ wt)
        got = oracle.dion_phi(d1, d2, tp)
        assert abs(got - ref) < 1e-8 * max(abs(ref), 1e-3), (D, delta, got, ref)


# Spot nodes of the refinement test: D from the first rows of a 48-bohr table
# to its last, sigma across [0, 1]; none sits on the zero crossing of phi
# (between D = 2 and 3, where a relative change is not meaningful).
REFINE_D = (48.0 / 2047, 0.5, 1.0, 2.0, 4.0, 8.0, 12.0, 20.0, 30.0, 40.0, 47.0)
REFINE_SIGMA = (0.0, 0.3, 0.7, 1.0)


def test_rule_converged_under_refinement(oracle):
    """Sec. 7 fixes the table's limits and node counts by checking that further
    refinement does not change the results.  The default rule against the rule
    with kappa, A0 and the points per panel doubled: every spot node moves by
    at most 1e-7 relative."""
    tp = oracle.table_params()
    fine = oracle.table_params(gl_points=2 * tp.gl_points, graded_levels=tp.graded_levels,
                               kappa=2 * tp.kappa, A0=2 * tp.A0)
    D = np.repeat(REFINE_D, len(REFINE_SIGMA))
    S = np.tile(REFINE_SIGMA, len(REFINE_D))
    a = oracle.phi_many(D, S, tp)
    b = oracle.phi_many(D, S, fine)
    rel = np.abs(a - b) / np.abs(b)
    worst = int(np.argmax(rel))
    assert rel.max() <= 1e-7, (D[worst], S[worst], a[worst], b[worst], rel.max())


def test_coarser_rules_fail_the_refinement_test(oracle):
    """The refinement test has teeth: halving kappa (the tail cut-off at large
    D) or A0 (at small D) moves the kernel by more than 1e-7."""
    tp = oracle.table_params()
    half_kappa = oracle.table_params(gl_points=tp.gl_points, graded_levels=tp.graded_levels,
                                     kappa=tp.kappa / 2, A0=tp.A0)
    half_A0 = oracle.table_params(gl_points=tp.gl_points, graded_levels=tp.graded_levels,
                                  kappa=tp.kappa, A0=tp.A0 / 8)
    D = np.array([40.0, 47.0, 1.0, 2.0])
    S = np.array([0.0, 0.0, 0.0, 0.0])
    ref = oracle.phi_many(D, S, tp)
    rk = np.abs(oracle.phi_many(D[:2], S[:2], half_kappa) / ref[:2] - 1)
    ra = np.abs(oracle.phi_many(D[2:], S[2:], half_A0) / ref[2:] - 1)
    assert rk.min() > 1e-7 and ra.min() > 1e-7, (rk, ra)


def test_table_layout_and_row0_extrapolation(oracle):
    tp = oracle.table_params(n_D=8, n_sigma=3, D_max=7.0)
    tab = oracle.build_table(tp)
    assert tab.shape == (8, 3)
    for k in (1, 4, 7):
        for l in range(3):
            assert tab[k, l] == pytest.approx(oracle.phi_Dsigma(float(k), l / 2.0, tp), rel=1e-15)
    assert np.allclose(tab[0], 2 * tab[1] - tab[2], rtol=0, atol=1e-15)
    nodes = oracle.table_nodes(tp, [0, 3, 7], [1, 2, 0])
    assert nodes == pytest.approx([tab[0, 1], tab[3, 2], tab[7, 0]], rel=1e-15)
