/*
 * vdw_oracle.c -- TEST ORACLE (test infrastructure only).
 *
 * Plain, slow, FP64 CPU implementation of the compute-heavy parts of the
 * vdW-DF nonlocal-correlation evaluation described in Lazic et al.,
 * "JuNoLo - Julich Non Local code for parallel calculation of vdW-DF
 * nonlocal density functional theory" (arXiv:0810.2273):
 *
 *   - the kernel phi(d1,d2) by the double integral of Dion et al. (their
 *     Eq. 14, which the paper names in Sec. 2 as the way the kernel is
 *     calculated), evaluated with one fixed, written quadrature rule;
 *   - the lookup table of phi over (D, sigma = delta^2) (Sec. 2, Sec. 7);
 *   - the interpolated pair kernel, with the large-D asymptote of Dion
 *     et al. (their Eq. 17, named in Sec. 2) beyond the table;
 *   - the discrete double sum of Eq. (2), with periodic images of the
 *     0th cell (Sec. 3, periodic problems; Sec. 6.2);
 *   - the per-point sums the adjoint needs (derivative of Eq. (2));
 *   - the far image shell with the large-D asymptote (Sec. 7 outlook).
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may
 * load this code.  It shares nothing with the HIP library: no headers,
 * no helpers, no constants tables.  Everything is written from the
 * mathematics, in the order the definitions state it, with no blocking
 * or reordering beyond what a plain loop does.
 *
 * Parity status: every function here is pinned by tests/test_oracle_*.py
 * (closed forms, symmetry, asymptote, brute force, invariants).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Parameters of the phi table and of the quadrature rule that fills it. */
typedef struct {
    int32_t n_D;            /* table rows, D_k = k * D_max / (n_D - 1)           */
    int32_t n_sigma;        /* table columns, sigma_l = l / (n_sigma - 1)        */
    double  D_max;          /* last row; D >= D_max uses the asymptote           */
    int32_t gl_points;      /* Gauss-Legendre points per panel                   */
    int32_t graded_levels;  /* number of halving panels below pi/2               */
    double  kappa;          /* cut-off A >= kappa * max(d1, d2)                  */
    double  A0;             /* cut-off A >= A0                                   */
    int32_t interp;         /* 0: bilinear; 1: cubic (C1) in D, linear in sigma  */
} vo_table_params;

static const double VO_PI = 3.14159265358979323846;

/* gamma = 4 pi / 9 in h(t) = 1 - exp(-gamma t^2) (Dion et al.). */
static double vo_gamma(void) { return 4.0 * VO_PI / 9.0; }

/* C = 12 (4 pi / 9)^3, the constant of the large-D asymptote. */
double vo_asym_C(void)
{
    double g = vo_gamma();
    return 12.0 * g * g * g;
}

/* ------------------------------------------------------------------ */
/* Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on   */
/* the Legendre polynomial P_n (three-term recurrence).                 */
/* ------------------------------------------------------------------ */
void vo_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(VO_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            /* derivative of P_n from P_n and P_{n-1} */
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* recompute the derivative at the converged node */
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = -z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* ------------------------------------------------------------------ */
/* Pieces of the Dion integrand.                                        */
/* ------------------------------------------------------------------ */

/* U(x) = (sin x - x cos x) / x.  Series for small x, where the direct
 * form cancels: U = sum_{k>=1} (-1)^{k+1} 2k x^{2k} / (2k+1)!. */
double vo_U(double x)
{
    if (fabs(x) < 0.5) {
        double x2 = x * x, term = x2, fact = 6.0; /* x^2k and (2k+1)! for k = 1 */
        double s = 0.0;
        for (int k = 1; k <= 12; ++k) {
            double sign = (k % 2 == 1) ? 1.0 : -1.0;
            s += sign * 2.0 * k * term / fact;
            term *= x2;
            fact *= (2.0 * k + 2.0) * (2.0 * k + 3.0);
        }
        return s;
    }
    return (sin(x) - x * cos(x)) / x;
}

/* a^2 b^2 W(a,b), with W the angular factor of the Dion kernel:
 *   W = 2[(3-a^2) b cos b sin a + (3-b^2) a cos a sin b
 *         + (a^2+b^2-3) sin a sin b - 3 a b cos a cos b] / (a^3 b^3).
 * Grouping the bracket as a^2 sin a u(b) + b^2 sin b u(a) - 3 u(a) u(b)
 * with u(x) = sin x - x cos x gives the same value without cancellation:
 *   a^2 b^2 W = 2 [P(a) U(b) + P(b) U(a) - 3 U(a) U(b)],  P(x) = x sin x. */
double vo_W2(double a, double b)
{
    double Pa = a * sin(a), Pb = b * sin(b);
    double Ua = vo_U(a), Ub = vo_U(b);
    return 2.0 * (Pa * Ub + Pb * Ua - 3.0 * Ua * Ub);
}

/* The literal W(a,b) (used only by tests of the identity above). */
double vo_W_literal(double a, double b)
{
    double sa = sin(a), ca = cos(a), sb = sin(b), cb = cos(b);
    double br = (3.0 - a * a) * b * cb * sa + (3.0 - b * b) * a * ca * sb
              + (a * a + b * b - 3.0) * sa * sb - 3.0 * a * b * ca * cb;
    return 2.0 * br / (a * a * a * b * b * b);
}

/* T(w,x,y,z) = 1/2 [1/(w+x) + 1/(y+z)] [1/((w+y)(x+z)) + 1/((w+z)(y+x))] */
double vo_T(double w, double x, double y, double z)
{
    return 0.5 * (1.0 / (w + x) + 1.0 / (y + z))
               * (1.0 / ((w + y) * (x + z)) + 1.0 / ((w + z) * (y + x)));
}

/* nu(y) = y^2 / (2 h(y/d)), h(t) = 1 - exp(-gamma t^2); h = 1 when d = 0. */
double vo_nu(double y, double d)
{
    if (d <= 0.0) return 0.5 * y * y;
    double t = y / d;
    double h = -expm1(-vo_gamma() * t * t);
    return 0.5 * y * y / h;
}

/* ------------------------------------------------------------------ */
/* The quadrature rule (the same written rule the GPU builder follows).   */
/*   width w = pi/2; A = (2m+1) w, the smallest odd multiple of w with    */
/*   A >= max(A0, kappa * max(d1, d2)); panels                            */
/*   [0, w 2^-K], [w 2^-(K-j+1), w 2^-(K-j)] (j = 1..K), then             */
/*   [t w, (t+1) w] for t = 1 .. 2m; gl_points GL nodes per panel.        */
/* ------------------------------------------------------------------ */
int vo_rule_nodes(double d1, double d2, const vo_table_params *p, double *a, double *wt, int cap)
{
    const double w = 0.5 * VO_PI;
    double dmax = d1 > d2 ? d1 : d2;
    double target = p->A0;
    if (p->kappa * dmax > target) target = p->kappa * dmax;
    long m = (long)ceil((target / w - 1.0) * 0.5);
    if (m < 0) m = 0;
    while ((2.0 * m + 1.0) * w < target) ++m;
    int ng = p->gl_points, K = p->graded_levels;
    long npan = (long)(K + 1) + 2 * m;
    long need = npan * ng;
    if (a == NULL) return (int)need;
    if (need > cap) return -1;

    double gx[64], gw[64];
    vo_gauss_legendre(ng, gx, gw);
    int c = 0;
    for (long pidx = 0; pidx < npan; ++pidx) {
        double lo, hi;
        if (pidx == 0) { lo = 0.0; hi = w * ldexp(1.0, -K); }
        else if (pidx <= K) { lo = w * ldexp(1.0, -(int)(K - pidx + 1)); hi = w * ldexp(1.0, -(int)(K - pidx)); }
        else { long t = pidx - K; lo = t * w; hi = (t + 1) * w; }
        double half = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
        for (int g = 0; g < ng; ++g) {
            a[c] = mid + half * gx[g];
            wt[c] = half * gw[g];
            ++c;
        }
    }
    return c;
}

/* phi(d1, d2) = (2/pi^2) int_0^A int_0^A a^2 b^2 W(a,b)
 *                          T(nu(a), nu(b), nu'(a), nu'(b)) da db,
 * nu from d1 and nu' from d2 (Dion et al. Eq. 14), with the rule above.
 * The integrand is symmetric in (a, b), so the sum runs over i <= j. */
double vo_dion_phi(double d1, double d2, const vo_table_params *p)
{
    int n = vo_rule_nodes(d1, d2, p, NULL, NULL, 0);
    double *a = (double *)malloc(sizeof(double) * 6 * (size_t)n);
    double *wt = a + n, *P = a + 2 * n, *U = a + 3 * n, *n1 = a + 4 * n, *n2 = a + 5 * n;
    vo_rule_nodes(d1, d2, p, a, wt, n);
    for (int i = 0; i < n; ++i) {
        P[i] = a[i] * sin(a[i]);
        U[i] = vo_U(a[i]);
        n1[i] = vo_nu(a[i], d1);
        n2[i] = vo_nu(a[i], d2);
    }
    double sum = 0.0;
    for (int i = 0; i < n; ++i) {
        double row = 0.0;
        for (int j = i; j < n; ++j) {
            double w2 = 2.0 * (P[i] * U[j] + P[j] * U[i] - 3.0 * U[i] * U[j]);
            double t = vo_T(n1[i], n1[j], n2[i], n2[j]);
            double f = wt[j] * w2 * t;
            row += (j == i) ? f : 2.0 * f;
        }
        sum += wt[i] * row;
    }
    free(a);
    return 2.0 / (VO_PI * VO_PI) * sum;
}

/* phi at table coordinates: d1 = D (1 + delta), d2 = D (1 - delta). */
double vo_phi_Dsigma(double D, double sigma, const vo_table_params *p)
{
    double delta = sqrt(sigma);
    return vo_dion_phi(D * (1.0 + delta), D * (1.0 - delta), p);
}

/* Fill the table: phi[k * n_sigma + l] = phi(D_k, sigma_l), row k = 0
 * (D = 0, where phi diverges logarithmically) by linear extrapolation
 * from rows 1 and 2. */
int vo_build_table(const vo_table_params *p, double *phi)
{
    if (p->n_D < 3 || p->n_sigma < 2 || !(p->D_max > 0.0)) return -1;
    const int nD = p->n_D, nS = p->n_sigma;
    const double dD = p->D_max / (nD - 1);
    long total = (long)(nD - 1) * nS;
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < total; ++t) {
        /* largest D first so dynamic scheduling balances the load */
        long idx = total - 1 - t;
        int k = 1 + (int)(idx / nS), l = (int)(idx % nS);
        double sigma = (double)l / (nS - 1);
        phi[(long)k * nS + l] = vo_phi_Dsigma(k * dD, sigma, p);
    }
    for (int l = 0; l < nS; ++l)
        phi[l] = 2.0 * phi[nS + l] - phi[2 * nS + l];
    return 0;
}

/* Only selected nodes (for sampled comparisons at large table sizes). */
int vo_table_nodes(const vo_table_params *p, long count, const int32_t *k, const int32_t *l, double *out)
{
    const double dD = p->D_max / (p->n_D - 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < count; ++t) {
        if (k[t] == 0) {
            double s = (double)l[t] / (p->n_sigma - 1);
            out[t] = 2.0 * vo_phi_Dsigma(dD, s, p) - vo_phi_Dsigma(2.0 * dD, s, p);
        } else {
            out[t] = vo_phi_Dsigma(k[t] * dD, (double)l[t] / (p->n_sigma - 1), p);
        }
    }
    return 0;
}

/* phi at arbitrary (D, sigma) points, one per loop iteration (refinement
 * and asymptote checks off the table nodes). */
int vo_phi_many(long count, const double *D, const double *sigma, const vo_table_params *p, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < count; ++t) out[t] = vo_phi_Dsigma(D[t], sigma[t], p);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Interpolated kernel.                                                  */
/* ------------------------------------------------------------------ */

/* Column l of the table at rows k-1 .. k+2 for the cubic form, with the rows
 * beyond the table ends extrapolated linearly (phi_{-1} = 2 phi_0 - phi_1,
 * phi_{nD} = 2 phi_{nD-1} - phi_{nD-2}). */
static double vo_row(const double *tab, int nD, int nS, int row, int l)
{
    if (row < 0) return 2.0 * tab[(long)l] - tab[(long)nS + l];
    if (row > nD - 1) return 2.0 * tab[(long)(nD - 1) * nS + l] - tab[(long)(nD - 2) * nS + l];
    return tab[(long)row * nS + l];
}

/* Cubic Hermite interpolation on [0, 1] between f1 and f2 with the
 * Catmull-Rom tangents (f2 - f0)/2 and (f3 - f1)/2, and its derivative. */
static double vo_catmull_rom(double f0, double f1, double f2, double f3, double t, double *dt)
{
    const double m1 = 0.5 * (f2 - f0), m2 = 0.5 * (f3 - f1);
    const double t2 = t * t, t3 = t2 * t;
    const double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + t, h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
    if (dt) *dt = (6 * t2 - 6 * t) * f1 + (3 * t2 - 4 * t + 1) * m1 + (-6 * t2 + 6 * t) * f2 + (3 * t2 - 2 * t) * m2;
    return h00 * f1 + h10 * m1 + h01 * f2 + h11 * m2;
}

/* Interpolation of the table at (D, sigma), D < D_max, with the partial
 * derivatives of the interpolant in D and sigma: bilinear (interp = 0), or
 * (interp = 1) cubic in D through the Catmull-Rom form of each of the two
 * sigma columns, which makes the interpolant C1 in D, then linear in sigma. */
double vo_table_interp(const double *tab, const vo_table_params *p, double D, double sigma,
                       double *dD_out, double *dS_out)
{
    const int nD = p->n_D, nS = p->n_sigma;
    if (p->interp == 1) {
        const double dD = p->D_max / (nD - 1);
        double tD = D / dD;
        int k = (int)floor(tD);
        if (k > nD - 2) k = nD - 2;
        if (k < 0) k = 0;
        const double fD = tD - k;
        double tS = sigma * (nS - 1);
        int l = (int)floor(tS);
        if (l > nS - 2) l = nS - 2;
        if (l < 0) l = 0;
        const double fS = tS - l;
        double d0, d1;
        const double c0 = vo_catmull_rom(vo_row(tab, nD, nS, k - 1, l), vo_row(tab, nD, nS, k, l),
                                         vo_row(tab, nD, nS, k + 1, l), vo_row(tab, nD, nS, k + 2, l), fD, &d0);
        const double c1 = vo_catmull_rom(vo_row(tab, nD, nS, k - 1, l + 1), vo_row(tab, nD, nS, k, l + 1),
                                         vo_row(tab, nD, nS, k + 1, l + 1), vo_row(tab, nD, nS, k + 2, l + 1), fD,
                                         &d1);
        if (dD_out) *dD_out = ((1.0 - fS) * d0 + fS * d1) / dD;
        if (dS_out) *dS_out = (c1 - c0) * (nS - 1);
        return (1.0 - fS) * c0 + fS * c1;
    }
    const double dD = p->D_max / (nD - 1);
    double tD = D / dD;
    int k = (int)floor(tD);
    if (k > nD - 2) k = nD - 2;
    if (k < 0) k = 0;
    double fD = tD - k;
    double tS = sigma * (nS - 1);
    int l = (int)floor(tS);
    if (l > nS - 2) l = nS - 2;
    if (l < 0) l = 0;
    double fS = tS - l;
    double p00 = tab[(long)k * nS + l], p01 = tab[(long)k * nS + l + 1];
    double p10 = tab[(long)(k + 1) * nS + l], p11 = tab[(long)(k + 1) * nS + l + 1];
    double v = (1.0 - fD) * (1.0 - fS) * p00 + (1.0 - fD) * fS * p01
             + fD * (1.0 - fS) * p10 + fD * fS * p11;
    if (dD_out) *dD_out = ((1.0 - fS) * (p10 - p00) + fS * (p11 - p01)) / dD;
    if (dS_out) *dS_out = ((1.0 - fD) * (p01 - p00) + fD * (p11 - p10)) * (nS - 1);
    return v;
}

/* The pair kernel phi~ for densities with q_i, q_j at distance r:
 *   D = (q_i + q_j) r / 2, delta = (q_i - q_j)/(q_i + q_j), sigma = delta^2;
 *   D <  D_max: the table interpolant;
 *   D >= D_max: -C / (d1^2 d2^2 (d1^2 + d2^2)), d1 = q_i r, d2 = q_j r.
 * Also returns d phi~ / d q_i (chain rule through D and sigma). */
double vo_pair_phi(double qi, double qj, double r, const double *tab, const vo_table_params *p,
                   double *dphi_dqi)
{
    double s = qi + qj;
    double D = 0.5 * s * r;
    if (D >= p->D_max) {
        double d1 = qi * r, d2 = qj * r;
        double v = -vo_asym_C() / (d1 * d1 * d2 * d2 * (d1 * d1 + d2 * d2));
        if (dphi_dqi) *dphi_dqi = v * (-2.0 / qi - 2.0 * qi / (qi * qi + qj * qj));
        return v;
    }
    double delta = (qi - qj) / s;
    double pD, pS;
    double v = vo_table_interp(tab, p, D, delta * delta, &pD, &pS);
    if (dphi_dqi) *dphi_dqi = pD * 0.5 * r + pS * 4.0 * delta * qj / (s * s);
    return v;
}

/* The on-site value phi~(q rho_s, 0) used by the self term, and its
 * derivative in q.  rho_s is passed in by the caller. */
double vo_self_phi(double q, double rho_s, const double *tab, const vo_table_params *p, double *dphi_dq)
{
    double D = q * rho_s;
    if (D >= p->D_max) {
        double C = vo_asym_C();
        double D6 = D * D * D * D * D * D;
        if (dphi_dq) *dphi_dq = rho_s * 3.0 * C / (D6 * D);
        return -C / (2.0 * D6);
    }
    double pD;
    double v = vo_table_interp(tab, p, D, 0.0, &pD, NULL);
    if (dphi_dq) *dphi_dq = rho_s * pD;
    return v;
}

/* The voxel double average of the kernel at delta = 0,
 *   Phi_V(q) = (1/dV^2) int_V int_V phi~(q |r - r'|, 0) dr dr'
 *            = int_{[-1,1]^3} phi~(q |t_0 e_0 + t_1 e_1 + t_2 e_2|, 0) prod_a (1 - |t_a|) dt,
 * V the grid cell spanned by the step vectors e_a (rows of E); the tent
 * weight is the overlap of V with its translate by r - r'.  Rule: the 8
 * octants, in each t_a = +-u_a^2 with u_a at the g Gauss-Legendre nodes of
 * [0, 1], node weight prod_a 2 u_a w_a (1 - u_a^2) (the substitution
 * clusters nodes at the log singularity of phi~ at r = r').  Also returns
 * d Phi_V / d q. */
double vo_self_voxel(double q, const double E[9], int g, const double *tab, const vo_table_params *p,
                     double *dphi_dq)
{
    double x[64], w[64];
    if (g < 1 || g > 64) return NAN;
    vo_gauss_legendre(g, x, w);
    double u[64], wt[64];
    for (int k = 0; k < g; ++k) {
        u[k] = 0.5 * (x[k] + 1.0);  /* [-1, 1] -> [0, 1] */
        double wk = 0.5 * w[k];
        wt[k] = 2.0 * u[k] * wk * (1.0 - u[k] * u[k]);
    }
    double acc = 0.0, dacc = 0.0;
    for (int oct = 0; oct < 8; ++oct) {
        const double s0 = (oct & 1) ? -1.0 : 1.0, s1 = (oct & 2) ? -1.0 : 1.0, s2 = (oct & 4) ? -1.0 : 1.0;
        for (int i = 0; i < g; ++i)
            for (int j = 0; j < g; ++j)
                for (int k = 0; k < g; ++k) {
                    const double t0 = s0 * u[i] * u[i], t1 = s1 * u[j] * u[j], t2 = s2 * u[k] * u[k];
                    const double rx = t0 * E[0] + t1 * E[3] + t2 * E[6];
                    const double ry = t0 * E[1] + t1 * E[4] + t2 * E[7];
                    const double rz = t0 * E[2] + t1 * E[5] + t2 * E[8];
                    const double r = sqrt(rx * rx + ry * ry + rz * rz);
                    const double wn = wt[i] * wt[j] * wt[k];
                    double d;
                    acc += wn * vo_self_phi(q, r, tab, p, &d);
                    dacc += wn * d;
                }
    }
    if (dphi_dq) *dphi_dq = dacc;
    return acc;
}

/* vo_self_voxel at many q values (one thread per value). */
int vo_self_voxel_many(long m, const double *q, const double E[9], int g, const double *tab,
                       const vo_table_params *p, double *phi, double *dphi_dq)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (long t = 0; t < m; ++t) {
        double d;
        phi[t] = vo_self_voxel(q[t], E, g, tab, p, &d);
        if (dphi_dq) dphi_dq[t] = d;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Row sums of the double sum of Eq. (2).                                */
/*                                                                        */
/* Points sit on an orthorhombic grid, r_i = (ix h_x, iy h_y, iz h_z).     */
/* Images L = (m nx h_x, n ny h_y, p nz h_z) with |m| <= image_max[0] on   */
/* periodic axes (0 otherwise).  For each selected row i:                 */
/*   S0_cell_i = sum_{j}      n_j phi~(q_i, q_j, |r_i - r_j|),  j != i      */
/*   S0_img_i  = sum_{j,L!=0} n_j phi~(q_i, q_j, |r_i - r_j - L|)          */
/*   Sq_i      = sum over the same (j, L) of n_j d phi~ / d q_i            */
/* with every (j, L) dropped when r_cut > 0 and |r_i - r_j - L| > r_cut.  */
/* ------------------------------------------------------------------ */
int vo_pair_rows(long npts, const int32_t *ix, const int32_t *iy, const int32_t *iz,
                 const double *n, const double *q,
                 const double h[3], const int32_t gdim[3], const int32_t periodic[3],
                 const int32_t image_max[3], double r_cut,
                 const double *tab, const vo_table_params *p,
                 long nrows, const int64_t *rows,
                 double *S0_cell, double *S0_img, double *Sq)
{
    int mx = periodic[0] ? image_max[0] : 0;
    int my = periodic[1] ? image_max[1] : 0;
    int mz = periodic[2] ? image_max[2] : 0;
    double Lx = gdim[0] * h[0], Ly = gdim[1] * h[1], Lz = gdim[2] * h[2];
#pragma omp parallel for schedule(dynamic, 16)
    for (long t = 0; t < nrows; ++t) {
        long i = rows ? (long)rows[t] : t;
        double xi = ix[i] * h[0], yi = iy[i] * h[1], zi = iz[i] * h[2];
        double sc = 0.0, si = 0.0, sq = 0.0;
        for (int a = -mx; a <= mx; ++a)
            for (int b = -my; b <= my; ++b)
                for (int c = -mz; c <= mz; ++c) {
                    int home = (a == 0 && b == 0 && c == 0);
                    for (long j = 0; j < npts; ++j) {
                        if (home && j == i) continue;
                        double dx = xi - ix[j] * h[0] - a * Lx;
                        double dy = yi - iy[j] * h[1] - b * Ly;
                        double dz = zi - iz[j] * h[2] - c * Lz;
                        double r = sqrt(dx * dx + dy * dy + dz * dz);
                        if (r_cut > 0.0 && r > r_cut) continue;
                        double dq;
                        double ph = vo_pair_phi(q[i], q[j], r, tab, p, &dq);
                        if (home) sc += n[j] * ph;
                        else si += n[j] * ph;
                        sq += n[j] * dq;
                    }
                }
        S0_cell[t] = sc;
        S0_img[t] = si;
        Sq[t] = sq;
    }
    return 0;
}

/* The double sum over the pairs of one image shift L = (m_x n_x h_x,
 * m_y n_y h_y, m_z n_z h_z):  sum_i n_i sum_j n_j phi~(q_i, q_j, |r_i - r_j - L|)
 * with the pair kept iff r <= r_cut (when r_cut > 0), (i, i) skipped for L = 0.
 * The terms of (i, j, L) and (j, i, -L) are equal (phi~ depends on q_i, q_j
 * through D and delta^2, and the distances agree), so the image part of Eq. (2)
 * is twice the sum over one half of the nonzero shifts.  Rows are summed in
 * row order after a parallel loop over them. */
double vo_image_pair_sum(long npts, const int32_t *ix, const int32_t *iy, const int32_t *iz,
                         const double *n, const double *q,
                         const double h[3], const int32_t gdim[3], const int32_t m[3], double r_cut,
                         const double *tab, const vo_table_params *p)
{
    const double Lx = m[0] * gdim[0] * h[0], Ly = m[1] * gdim[1] * h[1], Lz = m[2] * gdim[2] * h[2];
    const int home = (m[0] == 0 && m[1] == 0 && m[2] == 0);
    double *row = (double *)malloc(sizeof(double) * (size_t)(npts > 0 ? npts : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < npts; ++i) {
        double xi = ix[i] * h[0], yi = iy[i] * h[1], zi = iz[i] * h[2];
        double s = 0.0;
        for (long j = 0; j < npts; ++j) {
            if (home && j == i) continue;
            double dx = xi - ix[j] * h[0] - Lx;
            double dy = yi - iy[j] * h[1] - Ly;
            double dz = zi - iz[j] * h[2] - Lz;
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r_cut > 0.0 && r > r_cut) continue;
            s += n[j] * vo_pair_phi(q[i], q[j], r, tab, p, NULL);
        }
        row[i] = n[i] * s;
    }
    double total = 0.0;
    for (long i = 0; i < npts; ++i) total += row[i];
    free(row);
    return total;
}

/* Sum over one explicit set of pairs between two point lists (used by
 * the local-difference derivative check): sum_{a in A} sum_{b in B}
 * n_a n_b phi~(q_a, q_b, r_ab + images), skipping identical (a, b, 0). */
double vo_block_sum(long na, const int32_t *ia, long nb, const int32_t *ib,
                    const int32_t *ix, const int32_t *iy, const int32_t *iz,
                    const double *n, const double *q,
                    const double h[3], const int32_t gdim[3], const int32_t periodic[3],
                    const int32_t image_max[3], double r_cut,
                    const double *tab, const vo_table_params *p)
{
    int mx = periodic[0] ? image_max[0] : 0;
    int my = periodic[1] ? image_max[1] : 0;
    int mz = periodic[2] ? image_max[2] : 0;
    double Lx = gdim[0] * h[0], Ly = gdim[1] * h[1], Lz = gdim[2] * h[2];
    double *part = (double *)malloc(sizeof(double) * (size_t)(na > 0 ? na : 1));
#pragma omp parallel for schedule(dynamic, 4)
    for (long s = 0; s < na; ++s) {
        long i = ia[s];
        double acc = 0.0;
        for (int a = -mx; a <= mx; ++a)
            for (int b = -my; b <= my; ++b)
                for (int c = -mz; c <= mz; ++c) {
                    int home = (a == 0 && b == 0 && c == 0);
                    for (long u = 0; u < nb; ++u) {
                        long j = ib[u];
                        if (home && j == i) continue;
                        double dx = ix[i] * h[0] - ix[j] * h[0] - a * Lx;
                        double dy = iy[i] * h[1] - iy[j] * h[1] - b * Ly;
                        double dz = iz[i] * h[2] - iz[j] * h[2] - c * Lz;
                        double r = sqrt(dx * dx + dy * dy + dz * dz);
                        if (r_cut > 0.0 && r > r_cut) continue;
                        acc += n[i] * n[j] * vo_pair_phi(q[i], q[j], r, tab, p, NULL);
                    }
                }
        part[s] = acc;
    }
    double total = 0.0;
    for (long s = 0; s < na; ++s) total += part[s];
    free(part);
    return total;
}

/* ------------------------------------------------------------------ */
/* The same two sums on a general (possibly skew) grid: point (i0,i1,i2)  */
/* sits at r = i0 e_0 + i1 e_1 + i2 e_2 with the step vectors e_a as rows */
/* of E (e_a = lattice vector a / n_a), and image L = sum_a m_a n_a e_a.   */
/* The separation is formed in grid units first, then mapped by E.        */
/* ------------------------------------------------------------------ */
static double vo_cell_dist(const double E[9], double d0, double d1, double d2)
{
    double x = d0 * E[0] + d1 * E[3] + d2 * E[6];
    double y = d0 * E[1] + d1 * E[4] + d2 * E[7];
    double z = d0 * E[2] + d1 * E[5] + d2 * E[8];
    return sqrt(x * x + y * y + z * z);
}

int vo_pair_rows_cell(long npts, const int32_t *ix, const int32_t *iy, const int32_t *iz,
                      const double *n, const double *q,
                      const double E[9], const int32_t gdim[3], const int32_t periodic[3],
                      const int32_t image_max[3], double r_cut,
                      const double *tab, const vo_table_params *p,
                      long nrows, const int64_t *rows,
                      double *S0_cell, double *S0_img, double *Sq)
{
    int mx = periodic[0] ? image_max[0] : 0;
    int my = periodic[1] ? image_max[1] : 0;
    int mz = periodic[2] ? image_max[2] : 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (long t = 0; t < nrows; ++t) {
        long i = rows ? (long)rows[t] : t;
        double sc = 0.0, si = 0.0, sq = 0.0;
        for (int a = -mx; a <= mx; ++a)
            for (int b = -my; b <= my; ++b)
                for (int c = -mz; c <= mz; ++c) {
                    int home = (a == 0 && b == 0 && c == 0);
                    for (long j = 0; j < npts; ++j) {
                        if (home && j == i) continue;
                        double r = vo_cell_dist(E, (double)(ix[i] - ix[j]) - (double)a * gdim[0],
                                                (double)(iy[i] - iy[j]) - (double)b * gdim[1],
                                                (double)(iz[i] - iz[j]) - (double)c * gdim[2]);
                        if (r_cut > 0.0 && r > r_cut) continue;
                        double dq;
                        double ph = vo_pair_phi(q[i], q[j], r, tab, p, &dq);
                        if (home) sc += n[j] * ph;
                        else si += n[j] * ph;
                        sq += n[j] * dq;
                    }
                }
        S0_cell[t] = sc;
        S0_img[t] = si;
        Sq[t] = sq;
    }
    return 0;
}

double vo_block_sum_cell(long na, const int32_t *ia, long nb, const int32_t *ib,
                         const int32_t *ix, const int32_t *iy, const int32_t *iz,
                         const double *n, const double *q,
                         const double E[9], const int32_t gdim[3], const int32_t periodic[3],
                         const int32_t image_max[3], double r_cut,
                         const double *tab, const vo_table_params *p)
{
    int mx = periodic[0] ? image_max[0] : 0;
    int my = periodic[1] ? image_max[1] : 0;
    int mz = periodic[2] ? image_max[2] : 0;
    double *part = (double *)malloc(sizeof(double) * (size_t)(na > 0 ? na : 1));
#pragma omp parallel for schedule(dynamic, 4)
    for (long s = 0; s < na; ++s) {
        long i = ia[s];
        double acc = 0.0;
        for (int a = -mx; a <= mx; ++a)
            for (int b = -my; b <= my; ++b)
                for (int c = -mz; c <= mz; ++c) {
                    int home = (a == 0 && b == 0 && c == 0);
                    for (long u = 0; u < nb; ++u) {
                        long j = ib[u];
                        if (home && j == i) continue;
                        double r = vo_cell_dist(E, (double)(ix[i] - ix[j]) - (double)a * gdim[0],
                                                (double)(iy[i] - iy[j]) - (double)b * gdim[1],
                                                (double)(iz[i] - iz[j]) - (double)c * gdim[2]);
                        if (r_cut > 0.0 && r > r_cut) continue;
                        acc += n[i] * n[j] * vo_pair_phi(q[i], q[j], r, tab, p, NULL);
                    }
                }
        part[s] = acc;
    }
    double total = 0.0;
    for (long s = 0; s < na; ++s) total += part[s];
    free(part);
    return total;
}

/* ------------------------------------------------------------------ */
/* Far image shell.  The paper's outlook (Sec. 7) is to use the large-D */
/* form of the kernel to speed up the sum over repeated cells.  Here    */
/* the images L = sum_a m_a n_a e_a with |m_a| <= far_max[a] on the      */
/* periodic axes, except those with every |m_a| <= image_max[a] (the    */
/* near images, summed with the table), enter with the asymptote of     */
/* Dion et al. (their Eq. 17) whatever D.  Summed over the shell, the   */
/* ordered pair (i, j) -- i = j included: a point meets its own far      */
/* images -- then contributes                                           */
/*   phi_far(i, j) = -C T(r_i - r_j) / (q_i^2 q_j^2 (q_i^2 + q_j^2)),    */
/*   T(d) = sum over the shell of |d - L|^-6,                           */
/* and d phi_far / d q_i = -phi_far (2 / q_i + 2 q_i / (q_i^2 + q_j^2)).  */
/* ------------------------------------------------------------------ */
double vo_far_T(const double E[9], const int32_t gdim[3], const int32_t periodic[3],
                const int32_t image_max[3], const int32_t far_max[3],
                double d0, double d1, double d2)
{
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = periodic[a] ? image_max[a] : 0;
        hi[a] = periodic[a] ? far_max[a] : 0;
    }
    double s = 0.0;
    for (int a = -hi[0]; a <= hi[0]; ++a)
        for (int b = -hi[1]; b <= hi[1]; ++b)
            for (int c = -hi[2]; c <= hi[2]; ++c) {
                if (abs(a) <= lo[0] && abs(b) <= lo[1] && abs(c) <= lo[2]) continue;
                double r = vo_cell_dist(E, d0 - (double)a * gdim[0], d1 - (double)b * gdim[1],
                                        d2 - (double)c * gdim[2]);
                s += 1.0 / (r * r * r * r * r * r);
            }
    return s;
}

/* Per-row sums of the far shell: F0_i = sum_j n_j phi_far(i, j) and      */
/* Fq_i = sum_j n_j d phi_far(i, j) / d q_i, over every kept j (rows as   */
/* in vo_pair_rows).  T is tabulated first over all grid displacements.  */
int vo_far_rows(long npts, const int32_t *ix, const int32_t *iy, const int32_t *iz,
                const double *n, const double *q,
                const double E[9], const int32_t gdim[3], const int32_t periodic[3],
                const int32_t image_max[3], const int32_t far_max[3],
                long nrows, const int64_t *rows, double *F0, double *Fq)
{
    const long ex = 2L * gdim[0] - 1, ey = 2L * gdim[1] - 1, ez = 2L * gdim[2] - 1;
    const long ne = ex * ey * ez;
    double *T = (double *)malloc(sizeof(double) * (size_t)ne);
    if (!T) return -1;
#pragma omp parallel for schedule(dynamic, 64)
    for (long e = 0; e < ne; ++e) {
        long d0 = e % ex, rest = e / ex;
        long d1 = rest % ey, d2 = rest / ey;
        T[e] = vo_far_T(E, gdim, periodic, image_max, far_max, (double)(d0 - (gdim[0] - 1)),
                        (double)(d1 - (gdim[1] - 1)), (double)(d2 - (gdim[2] - 1)));
    }
    const double C = vo_asym_C();
#pragma omp parallel for schedule(dynamic, 16)
    for (long t = 0; t < nrows; ++t) {
        long i = rows ? (long)rows[t] : t;
        double f0 = 0.0, fq = 0.0;
        double qi2 = q[i] * q[i];
        for (long j = 0; j < npts; ++j) {
            long e = (ix[i] - ix[j] + gdim[0] - 1) + ex * ((iy[i] - iy[j] + gdim[1] - 1) + ey * (long)(iz[i] - iz[j] + gdim[2] - 1));
            double qj2 = q[j] * q[j];
            double ph = -C * T[e] / (qi2 * qj2 * (qi2 + qj2));
            f0 += n[j] * ph;
            fq += n[j] * (-ph) * (2.0 / q[i] + 2.0 * q[i] / (qi2 + qj2));
        }
        F0[t] = f0;
        Fq[t] = fq;
    }
    free(T);
    return 0;
}

int vo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
