// Kernel table builder: phi(D_k, sigma_l) by the double integral of Dion et
// al. (their Eq. 14; the paper, Sec. 2, computes phi this way), in FP64,
// one workgroup per table node.
//
// Quadrature rule (written in vdwdf.h): Gauss-Legendre points on panels
// [0, w 2^-K], [w 2^-(j+1), w 2^-j] (j = K-1..0), [t w, (t+1) w] up to A, with
// w = pi/2 and A the smallest odd multiple of w with A >= max(A0, kappa
// max(d1, d2)).  The integrand
//   a^2 b^2 W(a,b) T(nu1(a), nu1(b), nu2(a), nu2(b))
// is evaluated as
//   2 (U_b (P_a - 3 U_a) + P_b U_a) * S (c_a c_b + s5 s6) / (2 s1 s2 c_a c_b s5 s6)
// with P = x sin x, U = (sin x - x cos x)/x, c = nu1 + nu2, S = c_a + c_b,
// s1 = nu1(a)+nu1(b), s2 = nu2(a)+nu2(b), s5 = nu1(a)+nu2(b), s6 = nu2(a)+nu1(b):
// the factors 2 of a^2 b^2 W and 1/2 of T cancel, and T's four reciprocals
// become one (w+y = c_a and x+z = c_b), taken as the hardware estimate with
// two Newton steps.  The integrand is symmetric in (a, b): the double sum
// visits the pairs j >= i only.
#include <math.h>

#include <vector>

#include "common.h"

namespace vdw {

namespace {

constexpr int kTableThreads = 256;
constexpr int kChunk = kTableThreads;  // j-nodes staged in LDS per pass, one per thread

struct TableArgs {
    int nD, nS, ng, K;
    double dD, kappa, A0;
    double glx[32];
    double glw[32];
};

// Host: Gauss-Legendre nodes on [-1, 1]: Newton's method on P_n started from
// Tricomi's approximation, P_n and P_n' from the upward recurrences
//   k P_k = (2k-1) x P_{k-1} - (k-1) P_{k-2},   P_k' = P_{k-2}' + (2k-1) P_{k-1}.
void legendre_nodes(int n, double *x, double *w)
{
    const double pi = 3.14159265358979323846;
    for (int i = 1; i <= n; ++i) {
        double t = (1.0 - 1.0 / (8.0 * n * n) + 1.0 / (8.0 * n * n * n)) * cos(pi * (4.0 * i - 1.0) / (4.0 * n + 2.0));
        double d = 0.0;
        for (int it = 0; it < 60; ++it) {
            double pm2 = 1.0, pm1 = t, dm2 = 0.0, dm1 = 1.0;
            double p = (n == 1) ? t : 0.0, dp = (n == 1) ? 1.0 : 0.0;
            for (int k = 2; k <= n; ++k) {
                p = ((2.0 * k - 1.0) * t * pm1 - (k - 1.0) * pm2) / k;
                dp = dm2 + (2.0 * k - 1.0) * pm1;
                pm2 = pm1;
                pm1 = p;
                dm2 = dm1;
                dm1 = dp;
            }
            d = dp;
            double step = p / dp;
            t -= step;
            if (fabs(step) <= 1e-17) break;
        }
        // derivative at the final node
        {
            double pm2 = 1.0, pm1 = t, dm2 = 0.0, dm1 = 1.0, dp = 1.0;
            for (int k = 2; k <= n; ++k) {
                double p = ((2.0 * k - 1.0) * t * pm1 - (k - 1.0) * pm2) / k;
                dp = dm2 + (2.0 * k - 1.0) * pm1;
                pm2 = pm1;
                pm1 = p;
                dm2 = dm1;
                dm1 = dp;
            }
            d = dp;
        }
        x[n - i] = t;
        w[n - i] = 2.0 / ((1.0 - t * t) * d * d);
    }
}

struct Node {
    double P, U, n1, n2, c, w;
};

__device__ inline double node_U(double x)
{
    if (x < 0.5) {
        // (sin x - x cos x)/x = sum_k (-1)^(k+1) 2k x^(2k) / (2k+1)!, Horner in x^2
        double y = x * x;
        double s = 1.0 / 22230464256000.0;
        s = 1.0 / 93405312000.0 - y * s;
        s = 1.0 / 518918400.0 - y * s;
        s = 1.0 / 3991680.0 - y * s;
        s = 1.0 / 45360.0 - y * s;
        s = 1.0 / 840.0 - y * s;
        s = 1.0 / 30.0 - y * s;
        s = 1.0 / 3.0 - y * s;
        return y * s;
    }
    double sn, cs;
    sincos(x, &sn, &cs);
    return (sn - x * cs) / x;
}

__device__ inline double node_nu(double y, double d)
{
    // y^2 / (2 h(y/d)), h(t) = 1 - exp(-(4 pi/9) t^2); h = 1 for d = 0
    if (d == 0.0) return 0.5 * y * y;
    const double gamma = 4.0 * 3.14159265358979323846 / 9.0;
    double t = y / d;
    return 0.5 * y * y / (-expm1(-gamma * t * t));
}

__device__ inline Node make_node(const TableArgs &a, int idx, double d1, double d2)
{
    const double w0 = 0.5 * 3.14159265358979323846;
    int p = idx / a.ng, g = idx - p * a.ng;
    double lo, hi;
    if (p == 0) {
        lo = 0.0;
        hi = ldexp(w0, -a.K);
    } else if (p <= a.K) {
        lo = ldexp(w0, -(a.K - p + 1));
        hi = ldexp(w0, -(a.K - p));
    } else {
        double t = (double)(p - a.K);
        lo = t * w0;
        hi = (t + 1.0) * w0;
    }
    double half = 0.5 * (hi - lo);
    double x = 0.5 * (hi + lo) + half * a.glx[g];
    Node nd;
    nd.w = half * a.glw[g];
    nd.P = x * sin(x);
    nd.U = node_U(x);
    nd.n1 = node_nu(x, d1);
    nd.n2 = node_nu(x, d2);
    nd.c = nd.n1 + nd.n2;
    return nd;
}

// Points per axis of the rule at (d1, d2): the graded panels and the panels of
// width pi/2 up to A, the smallest odd multiple of pi/2 >= max(A0, kappa max(d1, d2)).
__host__ __device__ inline int64_t rule_points(int ng, int K, double kappa, double A0, double d1, double d2)
{
    const double w0 = 0.5 * 3.14159265358979323846;
    double target = fmax(A0, kappa * fmax(d1, d2));
    int64_t m = (int64_t)ceil((target / w0 - 1.0) * 0.5);
    if (m < 0) m = 0;
    while ((2.0 * m + 1.0) * w0 < target) ++m;
    return (K + 1 + 2 * m) * (int64_t)ng;
}

// FP64 reciprocal of a positive normal x: the hardware estimate and two Newton
// steps (each squares the relative error), about one ulp.
__device__ inline double rcp_refined(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// One workgroup per table node.  The integrand is symmetric under a <-> b, so
// only the blocks on and above the diagonal are visited: the 256 threads take
// one i-node each (a block of 256 consecutive nodes, set up once), and the
// j-nodes of each later chunk of 256 are staged in LDS with their weight folded
// into P and U.  Pairs j > i count twice, j = i once.  Padding nodes carry zero
// weight and finite values.
__global__ __launch_bounds__(kTableThreads) void phi_node_kernel(TableArgs a, double *__restrict__ phi)
{
    __shared__ double s1[kChunk], s2[kChunk], sc[kChunk], swP[kChunk], swU[kChunk];
    __shared__ double red[kTableThreads];

    const int node = blockIdx.x;
    const int k = 1 + node / a.nS, l = node - (node / a.nS) * a.nS;
    const double D = k * a.dD;
    const double delta = sqrt((double)l / (double)(a.nS - 1));
    const double d1 = D * (1.0 + delta), d2 = D * (1.0 - delta);
    const int n = (int)rule_points(a.ng, a.K, a.kappa, a.A0, d1, d2);
    const int nb = (n + kChunk - 1) / kChunk;
    const int tid = threadIdx.x;

    double acc = 0.0;
    for (int ib = 0; ib < nb; ++ib) {
        const int i = ib * kChunk + tid;
        Node ni = make_node(a, min(i, n - 1), d1, d2);
        const double wi = (i < n) ? ni.w : 0.0;
        const double Ai = ni.P - 3.0 * ni.U;  // a^2 b^2 W / 2 = U_j (P_i - 3 U_i) + P_j U_i
        double off = 0.0, diag = 0.0;
        for (int jb = ib; jb < nb; ++jb) {
            __syncthreads();
            {
                const int j = jb * kChunk + tid;
                Node nj = make_node(a, min(j, n - 1), d1, d2);
                const double wj = (j < n) ? nj.w : 0.0;
                s1[tid] = nj.n1;
                s2[tid] = nj.n2;
                sc[tid] = nj.c;
                swP[tid] = wj * nj.P;
                swU[tid] = wj * nj.U;
            }
            __syncthreads();
            if (jb == ib) {
                for (int t = 0; t < kChunk; ++t) {
                    const double cc = ni.c * sc[t];
                    const double s56 = (ni.n1 + s2[t]) * (ni.n2 + s1[t]);
                    const double num = (ni.c + sc[t]) * (cc + s56);
                    const double den = (ni.n1 + s1[t]) * (ni.n2 + s2[t]) * cc * s56;
                    const double wpart = fma(swU[t], Ai, swP[t] * ni.U);
                    const double f = (t > tid) ? 2.0 : (t == tid ? 1.0 : 0.0);
                    diag = fma(f * wpart * num, rcp_refined(den), diag);
                }
            } else {
                for (int t = 0; t < kChunk; ++t) {
                    const double cc = ni.c * sc[t];
                    const double s56 = (ni.n1 + s2[t]) * (ni.n2 + s1[t]);
                    const double num = (ni.c + sc[t]) * (cc + s56);
                    const double den = (ni.n1 + s1[t]) * (ni.n2 + s2[t]) * cc * s56;
                    const double wpart = fma(swU[t], Ai, swP[t] * ni.U);
                    off = fma(wpart * num, rcp_refined(den), off);
                }
            }
        }
        acc = fma(wi, fma(2.0, off, diag), acc);
    }
    red[tid] = acc;
    __syncthreads();
    for (int s = kTableThreads / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) {
        const double pi = 3.14159265358979323846;
        phi[(long)k * a.nS + l] = 2.0 / (pi * pi) * red[0];
    }
}

// Row 0 (D = 0) by linear extrapolation from rows 1 and 2, then the FP32 copy.
__global__ void phi_row0_kernel(int nS, double *__restrict__ phi)
{
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nS) phi[l] = 2.0 * phi[nS + l] - phi[2 * nS + l];
}

__global__ void phi_to_f32_kernel(long total, const double *__restrict__ phi, float *__restrict__ out)
{
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < total) out[t] = (float)phi[t];
}

}  // namespace

// Gauss-Legendre nodes (ascending) and weights on [-1, 1], for other parts of
// the library.
void gauss_legendre_nodes(int n, double *x, double *w) { legendre_nodes(n, x, w); }

int launch_phi_table(const vdw_table_params *tp, double *phi_d, float *phi_f, hipStream_t s)
{
    TableArgs a;
    a.nD = tp->n_D;
    a.nS = tp->n_sigma;
    a.ng = tp->gl_points;
    a.K = tp->graded_levels;
    a.dD = tp->D_max / (tp->n_D - 1);
    a.kappa = tp->kappa;
    a.A0 = tp->A0;
    legendre_nodes(a.ng, a.glx, a.glw);
    int nodes = (tp->n_D - 1) * tp->n_sigma;
    hipLaunchKernelGGL(phi_node_kernel, dim3(nodes), dim3(kTableThreads), 0, s, a, phi_d);
    VDW_HIP(hipGetLastError());
    hipLaunchKernelGGL(phi_row0_kernel, dim3((tp->n_sigma + 255) / 256), dim3(256), 0, s, tp->n_sigma, phi_d);
    VDW_HIP(hipGetLastError());
    if (phi_f) {
        long total = (long)tp->n_D * tp->n_sigma;
        hipLaunchKernelGGL(phi_to_f32_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total,
                           (const double *)phi_d, phi_f);
        VDW_HIP(hipGetLastError());
    }
    return VDW_OK;
}

}  // namespace vdw

extern "C" int build_phi_table(const vdw_table_params *tp, double *phi_d, float *phi_f, void *stream)
{
    int rc = vdw::validate_table(tp);
    if (rc) return rc;
    // the largest node count per axis is at D_max, delta = 1 (d1 = 2 D_max, d2 = 0)
    const int64_t npts = vdw::rule_points(tp->gl_points, tp->graded_levels, tp->kappa, tp->A0, 2.0 * tp->D_max, 0.0);
    if (npts > ((int64_t)1 << 20))
        return vdw::fail(VDW_EINVAL, "the quadrature rule needs %lld points per axis at D_max (at most 2^20)",
                         (long long)npts);
    if (!phi_d) return vdw::fail(VDW_EINVAL, "phi_d is NULL");
    hipStream_t s = (hipStream_t)stream;
    rc = vdw::launch_phi_table(tp, phi_d, phi_f, s);
    if (rc) return rc;
    VDW_HIP(hipStreamSynchronize(s));
    return VDW_OK;
}
