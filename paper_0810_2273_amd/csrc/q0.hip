// Density gradient by second-order finite differences (the paper's Sec. 3
// real-space option, perpendicular axes) and q0 of Dion et al. from the LDA
// exchange, the Perdew-Wang 1992 correlation and the gradient term.
// One thread per grid point, FP64 throughout (the logarithm of the PW92
// correlation is taken as log1p so it stays accurate near the cut-off).
#include <math.h>

#include "common.h"

namespace vdw {

namespace {

// d n / d axis at point i of an axis with N points, memory stride `st`.
__device__ inline double fd_axis(const double *__restrict__ n, long idx, int i, int N, long st, int per,
                                 double inv2h)
{
    if (per) {
        long up = (i + 1 == N) ? -(long)(N - 1) * st : st;
        long dn = (i == 0) ? (long)(N - 1) * st : -st;
        return (n[idx + up] - n[idx + dn]) * inv2h;
    }
    if (i == 0) return (-3.0 * n[idx] + 4.0 * n[idx + st] - n[idx + 2 * st]) * inv2h;
    if (i == N - 1) return (3.0 * n[idx] - 4.0 * n[idx - st] + n[idx - 2 * st]) * inv2h;
    return (n[idx + st] - n[idx - st]) * inv2h;
}

__global__ __launch_bounds__(256) void grad_q0_kernel(GridDev g, double n_cut, const double *__restrict__ n,
                                                      double *__restrict__ grad, double *__restrict__ q0,
                                                      double *__restrict__ dqdn, double *__restrict__ dqdg)
{
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.G) return;
    int ix = (int)(t % g.nx);
    long r = t / g.nx;
    int iy = (int)(r % g.ny);
    int iz = (int)(r / g.ny);
    double gx = fd_axis(n, t, ix, g.nx, 1, g.px, 0.5 / g.hx);
    double gy = fd_axis(n, t, iy, g.ny, g.nx, g.py, 0.5 / g.hy);
    double gz = fd_axis(n, t, iz, g.nz, (long)g.nx * g.ny, g.pz, 0.5 / g.hz);
    if (grad) {
        grad[t] = gx;
        grad[g.G + t] = gy;
        grad[2 * g.G + t] = gz;
    }
    double nn = n[t];
    double q = 0.0, a = 0.0, b = 0.0;
    if (nn >= n_cut) {
        const double pi = 3.14159265358979323846;
        const double A = 0.031091, a1 = 0.21370;
        const double b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294;
        const double Zab = -0.8491;
        double gg = gx * gx + gy * gy + gz * gz;
        double kF = cbrt(3.0 * pi * pi * nn);
        double rs = cbrt(3.0 / (4.0 * pi * nn));
        double srs = sqrt(rs);
        double Q = 2.0 * A * (srs * (b1 + b3 * rs) + rs * (b2 + b4 * rs));
        double Lg = log1p(1.0 / Q);
        double ec = -2.0 * A * (1.0 + a1 * rs) * Lg;
        double dQ = 2.0 * A * (0.5 * b1 / srs + b2 + 1.5 * b3 * srs + 2.0 * b4 * rs);
        double dec = -2.0 * A * a1 * Lg + 2.0 * A * (1.0 + a1 * rs) * dQ / (Q * (Q + 1.0));
        double inv_kn2 = 1.0 / (kF * nn * nn);
        q = kF - (4.0 * pi / 3.0) * ec - (Zab / 36.0) * gg * inv_kn2;
        a = kF / (3.0 * nn) + (4.0 * pi / 9.0) * dec * rs / nn + (7.0 * Zab / 108.0) * gg * inv_kn2 / nn;
        b = -(Zab / 36.0) * inv_kn2;
    }
    q0[t] = q;
    if (dqdn) dqdn[t] = a;
    if (dqdg) dqdg[t] = b;
}

}  // namespace

int launch_grad_q0(const GridDev &g, double n_cut, const double *n, double *grad, double *q0, double *dqdn,
                   double *dqdg, int64_t off, hipStream_t s)
{
    long blocks = (g.G + 255) / 256;
    hipLaunchKernelGGL(grad_q0_kernel, dim3((unsigned)blocks), dim3(256), 0, s, g, n_cut, n + off,
                       grad ? grad + 3 * off : nullptr, q0 + off, dqdn ? dqdn + off : nullptr,
                       dqdg ? dqdg + off : nullptr);
    VDW_HIP(hipGetLastError());
    return VDW_OK;
}

}  // namespace vdw

extern "C" int compute_q0(const vdw_grid *grid, double n_cut, const double *n_d, double *grad_d, double *q0_d,
                          double *dq_dn_d, double *dq_dg_d, void *stream)
{
    vdw::GridDev g;
    int rc = vdw::validate_grid(grid, &g);
    if (rc) return rc;
    if (!n_d || !q0_d) return vdw::fail(VDW_EINVAL, "n_d and q0_d must not be NULL");
    if (!(n_cut > 0.0) || !isfinite(n_cut)) return vdw::fail(VDW_EINVAL, "n_cut must be > 0");
    return vdw::launch_grad_q0(g, n_cut, n_d, grad_d, q0_d, dq_dn_d, dq_dg_d, 0, (hipStream_t)stream);
}
