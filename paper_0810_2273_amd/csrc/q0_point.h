// Gradient and q0 of one grid point, shared by the single-grid kernel, the
// batched one and the exchange-correlation energies: second-order finite
// differences along the grid axes (Sec. 3; or Fourier derivatives computed
// before), Cartesian components through the spacing or, on skew cells, the
// inverse step matrix; q0 of Dion et al. from the LDA exchange, the
// Perdew-Wang 1992 correlation (its logarithm as log1p) and the gradient
// term; FP64.
#pragma once

#include <math.h>
#include <stdint.h>

namespace vdw {

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

// Perdew-Wang 1992 correlation energy per electron of the unpolarised
// uniform gas, eps_c(r_s) = -2A (1 + a1 r_s) ln(1 + 1/Q), Q = 2A (b1 r_s^1/2
// + b2 r_s + b3 r_s^3/2 + b4 r_s^2), the logarithm as log1p; *dec = d eps_c / d r_s.
__device__ inline double pw92_ec(double rs, double *dec)
{
    const double A = 0.031091, a1 = 0.21370;
    const double b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294;
    double srs = sqrt(rs);
    double Q = 2.0 * A * (srs * (b1 + b3 * rs) + rs * (b2 + b4 * rs));
    double Lg = log1p(1.0 / Q);
    if (dec) {
        double dQ = 2.0 * A * (0.5 * b1 / srs + b2 + 1.5 * b3 * srs + 2.0 * b4 * rs);
        *dec = -2.0 * A * a1 * Lg + 2.0 * A * (1.0 + a1 * rs) * dQ / (Q * (Q + 1.0));
    }
    return -2.0 * A * (1.0 + a1 * rs) * Lg;
}

// Cartesian gradient at point t of an nx x ny x nz grid: differences along
// the grid axes, divided by h_a on orthorhombic grids (einv = NULL), or per
// grid step and mapped by E^-1 (row-major einv) on skew grids.  With spec
// (per-axis flags, or NULL) the derivative per grid step of a flagged axis
// is read from plane a of pre (the Fourier derivative, computed before).
__device__ inline void grad_point(const double *__restrict__ n, long t, int nx, int ny, int nz, int px, int py,
                                  int pz, double hx, double hy, double hz, const double *einv, const int *spec,
                                  const double *pre, long G, double &gx, double &gy, double &gz)
{
    int ix = (int)(t % nx);
    long r = t / nx;
    int iy = (int)(r % ny);
    int iz = (int)(r / ny);
    if (!einv && !spec) {
        gx = fd_axis(n, t, ix, nx, 1, px, 0.5 / hx);
        gy = fd_axis(n, t, iy, ny, nx, py, 0.5 / hy);
        gz = fd_axis(n, t, iz, nz, (long)nx * ny, pz, 0.5 / hz);
        return;
    }
    const double d0 = (spec && spec[0]) ? pre[t] : fd_axis(n, t, ix, nx, 1, px, 0.5);
    const double d1 = (spec && spec[1]) ? pre[G + t] : fd_axis(n, t, iy, ny, nx, py, 0.5);
    const double d2 = (spec && spec[2]) ? pre[2 * G + t] : fd_axis(n, t, iz, nz, (long)nx * ny, pz, 0.5);
    if (!einv) {
        gx = d0 / hx;
        gy = d1 / hy;
        gz = d2 / hz;
        return;
    }
    gx = einv[0] * d0 + einv[1] * d1 + einv[2] * d2;
    gy = einv[3] * d0 + einv[4] * d1 + einv[5] * d2;
    gz = einv[6] * d0 + einv[7] * d1 + einv[8] * d2;
}

// Point t (x fastest) of an nx x ny x nz grid of G points whose density
// starts at n: writes grad (3 planes of G, if non-null), q0, dq0/dn at fixed
// |grad n|^2 and dq0/d|grad n|^2 (0 where n < n_cut).  einv and spec as for
// grad_point; with spec the Fourier derivatives are read from grad (each
// point reads its own entries before it overwrites them).
__device__ inline void grad_q0_point(const double *__restrict__ n, long t, int nx, int ny, int nz, int px, int py,
                                     int pz, double hx, double hy, double hz, const double *einv, const int *spec,
                                     long G, double n_cut, double *grad, double *__restrict__ q0,
                                     double *__restrict__ dqdn, double *__restrict__ dqdg)
{
    double gx, gy, gz;
    grad_point(n, t, nx, ny, nz, px, py, pz, hx, hy, hz, einv, spec, grad, G, gx, gy, gz);
    if (grad) {
        grad[t] = gx;
        grad[G + t] = gy;
        grad[2 * G + t] = gz;
    }
    double nn = n[t];
    double q = 0.0, a = 0.0, b = 0.0;
    if (nn >= n_cut) {
        const double pi = 3.14159265358979323846;
        const double Zab = -0.8491;
        double gg = gx * gx + gy * gy + gz * gz;
        double kF = cbrt(3.0 * pi * pi * nn);
        double rs = cbrt(3.0 / (4.0 * pi * nn));
        double dec;
        double ec = pw92_ec(rs, &dec);
        double inv_kn2 = 1.0 / (kF * nn * nn);
        q = kF - (4.0 * pi / 3.0) * ec - (Zab / 36.0) * gg * inv_kn2;
        a = kF / (3.0 * nn) + (4.0 * pi / 9.0) * dec * rs / nn + (7.0 * Zab / 108.0) * gg * inv_kn2 / nn;
        b = -(Zab / 36.0) * inv_kn2;
    }
    q0[t] = q;
    if (dqdn) dqdn[t] = a;
    if (dqdg) dqdg[t] = b;
}

}  // namespace vdw
