// Density gradient by second-order finite differences (the paper's Sec. 3
// real-space option; along the grid axes, mapped to Cartesian components on
// skew cells) and q0 of Dion et al. from the LDA exchange, the Perdew-Wang
// 1992 correlation and the gradient term.
// One thread per grid point, FP64 throughout.
#include <math.h>

#include "common.h"
#include "q0_point.h"

namespace vdw {

namespace {

__global__ __launch_bounds__(256) void grad_q0_kernel(GridDev g, double n_cut, const double *__restrict__ n,
                                                      double *__restrict__ grad, double *__restrict__ q0,
                                                      double *__restrict__ dqdn, double *__restrict__ dqdg)
{
    long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.G) return;
    const bool spec = g.spec[0] || g.spec[1] || g.spec[2];
    grad_q0_point(n, t, g.nx, g.ny, g.nz, g.px, g.py, g.pz, g.hx, g.hy, g.hz, g.skew ? g.Einv : nullptr,
                  spec ? g.spec : nullptr, g.G, n_cut, grad, q0, dqdn, dqdg);
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
    if (g.spec[0] || g.spec[1] || g.spec[2]) {
        // Fourier derivatives per grid step into the gradient planes first
        if (!grad_d) return vdw::fail(VDW_EINVAL, "the spectral gradient needs grad_d");
        for (int a = 0; a < 3; ++a)
            if (g.spec[a]) {
                rc = vdw::launch_spectral_lines(g, a, n_d, grad_d + a * g.G, (hipStream_t)stream);
                if (rc) return rc;
            }
    }
    return vdw::launch_grad_q0(g, n_cut, n_d, grad_d, q0_d, dq_dn_d, dq_dg_d, 0, (hipStream_t)stream);
}
