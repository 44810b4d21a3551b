// Local and semilocal exchange-correlation energies of the recombination of
// Eq. (3): E_x^LDA, E_c^LDA (Perdew-Wang 1992), E_x^PBE, E_c^PBE and
// E_x^revPBE of one density, spin-unpolarised, FP64.  The paper's code
// evaluates them from the same density before the nonlocal sum (Sec. 3).
//
// One thread per grid point (the gradient by the finite differences of the
// q0 kernel, read through L1/L2 from the density), five per-thread sums,
// a fixed butterfly per wavefront and a fixed-order sum over the block's
// wavefronts, then one block that adds the block partials the same way: the
// result does not depend on scheduling.
#include <math.h>

#include "common.h"
#include "q0_point.h"

namespace vdw {

namespace {

constexpr int kXcThreads = 256;
constexpr int kXcMaxBlocks = 2048;
constexpr int kXcTerms = 5;

struct XcArgs {
    GridDev g;
    const double *n;
    double n_floor;
    double inv2h[3];  // 1 / (2 h) per axis
    int64_t chunk;    // grid points per block (multiple of kXcThreads)
    double *part;   // kXcTerms x blocks
    double *out;    // kXcTerms + 1 (the last: a non-finite flag)
    const double *pre;  // spectral gradient: Fourier derivatives per grid step (3 planes), else NULL
};

// n eps for the five energies at one point (0 at or below the floor).
__device__ inline void xc_point(const XcArgs &a, int64_t t, double e[kXcTerms])
{
    const double pi = 3.14159265358979323846;
    const double kappa_pbe = 0.804, kappa_rev = 1.245;
    const double beta = 0.06672455060314922;
    const double mu = beta * pi * pi / 3.0;
    const double gamma = (1.0 - 0.69314718055994530942) / (pi * pi);
    const double nn = a.n[t];
    for (int k = 0; k < kXcTerms; ++k) e[k] = 0.0;
    if (!(nn > a.n_floor)) return;
    // (3 pi^2)^(1/3) and (3 / (4 pi))^(1/3): k_F and r_s from one cube root
    const double c_kf = 3.0936677262801355, c_rs = 0.6203504908994001;
    const GridDev &g = a.g;
    double gx, gy, gz;
    if (g.skew || a.pre) {
        grad_point(a.n, t, g.nx, g.ny, g.nz, g.px, g.py, g.pz, g.hx, g.hy, g.hz, g.skew ? g.Einv : nullptr,
                   a.pre ? g.spec : nullptr, a.pre, g.G, gx, gy, gz);
    } else {
        const int ix = (int)(t % g.nx);
        const int64_t r = t / g.nx;
        const int iy = (int)(r % g.ny);
        const int iz = (int)(r / g.ny);
        gx = fd_axis(a.n, t, ix, g.nx, 1, g.px, a.inv2h[0]);
        gy = fd_axis(a.n, t, iy, g.ny, g.nx, g.py, a.inv2h[1]);
        gz = fd_axis(a.n, t, iz, g.nz, (int64_t)g.nx * g.ny, g.pz, a.inv2h[2]);
    }
    const double g2 = gx * gx + gy * gy + gz * gz;
    const double cr = cbrt(nn);
    const double kF = c_kf * cr;
    const double rs = c_rs / cr;
    const double ex = (-3.0 / (4.0 * pi)) * kF;
    const double ec = pw92_ec(rs, nullptr);
    const double gn = g2 / (kF * nn * nn);  // |grad n|^2 / (k_F n^2)
    // exchange: F_x(s) = 1 + kappa - kappa / (1 + mu s^2 / kappa), s = |grad n| / (2 k_F n)
    const double s2 = 0.25 * gn / kF;
    const double fx_pbe = 1.0 + kappa_pbe - kappa_pbe * kappa_pbe / (kappa_pbe + mu * s2);
    const double fx_rev = 1.0 + kappa_rev - kappa_rev * kappa_rev / (kappa_rev + mu * s2);
    // correlation: H = gamma ln(1 + (beta/gamma) t^2 (1 + A t^2) / (1 + A t^2 + A^2 t^4)),
    // A = (beta/gamma) / (exp(-eps_c/gamma) - 1), t = |grad n| / (2 k_s n), k_s^2 = 4 k_F / pi
    const double t2 = (pi / 16.0) * gn;
    const double bg = beta / gamma;
    const double A = bg / expm1(-ec * (1.0 / gamma));
    const double y = A * t2;
    const double H = gamma * log1p(bg * t2 * (1.0 + y) / (1.0 + y + y * y));
    e[0] = nn * ex;
    e[1] = nn * ec;
    e[2] = nn * ex * fx_pbe;
    e[3] = nn * (ec + H);
    e[4] = nn * ex * fx_rev;
}

// Block sums of the kXcTerms values of every thread (all threads call):
// each wavefront adds its 64 lanes by a fixed xor butterfly, then thread k
// adds the wavefronts' sums of term k in wavefront order.  Returns the sum
// in thread k < kXcTerms.
template <int NT>
__device__ inline double block_sums(double (&v)[kXcTerms], double *red)
{
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int k = 0; k < kXcTerms; ++k) {
        double x = v[k];
        for (int m = 32; m > 0; m >>= 1) x += __shfl_xor(x, m, 64);
        v[k] = x;
    }
    if (lane == 0)
        for (int k = 0; k < kXcTerms; ++k) red[k * NW + w] = v[k];
    __syncthreads();
    double s = 0.0;
    if ((int)threadIdx.x < kXcTerms)
        for (int u = 0; u < NW; ++u) s += red[threadIdx.x * NW + u];
    return s;
}

__global__ __launch_bounds__(kXcThreads) void xc_kernel(XcArgs a)
{
    __shared__ double red[kXcTerms * (kXcThreads / 64)];
    double acc[kXcTerms] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int64_t lo = (int64_t)blockIdx.x * a.chunk;
    const int64_t hi = min(a.g.G, lo + a.chunk);
    for (int64_t t = lo + threadIdx.x; t < hi; t += kXcThreads) {
        double e[kXcTerms];
        xc_point(a, t, e);
        for (int k = 0; k < kXcTerms; ++k) acc[k] += e[k];
    }
    const double s = block_sums<kXcThreads>(acc, red);
    if ((int)threadIdx.x < kXcTerms) a.part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
}

// One block of kXcReduceThreads: term k = dV x the block partials, each
// thread adding its strided share (all terms' loads in flight together),
// then the fixed-order block sums; out[kXcTerms] flags a non-finite term.
constexpr int kXcReduceThreads = 1024;

__global__ __launch_bounds__(kXcReduceThreads) void xc_reduce_kernel(const double *__restrict__ part, int blocks,
                                                                     double dV, double *__restrict__ out)
{
    __shared__ double red[kXcTerms * (kXcReduceThreads / 64)];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    double s[kXcTerms] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < blocks; b += kXcReduceThreads)
        for (int k = 0; k < kXcTerms; ++k) s[k] += part[(int64_t)k * blocks + b];
    const double t = block_sums<kXcReduceThreads>(s, red);
    if ((int)threadIdx.x < kXcTerms) {
        out[threadIdx.x] = dV * t;
        if (!isfinite(t)) atomicOr(&bad, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) out[kXcTerms] = bad ? 1.0 : 0.0;
}

int xc_blocks(int64_t G)
{
    const int64_t b = (G + kXcThreads - 1) / kXcThreads;
    return (int)(b < kXcMaxBlocks ? b : kXcMaxBlocks);
}

}  // namespace

}  // namespace vdw

extern "C" size_t xc_workspace_size(const vdw_grid *grid)
{
    vdw::GridDev g;
    if (vdw::validate_grid(grid, &g)) return 0;
    const int blocks = vdw::xc_blocks(g.G);
    size_t bytes = ((size_t)vdw::kXcTerms * blocks + vdw::kXcTerms + 1) * sizeof(double);
    if (g.spec[0] || g.spec[1] || g.spec[2]) bytes = (bytes + 255) / 256 * 256 + 3 * (size_t)g.G * sizeof(double);
    return bytes;
}

extern "C" int xc_energies(const vdw_grid *grid, const double *n_d, double n_floor, void *ws, size_t ws_bytes,
                           double *E, void *stream)
{
    vdw::GridDev g;
    int rc = vdw::validate_grid(grid, &g);
    if (rc) return rc;
    if (!n_d || !ws || !E) return vdw::fail(VDW_EINVAL, "n_d, ws and E must not be NULL");
    if (!(n_floor >= 0.0) || !isfinite(n_floor)) return vdw::fail(VDW_EINVAL, "n_floor must be finite and >= 0");
    const size_t need = xc_workspace_size(grid);
    if (ws_bytes < need) return vdw::fail(VDW_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    const int blocks = vdw::xc_blocks(g.G);
    vdw::XcArgs a;
    a.g = g;
    a.n = n_d;
    a.n_floor = n_floor;
    a.inv2h[0] = 0.5 / g.hx;
    a.inv2h[1] = 0.5 / g.hy;
    a.inv2h[2] = 0.5 / g.hz;
    const int64_t per = (g.G + blocks - 1) / blocks;
    a.chunk = (per + vdw::kXcThreads - 1) / vdw::kXcThreads * vdw::kXcThreads;
    a.part = (double *)ws;
    a.out = a.part + (int64_t)vdw::kXcTerms * blocks;
    a.pre = nullptr;
    if (g.spec[0] || g.spec[1] || g.spec[2]) {
        // Fourier derivatives per grid step of the periodic axes, before the energies
        const size_t head = (((size_t)vdw::kXcTerms * blocks + vdw::kXcTerms + 1) * sizeof(double) + 255) / 256 * 256;
        double *pre = (double *)((char *)ws + head);
        for (int ax = 0; ax < 3; ++ax)
            if (g.spec[ax]) {
                rc = vdw::launch_spectral_lines(g, ax, n_d, pre + ax * g.G, s);
                if (rc) return rc;
            }
        a.pre = pre;
    }
    // blocks whose chunk starts beyond the grid (chunk rounding) write zero partials
    hipLaunchKernelGGL(vdw::xc_kernel, dim3(blocks), dim3(vdw::kXcThreads), 0, s, a);
    VDW_HIP(hipGetLastError());
    hipLaunchKernelGGL(vdw::xc_reduce_kernel, dim3(1), dim3(vdw::kXcReduceThreads), 0, s, (const double *)a.part,
                       blocks, g.dV, a.out);
    VDW_HIP(hipGetLastError());
    double out[vdw::kXcTerms + 1];
    VDW_HIP(hipMemcpyAsync(out, a.out, sizeof(out), hipMemcpyDeviceToHost, s));
    VDW_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < vdw::kXcTerms; ++k) E[k] = out[k];
    if (out[vdw::kXcTerms] != 0.0) return vdw::fail(VDW_ENONFINITE, "non-finite exchange-correlation energy "
                                                                    "(a density at or near zero above n_floor?)");
    return VDW_OK;
}

extern "C" double vdw_recombine(const double *E_xc, double E_nl, double E_dft, int32_t exchange)
{
    if (!E_xc || (exchange != 0 && exchange != 1)) return NAN;
    const double ex = exchange == 1 ? E_xc[4] : E_xc[2];
    return E_dft - E_xc[2] - E_xc[3] + (ex + E_xc[1] + E_nl);
}
