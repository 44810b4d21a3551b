// Fourier derivative along periodic axes: the spectral gradient that the
// paper's code takes by FFT (Sec. 3; App. A timing).  On N periodic points
// the derivative per grid step is the circulant operator
//   (D f)_j = sum_{m=1}^{N-1} w(m) f_{j-m},
//   w(m) = (pi/N) (-1)^m cot(pi m / N)   (N even; the unpaired Nyquist
//                                          frequency differentiates to 0)
//   w(m) = (pi/N) (-1)^m / sin(pi m / N) (N odd)
// (the closed form of multiplying the DFT by i k; e.g. L. N. Trefethen,
// Spectral Methods in MATLAB, ch. 3).  With N <= 4096 a direct product is
// cheap (N - 1 FMAs per point), exact like the FFT up to rounding, and needs
// no FFT library: one workgroup per grid line stages the line and the
// weights in LDS.
#include <math.h>

#include "common.h"

namespace vdw {

namespace {

constexpr int kSpecThreads = 256;
constexpr int kSpecMaxN = 4096;

// Line `line` of the lines along `axis`: base index and stride.
__device__ inline void line_base(const GridDev &g, int axis, int64_t line, int64_t &base, int64_t &stride, int &N)
{
    const int64_t nx = g.nx, ny = g.ny;
    if (axis == 0) {
        N = g.nx;
        stride = 1;
        base = line * nx;  // lines are (y, z) pairs
    } else if (axis == 1) {
        N = g.ny;
        stride = nx;
        const int64_t x = line % nx, z = line / nx;
        base = z * nx * ny + x;
    } else {
        N = g.nz;
        stride = nx * ny;
        base = line;  // lines are (x, y) pairs
    }
}

__device__ inline void fill_weights(double *w, int N)
{
    const double pi = 3.14159265358979323846;
    for (int m = threadIdx.x; m < N; m += kSpecThreads) {
        double v = 0.0;
        if (m > 0) {
            const double x = pi * m / N;
            const double sgn = (m & 1) ? -1.0 : 1.0;
            v = (N % 2 == 0) ? sgn * (pi / N) * cos(x) / sin(x) : sgn * (pi / N) / sin(x);
        }
        w[m] = v;
    }
}

__global__ __launch_bounds__(kSpecThreads) void spectral_line_kernel(GridDev g, int axis,
                                                                     const double *__restrict__ src,
                                                                     double *__restrict__ dst)
{
    __shared__ double f[kSpecMaxN], w[kSpecMaxN];
    int64_t base, stride;
    int N;
    line_base(g, axis, blockIdx.x, base, stride, N);
    fill_weights(w, N);
    for (int i = threadIdx.x; i < N; i += kSpecThreads) f[i] = src[base + i * stride];
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += kSpecThreads) {
        double acc = 0.0;
        for (int m = 1; m < N; ++m) {
            int k = j - m;
            k += (k < 0) ? N : 0;
            acc += w[m] * f[k];
        }
        dst[base + j * stride] = acc;
    }
}

__global__ __launch_bounds__(kSpecThreads) void spectral_adjoint_kernel(GridDev g, int axis,
                                                                        const double *__restrict__ dEdq,
                                                                        const double *__restrict__ dqdg,
                                                                        const double *__restrict__ grad,
                                                                        double *__restrict__ dst)
{
    __shared__ double f[kSpecMaxN], w[kSpecMaxN];
    int64_t base, stride;
    int N;
    line_base(g, axis, blockIdx.x, base, stride, N);
    fill_weights(w, N);
    const int64_t G = g.G;
    for (int i = threadIdx.x; i < N; i += kSpecThreads) {
        const int64_t p = base + i * stride;
        double ga;
        if (g.skew)
            ga = g.Einv[axis] * grad[p] + g.Einv[3 + axis] * grad[G + p] + g.Einv[6 + axis] * grad[2 * G + p];
        else
            ga = g.Einv[4 * axis] * grad[axis * G + p];
        f[i] = dEdq[p] * dqdg[p] * 2.0 * ga;
    }
    __syncthreads();
    // transpose of (D f)_j = sum_m w(m) f_{j-m}: dst_k += sum_m w(m) B_{k+m}
    for (int k = threadIdx.x; k < N; k += kSpecThreads) {
        double acc = 0.0;
        for (int m = 1; m < N; ++m) {
            int j = k + m;
            j -= (j >= N) ? N : 0;
            acc += w[m] * f[j];
        }
        dst[base + k * stride] += acc;
    }
}

int64_t lines_of(const GridDev &g, int axis)
{
    const int64_t n3[3] = {g.nx, g.ny, g.nz};
    return g.G / n3[axis];
}

}  // namespace

int launch_spectral_lines(const GridDev &g, int axis, const double *src, double *dst, hipStream_t s)
{
    const int n3[3] = {g.nx, g.ny, g.nz};
    if (axis < 0 || axis > 2 || n3[axis] > kSpecMaxN) return fail(VDW_EINVAL, "spectral axis out of range");
    hipLaunchKernelGGL(spectral_line_kernel, dim3((unsigned)lines_of(g, axis)), dim3(kSpecThreads), 0, s, g, axis, src,
                       dst);
    VDW_HIP(hipGetLastError());
    return VDW_OK;
}

int launch_spectral_adjoint(const GridDev &g, int axis, const double *dEdq, const double *dqdg, const double *grad,
                            double *dst, hipStream_t s)
{
    const int n3[3] = {g.nx, g.ny, g.nz};
    if (axis < 0 || axis > 2 || n3[axis] > kSpecMaxN) return fail(VDW_EINVAL, "spectral axis out of range");
    hipLaunchKernelGGL(spectral_adjoint_kernel, dim3((unsigned)lines_of(g, axis)), dim3(kSpecThreads), 0, s, g, axis,
                       dEdq, dqdg, grad, dst);
    VDW_HIP(hipGetLastError());
    return VDW_OK;
}

}  // namespace vdw
