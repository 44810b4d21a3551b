// Far image shell: the images beyond the near range (image_max) up to
// far_max enter with the kernel's large-D asymptote (Dion et al., their
// Eq. 17, named in Sec. 2), the form the paper's outlook (Sec. 7) proposes
// for the sums over repeated cells.  Summed over the shell, pair (i, j)
// contributes -C T(r_i - r_j) / (q_i^2 q_j^2 (q_i^2 + q_j^2)) with the
// lattice sum T(d) = sum_L |d - L|^-6, so the shell costs one table of T
// over the grid displacements and one O(N^2) pass, whatever its size.
//
//   far_table  one thread per displacement: the shell's lattice sum in
//              FP64, in a fixed order
//   far_rows   one lane per kept point i (two per thread), every j of the
//              density streamed through scalar loads; T gathered at the
//              displacement (the lanes of a wavefront are one brick of
//              points, so their gathers hit a few cache lines); FP64
//              sums, the pair i = j included
#include <math.h>

#include "common.h"

namespace vdw {

namespace {

constexpr int kFarThreads = 256;
constexpr int kFarIPL = 2;  // kept points per thread (amortises the wave-uniform j work)

__global__ __launch_bounds__(kFarThreads) void far_table_kernel(FarGeo g, int64_t ne, double *__restrict__ T)
{
    const int64_t e = (int64_t)blockIdx.x * kFarThreads + threadIdx.x;
    if (e >= ne) return;
    const int64_t ex = 2 * g.nx - 1, ey = 2 * g.ny - 1;
    const double d0 = (double)(e % ex - (g.nx - 1));
    const int64_t rest = e / ex;
    const double d1 = (double)(rest % ey - (g.ny - 1));
    const double d2 = (double)(rest / ey - (g.nz - 1));
    double s = 0.0;
    for (int c = -g.hi[2]; c <= g.hi[2]; ++c)
        for (int b = -g.hi[1]; b <= g.hi[1]; ++b) {
            const bool inner = abs(b) <= g.lo[1] && abs(c) <= g.lo[2];
            for (int a = -g.hi[0]; a <= g.hi[0]; ++a) {
                if (inner && abs(a) <= g.lo[0]) continue;
                const double t0 = d0 - (double)a * g.nx, t1 = d1 - (double)b * g.ny, t2 = d2 - (double)c * g.nz;
                const double x = t0 * g.en[0] + t1 * g.en[3] + t2 * g.en[6];
                const double y = t0 * g.en[1] + t1 * g.en[4] + t2 * g.en[7];
                const double z = t0 * g.en[2] + t1 * g.en[5] + t2 * g.en[8];
                const double m = x * x + y * y + z * z;
                s += 1.0 / (m * m * m);
            }
        }
    T[e] = s;
}

template <typename Rec>
__global__ __launch_bounds__(kFarThreads) void far_rows_kernel(FarGeo g, const Rec *__restrict__ recs,
                                                               const int64_t *__restrict__ nkept,
                                                               const double *__restrict__ T, double casym,
                                                               double qscale, double *__restrict__ far0,
                                                               double *__restrict__ far_q)
{
    const int64_t N = *nkept;
    const int64_t i0 = (int64_t)blockIdx.x * (kFarThreads * kFarIPL);
    if (i0 >= N) return;  // N >= 1 below
    const int64_t ex = 2 * g.nx - 1, ey = 2 * g.ny - 1;
    int64_t base[kFarIPL];
    double pi[kFarIPL], g2[kFarIPL], a2[kFarIPL], acc[kFarIPL], accq[kFarIPL];
#pragma unroll
    for (int p = 0; p < kFarIPL; ++p) {
        const int64_t i = i0 + threadIdx.x + (int64_t)kFarThreads * p;
        const Rec R = recs[i < N ? i : N - 1];
        // table entry of displacement r_i - r_j is base - offset(j)
        base[p] = ((int64_t)R.x + g.nx - 1) + ex * (((int64_t)R.y + g.ny - 1) + ey * ((int64_t)R.z + g.nz - 1));
        const double a = (double)R.a;
        pi[p] = a * a;
        g2[p] = 2.0 / a;
        a2[p] = 2.0 * a;
        acc[p] = accq[p] = 0.0;
    }
    const bool adj = far_q != nullptr;
    for (int64_t j = 0; j < N; ++j) {
        const Rec J = recs[j];
        const int64_t oj = (int64_t)J.x + ex * ((int64_t)J.y + ey * (int64_t)J.z);
        const double aj = (double)J.a, pj = aj * aj, nj = (double)J.n;
#pragma unroll
        for (int p = 0; p < kFarIPL; ++p) {
            const double t = T[base[p] - oj];
            const double X = pi[p] * pj, pp = pi[p] + pj;
            const double Rinv = 1.0 / (X * pp);
            const double w = nj * t * Rinv;
            acc[p] += w;
            // d/da_i of -1 / (a_i^2 a_j^2 pp) is (2 / a_i + 2 a_i / pp) / (a_i^2 a_j^2 pp)
            if (adj) accq[p] += w * (g2[p] + a2[p] * (Rinv * X));
        }
    }
#pragma unroll
    for (int p = 0; p < kFarIPL; ++p) {
        const int64_t i = i0 + threadIdx.x + (int64_t)kFarThreads * p;
        if (i >= N) continue;
        far0[i] = -casym * acc[p];
        if (adj) far_q[i] = casym * qscale * accq[p];
    }
}

}  // namespace

int64_t far_table_entries(const FarGeo &g)
{
    return (int64_t)(2 * g.nx - 1) * (2 * g.ny - 1) * (2 * g.nz - 1);
}

int launch_far_table(const FarGeo &g, double *T, hipStream_t s)
{
    const int64_t ne = far_table_entries(g);
    hipLaunchKernelGGL(far_table_kernel, dim3((unsigned)((ne + kFarThreads - 1) / kFarThreads)), dim3(kFarThreads), 0,
                       s, g, ne, T);
    VDW_HIP(hipGetLastError());
    return VDW_OK;
}

int launch_far_rows(const FarGeo &g, int fp64, const void *recs, const int64_t *nkept, int64_t nmax,
                    const double *T, double casym, double qscale, double *far0, double *far_q, hipStream_t s)
{
    if (nmax < 1) return VDW_OK;
    const unsigned blocks = (unsigned)((nmax + kFarThreads * kFarIPL - 1) / (kFarThreads * kFarIPL));
    if (fp64)
        hipLaunchKernelGGL(far_rows_kernel<RecD>, dim3(blocks), dim3(kFarThreads), 0, s, g, (const RecD *)recs, nkept,
                           T, casym, qscale, far0, far_q);
    else
        hipLaunchKernelGGL(far_rows_kernel<RecF>, dim3(blocks), dim3(kFarThreads), 0, s, g, (const RecF *)recs, nkept,
                           T, casym, qscale, far0, far_q);
    VDW_HIP(hipGetLastError());
    return VDW_OK;
}

}  // namespace vdw
