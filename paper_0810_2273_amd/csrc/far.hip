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
//   far_rows   one lane per kept point i (two per thread), the j-points of
//              one chunk of the density streamed through scalar loads in
//              tiles; T read from an LDS copy of the tile's displacement
//              box (or gathered where the box is too large); FP64 sums per
//              chunk, the pair i = j included; the chunk partials are added
//              in a fixed order later
#include <limits.h>
#include <math.h>

#include "common.h"

namespace vdw {

namespace {

constexpr int kFarThreads = 256;
constexpr int kFarIPL = 2;  // kept points per thread (four: 106 VGPRs, measured no faster)

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

// 1 / x for x > 0 in the normal range: the hardware estimate refined by two
// Newton steps (each squares the relative error), to about one ulp.
__device__ inline double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Rows of block x, j chunk y (of gridDim.y): partial sums of the chunk's
// j-points, written to part[y][i] (energy) and (ADJ) part[C + y][i]
// (dE/da_i).  The j-points go in tiles of kFarTile consecutive records: the
// displacements between the block's i-points and a tile's j-points fill a
// box of the grid displacements, which the block copies from T into LDS
// (one coalesced pass) when it holds at most kFarStage entries, so each pair
// reads T from LDS; a tile whose box is larger (scattered points) gathers T
// directly, kFarJ j-points at a time so that their gathers are in flight
// together.  Either way the j-points are summed in their order.
constexpr int kFarJ = 4;
constexpr int kFarTile = 64;
constexpr int kFarStage = 4096;  // FP64 entries (32 KiB of LDS)

// Block-wide min and max of six integers (every thread gets them); `red`
// holds kFarThreads / 64 x 6 values.
__device__ inline void block_box(int (&v)[6], int *red)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        int x = v[k];
        for (int o = 32; o > 0; o >>= 1) {
            const int y = __shfl_xor(x, o);
            x = (k & 1) ? max(x, y) : min(x, y);
        }
        if (lane == 0) red[w * 6 + k] = x;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        int x = red[k];
        for (int u = 1; u < kFarThreads / 64; ++u) x = (k & 1) ? max(x, red[u * 6 + k]) : min(x, red[u * 6 + k]);
        v[k] = x;
    }
    __syncthreads();
}

template <typename Rec, bool ADJ>
__global__ __launch_bounds__(kFarThreads) void far_rows_kernel(FarGeo g, const Rec *__restrict__ recs,
                                                               const int64_t *__restrict__ nkept,
                                                               const int64_t *__restrict__ first,
                                                               const double *__restrict__ T, double casym,
                                                               double qscale, int64_t stride,
                                                               double *__restrict__ part)
{
    __shared__ double Ts[kFarStage];
    __shared__ int red[(kFarThreads / 64) * 6];
    const int64_t N = *nkept;
    recs += *first;
    const int64_t i0 = (int64_t)blockIdx.x * (kFarThreads * kFarIPL);
    if (i0 >= N) return;  // N >= 1 below (the whole block leaves together)
    const int C = gridDim.y, c = blockIdx.y;
    const int64_t len = (N + C - 1) / C;
    const int64_t j0 = min(N, (int64_t)c * len), j1 = min(N, j0 + len);
    // table offsets fit 32 bits (the host bounds the table); a record's
    // `off` is its x + ex (y + ey z)
    const int ex = 2 * g.nx - 1, ey = 2 * g.ny - 1;
    const int k0 = (g.nx - 1) + ex * ((g.ny - 1) + ey * (g.nz - 1));
    int base[kFarIPL], ix[kFarIPL], iy[kFarIPL], iz[kFarIPL];
    double pi[kFarIPL], g2[kFarIPL], a2[kFarIPL], acc[kFarIPL], accq[kFarIPL];
    int ib[6] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN, INT_MAX, INT_MIN};
#pragma unroll
    for (int p = 0; p < kFarIPL; ++p) {
        const int64_t i = i0 + threadIdx.x + (int64_t)kFarThreads * p;
        const Rec R = recs[i < N ? i : N - 1];
        // table entry of displacement r_i - r_j is base - off(j)
        base[p] = rec_off(R) + k0;
        ix[p] = (int)R.x;
        iy[p] = (int)R.y;
        iz[p] = (int)R.z;
        ib[0] = min(ib[0], ix[p]);
        ib[1] = max(ib[1], ix[p]);
        ib[2] = min(ib[2], iy[p]);
        ib[3] = max(ib[3], iy[p]);
        ib[4] = min(ib[4], iz[p]);
        ib[5] = max(ib[5], iz[p]);
        const double a = (double)R.a;
        pi[p] = a * a;
        g2[p] = 2.0 / a;
        a2[p] = 2.0 * a;
        acc[p] = accq[p] = 0.0;
    }
    block_box(ib, red);  // the block's i box (padding lanes repeat point N - 1)
    // one pair: w = n_j T / (p_i p_j (p_i + p_j)); d/da_i of -1 / (a_i^2 a_j^2 pp)
    // is (2 / a_i + 2 a_i / pp) / (a_i^2 a_j^2 pp)
    auto term = [&](int p, double t, double pj, double nj) {
        const double X = pi[p] * pj, pp = pi[p] + pj;
        const double Rinv = rcp64(X * pp);
        const double w = nj * t * Rinv;
        acc[p] += w;
        if (ADJ) accq[p] += w * (g2[p] + a2[p] * (Rinv * X));
    };
    for (int64_t jt = j0; jt < j1; jt += kFarTile) {
        const int64_t je = min(j1, jt + kFarTile);
        // the tile's j box, then the displacement box r_i - r_j
        int jb[6];
        {
            const int64_t jj = jt + (threadIdx.x & 63);
            const Rec J = recs[jj < je ? jj : je - 1];
            jb[0] = jb[1] = (int)J.x;
            jb[2] = jb[3] = (int)J.y;
            jb[4] = jb[5] = (int)J.z;
        }
        block_box(jb, red);
        const int dx0 = ib[0] - jb[1], dy0 = ib[2] - jb[3], dz0 = ib[4] - jb[5];
        const int bx = ib[1] - jb[0] - dx0 + 1, by = ib[3] - jb[2] - dy0 + 1, bz = ib[5] - jb[4] - dz0 + 1;
        const bool staged = (int64_t)bx * by * bz <= kFarStage;
        if (staged) {
            const int vol = bx * by * bz, bxy = bx * by;
            for (int e = threadIdx.x; e < vol; e += kFarThreads) {
                const int ez = e / bxy, r = e - ez * bxy, ey_ = r / bx, ex_ = r - ey_ * bx;
                Ts[e] = T[(unsigned)((dx0 + ex_) + ex * ((dy0 + ey_) + ey * (dz0 + ez)) + k0)];
            }
            __syncthreads();
            // local index of r_i - r_j in the box: Li - Lj
            int Li[kFarIPL];
#pragma unroll
            for (int p = 0; p < kFarIPL; ++p) Li[p] = (ix[p] - dx0) + bx * ((iy[p] - dy0) + by * (iz[p] - dz0));
            int64_t j = jt;
            for (; j + kFarJ <= je; j += kFarJ) {
                int Lj[kFarJ];
                double pj[kFarJ], nj[kFarJ], t[kFarJ][kFarIPL];
#pragma unroll
                for (int u = 0; u < kFarJ; ++u) {
                    const Rec J = recs[j + u];
                    Lj[u] = (int)J.x + bx * ((int)J.y + by * (int)J.z);
                    const double aj = (double)J.a;
                    pj[u] = aj * aj;
                    nj[u] = (double)J.n;
                }
#pragma unroll
                for (int u = 0; u < kFarJ; ++u)
#pragma unroll
                    for (int p = 0; p < kFarIPL; ++p) t[u][p] = Ts[Li[p] - Lj[u]];
#pragma unroll
                for (int u = 0; u < kFarJ; ++u)
#pragma unroll
                    for (int p = 0; p < kFarIPL; ++p) term(p, t[u][p], pj[u], nj[u]);
            }
            for (; j < je; ++j) {
                const Rec J = recs[j];
                const int Lj = (int)J.x + bx * ((int)J.y + by * (int)J.z);
                const double aj = (double)J.a;
#pragma unroll
                for (int p = 0; p < kFarIPL; ++p) term(p, Ts[Li[p] - Lj], aj * aj, (double)J.n);
            }
            __syncthreads();  // the box is rewritten for the next tile
        } else {
            int64_t j = jt;
            for (; j + kFarJ <= je; j += kFarJ) {
                int oj[kFarJ];
                double pj[kFarJ], nj[kFarJ], t[kFarJ][kFarIPL];
#pragma unroll
                for (int u = 0; u < kFarJ; ++u) {
                    const Rec J = recs[j + u];
                    oj[u] = rec_off(J);
                    const double aj = (double)J.a;
                    pj[u] = aj * aj;
                    nj[u] = (double)J.n;
                }
#pragma unroll
                for (int u = 0; u < kFarJ; ++u)
#pragma unroll
                    for (int p = 0; p < kFarIPL; ++p) t[u][p] = T[(unsigned)(base[p] - oj[u])];
#pragma unroll
                for (int u = 0; u < kFarJ; ++u)
#pragma unroll
                    for (int p = 0; p < kFarIPL; ++p) term(p, t[u][p], pj[u], nj[u]);
            }
            for (; j < je; ++j) {
                const Rec J = recs[j];
                const int oj = rec_off(J);
                const double aj = (double)J.a;
#pragma unroll
                for (int p = 0; p < kFarIPL; ++p) term(p, T[(unsigned)(base[p] - oj)], aj * aj, (double)J.n);
            }
        }
    }
#pragma unroll
    for (int p = 0; p < kFarIPL; ++p) {
        const int64_t i = i0 + threadIdx.x + (int64_t)kFarThreads * p;
        if (i >= N) continue;
        part[(int64_t)c * stride + i] = -casym * acc[p];
        if (ADJ) part[(int64_t)(C + c) * stride + i] = casym * qscale * accq[p];
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

int far_chunks(int64_t nmax)
{
    // enough blocks for about 16 wavefronts per SIMD when every point is
    // kept, chunks of at least 1024 points
    const int64_t rb = (nmax + kFarThreads * kFarIPL - 1) / (kFarThreads * kFarIPL);
    int64_t C = rb > 0 ? (4096 + rb - 1) / rb : 1;
    if (C > nmax / 1024) C = nmax / 1024;
    if (C > kFarMaxChunks) C = kFarMaxChunks;
    return C < 1 ? 1 : (int)C;
}

int launch_far_rows(const FarGeo &g, int fp64, const void *recs, const int64_t *nkept, const int64_t *first,
                    int64_t nmax, const double *T, double casym, double qscale, int chunks, int adj, double *part,
                    hipStream_t s)
{
    if (nmax < 1) return VDW_OK;
    if (chunks < 1 || chunks > kFarMaxChunks) return fail(VDW_EINVAL, "internal: %d far chunks", chunks);
    const dim3 grid((unsigned)((nmax + kFarThreads * kFarIPL - 1) / (kFarThreads * kFarIPL)), (unsigned)chunks);
    const RecD *rd = (const RecD *)recs;
    const RecF *rf = (const RecF *)recs;
    const dim3 blk(kFarThreads);
    if (fp64 && adj)
        hipLaunchKernelGGL((far_rows_kernel<RecD, true>), grid, blk, 0, s, g, rd, nkept, first, T, casym, qscale, nmax,
                           part);
    else if (fp64)
        hipLaunchKernelGGL((far_rows_kernel<RecD, false>), grid, blk, 0, s, g, rd, nkept, first, T, casym, qscale, nmax,
                           part);
    else if (adj)
        hipLaunchKernelGGL((far_rows_kernel<RecF, true>), grid, blk, 0, s, g, rf, nkept, first, T, casym, qscale, nmax,
                           part);
    else
        hipLaunchKernelGGL((far_rows_kernel<RecF, false>), grid, blk, 0, s, g, rf, nkept, first, T, casym, qscale, nmax,
                           part);
    VDW_HIP(hipGetLastError());
    return VDW_OK;
}

}  // namespace vdw
