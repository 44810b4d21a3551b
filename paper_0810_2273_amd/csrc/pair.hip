// The O(N^2) double sum of Eq. (2) (paper, Sec. 2) over the points kept by
// the density cut-off (Sec. 3), with periodic images of the 0th cell
// (Sec. 3), the on-site term (sphere or cell average), the deterministic
// FP64 reductions, and the adjoint dE/dn through q0 and the gradient, on
// orthorhombic or skew cells.
//
// Pipeline of one call (all on the caller's stream, no host round trip
// before the final copy of the energies):
//   fill      zero the work counter, flags, and (potential) dE/dn buffers
//   count     brick-ordered scan of n >= n_cut, per-block counts
//   scan      one workgroup: exclusive prefix, per-density offsets and the
//             work-item table
//   scatter   compact the kept points into 32-byte (FP32) or 64-byte (FP64)
//             records in brick order (4x4x4 bricks, so a wavefront's
//             i-points are spatially compact and their table rows coherent)
//   pair      persistent workgroups (one per CU) pull work items from an
//             atomic counter.  The kept points of a density are cut into
//             row blocks of IPL x (workgroup size) points, IPL i-points per
//             lane (four for the FP32 n_sigma = 64 kernels without images in
//             1024-thread workgroups, eight in 512-thread ones, two
//             elsewhere).  Row block I owns ND diagonal items (ordered pairs
//             of the block's points with one of ND j sub-ranges of it, j
//             records streamed through scalar registers) and items (I, c)
//             pairing it with chunks of the points after the block.  Off-diagonal pairs are evaluated once
//             for both orders: each wavefront loads a 64-record j tile into
//             its lanes and rotates it one lane per step (DPP wave rotate),
//             carrying the j-side sums with the records, so after 64 steps
//             every lane has met every j and every j-side sum is back in its
//             home lane; the wavefronts then add their j-side sums in a fixed
//             order through LDS.  The first table rows sit in static LDS
//             (row stride n_sigma + 1), the rest is read through L2 in a
//             second pass taken only by the pairs beyond them.
//   finalize  per point: fixed-order sum of its item partials, on-site term,
//             energy terms, and (potential) the direct part of dE/dn
//   reduce    per density: fixed-order sum of the block partials
//   assemble  (potential) transposed gradient stencil on the whole grid (the
//             axes with the Fourier derivative follow as line kernels)
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "common.h"
#include "q0_point.h"

namespace vdw {

namespace {

constexpr int kCompactBlock = 1024;  // brick-order positions per count/scatter block
constexpr int kCompactThreads = 256;  // 4 positions (one brick row) per thread
constexpr int kPairThreads = 1024;    // default pair workgroup size (variants: 512 and 256)
constexpr int kFinThreads = 256;      // points per finalize block
constexpr int kRun = 64;              // j-terms per FP32 run before the FP64 carry (diagonal items)
constexpr int kLdsBytes = 160 * 1024; // LDS of one gfx950 workgroup

// Table elements a pair workgroup of NW wavefronts keeps in LDS, next to
// its j-side reduction buffer (NW x 64 doubles, one accumulator array at a
// time) and the work-item slot.
template <typename R>
constexpr int tab_elems(int NW)
{
    return (int)((kLdsBytes - NW * 64 * sizeof(double) - 64) / sizeof(R));
}

enum { HDR_ITEMS = 0, HDR_NTOTAL = 1, HDR_BLKS = 2, HDR_WORDS = 8 };

struct Seg {
    // filled on the host
    int32_t nx, ny, nz, px, py, pz;
    double hx, hy, hz, dV;  // |e_a| (the unit of the kernel's distances is h_x = |e_x|), cell volume / G
    int32_t skew, pad1;
    int32_t spec[3], pad2;  // Fourier derivative on axis a (its adjoint runs as line kernels)
    double einv[9];     // E^-1 (skew cells; gradient and its adjoint)
    double e[9];        // the step vectors e_a (rows; diag(h) on orthorhombic cells), for the voxel term
    double m01, m02, m12;  // skew: 2 e_x.e_y / h_x^2, 2 e_x.e_z / h_x^2, 2 e_y.e_z / h_x^2
    double en[9];          // skew: the step vectors e_a / h_x (row-major), for Cartesian tile boxes
    int64_t G, grid_off;
    int32_t nbx, nby, nbz, pad0;
    int64_t t_off, T;     // brick-order positions: offset (multiple of kCompactBlock), padded length
    int64_t row_base;     // first entry of this density in the row-offset table
    int64_t slot_base;    // first partial slot of this density
    int64_t far_tab_off;  // far shell: first entry of this density's lattice-sum table
    int64_t far_part_off; // far shell: first element of its row partials (2 far_chunks arrays of G)
    int32_t far_chunks, pad3;
    // filled on the device by scan_kernel
    int64_t N, p_off, item_off, blk_off, nIB, items;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ inline int find_seg(const Seg *__restrict__ segs, int B, int64_t key, int which)
{
    // largest b with offset(b) <= key; offsets are non-decreasing
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        int64_t off = which == 0 ? segs[mid].t_off
                    : which == 1 ? segs[mid].p_off
                    : which == 2 ? segs[mid].item_off
                    : which == 3 ? segs[mid].blk_off
                                 : segs[mid].grid_off;
        if (off <= key) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void fill_kernel(double *__restrict__ a, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = 0.0;
}

__global__ void zero_words_kernel(int64_t *__restrict__ a, int n)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = 0;
}

__global__ void max_words_kernel(unsigned long long *__restrict__ a, int n)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = ~0ull;
}

// The FP32 table's cells as corner quadruples (k, l), (k, l+1), (k+1, l),
// (k+1, l+1), cell k (nS - 1) + l: one 16-byte load per pair beyond the LDS rows.
__global__ void quad_kernel(const float *__restrict__ t, float4 *__restrict__ quad, int nD, int nS)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t)(nD - 1) * (nS - 1)) return;
    const int k = (int)(c / (nS - 1)), l = (int)(c - (int64_t)k * (nS - 1));
    const float *r = t + (int64_t)k * nS + l;
    quad[c] = make_float4(r[0], r[1], r[nS], r[nS + 1]);
}

// Brick-order position -> grid coordinates of one segment; false if outside.
__device__ inline bool brick_pos(const Seg &s, int64_t lt, int &x, int &y, int &z)
{
    int64_t brick = lt >> 6;
    int l = (int)(lt & 63);
    int64_t nb_xy = (int64_t)s.nbx * s.nby;
    int bz = (int)(brick / nb_xy);
    int64_t rem = brick - bz * nb_xy;
    int by = (int)(rem / s.nbx);
    int bx = (int)(rem - (int64_t)by * s.nbx);
    x = 4 * bx + (l & 3);
    y = 4 * by + ((l >> 2) & 3);
    z = 4 * bz + (l >> 4);
    return bz < s.nbz && x < s.nx && y < s.ny && z < s.nz;
}

// ---------------------------------------------------------------------------
// compaction
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kCompactThreads) void count_kernel(const Seg *__restrict__ segs, int B,
                                                                const double *__restrict__ n, double n_cut,
                                                                int64_t *__restrict__ counts,
                                                                int *__restrict__ flag)
{
    __shared__ int red[kCompactThreads];
    int64_t base = (int64_t)blockIdx.x * kCompactBlock;
    int b = find_seg(segs, B, base, 0);
    const Seg s = segs[b];
    int cnt = 0;
    bool bad = false;
    for (int u = 0; u < 4; ++u) {
        int64_t lt = base - s.t_off + 4 * threadIdx.x + u;
        int x, y, z;
        if (lt < s.T && brick_pos(s, lt, x, y, z)) {
            double v = n[s.grid_off + x + (int64_t)s.nx * (y + (int64_t)s.ny * z)];
            if (!isfinite(v)) bad = true;
            cnt += (v >= n_cut) ? 1 : 0;
        }
    }
    if (bad) atomicOr(flag, 1);
    red[threadIdx.x] = cnt;
    __syncthreads();
    for (int st = kCompactThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

// One workgroup: exclusive prefix of the block counts (in place, with the
// total appended), then the per-density offsets the later kernels use.
__global__ __launch_bounds__(1024) void scan_kernel(int64_t *__restrict__ counts, int64_t nblocks,
                                                    Seg *__restrict__ segs, int B, int64_t *__restrict__ hdr,
                                                    int64_t *__restrict__ rowoff, int64_t JC, int64_t BI, int64_t ND)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    int64_t per = (nblocks + 1023) / 1024;
    int64_t lo = t * per, hi = min(nblocks, lo + per);
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += counts[i];
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 1024 thread sums
    for (int d = 1; d < 1024; d <<= 1) {
        int64_t v = (t >= d) ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = (t == 0) ? 0 : part[t - 1];
    for (int64_t i = lo; i < hi; ++i) {
        int64_t c = counts[i];
        counts[i] = run;
        run += c;
    }
    if (t == 1023) counts[nblocks] = part[1023];
    __syncthreads();
    if (t == 0) {
        int64_t item_off = 0, blk_off = 0;
        for (int b = 0; b < B; ++b) {
            Seg &g = segs[b];
            int64_t first = g.t_off / kCompactBlock, last = (g.t_off + g.T) / kCompactBlock;
            g.p_off = counts[first];
            g.N = counts[last] - counts[first];
            g.nIB = (g.N + BI - 1) / BI;
            // row I: ND diagonal items, then ceil((N - (I+1) BI) / JC) chunks
            int64_t items = 0;
            for (int64_t I = 0; I < g.nIB; ++I) {
                rowoff[g.row_base + I] = items;
                int64_t rest = g.N - (I + 1) * BI;
                items += ND + (rest > 0 ? (rest + JC - 1) / JC : 0);
            }
            rowoff[g.row_base + g.nIB] = items;
            g.items = items;
            g.item_off = item_off;
            g.blk_off = blk_off;
            item_off += items;
            blk_off += (g.N + kFinThreads - 1) / kFinThreads;
        }
        hdr[HDR_ITEMS] = item_off;
        hdr[HDR_NTOTAL] = counts[nblocks];
        hdr[HDR_BLKS] = blk_off;
    }
}

struct ScatterArgs {
    const Seg *segs;
    int B;
    const double *n;
    const double *q0;
    double n_cut;
    const int64_t *offs;
    void *recs;
    int32_t *gidx;
    double inv2dD;  // 1 / (2 dD): a = q h_x / (2 dD) is D / dD per grid spacing h_x
    double csig;    // sqrt(n_sigma - 1): b = csig a, so (b_i - b_j)/(a_i + a_j) = csig delta
    int fp64;
};

__global__ __launch_bounds__(kCompactThreads) void scatter_kernel(ScatterArgs A)
{
    __shared__ int pre[kCompactThreads];
    int64_t base = (int64_t)blockIdx.x * kCompactBlock;
    int b = find_seg(A.segs, A.B, base, 0);
    const Seg s = A.segs[b];
    int keep[4];
    int64_t gi[4];
    int xs[4], ys[4], zs[4];
    int cnt = 0;
    for (int u = 0; u < 4; ++u) {
        int64_t lt = base - s.t_off + 4 * threadIdx.x + u;
        int x = 0, y = 0, z = 0;
        keep[u] = 0;
        gi[u] = 0;
        if (lt < s.T && brick_pos(s, lt, x, y, z)) {
            gi[u] = s.grid_off + x + (int64_t)s.nx * (y + (int64_t)s.ny * z);
            keep[u] = (A.n[gi[u]] >= A.n_cut) ? 1 : 0;
        }
        xs[u] = x;
        ys[u] = y;
        zs[u] = z;
        cnt += keep[u];
    }
    // block-wide exclusive scan of the per-thread counts (fixed order)
    pre[threadIdx.x] = cnt;
    __syncthreads();
    for (int d = 1; d < kCompactThreads; d <<= 1) {
        int v = (threadIdx.x >= d) ? pre[threadIdx.x - d] : 0;
        __syncthreads();
        pre[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t pos = A.offs[blockIdx.x] + pre[threadIdx.x] - cnt;
    const uint32_t ex = 2u * (uint32_t)s.nx - 1u, ey = 2u * (uint32_t)s.ny - 1u;
    for (int u = 0; u < 4; ++u) {
        if (!keep[u]) continue;
        // far-shell table term (wraps harmlessly when no table is built)
        const uint32_t off = (uint32_t)xs[u] + ex * ((uint32_t)ys[u] + ey * (uint32_t)zs[u]);
        double nn = A.n[gi[u]], q = A.q0[gi[u]];
        double a = q * s.hx * A.inv2dD;
        if (A.fp64) {
            RecD r;
            r.x = xs[u];
            r.y = ys[u];
            r.z = zs[u];
            r.n = nn;
            r.a = a;
            r.b = a * A.csig;
            r.w = (double)xs[u] * xs[u] + (double)ys[u] * ys[u] + (double)zs[u] * zs[u];
            r.off = __builtin_bit_cast(double, (uint64_t)off);
            ((RecD *)A.recs)[pos] = r;
        } else {
            RecF r;
            r.x = (float)xs[u];
            r.y = (float)ys[u];
            r.z = (float)zs[u];
            r.n = (float)nn;
            r.a = (float)a;
            r.b = (float)(a * A.csig);
            r.w = (float)((double)xs[u] * xs[u] + (double)ys[u] * ys[u] + (double)zs[u] * zs[u]);
            r.off = __builtin_bit_cast(float, off);
            ((RecF *)A.recs)[pos] = r;
        }
        A.gidx[pos] = (int32_t)gi[u];
        ++pos;
    }
}

// ---------------------------------------------------------------------------
// pair kernel
// ---------------------------------------------------------------------------

struct PairArgs {
    int B;
    int nD, nS, S, K;   // S: LDS row stride (n_sigma + 1); K: rows held in LDS
    int JC;             // j-points per off-diagonal item (multiple of 64)
    int BI;             // i-points per row block (IPL x threads of the variant)
    int ND, DS;         // diagonal items per row block, each over a j sub-range of DS = BI / ND points
    int interp;         // 1: cubic in D (FP64 form)
    double tDmax;       // n_D - 1: table branch iff t_D = D / dD < n_D - 1
    double tSclamp;     // largest value below n_sigma - 1 (sigma index clamp)
    double csig;        // sqrt(n_sigma - 1)
    double casym;       // C / (2 dD)^6, C = 12 (4 pi/9)^3 (asymptote in h_x units)
    double dD2;         // 2 dD
    double rc2;         // squared distance cut (inf: none)
    int nimg, home;     // number of images, index of (0, 0, 0)
    int NI, NJ;         // accumulator arrays: S0c, (S0L if images), (Sq if potential)
    int64_t istride;    // doubles per i-side accumulator array
    int64_t jstride;    // elements per j-side accumulator array
};

template <typename R>
struct RecOf;
template <>
struct RecOf<float> {
    using T = RecF;
};
template <>
struct RecOf<double> {
    using T = RecD;
};

__device__ inline float dsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline float drcp(float x) { return __builtin_amdgcn_rcpf(x); }
// FP64 reciprocal of a positive normal x: the hardware estimate refined by
// two Newton steps (each squares the relative error), to about one ulp.
__device__ inline double drcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
// FP64 square root of a positive normal x from the hardware reciprocal-root
// estimate y: g = x y and h = y / 2 refined by one Goldschmidt step, then two
// Newton corrections of g (about one ulp).  x = 0 (only the excluded pair
// (i, i, 0) of weight zero has it) gives 0, which keeps that pair on the
// table branch, where every value stays finite.
__device__ inline double dsqrt(double x)
{
    const bool pos = x > 0.0;
    const double xs = pos ? x : 1.0;
    const double y = __builtin_amdgcn_rsq(xs);
    double g = xs * y, h = 0.5 * y;
    const double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    double d = fma(-g, g, xs);
    g = fma(d, h, g);
    d = fma(-g, g, xs);
    g = fma(d, h, g);
    return pos ? g : 0.0;
}
__device__ inline float dfract(float x) { return __builtin_amdgcn_fractf(x); }
__device__ inline double dfract(double x) { return __builtin_amdgcn_fract(x); }  // x - floor(x), exact for x >= 0

// Rotate a wavefront-wide value by one lane (DPP wave_ror:1): 64 rotations
// bring every value back to its lane.
__device__ inline float wrot(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x13C, 0xF, 0xF, true));
}
__device__ inline double wrot(double x)
{
    int2 v = __builtin_bit_cast(int2, x);
    v.x = __builtin_amdgcn_mov_dpp(v.x, 0x13C, 0xF, 0xF, true);
    v.y = __builtin_amdgcn_mov_dpp(v.y, 0x13C, 0xF, 0xF, true);
    return __builtin_bit_cast(double, v);
}

// Two f16 values in one register (the x, y grid coordinates of the cubic
// squared distance, exact as f16 for |value| <= 2048), rotated as one.
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
__device__ inline half2v wrot(half2v x)
{
    return __builtin_bit_cast(half2v, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x13C, 0xF, 0xF, true));
}

template <typename R>
struct PairK {
    R tDmax, tDlds, tSclamp, csig, c4, rc4, casym, wy, wz;  // rc4 = 1 / c4
    R m01, m02, m12;  // skew cells (see Seg)
    R en[9];
    int S, nS, K;
    int nD;           // table rows
    // FP32 bilinear kernels: the global table as one float4 per cell, the
    // corners (k, l), (k, l+1), (k+1, l), (k+1, l+1) of cell k (n_sigma - 1) + l
    const float4 *quad;
};

// Grid geometry of a pair-kernel variant: orthorhombic, cubic (equal
// spacings), skew (general metric), or square (orthorhombic with h_x = h_y,
// the slab's layout: x, y enter the squared distance exactly, as on cubic
// grids, and z through its weight).
constexpr int kOrtho = 0, kCubic = 1, kSkew = 2, kSquare = 3;

// The NSIG template value of the FP64 kernels that read the table cubic in D
// (any n_sigma); NSIG = 0: any n_sigma, bilinear; NSIG > 0: that n_sigma.
constexpr int kCubicD = -1;

// min of two non-negative values; for FP32 an integer min on the bit
// patterns (same order for non-negative floats, no NaN quieting needed)
__device__ inline float dmin(float a, float b)
{
    return __builtin_bit_cast(float, min(__builtin_bit_cast(int, a), __builtin_bit_cast(int, b)));
}
__device__ inline double dmin(double a, double b) { return __builtin_fmin(a, b); }

// Squared distance in units of h_x^2 from exact integer grid deltas
// (wy = (h_y/h_x)^2, wz = (h_z/h_x)^2; both 1 on cubic grids; on skew grids
// |e_a|^2 / h_x^2 and the cross terms m01 = 2 e_x.e_y / h_x^2, ...).
template <typename R, int GEO>
__device__ __forceinline__ R dist2(const PairK<R> &k, R dx, R dy, R dz)
{
    if (GEO == kCubic) return dx * dx + dy * dy + dz * dz;
    if (GEO == kSkew) return dx * dx + (k.wy * dy) * dy + (k.wz * dz) * dz + dx * (k.m01 * dy + k.m02 * dz) + (k.m12 * dy) * dz;
    return dx * dx + (k.wy * dy) * dy + (k.wz * dz) * dz;
}

// Squared distance on a cubic grid as |x_i|^2 + |x_j|^2 - 2 x_i . x_j with
// (mx, my, mz) = -2 x_i and w = |x_i|^2 + |x_j|^2: every term and partial
// sum is an integer below 2^24 (the host checks the coordinate range), so
// the FP32 result is exact and equals the difference form.
__device__ __forceinline__ float dist2n(float mx, float my, float mz, float w, float xj, float yj, float zj)
{
    return fmaf(mx, xj, fmaf(my, yj, fmaf(mz, zj, w)));
}

// The table interpolant at fractions (fD, fS) of the cell whose corners are
// p00 = phi(k, l), p01 = phi(k, l+1), p10 = phi(k+1, l), p11 = phi(k+1, l+1),
// and (ADJ) the q-derivatives: gD r + gS u inv^2 4 csig a_j for q_i, and the
// sigma term with the sign flipped and a_j -> a_i for q_j.
template <typename R, bool ADJ, bool JSIDE>
__device__ __forceinline__ void bilinear(R p00, R p01, R p10, R p11, R fD, R fS, R r, R u, R inv, R c4, R ai, R aj,
                                         R &phi, R &dqi, R &dqj)
{
    const R d0 = p01 - p00, d1 = p11 - p10;
    const R lo = p00 + fS * d0, hi = p10 + fS * d1;
    const R gD = hi - lo;
    phi = lo + fD * gD;
    if (ADJ) {
        const R gS = d0 + fD * (d1 - d0);
        const R X = gD * r;
        const R Y = (gS * (u * inv)) * (inv * c4);
        dqi = X + Y * aj;
        if (JSIDE) dqj = X - Y * ai;
    }
}

// The large-D asymptote -C' / (m^3 a_i^2 a_j^2 (a_i^2 + a_j^2)) and its
// q-derivatives.
template <typename R, bool ADJ, bool JSIDE>
__device__ __forceinline__ void asymptote(const PairK<R> &k, R m, R ai, R aj, R &phi, R &dqi, R &dqj)
{
    // a private copy keeps these rare-branch products from being hoisted
    R ajx = aj;
    asm("" : "+v"(ajx));
    const R pi = ai * ai, pj = ajx * ajx, pp = pi + pj;
    phi = -k.casym * drcp(m * m * m * pi * pj * pp);
    if (ADJ) {
        const R rp = drcp(pp);
        dqi = -phi * ((R)2 * drcp(ai) + (R)2 * ai * rp);
        if (JSIDE) dqj = -phi * ((R)2 * drcp(ajx) + (R)2 * ajx * rp);
    }
}

// phi~ of one pair and (ADJ) the q-derivatives, from m = r^2 / h_x^2 and
// a = q h_x / (2 dD) of both points:
//   t_D = (a_i + a_j) sqrt(m) = D / dD,  u = csig (a_i - a_j)/(a_i + a_j),  t_s = u^2 = sigma (n_sigma - 1)
//   table branch: bilinear in (t_D, t_s);  beyond: -C' / (m^3 a_i^2 a_j^2 (a_i^2 + a_j^2)),  C' = C / (2 dD)^6
// dqi, dqj are 2 dD / h_x times d phi~ / d q_i and d phi~ / d q_j.
// Catmull-Rom cubic on [0, 1] between f[1] and f[2] (tangents (f[2]-f[0])/2,
// (f[3]-f[1])/2) and its derivative in t.
__device__ __forceinline__ double catmull_rom(const double (&f)[4], double t, double &dt)
{
    const double m1 = 0.5 * (f[2] - f[0]), m2 = 0.5 * (f[3] - f[1]);
    const double t2 = t * t, t3 = t2 * t;
    dt = (6.0 * t2 - 6.0 * t) * (f[1] - f[2]) + (3.0 * t2 - 4.0 * t + 1.0) * m1 + (3.0 * t2 - 2.0 * t) * m2;
    return (2.0 * t3 - 3.0 * t2 + 1.0) * f[1] + (t3 - 2.0 * t2 + t) * m1 + (-2.0 * t3 + 3.0 * t2) * f[2] +
           (t3 - t2) * m2;
}

// The C1 interpolant at cell (kk, l) with fractions (fD, fS): rows kk-1 ..
// kk+2 of columns l and l+1 (from LDS when they are all held there, else
// from the global table; beyond the table ends extrapolated linearly), the
// cubic in D per column, then linear in sigma; gD, gS per unit t_D, t_s.
template <int NSIG>
__device__ __forceinline__ double cubic_d(const PairK<double> &k, const double *tab, const double *__restrict__ tabg,
                                          int kk, int l, double fD, double fS, double &gD, double &gS)
{
    const int S = NSIG > 0 ? NSIG + 1 : k.S;
    const int nS = NSIG > 0 ? NSIG : k.nS;
    const bool lds = kk >= 1 && kk + 2 <= k.K - 1;
    double c0[4], c1[4];
    for (int i = 0; i < 4; ++i) {
        const int rr = min(max(kk - 1 + i, 0), k.nD - 1);
        const double *t = lds ? tab + (int64_t)rr * S + l : tabg + (int64_t)rr * nS + l;
        c0[i] = t[0];
        c1[i] = t[1];
    }
    if (kk == 0) {
        c0[0] = 2.0 * c0[1] - c0[2];
        c1[0] = 2.0 * c1[1] - c1[2];
    }
    if (kk + 2 > k.nD - 1) {
        c0[3] = 2.0 * c0[2] - c0[1];
        c1[3] = 2.0 * c1[2] - c1[1];
    }
    double d0, d1;
    const double v0 = catmull_rom(c0, fD, d0), v1 = catmull_rom(c1, fD, d1);
    gD = d0 + fS * (d1 - d0);
    gS = v1 - v0;
    return v0 + fS * (v1 - v0);
}

// FP32 form of cubic_d: the same rows (LDS when all four are held there,
// else global, whose rows lack the extra column: there the last cell and its
// fraction), the Catmull-Rom cubic per column, linear in sigma.
__device__ __forceinline__ float catmull_rom(const float (&f)[4], float t, float &dt)
{
    const float m1 = 0.5f * (f[2] - f[0]), m2 = 0.5f * (f[3] - f[1]);
    const float t2 = t * t, t3 = t2 * t;
    dt = (6.0f * t2 - 6.0f * t) * (f[1] - f[2]) + (3.0f * t2 - 4.0f * t + 1.0f) * m1 + (3.0f * t2 - 2.0f * t) * m2;
    return (2.0f * t3 - 3.0f * t2 + 1.0f) * f[1] + (t3 - 2.0f * t2 + t) * m1 + (-2.0f * t3 + 3.0f * t2) * f[2] +
           (t3 - t2) * m2;
}

__device__ __forceinline__ float cubic_d32(const PairK<float> &k, const float *tab, const float *__restrict__ tabg,
                                           int kk, int l, float fD, float ts, float &gD, float &gS)
{
    const bool lds = kk >= 1 && kk + 2 <= k.K - 1;
    const int lg = lds ? l : min(l, k.nS - 2);
    const float fS = ts - (float)lg;
    float c0[4], c1[4];
    for (int i = 0; i < 4; ++i) {
        const int rr = min(max(kk - 1 + i, 0), k.nD - 1);
        const float *t = lds ? tab + (int64_t)rr * k.S + lg : tabg + (int64_t)rr * k.nS + lg;
        c0[i] = t[0];
        c1[i] = t[1];
    }
    if (kk == 0) {
        c0[0] = 2.0f * c0[1] - c0[2];
        c1[0] = 2.0f * c1[1] - c1[2];
    }
    if (kk + 2 > k.nD - 1) {
        c0[3] = 2.0f * c0[2] - c0[1];
        c1[3] = 2.0f * c1[2] - c1[1];
    }
    float d0, d1;
    const float v0 = catmull_rom(c0, fD, d0), v1 = catmull_rom(c1, fD, d1);
    gD = d0 + fS * (d1 - d0);
    gS = v1 - v0;
    return v0 + fS * (v1 - v0);
}

// FP64 form: ci = b_i = csig a_i and cj = csig a_j, u = (b_i - csig a_j) / s.
// (NEAR and GLOB are properties of the FP32 form; the FP64 form always checks
// the rows.)
template <bool ADJ, bool JSIDE, int NSIG, bool SPLIT, bool NEAR = false, bool GLOB = false>
__device__ __forceinline__ void pair_eval(const PairK<double> &k, const double *tab, const double *__restrict__ tabg,
                                          double m, double ai, double ci, double aj, double cj, double &phi,
                                          double &dqi, double &dqj)
{
    const int S = NSIG > 0 ? NSIG + 1 : k.S;
    const int nS = NSIG > 0 ? NSIG : k.nS;
    const double r = dsqrt(m);
    const double s = ai + aj;
    const double tD = s * r;
    if (tD < k.tDmax) {
        const double inv = drcp(s);
        const double u = (ci - cj) * inv;
        const double ts = dmin(u * u, k.tSclamp);
        const int kk = (int)tD;
        const int l = (int)ts;
        const double fD = dfract(tD), fS = dfract(ts);
        if constexpr (NSIG == kCubicD) {
            double gD, gS;
            phi = cubic_d<NSIG>(k, tab, tabg, kk, l, fD, fS, gD, gS);
            if (ADJ) {
                const double X = gD * r;
                const double Y = (gS * (u * inv)) * (inv * k.c4);
                dqi = X + Y * aj;
                if (JSIDE) dqj = X - Y * ai;
            }
            return;
        }
        // rows below K come from LDS; the clamped LDS read is always in
        // bounds and is replaced for rows >= K - 1
        const int kl = min(kk, k.K - 2);
        const double *t = tab + (__umul24((unsigned)kl, (unsigned)S) + (unsigned)l);
        double p00 = t[0], p01 = t[1], p10 = t[S], p11 = t[S + 1];
        // keep the LDS reads unconditional: without this the compiler folds
        // the two sources into one FLAT load
        asm("" : "+v"(p00), "+v"(p01), "+v"(p10), "+v"(p11));
        if (kk >= k.K - 1) {
            const double *t0 = tabg + (int64_t)kk * nS + l;
            p00 = t0[0];
            p01 = t0[1];
            p10 = t0[nS];
            p11 = t0[nS + 1];
        }
        bilinear<double, ADJ, JSIDE>(p00, p01, p10, p11, fD, fS, r, u, inv, k.c4, ai, aj, phi, dqi, dqj);
    } else {
        asymptote<double, ADJ, JSIDE>(k, m, ai, aj, phi, dqi, dqj);
    }
}

// FP32 form: ci = 2 csig a_i, so u = ci / s - csig in one FMA; the j point
// comes as ej = 4 csig a_j and the i point also as ei = 4 csig a_i, which
// puts the factor 4 csig of the sigma slope into the q-derivative products:
// dq_i = gD r + Z ej, dq_j = gD r - Z ei, Z = gS (u / s) / s.
// The LDS rows are read and interpolated for every pair; one compare
// (t_D >= K - 1) sends the pairs beyond them to a second pass with the
// global table or the asymptote, which few pairs take.  NEAR: the caller has
// shown t_D < K - 1 for every pair (a bound over the two tiles' boxes and
// q ranges), so the LDS cell is read unclamped and nothing is checked.
template <bool ADJ, bool JSIDE, int NSIG, bool SPLIT, bool NEAR = false, bool GLOB = false>
__device__ __forceinline__ void pair_eval(const PairK<float> &k, const float *tab, const float *__restrict__ tabg,
                                          float m, float ai, float ci, float ej, float ei, float &phi, float &dqi,
                                          float &dqj)
{
    const int S = NSIG > 0 ? NSIG + 1 : k.S;
    const int nS = NSIG > 0 ? NSIG : k.nS;
    const float r = dsqrt(m);
    const float s = fmaf(ej, k.rc4, ai);
    const float tD = s * r;
    const float inv = drcp(s);
    const float u = fmaf(ci, inv, -k.csig);
    // t_s < n_sigma (|delta| < 1 up to rounding), so l + 1 <= n_sigma: the
    // LDS rows carry a column n_sigma that continues the last cell linearly,
    // which is the interpolant's own extrapolation beyond sigma = 1
    const float ts = u * u;
    const int kk = (int)tD;
    const int l = (int)ts;
    const float fD = dfract(tD), fS = dfract(ts);
    if constexpr (NSIG == kCubicD) {
        if (tD < k.tDmax) {
            float gD, gS;
            phi = cubic_d32(k, tab, tabg, kk, l, fD, ts, gD, gS);
            if (ADJ) {
                const float X = gD * r;
                const float Z = (gS * (u * inv)) * inv;
                dqi = fmaf(Z, ej, X);
                if (JSIDE) dqj = fmaf(-Z, ei, X);
            }
        } else {
            asymptote<float, ADJ, JSIDE>(k, m, ai, ej * k.rc4, phi, dqi, dqj);
        }
        return;
    }
    // SPLIT (the image kernels, where many pairs lie beyond the LDS rows):
    // each lane reads one table source, the LDS rows (t_D < K - 1, so the
    // cell's rows kk and kk + 1 are both there), the global rows, or the
    // asymptote, and a wavefront runs only the sources its lanes need.
    // GLOB: the caller has shown K - 1 <= t_D < n_D - 1 for every pair, so
    // every lane reads the global rows with no branch (the loads of a step's
    // pairs can then be issued together)
    if (NEAR) {
        const float *t = tab + (__umul24((unsigned)kk, (unsigned)S) + (unsigned)l);
        bilinear<float, ADJ, JSIDE>(t[0], t[1], t[S], t[S + 1], fD, fS, r, u, inv, 1.0f, ei, ej, phi, dqi, dqj);
    } else if (GLOB) {
        // the cell's corners in one 16-byte load; the table has no column
        // beyond n_sigma - 1: last cell and its fraction
        const int lg = min(l, nS - 2);
        const float4 c = k.quad[(uint32_t)(kk * (nS - 1) + lg)];
        bilinear<float, ADJ, JSIDE>(c.x, c.y, c.z, c.w, fD, ts - (float)lg, r, u, inv, 1.0f, ei, ej, phi, dqi, dqj);
    } else if (SPLIT) {
        if (tD < k.tDlds) {
            const float *t = tab + (__umul24((unsigned)kk, (unsigned)S) + (unsigned)l);
            bilinear<float, ADJ, JSIDE>(t[0], t[1], t[S], t[S + 1], fD, fS, r, u, inv, 1.0f, ei, ej, phi, dqi, dqj);
        } else if (tD < k.tDmax) {
            const int lg = min(l, nS - 2);
            const float4 c = k.quad[(uint32_t)(kk * (nS - 1) + lg)];
            bilinear<float, ADJ, JSIDE>(c.x, c.y, c.z, c.w, fD, ts - (float)lg, r, u, inv, 1.0f, ei, ej, phi, dqi,
                                        dqj);
        } else {
            asymptote<float, ADJ, JSIDE>(k, m, ai, ej * k.rc4, phi, dqi, dqj);
        }
    } else {
        // every lane reads the LDS copy (the clamped read is in bounds); the
        // pairs beyond it are redone from the global rows (the cell's corner
        // quadruple, one 16-byte load) or the asymptote
        const int kl = min(kk, k.K - 2);
        const float *t = tab + (__umul24((unsigned)kl, (unsigned)S) + (unsigned)l);
        bilinear<float, ADJ, JSIDE>(t[0], t[1], t[S], t[S + 1], fD, fS, r, u, inv, 1.0f, ei, ej, phi, dqi, dqj);
        if (tD >= k.tDlds) {
            if (tD < k.tDmax) {
                const int lg = min(l, nS - 2);
                const float4 c = k.quad[(uint32_t)(kk * (nS - 1) + lg)];
                bilinear<float, ADJ, JSIDE>(c.x, c.y, c.z, c.w, fD, ts - (float)lg, r, u, inv, 1.0f, ei, ej, phi, dqi,
                                            dqj);
            } else {
                asymptote<float, ADJ, JSIDE>(k, m, ai, ej * k.rc4, phi, dqi, dqj);
            }
        }
    }
}

// i-side constant of the sigma argument: b_i (FP64) or 2 csig a_i (FP32).
__device__ inline double ci_of(const PairK<double> &, double a, double b) { return b; }
__device__ inline float ci_of(const PairK<float> &k, float a, float) { return (2.0f * k.csig) * a; }
// j-side constant: csig a_j (FP64), unused in FP32.
__device__ inline double cj_of(const PairK<double> &k, double a) { return k.csig * a; }
__device__ inline float cj_of(const PairK<float> &, float) { return 0.0f; }

// Kahan-compensated sum step: s + y with the running error in c.
template <typename R>
__device__ __forceinline__ void kadd(R &sum, R &c, R y)
{
    const R t0 = y - c, t1 = sum + t0;
    c = (t1 - sum) - t0;
    sum = t1;
}

// One 64-step ring of an off-diagonal tile against one image shift: every
// lane meets every j of the tile with each of its IPL i-points; the j values
// and the j-side sums rotate with the records.  MASK applies the distance cut
// pair by pair (only for tiles that straddle it).  NORM (FP32 on cubic
// grids) takes the squared distance from the exact integer form of dist2n,
// with |x_j|^2 rotating along.  NEAR: every pair of the ring lies below the
// LDS rows; GLOB: every pair lies in the global rows (see pair_eval).
template <typename R, bool ADJ, bool MASK, bool KAHAN, int NSIG, int GEO, int IPL, bool SPLIT, bool NEAR = false,
          bool GLOB = false>
__device__ __forceinline__ void ring64(const PairK<R> &kc, const R *tab, const R *__restrict__ tabg, R rcm,
                                       const R (&sx)[IPL], const R (&sy)[IPL], const R (&sz)[IPL], const R (&ai)[IPL],
                                       const R (&ci)[IPL], const R (&ni)[IPL], R xj, R yj, R zj, R wj, R aj, R nj,
                                       R (&acc)[IPL], R (&accq)[IPL], R &accj, R &accqj)
{
    constexpr bool NORM = GEO == kCubic && sizeof(R) == 4;
    // square grids: x, y exactly as NORM (|x_i|^2 + |x_j|^2 - 2 x_i . x_j over
    // x and y), then the z term w_z (z_i - z_j)^2
    constexpr bool SQXY = GEO == kSquare && sizeof(R) == 4;
    // FP64 on cubic grids: the same exact integer as NORM, formed in FP32 and
    // widened (it equals the FP64 difference form bit for bit); the j
    // coordinates travel as one f16 pair and two FP32 values
    constexpr bool NORM64 = GEO == kCubic && sizeof(R) == 8;
    constexpr bool XY16 = NORM || SQXY || NORM64;
    R mz[IPL], wi[IPL], ca[IPL], cq[IPL];
    float mz32[IPL], wi32[IPL];
    half2v mxy[IPL];
#pragma unroll
    for (int p = 0; p < IPL; ++p) {
        if (XY16) mxy[p] = half2v{(_Float16)(float)(-2 * sx[p]), (_Float16)(float)(-2 * sy[p])};
        mz[p] = -2 * sz[p];
        wi[p] = SQXY ? sx[p] * sx[p] + sy[p] * sy[p] : sx[p] * sx[p] + sy[p] * sy[p] + sz[p] * sz[p];
        mz32[p] = (float)mz[p];
        wi32[p] = (float)wi[p];
        ca[p] = 0;  // Kahan terms (KAHAN only)
        cq[p] = 0;
    }
    // NORM, SQXY, NORM64: the x, y coordinates of the j records as one f16
    // pair; SQXY carries x_j^2 + y_j^2 in wj
    half2v xyj = XY16 ? half2v{(_Float16)(float)xj, (_Float16)(float)yj} : half2v{};
    if (SQXY) wj = xj * xj + yj * yj;
    float zj32 = (float)zj, wj32 = (float)wj;
    // FP32: the j point travels as ej = 4 csig a_j, the i points also carry ei
    constexpr bool F32 = sizeof(R) == 4;
    R ei[IPL];
#pragma unroll
    for (int p = 0; p < IPL; ++p) ei[p] = F32 ? kc.c4 * ai[p] : (R)0;
    if (F32) aj = kc.c4 * aj;
    R cj = 0, cqj = 0;
    for (int st = 0; st < 64; ++st) {
        const R cj_ = cj_of(kc, aj);
        R sj = 0, sqj = 0;  // j-side terms of this step (KAHAN only)
#pragma unroll
        for (int p = 0; p < IPL; ++p) {
            R m;
            if (NORM)
                m = (R)__builtin_amdgcn_fdot2(mxy[p], xyj, fmaf((float)mz[p], (float)zj, (float)(wi[p] + wj)), false);
            else if (NORM64)
                m = (R)__builtin_amdgcn_fdot2(mxy[p], xyj, fmaf(mz32[p], zj32, wi32[p] + wj32), false);
            else if (SQXY) {
                const float dz = (float)sz[p] - (float)zj;
                m = (R)fmaf((float)kc.wz * dz, dz, __builtin_amdgcn_fdot2(mxy[p], xyj, (float)(wi[p] + wj), false));
            } else
                m = dist2<R, GEO>(kc, sx[p] - xj, sy[p] - yj, sz[p] - zj);
            R ph, q = 0, jq = 0;
            pair_eval<ADJ, true, NSIG, SPLIT, NEAR, GLOB>(kc, tab, tabg, m, ai[p], ci[p], aj, F32 ? ei[p] : cj_, ph, q,
                                                          jq);
            R wjp = nj, wip = ni[p];
            if (MASK) {
                wjp = (m <= rcm) ? nj : (R)0;
                wip = (m <= rcm) ? ni[p] : (R)0;
            }
            if (KAHAN) {
                kadd(acc[p], ca[p], wjp * ph);
                sj = fma(wip, ph, sj);
                if (ADJ) {
                    kadd(accq[p], cq[p], wjp * q);
                    sqj = fma(wip, jq, sqj);
                }
            } else {
                acc[p] = fma(wjp, ph, acc[p]);
                accj = fma(wip, ph, accj);
                if (ADJ) {
                    accq[p] = fma(wjp, q, accq[p]);
                    accqj = fma(wip, jq, accqj);
                }
            }
        }
        if (KAHAN) {
            kadd(accj, cj, sj);
            if (ADJ) kadd(accqj, cqj, sqj);
        }
        if (XY16) {
            xyj = wrot(xyj);
        } else {
            xj = wrot(xj);
            yj = wrot(yj);
        }
        if (NORM64) {
            zj32 = wrot(zj32);
            wj32 = wrot(wj32);
        } else {
            zj = wrot(zj);
            if (NORM || SQXY) wj = wrot(wj);
        }
        aj = wrot(aj);
        nj = wrot(nj);
        accj = wrot(accj);
        if (ADJ) accqj = wrot(accqj);
        if (KAHAN) {
            cj = wrot(cj);
            if (ADJ) cqj = wrot(cqj);
        }
    }
    if (KAHAN) {
        // fold the compensation into the sums
#pragma unroll
        for (int p = 0; p < IPL; ++p) {
            acc[p] -= ca[p];
            accq[p] -= cq[p];
        }
        accj -= cj;
        accqj -= cqj;
    }
}

// One image shift of a pair in ring64_img: the shift-independent parts (s,
// the sigma cell l, its fraction fS, w = u / s^2) come in; r, t_D and the D
// cell are the shift's own.  NEAR / GLOB as in pair_eval; otherwise each lane
// reads its own source (LDS rows, global rows or the asymptote).
template <bool ADJ, bool NEAR, bool GLOB>
__device__ __forceinline__ void img_eval(const PairK<float> &k, const float *tab, float m, float s, float w, int l,
                                         float fS, int lg, float fSg, float ai, float ej, float ei, float &phi,
                                         float &dqi, float &dqj)
{
    constexpr int S = 65, nS = 64;  // n_sigma = 64: LDS row stride n_sigma + 1
    const float r = dsqrt(m);
    const float tD = s * r;
    const int kk = (int)tD;
    const float fD = dfract(tD);
    if (NEAR) {
        const float *t = tab + (__umul24((unsigned)kk, (unsigned)S) + (unsigned)l);
        bilinear<float, ADJ, true>(t[0], t[1], t[S], t[S + 1], fD, fS, r, w, 1.0f, 1.0f, ei, ej, phi, dqi, dqj);
    } else if (GLOB) {
        const float4 c = k.quad[(uint32_t)(kk * (nS - 1) + lg)];
        bilinear<float, ADJ, true>(c.x, c.y, c.z, c.w, fD, fSg, r, w, 1.0f, 1.0f, ei, ej, phi, dqi, dqj);
    } else {
        if (tD < k.tDlds) {
            const float *t = tab + (__umul24((unsigned)kk, (unsigned)S) + (unsigned)l);
            bilinear<float, ADJ, true>(t[0], t[1], t[S], t[S + 1], fD, fS, r, w, 1.0f, 1.0f, ei, ej, phi, dqi, dqj);
        } else if (tD < k.tDmax) {
            const float4 c = k.quad[(uint32_t)(kk * (nS - 1) + lg)];
            bilinear<float, ADJ, true>(c.x, c.y, c.z, c.w, fD, fSg, r, w, 1.0f, 1.0f, ei, ej, phi, dqi, dqj);
        } else {
            asymptote<float, ADJ, true>(k, m, ai, ej * k.rc4, phi, dqi, dqj);
        }
    }
}

constexpr int kImgGroup = 4;  // shifts per ring (groups of six or eight spill)
template <int N>
struct IntC {
    static constexpr int value = N;
};

// G image shifts of one j tile in one 64-step ring (FP32, n_sigma = 64,
// square or skew grids, shifts in x and y only, none of them the home cell).
// Per step and pair, what does not depend on the shift is formed once: s =
// a_i + a_j, 1/s, u, the sigma cell and w = u / s^2, and the shift-free part
// of the squared distance.  MASK, NEAR and GLOB hold for every shift of the
// group.  The caller runs groups of kImgGroup shifts, then at most one group
// of two per ring class.
//
// Square grids: x_i - x_j is an exact f16 pair and Q0 its squared length
// plus the z term; per shift L the squared distance is Q0 + |L|^2 - 2 L .
// (x_i - x_j), one add and one f16 dot product (L and x_i - x_j are exact
// integers in f16).  ml holds (-2 L_x, -2 L_y) as f16, cl |L|^2.
//
// Skew cells: the components of d - L (grid steps) are formed exactly and
// the metric is evaluated on them with the pair's z terms hoisted (wz dz^2,
// m02 dz, m12 dz); expanding |d - L|^2 about |d|^2 instead would cancel for
// pairs close only across the cell boundary.  lxy holds (L_x, L_y); ml and cl
// are unused there.
template <bool ADJ, bool MASK, int IPL, bool NEAR, bool GLOB, int G, int GEO = kSquare>
__device__ __forceinline__ void ring64_img(const PairK<float> &kc, const float *tab, float rcm,
                                           const RecF (&Ir)[IPL], const float (&ai)[IPL], const float (&ci)[IPL],
                                           const float (&ni)[IPL], float xj, float yj, float zj, float aj, float nj,
                                           const half2v (&ml)[G], const float (&cl)[G], const float2 (&lxy)[G],
                                           float (&acc)[IPL], float (&accq)[IPL], float &accj, float &accqj)
{
    constexpr bool SKEW = GEO == kSkew;
    half2v xyi[IPL];
    float ei[IPL];
#pragma unroll
    for (int p = 0; p < IPL; ++p) {
        xyi[p] = half2v{(_Float16)Ir[p].x, (_Float16)Ir[p].y};
        ei[p] = kc.c4 * ai[p];
    }
    half2v xyj = half2v{(_Float16)xj, (_Float16)yj};
    float ej = kc.c4 * aj;  // the j point as 4 csig a_j (see pair_eval)
    const float wz = kc.wz;
    for (int st = 0; st < 64; ++st) {
#pragma unroll
        for (int p = 0; p < IPL; ++p) {
            half2v dxy;
            float q0 = 0.0f, dx = 0.0f, dy = 0.0f, zA = 0.0f, zx = 0.0f, zy = 0.0f;
            if constexpr (SKEW) {
                const float dz = Ir[p].z - zj;
                dx = Ir[p].x - xj;
                dy = Ir[p].y - yj;
                zA = (kc.wz * dz) * dz;
                zx = kc.m02 * dz;
                zy = kc.m12 * dz;
            } else {
                dxy = xyi[p] - xyj;
                const float dz = Ir[p].z - zj;
                q0 = fmaf(wz * dz, dz, __builtin_amdgcn_fdot2(dxy, dxy, 0.0f, false));
            }
            const float s = fmaf(ej, kc.rc4, ai[p]);
            const float inv = drcp(s);
            const float u = fmaf(ci[p], inv, -kc.csig);
            const float ts = u * u;
            const int l = (int)ts;
            const float fS = dfract(ts);
            const int lg = min(l, 64 - 2);  // the global rows have no column beyond n_sigma - 1
            const float fSg = ts - (float)lg;
            const float w = (u * inv) * inv;
            // NEAR, GLOB: the group's table cells are read first, then
            // interpolated, so that their loads are in flight together
            float mg[G], rg[G], fDg[G];
            float4 cg[G];
            if (NEAR || GLOB) {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    if constexpr (SKEW) {
                        const float ex = dx - lxy[g].x, ey = dy - lxy[g].y;
                        mg[g] = fmaf(ex, fmaf(kc.m01, ey, ex + zx), fmaf(ey, fmaf(kc.wy, ey, zy), zA));
                    } else {
                        mg[g] = __builtin_amdgcn_fdot2(ml[g], dxy, q0 + cl[g], false);
                    }
                    rg[g] = dsqrt(mg[g]);
                    const float tD = s * rg[g];
                    const int kk = (int)tD;
                    fDg[g] = dfract(tD);
                    if (NEAR) {
                        const float *t = tab + (__umul24((unsigned)kk, 65u) + (unsigned)l);
                        cg[g] = make_float4(t[0], t[1], t[65], t[66]);
                    } else {
                        cg[g] = kc.quad[(uint32_t)(kk * (64 - 1) + lg)];
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                float m, ph, dqi = 0.0f, dqj = 0.0f;
                if (NEAR || GLOB) {
                    m = mg[g];
                    bilinear<float, ADJ, true>(cg[g].x, cg[g].y, cg[g].z, cg[g].w, fDg[g], NEAR ? fS : fSg, rg[g], w,
                                               1.0f, 1.0f, ei[p], ej, ph, dqi, dqj);
                } else {
                    if constexpr (SKEW) {
                        const float ex = dx - lxy[g].x, ey = dy - lxy[g].y;
                        m = fmaf(ex, fmaf(kc.m01, ey, ex + zx), fmaf(ey, fmaf(kc.wy, ey, zy), zA));
                    } else {
                        m = __builtin_amdgcn_fdot2(ml[g], dxy, q0 + cl[g], false);
                    }
                    img_eval<ADJ, NEAR, GLOB>(kc, tab, m, s, w, l, fS, lg, fSg, ai[p], ej, ei[p], ph, dqi, dqj);
                }
                float wjp = nj, wip = ni[p];
                if (MASK) {
                    wjp = (m <= rcm) ? nj : 0.0f;
                    wip = (m <= rcm) ? ni[p] : 0.0f;
                }
                acc[p] = fmaf(wjp, ph, acc[p]);
                accj = fmaf(wip, ph, accj);
                if (ADJ) {
                    accq[p] = fmaf(wjp, dqi, accq[p]);
                    accqj = fmaf(wip, dqj, accqj);
                }
            }
        }
        if constexpr (SKEW) {
            xj = wrot(xj);
            yj = wrot(yj);
        } else {
            xyj = wrot(xyj);
        }
        zj = wrot(zj);
        ej = wrot(ej);
        nj = wrot(nj);
        accj = wrot(accj);
        if (ADJ) accqj = wrot(accqj);
    }
}

// Wavefront-wide min / max (every lane gets the result; all 64 lanes active).
// FP32: rotations within each row of 16 lanes (DPP row_ror 8, 4, 2, 1) leave
// every lane with its row's result, then the four rows are read out, all
// without the LDS unit; FP64: lane exchanges.
template <int CTRL>
__device__ inline float dpp_row(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
__device__ inline float lane_value(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
template <typename R>
__device__ inline R wave_min(R v)
{
    if constexpr (sizeof(R) == 4) {
        v = min(v, dpp_row<0x128>(v));
        v = min(v, dpp_row<0x124>(v));
        v = min(v, dpp_row<0x122>(v));
        v = min(v, dpp_row<0x121>(v));
        return min(min(lane_value(v, 0), lane_value(v, 16)), min(lane_value(v, 32), lane_value(v, 48)));
    } else {
        for (int o = 32; o > 0; o >>= 1) v = min(v, (R)__shfl_xor(v, o));
        return v;
    }
}
template <typename R>
__device__ inline R wave_max(R v)
{
    if constexpr (sizeof(R) == 4) {
        v = max(v, dpp_row<0x128>(v));
        v = max(v, dpp_row<0x124>(v));
        v = max(v, dpp_row<0x122>(v));
        v = max(v, dpp_row<0x121>(v));
        return max(max(lane_value(v, 0), lane_value(v, 16)), max(lane_value(v, 32), lane_value(v, 48)));
    } else {
        for (int o = 32; o > 0; o >>= 1) v = max(v, (R)__shfl_xor(v, o));
        return v;
    }
}

// A wavefront-uniform copy of lane 0's value.  The builtin moves 32-bit
// integers, so floating-point values travel as their bit patterns (a plain
// call would convert them to int and truncate).
__device__ inline float uniform(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ inline double uniform(double v)
{
    int2 b = __builtin_bit_cast(int2, v);
    b.x = __builtin_amdgcn_readfirstlane(b.x);
    b.y = __builtin_amdgcn_readfirstlane(b.y);
    return __builtin_bit_cast(double, b);
}

// Position used for the tile boxes of the image pruning: the grid indices
// on orthorhombic grids (the distance weights wy, wz apply), Cartesian
// coordinates in units of h_x on skew grids (unit weights).
template <typename R, int GEO>
__device__ __forceinline__ void box_pos(const PairK<R> &k, R x, R y, R z, R &px, R &py, R &pz)
{
    if (GEO == kSkew) {
        px = x * k.en[0] + y * k.en[3] + z * k.en[6];
        py = x * k.en[1] + y * k.en[4] + z * k.en[7];
        pz = x * k.en[2] + y * k.en[5] + z * k.en[8];
    } else {
        px = x;
        py = y;
        pz = z;
    }
}

// Smallest and largest squared distance (units of h_x^2) between two boxes
// of box_pos coordinates, after shifting the second by (sx, sy, sz).  On
// skew grids the Cartesian boxes come from rounded products, so the bounds
// are widened by 2^-12 relative.
template <typename R, bool SKEW>
__device__ inline void box_dist2(const PairK<R> &k, const R *bi, const R *bj, R sx, R sy, R sz, R &dmin2, R &dmax2)
{
    const R sh[3] = {sx, sy, sz};
    const R wt[3] = {(R)1, SKEW ? (R)1 : k.wy, SKEW ? (R)1 : k.wz};
    dmin2 = 0;
    dmax2 = 0;
    for (int a = 0; a < 3; ++a) {
        // i range [bi[2a], bi[2a+1]], shifted j range [bj[2a] + s, bj[2a+1] + s]
        const R lo = bj[2 * a] + sh[a], hi = bj[2 * a + 1] + sh[a];
        const R gap = max((R)0, max(bi[2 * a] - hi, lo - bi[2 * a + 1]));
        const R far = max(bi[2 * a + 1] - lo, hi - bi[2 * a]);
        dmin2 += wt[a] * gap * gap;
        dmax2 += wt[a] * far * far;
    }
    if (SKEW) {
        dmin2 *= (R)(1.0 - 1.0 / 4096.0);
        dmax2 *= (R)(1.0 + 1.0 / 4096.0);
    }
}

// Pointers are separate __restrict__ parameters so the compiler knows the
// records, segments and table are not written during the kernel and can
// fetch wave-uniform records with scalar loads.
template <typename R, bool ADJ, bool IMG, bool KAHAN, int NSIG, int GEO, int IPL, int TPB>
__global__ __launch_bounds__(TPB) void pair_kernel(PairArgs A, const typename RecOf<R>::T *__restrict__ recs,
                                                            const Seg *__restrict__ segs,
                                                            const int64_t *__restrict__ hdr, int *__restrict__ counter,
                                                            const R *__restrict__ tabg, const int *__restrict__ imgs,
                                                            const int64_t *__restrict__ rowoff,
                                                            double *__restrict__ ipart, double *__restrict__ jpart,
                                                            const float4 *__restrict__ quad)
{
    using Rec = typename RecOf<R>::T;
    constexpr int NJc = 1 + (IMG ? 1 : 0) + (ADJ ? 1 : 0);
    constexpr bool NORM = GEO == kCubic && sizeof(R) == 4;
    // static LDS: the table rows (K x S, row stride S = n_sigma + 1), the
    // j-side sums of one tile from every wavefront (one accumulator array at
    // a time, FP64), the work-item slot
    constexpr int NW = TPB / 64;  // wavefronts of the workgroup
    __shared__ __align__(16) R tab[tab_elems<R>(NW)];
    __shared__ double red[NW * 64];
    __shared__ int s_item_v;
    int *s_item = &s_item_v;

    const int nS = A.nS;
    PairK<R> kc;
    kc.tDmax = (R)A.tDmax;
    kc.tDlds = (R)(A.K - 1);
    kc.tSclamp = (R)A.tSclamp;
    kc.csig = (R)A.csig;
    kc.c4 = (R)(4.0 * A.csig);
    kc.rc4 = (R)(0.25 / A.csig);
    kc.casym = (R)A.casym;
    kc.S = A.S;
    kc.nS = nS;
    kc.K = A.K;
    kc.nD = A.nD;
    kc.quad = quad;

    for (int t = threadIdx.x; t < A.K * nS; t += TPB) {
        int r = t / nS, c = t - r * nS;
        tab[r * A.S + c] = tabg[t];
        // column n_sigma: linear continuation of the last cell (FP32 form)
        if (sizeof(R) == 4 && c == nS - 1) tab[r * A.S + nS] = (R)2 * tabg[t] - tabg[t - 1];
    }
    __syncthreads();

    const int64_t total = hdr[HDR_ITEMS];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int iS0L = 1, iSq = A.NI - 1;  // accumulator array indices

    for (;;) {
        if (threadIdx.x == 0) *s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(*s_item);
        __syncthreads();
        if (item >= total) break;

        const int b = (A.B > 1) ? __builtin_amdgcn_readfirstlane(find_seg(segs, A.B, item, 2)) : 0;
        const Seg &sg = segs[b];
        const int N = __builtin_amdgcn_readfirstlane((int)sg.N);
        const int nIB = __builtin_amdgcn_readfirstlane((int)sg.nIB);
        const int local = __builtin_amdgcn_readfirstlane((int)(item - sg.item_off));
        const int64_t *__restrict__ ro = rowoff + sg.row_base;
        int I = 0;
        {
            int lo = 0, hi = nIB - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (ro[mid] <= local) lo = mid;
                else hi = mid - 1;
            }
            I = __builtin_amdgcn_readfirstlane(lo);
        }
        const int c = local - (int)ro[I];
        const int64_t slot = sg.slot_base + local;
        kc.wy = (R)((sg.hy / sg.hx) * (sg.hy / sg.hx));
        kc.wz = (R)((sg.hz / sg.hx) * (sg.hz / sg.hx));
        if (GEO == kSkew) {
            kc.m01 = (R)sg.m01;
            kc.m02 = (R)sg.m02;
            kc.m12 = (R)sg.m12;
            for (int k = 0; k < 9; ++k) kc.en[k] = (R)sg.en[k];
        }
        const R rcm = (R)(A.rc2 / (sg.hx * sg.hx));  // distance cut in units of h_x^2
        const Rec *__restrict__ P = recs + sg.p_off;

        // IPL i-points per lane: point p of lane l of wavefront w is number
        // w (64 IPL) + 64 p + l of the row block
        constexpr int BI = IPL * TPB;
        bool act[IPL];
        Rec Ir[IPL];
        R ai[IPL], ci[IPL], ni[IPL];
#pragma unroll
        for (int p = 0; p < IPL; ++p) {
            const int il = I * BI + w * (64 * IPL) + 64 * p + lane;
            act[p] = il < N;
            Ir[p] = P[act[p] ? il : N - 1];
            ai[p] = Ir[p].a;
            ci[p] = ci_of(kc, Ir[p].a, Ir[p].b);
            ni[p] = act[p] ? Ir[p].n : (R)0;
        }
        double Sc[IPL], SL[IPL], Sq[IPL];
#pragma unroll
        for (int p = 0; p < IPL; ++p) Sc[p] = SL[p] = Sq[p] = 0.0;
        const int nimg = IMG ? A.nimg : 1;

        if (c < A.ND) {
            // diagonal item c: ordered pairs of the row block's points with its
            // c-th j sub-range, j through scalar loads
            const int j0 = I * BI + c * A.DS, j1 = min(N, j0 + A.DS);
            for (int L = 0; L < (j0 < j1 ? nimg : 0); ++L) {
                R sx[IPL], sy[IPL], sz[IPL], mx[IPL], my[IPL], mz[IPL], wi[IPL];
                bool home = true;
                R lx = 0, ly = 0, lz = 0;
                if (IMG) {
                    lx = (R)(imgs[4 * L + 0] * sg.nx);
                    ly = (R)(imgs[4 * L + 1] * sg.ny);
                    lz = (R)(imgs[4 * L + 2] * sg.nz);
                    home = (L == A.home);
                }
#pragma unroll
                for (int p = 0; p < IPL; ++p) {
                    sx[p] = Ir[p].x - lx;
                    sy[p] = Ir[p].y - ly;
                    sz[p] = Ir[p].z - lz;
                    mx[p] = -2 * sx[p];
                    my[p] = -2 * sy[p];
                    mz[p] = -2 * sz[p];
                    wi[p] = sx[p] * sx[p] + sy[p] * sy[p] + sz[p] * sz[p];
                }
                Rec Jn = P[j0];
                for (int jr = j0; jr < j1; jr += kRun) {
                    const int je = min(j1, jr + kRun);
                    R acc[IPL], accq[IPL], cm[IPL];
#pragma unroll
                    for (int p = 0; p < IPL; ++p) acc[p] = accq[p] = cm[p] = 0;
                    for (int j = jr; j < je; ++j) {
                        const Rec J = Jn;
                        Jn = P[min(j + 1, j1 - 1)];  // prefetch the next record (wave-uniform)
                        // FP32: the j point as ej = 4 csig a_j (see pair_eval)
                        const R ajx = sizeof(R) == 4 ? kc.c4 * J.a : J.a;
                        const R cj = cj_of(kc, J.a);
#pragma unroll
                        for (int p = 0; p < IPL; ++p) {
                            R m;
                            if (NORM)
                                m = (R)dist2n((float)mx[p], (float)my[p], (float)mz[p], (float)(wi[p] + J.w),
                                              (float)J.x, (float)J.y, (float)J.z);
                            else
                                m = dist2<R, GEO>(kc, sx[p] - J.x, sy[p] - J.y, sz[p] - J.z);
                            R wt = (m > (R)0) ? J.n : (R)0;
                            if (IMG) wt = (m <= rcm) ? wt : (R)0;
                            R ph, q = 0, unused;
                            pair_eval<ADJ, false, NSIG, IMG>(kc, tab, tabg, m, ai[p], ci[p], ajx, cj, ph, q, unused);
                            if (KAHAN) {
                                R y = wt * ph - cm[p], t = acc[p] + y;
                                cm[p] = (t - acc[p]) - y;
                                acc[p] = t;
                            } else {
                                acc[p] += wt * ph;
                            }
                            if (ADJ) accq[p] += wt * q;
                        }
                    }
#pragma unroll
                    for (int p = 0; p < IPL; ++p) {
                        if (home) Sc[p] += (double)acc[p] - (double)cm[p];
                        else SL[p] += (double)acc[p] - (double)cm[p];
                        if (ADJ) Sq[p] += (double)accq[p];
                    }
                }
            }
        } else {
            // off-diagonal item: both orders of every pair, j tiles rotating through the lanes
            const int J0 = (I + 1) * BI + (c - A.ND) * A.JC, J1 = min(N, J0 + A.JC);
            const bool prune = IMG && A.rc2 < 1e300;
            // FP32 bilinear image kernels: rings whose pairs provably stay
            // below the LDS rows take the NEAR ring (bound from the tile boxes
            // and the largest a of either tile, widened by 2^-10 for the FP32
            // rounding of s r); without images the plain ring was as fast
            constexpr bool NEARABLE = sizeof(R) == 4 && NSIG != kCubicD && IMG;
            // image kernels: rings whose pairs provably lie in the global rows
            // (K - 1 <= t_D < n_D - 1) take the GLOB ring
            constexpr bool GLOBABLE = NEARABLE && IMG;
            R ib[6] = {0, 0, 0, 0, 0, 0};
            R aimax = 0, aimin = 0;
            if (NEARABLE) {
                R am = ai[0], an = ai[0];
#pragma unroll
                for (int p = 1; p < IPL; ++p) {
                    am = max(am, ai[p]);
                    an = min(an, ai[p]);
                }
                aimax = uniform(wave_max<R>(am));
                aimin = uniform(wave_min<R>(an));
            }
            if (prune || NEARABLE) {
                // bounding box of this wavefront's i-points
                R lo[3], hi[3];
                box_pos<R, GEO>(kc, Ir[0].x, Ir[0].y, Ir[0].z, lo[0], lo[1], lo[2]);
                hi[0] = lo[0];
                hi[1] = lo[1];
                hi[2] = lo[2];
#pragma unroll
                for (int p = 1; p < IPL; ++p) {
                    R q[3];
                    box_pos<R, GEO>(kc, Ir[p].x, Ir[p].y, Ir[p].z, q[0], q[1], q[2]);
                    for (int a3 = 0; a3 < 3; ++a3) {
                        lo[a3] = min(lo[a3], q[a3]);
                        hi[a3] = max(hi[a3], q[a3]);
                    }
                }
                for (int a3 = 0; a3 < 3; ++a3) {
                    ib[2 * a3] = uniform(wave_min<R>(lo[a3]));
                    ib[2 * a3 + 1] = uniform(wave_max<R>(hi[a3]));
                }
            }
            for (int t0 = J0; t0 < J1; t0 += 64) {
                const int jj = t0 + lane;
                const bool jv = jj < J1;
                const Rec Jr = P[jv ? jj : J1 - 1];
                R jb6[6] = {0, 0, 0, 0, 0, 0};
                const R ajmax = NEARABLE ? uniform(wave_max<R>(Jr.a)) : (R)0;
                const R ajmin = GLOBABLE ? uniform(wave_min<R>(Jr.a)) : (R)0;
                if (prune || NEARABLE) {
                    R q[3];
                    box_pos<R, GEO>(kc, Jr.x, Jr.y, Jr.z, q[0], q[1], q[2]);
                    jb6[0] = uniform(wave_min<R>(q[0]));
                    jb6[1] = uniform(wave_max<R>(q[0]));
                    jb6[2] = uniform(wave_min<R>(q[1]));
                    jb6[3] = uniform(wave_max<R>(q[1]));
                    jb6[4] = uniform(wave_min<R>(q[2]));
                    jb6[5] = uniform(wave_max<R>(q[2]));
                }
                // j-side sums of the tile over the image shifts, carried in
                // FP64 after every 64-step ring (as the i side)
                double jSc = 0.0, jSL = 0.0, jSq = 0.0;
                // FP32 n_sigma = 64 image kernels on square and skew grids: the
                // image shifts of the first 64 (those in x and y only, not the
                // home cell) are sorted by ring class (masked or not; NEAR, GLOB
                // or per-lane source) and run kImgGroup at a time (ring64_img),
                // two or three left of a class two at a time; the last one of a
                // class, and every other shift, one at a time
                constexpr bool GRP = IMG && (GEO == kSquare || GEO == kSkew) && sizeof(R) == 4 && !KAHAN && NSIG == 64;
                if constexpr (GRP) {
                    const R nj0 = jv ? Jr.n : (R)0;
                    // one 64-step ring of the tile against one shift, carried into
                    // the FP64 sums of the home cell or of the images
                    auto one_ring = [&](R lx, R ly, R lz, bool home, bool masked, bool near, bool glob) {
                        R sx[IPL], sy[IPL], sz[IPL], acc[IPL], accq[IPL];
#pragma unroll
                        for (int p = 0; p < IPL; ++p) {
                            sx[p] = Ir[p].x - lx;
                            sy[p] = Ir[p].y - ly;
                            sz[p] = Ir[p].z - lz;
                            acc[p] = accq[p] = 0;
                        }
                        R accj = 0, accqj = 0;
#define RING(MSK, NR, GL)                                                                                          \
        ring64<R, ADJ, MSK, KAHAN, NSIG, GEO, IPL, IMG, NR, GL>(kc, tab, tabg, rcm, sx, sy, sz, ai, ci, ni, Jr.x, Jr.y, Jr.z, \
                                                             Jr.w, Jr.a, nj0, acc, accq, accj, accqj)
                        if (masked) {
                            if (NEARABLE && near) RING(true, NEARABLE, false);
                            else if (GLOBABLE && glob) RING(true, false, GLOBABLE);
                            else RING(true, false, false);
                        } else {
                            if (NEARABLE && near) RING(false, NEARABLE, false);
                            else if (GLOBABLE && glob) RING(false, false, GLOBABLE);
                            else RING(false, false, false);
                        }
#undef RING
#pragma unroll
                        for (int p = 0; p < IPL; ++p) {
                            if (home) Sc[p] += (double)acc[p];
                            else SL[p] += (double)acc[p];
                            if (ADJ) Sq[p] += (double)accq[p];
                        }
                        if (home) jSc += (double)accj;
                        else jSL += (double)accj;
                        if (ADJ) jSq += (double)accqj;
                    };
                    uint64_t gm[6] = {0, 0, 0, 0, 0, 0};  // class 3 masked + (0 NEAR, 1 GLOB, 2 per lane)
                    for (int L = 0; L < nimg; ++L) {
                        R lx = 0, ly = 0, lz = 0;
                        bool home = true, masked = prune;  // no cut: every tile unmasked
                        bool near = false, glob = false;
                        if (IMG) {
                            lx = (R)(imgs[4 * L + 0] * sg.nx);
                            ly = (R)(imgs[4 * L + 1] * sg.ny);
                            lz = (R)(imgs[4 * L + 2] * sg.nz);
                            home = (L == A.home);
                        }
                        if (prune || NEARABLE) {
                            // r_i - r_j - L: the j box shifted by +L against the i box
                            R dmin2, dmax2, bx, by, bz;
                            box_pos<R, GEO>(kc, lx, ly, lz, bx, by, bz);
                            box_dist2<R, GEO == kSkew>(kc, ib, jb6, bx, by, bz, dmin2, dmax2);
                            if (prune) {
                                if (dmin2 > rcm) continue;  // the whole tile is beyond the cut
                                masked = dmax2 > rcm;
                            }
                            if (NEARABLE) {
                                const R hi = (aimax + ajmax) * sqrt(dmax2) * (R)(1.0 + 1.0 / 1024.0);
                                near = hi < kc.tDlds;
                                glob = GLOBABLE && hi < kc.tDmax &&
                                       (aimin + ajmin) * sqrt(dmin2) * (R)(1.0 - 1.0 / 1024.0) >= kc.tDlds;
                            }
                        }
                        if (GRP && !home && lz == (R)0 && L < 64) {
                            const int cls = (masked ? 3 : 0) + (near ? 0 : glob ? 1 : 2);
#pragma unroll
                            for (int c6 = 0; c6 < 6; ++c6)  // constant indices: the masks stay in registers
                                if (c6 == cls) gm[c6] |= 1ull << L;
                            continue;
                        }
                        one_ring(lx, ly, lz, home, masked, near, glob);
                    }
                    if constexpr (GRP) {
#pragma unroll
                        for (int cl6 = 0; cl6 < 6; ++cl6) {
                            uint64_t mk = gm[cl6];
                            // the next Gc::value shifts of mk as one ring of class cl6
                            auto group_ring = [&](auto Gc) {
                                constexpr int G = decltype(Gc)::value;
                                half2v ml[G];
                                float cL[G];
                                float2 lxy[G];
#pragma unroll
                                for (int g = 0; g < G; ++g) {
                                    const int L = __builtin_ctzll(mk);
                                    mk &= mk - 1;
                                    const float lx = (float)(imgs[4 * L + 0] * sg.nx);
                                    const float ly = (float)(imgs[4 * L + 1] * sg.ny);
                                    ml[g] = half2v{(_Float16)(-2.0f * lx), (_Float16)(-2.0f * ly)};
                                    cL[g] = lx * lx + ly * ly;
                                    lxy[g] = make_float2(lx, ly);
                                }
                                R acc[IPL], accq[IPL];
#pragma unroll
                                for (int p = 0; p < IPL; ++p) acc[p] = accq[p] = 0;
                                R accj = 0, accqj = 0;
#define RINGI(MSK, NR, GL)                                                                                          \
    ring64_img<ADJ, MSK, IPL, NR, GL, G, GEO>(kc, tab, rcm, Ir, ai, ci, ni, Jr.x, Jr.y, Jr.z, Jr.a, nj0, ml, cL, lxy, \
                                              acc, accq, accj, accqj)
                                switch (cl6) {
                                case 0: RINGI(false, true, false); break;
                                case 1: RINGI(false, false, true); break;
                                case 2: RINGI(false, false, false); break;
                                case 3: RINGI(true, true, false); break;
                                case 4: RINGI(true, false, true); break;
                                default: RINGI(true, false, false); break;
                                }
#undef RINGI
#pragma unroll
                                for (int p = 0; p < IPL; ++p) {
                                    SL[p] += (double)acc[p];
                                    if (ADJ) Sq[p] += (double)accq[p];
                                }
                                jSL += (double)accj;
                                if (ADJ) jSq += (double)accqj;
                            };
                            while (__builtin_popcountll(mk) >= kImgGroup) group_ring(IntC<kImgGroup>{});
                            if (__builtin_popcountll(mk) >= 2) group_ring(IntC<2>{});
                            while (mk) {
                                const int L = __builtin_ctzll(mk);
                                mk &= mk - 1;
                                one_ring((R)(imgs[4 * L + 0] * sg.nx), (R)(imgs[4 * L + 1] * sg.ny), (R)0, false,
                                         cl6 >= 3, cl6 % 3 == 0, cl6 % 3 == 1);
                            }
                        }
                    }
                } else {
                    for (int L = 0; L < nimg; ++L) {
                        R lx = 0, ly = 0, lz = 0;
                        bool home = true, masked = prune;  // no cut: every tile unmasked
                        bool near = false, glob = false;
                        if (IMG) {
                            lx = (R)(imgs[4 * L + 0] * sg.nx);
                            ly = (R)(imgs[4 * L + 1] * sg.ny);
                            lz = (R)(imgs[4 * L + 2] * sg.nz);
                            home = (L == A.home);
                        }
                        if (prune || NEARABLE) {
                            // r_i - r_j - L: the j box shifted by +L against the i box
                            R dmin2, dmax2, bx, by, bz;
                            box_pos<R, GEO>(kc, lx, ly, lz, bx, by, bz);
                            box_dist2<R, GEO == kSkew>(kc, ib, jb6, bx, by, bz, dmin2, dmax2);
                            if (prune) {
                                if (dmin2 > rcm) continue;  // the whole tile is beyond the cut
                                masked = dmax2 > rcm;
                            }
                            if (NEARABLE) {
                                const R hi = (aimax + ajmax) * sqrt(dmax2) * (R)(1.0 + 1.0 / 1024.0);
                                near = hi < kc.tDlds;
                                glob = GLOBABLE && hi < kc.tDmax &&
                                       (aimin + ajmin) * sqrt(dmin2) * (R)(1.0 - 1.0 / 1024.0) >= kc.tDlds;
                            }
                        }
                        R sx[IPL], sy[IPL], sz[IPL], acc[IPL], accq[IPL];
#pragma unroll
                        for (int p = 0; p < IPL; ++p) {
                            sx[p] = Ir[p].x - lx;
                            sy[p] = Ir[p].y - ly;
                            sz[p] = Ir[p].z - lz;
                            acc[p] = accq[p] = 0;
                        }
                        R accj = 0, accqj = 0;
                        const R nj0 = jv ? Jr.n : (R)0;
#define RING(MSK, NR, GL)                                                                                          \
        ring64<R, ADJ, MSK, KAHAN, NSIG, GEO, IPL, IMG, NR, GL>(kc, tab, tabg, rcm, sx, sy, sz, ai, ci, ni, Jr.x, Jr.y, Jr.z, \
                                                             Jr.w, Jr.a, nj0, acc, accq, accj, accqj)
                        if (masked) {
                            if (NEARABLE && near) RING(true, NEARABLE, false);
                            else if (GLOBABLE && glob) RING(true, false, GLOBABLE);
                            else RING(true, false, false);
                        } else {
                            if (NEARABLE && near) RING(false, NEARABLE, false);
                            else if (GLOBABLE && glob) RING(false, false, GLOBABLE);
                            else RING(false, false, false);
                        }
#undef RING
#pragma unroll
                        for (int p = 0; p < IPL; ++p) {
                            if (home) Sc[p] += (double)acc[p];
                            else SL[p] += (double)acc[p];
                            if (ADJ) Sq[p] += (double)accq[p];
                        }
                        if (home) jSc += (double)accj;
                        else jSL += (double)accj;
                        if (ADJ) jSq += (double)accqj;
                    }
                }
                // j-side sums of the tile: the wavefronts' FP64 partials added
                // in a fixed order, one accumulator array at a time
#pragma unroll
                for (int a = 0; a < NJc; ++a) {
                    red[w * 64 + lane] = (a == 0) ? jSc : (IMG && a == iS0L) ? jSL : jSq;
                    __syncthreads();
                    if (threadIdx.x < 64) {
                        double sum = 0.0;
                        for (int v = 0; v < NW; ++v) sum += red[v * 64 + threadIdx.x];
                        if (t0 + (int)threadIdx.x < J1)
                            jpart[a * A.jstride + slot * A.JC + (t0 + threadIdx.x - J0)] = sum;
                    }
                    __syncthreads();
                }
            }
        }
        const int64_t base = slot * BI + w * (64 * IPL) + lane;
        const double qscale = sg.hx / A.dD2;  // d/dq = h_x / (2 dD) times the sums above
#pragma unroll
        for (int p = 0; p < IPL; ++p) {
            if (!act[p]) continue;
            ipart[base + 64 * p] = Sc[p];
            if (IMG) ipart[iS0L * A.istride + base + 64 * p] = SL[p];
            if (ADJ) ipart[iSq * A.istride + base + 64 * p] = Sq[p] * qscale;
        }
    }
}

// ---------------------------------------------------------------------------
// finalize, reduce, assemble
// ---------------------------------------------------------------------------

constexpr int kVoxelGL = 8;  // Gauss-Legendre points per octant axis of the voxel on-site rule
// The voxel on-site term is read from a table of Phi_V over ln q: kVoxNodes
// nodes from ln 2^-6 to ln 2^7 (q outside takes the rule directly).
constexpr int kVoxNodes = 4096;
constexpr double kVoxLnLo = -6.0 * 0.69314718055994530942, kVoxLnHi = 7.0 * 0.69314718055994530942;

struct FinArgs {
    const Seg *segs;
    int B;
    const int64_t *hdr;
    const int64_t *rowoff;
    const double *ipart;
    const double *jpart;
    int64_t istride, jstride;
    int JC, BI, ND, NI, NJ;
    int img, adj, self_term;
    int vg;                   // voxel term: Gauss-Legendre points per octant axis
    int interp;               // 1: the table is read cubic in D
    double vu[kVoxelGL], vw[kVoxelGL];  // voxel term: nodes u in (0, 1) and weights 2 u w (1 - u^2)
    const int32_t *gidx;
    const double *n, *q0, *dqdn;
    const double *tab;  // FP64 table for the on-site term
    int nD, nS;
    double dD, Dmax, casym;
    double *blockE;
    const double *vox;  // self_term = 2: Phi_V at the ln q nodes, kVoxNodes per density
    unsigned long long *qmin;  // per density: bits of the smallest q0 of a kept point (positive doubles order as integers)
    double *dEdn;   // direct part scattered to the grid (potential)
    double *dEdq;   // dE/dq scattered to the grid (potential)
    const double *far;   // far-shell row partials, per density from Seg::far_part_off (compact order):
                         // far_chunks S0 arrays, then (potential) far_chunks Sq arrays, G apart; or NULL
};

// phi~(D, 0) and d phi~/dD from the FP64 table (asymptote at D >= D_max).
__device__ inline double self_phi(const FinArgs &F, double D, double *dphi)
{
    if (D >= F.Dmax) {
        double D6 = D * D * D * D * D * D;
        *dphi = 3.0 * F.casym / (D6 * D);
        return -F.casym / (2.0 * D6);
    }
    double tD = D / F.dD;
    int k = (int)floor(tD);
    if (k > F.nD - 2) k = F.nD - 2;
    double fD = tD - k;
    if (F.interp == VDW_INTERP_CUBIC_D) {
        // column sigma = 0, rows k-1 .. k+2 (extrapolated linearly beyond the ends)
        double c[4];
        for (int i = 0; i < 4; ++i) c[i] = F.tab[(int64_t)min(max(k - 1 + i, 0), F.nD - 1) * F.nS];
        if (k == 0) c[0] = 2.0 * c[1] - c[2];
        if (k + 2 > F.nD - 1) c[3] = 2.0 * c[2] - c[1];
        double dt;
        const double v = catmull_rom(c, fD, dt);
        *dphi = dt / F.dD;
        return v;
    }
    double p0 = F.tab[(int64_t)k * F.nS], p1 = F.tab[(int64_t)(k + 1) * F.nS];
    *dphi = (p1 - p0) / F.dD;
    return p0 + fD * (p1 - p0);
}

// The voxel double average of phi~(., 0) over the grid cell spanned by the
// step vectors e (rows):
//   Phi_V(q) = int_{[-1,1]^3} phi~(q |sum_a t_a e_a|, 0) prod_a (1 - |t_a|) dt,
// by the rule of 8 octants with t_a = +-u^2 at the Gauss-Legendre nodes u of
// [0, 1] (node weight prod 2 u w (1 - u^2)); *dPhi = d Phi_V / d q.
__device__ inline double voxel_phi(const FinArgs &F, const double *e, double q, double *dPhi)
{
    double acc = 0.0, dacc = 0.0;
    for (int oct = 0; oct < 8; ++oct) {
        const double s0 = (oct & 1) ? -1.0 : 1.0, s1 = (oct & 2) ? -1.0 : 1.0, s2 = (oct & 4) ? -1.0 : 1.0;
        for (int i = 0; i < F.vg; ++i)
            for (int j = 0; j < F.vg; ++j)
                for (int k = 0; k < F.vg; ++k) {
                    const double t0 = s0 * F.vu[i] * F.vu[i], t1 = s1 * F.vu[j] * F.vu[j], t2 = s2 * F.vu[k] * F.vu[k];
                    const double rx = t0 * e[0] + t1 * e[3] + t2 * e[6];
                    const double ry = t0 * e[1] + t1 * e[4] + t2 * e[7];
                    const double rz = t0 * e[2] + t1 * e[5] + t2 * e[8];
                    const double r = sqrt(rx * rx + ry * ry + rz * rz);
                    const double w = F.vw[i] * F.vw[j] * F.vw[k];
                    double dD;
                    acc += w * self_phi(F, q * r, &dD);
                    dacc += w * r * dD;
                }
    }
    *dPhi = dacc;
    return acc;
}

// Phi_V at the ln q nodes of every density: one thread per node.
__global__ __launch_bounds__(256) void voxel_table_kernel(FinArgs F, double *__restrict__ vox)
{
    const int k = blockIdx.x * 256 + threadIdx.x, b = blockIdx.y;
    if (k >= kVoxNodes) return;
    const double x = kVoxLnLo + k * ((kVoxLnHi - kVoxLnLo) / (kVoxNodes - 1));
    double d;
    vox[(int64_t)b * kVoxNodes + k] = voxel_phi(F, F.segs[b].e, exp(x), &d);
}

// Phi_V(q) and dPhi_V/dq from the node values of one density: the
// Catmull-Rom cubic in ln q (rows beyond the ends extrapolated linearly).
__device__ inline double voxel_interp(const double *__restrict__ vt, double q, double *dPhi)
{
    const double dx = (kVoxLnHi - kVoxLnLo) / (kVoxNodes - 1);
    const double xs = (log(q) - kVoxLnLo) / dx;
    const int k = min(max((int)floor(xs), 0), kVoxNodes - 2);
    const double t = xs - k;
    double f[4];
    f[1] = vt[k];
    f[2] = vt[k + 1];
    f[0] = k > 0 ? vt[k - 1] : 2.0 * f[1] - f[2];
    f[3] = k + 2 < kVoxNodes ? vt[k + 2] : 2.0 * f[2] - f[1];
    double dt;
    const double v = catmull_rom(f, t, dt);
    *dPhi = dt / (dx * q);
    return v;
}

__global__ __launch_bounds__(kFinThreads) void finalize_kernel(FinArgs F)
{
    __shared__ double r0[kFinThreads], r1[kFinThreads], r2[kFinThreads];
    __shared__ unsigned long long r3[kFinThreads];
    const int64_t blk = blockIdx.x;
    if (blk >= F.hdr[HDR_BLKS]) return;
    const int b = find_seg(F.segs, F.B, blk, 3);
    const Seg &sg = F.segs[b];
    const int64_t lp = (blk - sg.blk_off) * kFinThreads + threadIdx.x;
    double e0 = 0.0, eL = 0.0, es = 0.0;
    unsigned long long qb = ~0ull;
    if (lp < sg.N) {
        const int64_t p = sg.p_off + lp;
        double S0c = 0.0, S0L = 0.0, Sq = 0.0;
        const int iL = 1, iq = F.NI - 1;
        const int64_t *ro = F.rowoff + sg.row_base;
        // as an i-point: the diagonal items and the chunks of its own row block
        const int64_t Bk = lp / F.BI, t = lp - Bk * F.BI;
        for (int64_t it = ro[Bk]; it < ro[Bk + 1]; ++it) {
            const int64_t k = (sg.slot_base + it) * F.BI + t;
            S0c += F.ipart[k];
            if (F.img) S0L += F.ipart[iL * F.istride + k];
            if (F.adj) Sq += F.ipart[iq * F.istride + k];
        }
        // as a j-point: one chunk in each earlier row block
        for (int64_t I = 0; I < Bk; ++I) {
            const int64_t off = lp - (I + 1) * F.BI;
            const int64_t cc = off / F.JC;
            const int64_t k = (sg.slot_base + ro[I] + F.ND + cc) * F.JC + (off - cc * F.JC);
            S0c += F.jpart[k];
            if (F.img) S0L += F.jpart[iL * F.jstride + k];
            if (F.adj) Sq += F.jpart[iq * F.jstride + k] * (sg.hx / (2.0 * F.dD));
        }
        if (F.far) {
            const double *fp = F.far + sg.far_part_off;
            for (int c = 0; c < sg.far_chunks; ++c) {
                S0L += fp[c * sg.G + lp];
                if (F.adj) Sq += fp[(sg.far_chunks + c) * sg.G + lp];
            }
        }
        const int64_t g = F.gidx[p];
        const double nn = F.n[g], q = F.q0[g];
        qb = (unsigned long long)__builtin_bit_cast(uint64_t, q);
        const double rho_s = cbrt(3.0 * sg.dV / (4.0 * 3.14159265358979323846)) * exp(-1.0 / 3.0);
        double Phi = 0.0, dPhi = 0.0;
        if (F.self_term == 2) {
            if (q >= exp(kVoxLnLo) && q <= exp(kVoxLnHi))
                Phi = voxel_interp(F.vox + (int64_t)b * kVoxNodes, q, &dPhi);
            else
                Phi = voxel_phi(F, sg.e, q, &dPhi);
        } else if (F.self_term) {
            double dphi_dD;
            Phi = self_phi(F, q * rho_s, &dphi_dD);
            dPhi = rho_s * dphi_dD;
        }
        e0 = nn * S0c;
        eL = nn * S0L;
        es = nn * nn * Phi;
        if (F.adj) {
            const double dV2 = sg.dV * sg.dV;
            const double dEdq = dV2 * nn * (Sq + 0.5 * nn * dPhi);
            F.dEdn[g] = dV2 * (S0c + S0L + nn * Phi) + dEdq * F.dqdn[g];
            F.dEdq[g] = dEdq;
        }
    }
    r0[threadIdx.x] = e0;
    r1[threadIdx.x] = eL;
    r2[threadIdx.x] = es;
    r3[threadIdx.x] = qb;
    __syncthreads();
    for (int st = kFinThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            r0[threadIdx.x] += r0[threadIdx.x + st];
            r1[threadIdx.x] += r1[threadIdx.x + st];
            r2[threadIdx.x] += r2[threadIdx.x + st];
            r3[threadIdx.x] = min(r3[threadIdx.x], r3[threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        F.blockE[3 * blk + 0] = r0[0];
        F.blockE[3 * blk + 1] = r1[0];
        F.blockE[3 * blk + 2] = r2[0];
        atomicMin(F.qmin + b, r3[0]);
    }
}

__global__ __launch_bounds__(256) void seg_reduce_kernel(const Seg *__restrict__ segs, const double *__restrict__ blockE,
                                                         double *__restrict__ res, int B, const int *__restrict__ flag)
{
    __shared__ double r0[256], r1[256], r2[256];
    const int b = blockIdx.x;
    const Seg &sg = segs[b];
    const int64_t nb = (sg.N + kFinThreads - 1) / kFinThreads;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t k = threadIdx.x; k < nb; k += 256) {
        a0 += blockE[3 * (sg.blk_off + k) + 0];
        a1 += blockE[3 * (sg.blk_off + k) + 1];
        a2 += blockE[3 * (sg.blk_off + k) + 2];
    }
    r0[threadIdx.x] = a0;
    r1[threadIdx.x] = a1;
    r2[threadIdx.x] = a2;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            r0[threadIdx.x] += r0[threadIdx.x + st];
            r1[threadIdx.x] += r1[threadIdx.x + st];
            r2[threadIdx.x] += r2[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double h = 0.5 * sg.dV * sg.dV;
        res[3 * b + 0] = h * r0[0];
        res[3 * b + 1] = h * r1[0];
        res[3 * b + 2] = h * r2[0];
        res[3 * B + b] = (double)sg.N;
        if (b == 0) res[4 * B] = (double)*flag;
    }
}

// Transposed second-order stencil along one axis at index k, applied to
// B_i = dE/dq_i dq/dg_i 2 (d_a n)_i (zero where i is not kept).
struct AsmArgs {
    const Seg *segs;
    int B;
    int64_t Gtot;
    const double *dEdq, *dqdg, *grad;
    double *dEdn;
};

// B_a at grid point gl: dE/dq dq/dg 2 (grad n)_a on orthorhombic grids; on
// skew grids the same Cartesian vector mapped back to the grid axes by the
// transpose of E^-1 (the derivative with respect to the difference d_a).
template <bool SKEW>
__device__ inline double bval(const AsmArgs &A, const Seg &s, int axis, int64_t gl)
{
    int64_t g = s.grid_off + gl;
    const double *gr = A.grad + 3 * s.grid_off + gl;
    if (SKEW)
        return A.dEdq[g] * A.dqdg[g] * 2.0 *
               (s.einv[axis] * gr[0] + s.einv[3 + axis] * gr[s.G] + s.einv[6 + axis] * gr[2 * s.G]);
    return A.dEdq[g] * A.dqdg[g] * 2.0 * gr[axis * s.G];
}

// Transposed difference stencil of axis `axis` applied to B at point idx
// (index k of N along the axis, stride st); h = 1 on skew grids (differences
// per grid step).
template <bool SKEW>
__device__ inline double tstencil(const AsmArgs &A, const Seg &s, int axis, int64_t idx, int k, int N, int64_t st,
                                  int per, double h)
{
    double acc = 0.0;
    if (per) {
        int64_t up = (k + 1 == N) ? -(int64_t)(N - 1) * st : st;
        int64_t dn = (k == 0) ? (int64_t)(N - 1) * st : -st;
        acc = bval<SKEW>(A, s, axis, idx + dn) - bval<SKEW>(A, s, axis, idx + up);
    } else {
        // interior rows i = k-1 (coefficient +1 at k) and i = k+1 (coefficient -1 at k)
        if (k - 1 >= 1 && k - 1 <= N - 2) acc += bval<SKEW>(A, s, axis, idx - st);
        if (k + 1 >= 1 && k + 1 <= N - 2) acc -= bval<SKEW>(A, s, axis, idx + st);
        // face row i = 0: (-3, 4, -1) on (0, 1, 2)
        if (k <= 2) {
            const double c0[3] = {-3.0, 4.0, -1.0};
            acc += c0[k] * bval<SKEW>(A, s, axis, idx - (int64_t)k * st);
        }
        // face row i = N-1: (1, -4, 3) on (N-3, N-2, N-1)
        if (k >= N - 3) {
            const double c1[3] = {1.0, -4.0, 3.0};
            acc += c1[k - (N - 3)] * bval<SKEW>(A, s, axis, idx + (int64_t)(N - 1 - k) * st);
        }
    }
    return acc * (0.5 / h);
}

__global__ __launch_bounds__(256) void assemble_kernel(AsmArgs A)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A.Gtot) return;
    const int b = find_seg(A.segs, A.B, t, 4);
    const Seg &s = A.segs[b];
    const int64_t gl = t - s.grid_off;
    const int ix = (int)(gl % s.nx);
    const int64_t r = gl / s.nx;
    const int iy = (int)(r % s.ny);
    const int iz = (int)(r / s.ny);
    // (axes with the Fourier derivative are added by their own line kernels)
    double v = 0.0;
    if (s.skew) {
        if (!s.spec[0]) v += tstencil<true>(A, s, 0, gl, ix, s.nx, 1, s.px, 1.0);
        if (!s.spec[1]) v += tstencil<true>(A, s, 1, gl, iy, s.ny, s.nx, s.py, 1.0);
        if (!s.spec[2]) v += tstencil<true>(A, s, 2, gl, iz, s.nz, (int64_t)s.nx * s.ny, s.pz, 1.0);
    } else {
        if (!s.spec[0]) v += tstencil<false>(A, s, 0, gl, ix, s.nx, 1, s.px, s.hx);
        if (!s.spec[1]) v += tstencil<false>(A, s, 1, gl, iy, s.ny, s.nx, s.py, s.hy);
        if (!s.spec[2]) v += tstencil<false>(A, s, 2, gl, iz, s.nz, (int64_t)s.nx * s.ny, s.pz, s.hz);
    }
    A.dEdn[t] += v;
}

// ---------------------------------------------------------------------------
// gradient and q0 of every density of a packed batch (one launch)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void grad_q0_batched_kernel(const Seg *__restrict__ segs, int B, int64_t Gtot,
                                                              double n_cut, const double *__restrict__ n,
                                                              double *__restrict__ grad, double *__restrict__ q0,
                                                              double *__restrict__ dqdn, double *__restrict__ dqdg)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Gtot) return;
    const Seg &s = segs[find_seg(segs, B, t, 4)];
    const int64_t o = s.grid_off;
    // densities with the Fourier derivative have it staged in their grad planes
    const bool spec = s.spec[0] || s.spec[1] || s.spec[2];
    grad_q0_point(n + o, (long)(t - o), s.nx, s.ny, s.nz, s.px, s.py, s.pz, s.hx, s.hy, s.hz, s.skew ? s.einv : nullptr,
                  spec ? s.spec : nullptr, (long)s.G, n_cut,
                  grad ? grad + 3 * o : nullptr, q0 + o, dqdn ? dqdn + o : nullptr, dqdg ? dqdg + o : nullptr);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct Layout {
    size_t hdr, counter, flag, segs, imgs, counts, rowoff, recs, gidx, ipart, jpart, blockE, res, qmin, quad, vox,
        dEdq, fartab, far, total;
    int64_t nblocks, slots, rows, fin_blocks, Gtot;
    int64_t quad_cells;  // FP32 bilinear runs: cells of the global table held as corner quadruples
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Plan {
    std::vector<Seg> segs;
    std::vector<int> imgs;  // 4 ints per image
    int nimg = 1, home = 0;
    int mimg[3] = {0, 0, 0};  // image range per axis (0 on open axes)
    bool img = false;
    bool skew = false;  // some density has a skew cell: the general-metric kernels
    bool spec = false;  // some density takes the Fourier derivative on some axis
    GridDev g0;         // the first density's grid
    std::vector<GridDev> gds;  // every density's grid (spectral line kernels)
    bool far = false;   // far image shell
    std::vector<FarGeo> fgs;        // its shell and geometry per density
    int64_t far_tab = 0, far_part = 0;  // elements of all lattice-sum tables, of all row partials
    int JC = 8192;
    int tpb = kPairThreads;     // pair-kernel workgroup size
    int BI = 2 * kPairThreads;  // i-points per row block (IPL per lane)
    int ND = 1;                 // diagonal items per row block
    int NI = 1, NJ = 1;
    Layout L;
};

// i-points per lane of the pair-kernel variant these options select in
// 1024-thread workgroups: four for the FP32 n_sigma = 64 kernels without
// images, two elsewhere.  (With images, four points per lane was measured
// slower on the slab: the wider i box of a wavefront lets fewer tiles skip
// or run unmasked against the cut, and the per-image set-up spills
// registers.)
int ipl_for(int fp64, int kahan, int nsig, bool img) { return (!fp64 && !kahan && nsig == 64 && !img) ? 4 : 2; }

// Work items of one density's list if every point were kept (an upper
// bound for any density on that grid): per row block ND diagonal items and
// the chunks of the points after it.
int64_t items_bound(int64_t G, int64_t BI, int64_t JC, int64_t ND)
{
    const int64_t nib = (G + BI - 1) / BI;
    int64_t items = 0;
    for (int64_t I = 0; I < nib; ++I) {
        const int64_t rest = G - (I + 1) * BI;
        items += ND + (rest > 0 ? (rest + JC - 1) / JC : 0);
    }
    return items;
}

// Diagonal items per row block: a diagonal item evaluates each ordered pair
// on its own (twice the work per pair of the two-sided off-diagonal rings),
// so BI x BI / ND ordered pairs cost about as much as one BI x JC chunk
// when ND = BI / JC.
int diag_items(int64_t BI, int64_t JC) { return BI > JC ? (int)(BI / JC) : 1; }

// Nodes and weights of the voxel on-site rule: the kVoxelGL-point
// Gauss-Legendre rule mapped to [0, 1], each weight times 2 u (1 - u^2) for
// the substitution t = u^2 and the tent 1 - t.
void voxel_rule(double *u, double *wt)
{
    double x[kVoxelGL], w[kVoxelGL];
    gauss_legendre_nodes(kVoxelGL, x, w);
    for (int j = 0; j < kVoxelGL; ++j) {
        u[j] = 0.5 * (x[j] + 1.0);
        wt[j] = 2.0 * u[j] * (0.5 * w[j]) * (1.0 - u[j] * u[j]);
    }
}

// Compute units of the target (gfx950): the pair kernel runs one persistent
// workgroup per CU, so the work list needs many more items than this to
// keep every CU busy to the end.
constexpr int64_t kCUs = 256;

// The n_sigma the work layout is planned for: the table's, except for the
// cubic-in-D interpolant, whose kernels have two i-points per lane (the
// layout of any n_sigma).
int plan_nsig(const vdw_table_params *tp) { return tp->interp == VDW_INTERP_CUBIC_D ? kCubicD : tp->n_sigma; }

int make_plan(int B, const vdw_grid *grids, const int64_t *grid_off, const vdw_opts *o, int nsig, int nD, int fp64,
              int adj, Plan *P)
{
    P->segs.resize(B);
    P->gds.resize(B);
    P->skew = false;
    P->spec = false;
    int64_t Gtot = 0;
    for (int b = 0; b < B; ++b) {
        GridDev g;
        int rc = validate_grid(&grids[b], &g);
        if (rc) return rc;
        if (b > 0 && (g.px != P->segs[0].px || g.py != P->segs[0].py || g.pz != P->segs[0].pz))
            return fail(VDW_EINVAL, "all densities of a batch must share the periodic flags");
        Seg &s = P->segs[b];
        memset(&s, 0, sizeof(s));
        s.nx = g.nx;
        s.ny = g.ny;
        s.nz = g.nz;
        s.px = g.px;
        s.py = g.py;
        s.pz = g.pz;
        s.hx = g.hx;
        s.hy = g.hy;
        s.hz = g.hz;
        s.dV = g.dV;
        s.skew = g.skew;
        for (int k = 0; k < 9; ++k) s.einv[k] = g.Einv[k];
        for (int k = 0; k < 9; ++k) s.e[k] = g.E[k];
        {
            // metric e_a.e_b / h_x^2 (diagonal on orthorhombic cells)
            double M[3][3];
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c)
                    M[a][c] = (g.E[3 * a] * g.E[3 * c] + g.E[3 * a + 1] * g.E[3 * c + 1] + g.E[3 * a + 2] * g.E[3 * c + 2]) /
                              (g.hx * g.hx);
            s.m01 = 2.0 * M[0][1];
            s.m02 = 2.0 * M[0][2];
            s.m12 = 2.0 * M[1][2];
            for (int k = 0; k < 9; ++k) s.en[k] = g.E[k] / g.hx;
        }
        if (g.skew) P->skew = true;
        for (int a = 0; a < 3; ++a) {
            s.spec[a] = g.spec[a];
            if (g.spec[a]) P->spec = true;
        }
        if (b == 0) P->g0 = g;
        P->gds[b] = g;
        s.G = g.G;
        s.grid_off = grid_off ? grid_off[b] : 0;
        if (grid_off && grid_off[b + 1] - grid_off[b] != g.G)
            return fail(VDW_EINVAL, "grid_off[%d+1] - grid_off[%d] != grid %d size", b, b, b);
        Gtot += g.G;
    }
    if (Gtot > ((int64_t)1 << 31) - 1) return fail(VDW_EINVAL, "total grid size exceeds 2^31 - 1");
    auto bound = [&](int64_t BI, int64_t JC) {
        int64_t n = 0;
        for (int b = 0; b < B; ++b) n += items_bound(P->segs[b].G, BI, JC, diag_items(BI, JC));
        return n;
    };
    {
        // the image loop runs when a periodic axis has images or a cut is set
        int nimg = 1;
        for (int a = 0; a < 3; ++a)
            if (grids[0].periodic[a] && o->image_max[a] > 0) nimg *= 2 * o->image_max[a] + 1;
        const bool img = nimg > 1 || o->r_cut > 0.0;
        const bool fast = !fp64 && !o->kahan && nsig == 64;
        // workgroup shape: 512 threads with eight i-points per lane on request
        // (FP32 n_sigma = 64 kernels without images); 256 threads with two on
        // request or, by default, when even the finest chunking of the
        // 1024-thread list leaves half the CUs idle (no images); else 1024.
        // Skew cells: 1024 threads, two i-points per lane.
        const int64_t BI_big = (int64_t)(P->skew ? 2 : ipl_for(fp64, o->kahan, nsig, img)) * kPairThreads;
        if (P->skew) {
            P->tpb = kPairThreads;
            P->BI = (int)BI_big;
        } else if (fast && !img && o->block_threads == 512) {
            P->tpb = 512;
            P->BI = 8 * 512;
        } else if (!img && (o->block_threads == 256 || (o->block_threads == 0 && bound(BI_big, 1024) < kCUs / 2))) {
            P->tpb = 256;
            P->BI = 2 * 256;
        } else {
            P->tpb = kPairThreads;
            P->BI = (int)BI_big;
        }
        // chunk length: as requested, or the longest of 8192 ... 1024 points
        // that still gives 16 items per CU when every point is kept (the
        // last items to finish then leave little of the launch idle)
        if (o->j_chunks > 0) {
            P->JC = 1024 * o->j_chunks;
        } else {
            P->JC = 8192;
            while (P->JC > 1024 && bound(P->BI, P->JC) < 16 * kCUs) P->JC /= 2;
        }
    }
    P->ND = diag_items(P->BI, P->JC);
    const int64_t BI = P->BI, JC = P->JC;
    int64_t t_off = 0, slots = 0, rows = 0, fin = 0;
    for (int b = 0; b < B; ++b) {
        Seg &s = P->segs[b];
        s.nbx = (s.nx + 3) / 4;
        s.nby = (s.ny + 3) / 4;
        s.nbz = (s.nz + 3) / 4;
        int64_t T = (int64_t)s.nbx * s.nby * s.nbz * 64;
        s.T = (T + kCompactBlock - 1) / kCompactBlock * kCompactBlock;
        s.t_off = t_off;
        t_off += s.T;
        const int64_t nib = (s.G + BI - 1) / BI;
        s.row_base = rows;
        rows += nib + 1;
        s.slot_base = slots;
        slots += items_bound(s.G, BI, JC, P->ND);
        fin += (s.G + kFinThreads - 1) / kFinThreads;
    }
    // images on periodic axes
    int m[3];
    for (int a = 0; a < 3; ++a) {
        int per = a == 0 ? P->segs[0].px : a == 1 ? P->segs[0].py : P->segs[0].pz;
        if (o->image_max[a] < 0) return fail(VDW_EINVAL, "image_max must be >= 0");
        m[a] = per ? o->image_max[a] : 0;
        P->mimg[a] = m[a];
    }
    P->imgs.clear();
    P->nimg = 0;
    for (int x = -m[0]; x <= m[0]; ++x)
        for (int y = -m[1]; y <= m[1]; ++y)
            for (int z = -m[2]; z <= m[2]; ++z) {
                if (x == 0 && y == 0 && z == 0) P->home = P->nimg;
                P->imgs.push_back(x);
                P->imgs.push_back(y);
                P->imgs.push_back(z);
                P->imgs.push_back(0);
                ++P->nimg;
            }
    if (P->nimg > 4096) return fail(VDW_EINVAL, "too many images (%d)", P->nimg);
    P->img = P->nimg > 1 || o->r_cut > 0.0;
    // far image shell: the lattice vectors up to far_max on periodic axes
    // that are not near images
    P->far = false;
    {
        const int per[3] = {P->segs[0].px, P->segs[0].py, P->segs[0].pz};
        double vecs = 1.0;
        for (int a = 0; a < 3; ++a) {
            if (o->far_max[a] < 0) return fail(VDW_EINVAL, "far_max must be >= 0");
            if (per[a] && o->far_max[a] > 0) P->far = true;
            if (per[a]) vecs *= 2.0 * o->far_max[a] + 1.0;
        }
        P->fgs.clear();
        P->far_tab = P->far_part = 0;
        if (P->far) {
            if (o->r_cut > 0.0) return fail(VDW_EINVAL, "the far image shell is defined without a distance cut");
            for (int a = 0; a < 3; ++a)
                if (per[a] && o->far_max[a] < m[a])
                    return fail(VDW_EINVAL, "far_max[%d] = %d is below image_max[%d] = %d", a, o->far_max[a], a, m[a]);
            if (vecs > 4194304.0) return fail(VDW_EINVAL, "far shell of %.0f lattice vectors (at most 2^22)", vecs);
            P->fgs.resize(B);
            for (int b = 0; b < B; ++b) {
                Seg &sb = P->segs[b];
                FarGeo &f = P->fgs[b];
                f.nx = sb.nx;
                f.ny = sb.ny;
                f.nz = sb.nz;
                for (int a = 0; a < 3; ++a) {
                    f.lo[a] = per[a] ? m[a] : 0;
                    f.hi[a] = per[a] ? o->far_max[a] : 0;
                }
                for (int k = 0; k < 9; ++k) f.en[k] = sb.e[k] / sb.hx;
                const int64_t ne = far_table_entries(f);
                if (ne >= ((int64_t)1 << 31))
                    return fail(VDW_EINVAL, "grid %d too large for the far-shell table (2^31 displacements)", b);
                sb.far_chunks = far_chunks(sb.G);
                sb.far_tab_off = P->far_tab;
                sb.far_part_off = P->far_part;
                P->far_tab += ne;
                P->far_part += 2 * (int64_t)sb.far_chunks * sb.G;
            }
        }
    }
    P->NI = P->NJ = 1 + (P->img ? 1 : 0) + (adj ? 1 : 0);

    Layout &L = P->L;
    L.nblocks = t_off / kCompactBlock;
    L.slots = slots;
    L.rows = rows;
    L.fin_blocks = fin;
    L.Gtot = Gtot;
    size_t off = 0;
    L.hdr = off;
    off = align256(off + HDR_WORDS * sizeof(int64_t));
    L.counter = off;
    off = align256(off + sizeof(int64_t));
    L.flag = off;
    off = align256(off + sizeof(int64_t));
    L.segs = off;
    off = align256(off + B * sizeof(Seg));
    L.imgs = off;
    off = align256(off + P->imgs.size() * sizeof(int));
    L.counts = off;
    off = align256(off + (L.nblocks + 1) * sizeof(int64_t));
    L.rowoff = off;
    off = align256(off + rows * sizeof(int64_t));
    L.recs = off;
    off = align256(off + Gtot * (fp64 ? sizeof(RecD) : sizeof(RecF)));
    L.gidx = off;
    off = align256(off + Gtot * sizeof(int32_t));
    L.ipart = off;
    off = align256(off + (size_t)P->NI * slots * BI * sizeof(double));
    L.jpart = off;
    off = align256(off + (size_t)P->NJ * slots * JC * sizeof(double));
    L.blockE = off;
    off = align256(off + 3 * fin * sizeof(double));
    L.res = off;
    off = align256(off + (4 * B + 1) * sizeof(double));
    L.qmin = off;
    off = align256(off + B * sizeof(uint64_t));
    L.quad = off;
    L.quad_cells = (!fp64 && nsig > 0) ? (int64_t)(nD - 1) * (nsig - 1) : 0;
    off = align256(off + (size_t)L.quad_cells * sizeof(float4));
    L.vox = off;
    if (o->self_term == 2) off = align256(off + (size_t)B * kVoxNodes * sizeof(double));
    L.dEdq = off;
    if (adj) off = align256(off + Gtot * sizeof(double));
    L.fartab = off;
    if (P->far) off = align256(off + (size_t)P->far_tab * sizeof(double));
    L.far = off;
    if (P->far) off = align256(off + (size_t)P->far_part * sizeof(double));
    L.total = off;
    return VDW_OK;
}

int validate_opts(const vdw_opts *o)
{
    if (!o) return fail(VDW_EINVAL, "opts is NULL");
    if (!(o->n_cut > 0.0) || !isfinite(o->n_cut)) return fail(VDW_EINVAL, "n_cut must be > 0");
    if (o->precision != VDW_FP64 && o->precision != VDW_FP32C) return fail(VDW_EINVAL, "precision must be 0 or 1");
    if (o->self_term < 0 || o->self_term > 2) return fail(VDW_EINVAL, "self_term must be 0, 1 or 2");
    if (o->block_threads != 0 && o->block_threads != 1024 && o->block_threads != 512 && o->block_threads != 256)
        return fail(VDW_EINVAL, "block_threads must be 0, 256, 512 or 1024");
    if (o->j_chunks < 0 || o->j_chunks > 64) return fail(VDW_EINVAL, "j_chunks must be in 0..64");
    if (o->grid_blocks < 0) return fail(VDW_EINVAL, "grid_blocks must be >= 0");
    if (o->kahan != 0 && o->kahan != 1) return fail(VDW_EINVAL, "kahan must be 0 or 1");
    if (!isfinite(o->r_cut)) return fail(VDW_EINVAL, "r_cut must be finite");
    return VDW_OK;
}

struct PairPtrs {
    const float4 *quad;
    const void *recs;
    const Seg *segs;
    const int64_t *hdr;
    int *counter;
    const void *tabg;
    const int *imgs;
    const int64_t *rowoff;
    double *ipart;
    void *jpart;
};

template <typename R, bool ADJ, bool IMG, bool KAHAN, int NSIG, int GEO, int IPL, int TPB>
int launch_pair_t(const PairArgs &a, const PairPtrs &p, int grid, size_t lds, hipStream_t s, bool attr_only)
{
    // the work layout was made for this row-block length
    if (a.BI != IPL * TPB)
        return fail(VDW_EINVAL, "internal: row blocks of %d points planned for a kernel with %d", a.BI, IPL * TPB);
    // the kernel's LDS is static (kLdsBytes); nothing else to set up
    if (attr_only) return VDW_OK;
    hipLaunchKernelGGL((pair_kernel<R, ADJ, IMG, KAHAN, NSIG, GEO, IPL, TPB>), dim3(grid), dim3(TPB), lds, s, a,
                       (const typename RecOf<R>::T *)p.recs, p.segs, p.hdr, p.counter, (const R *)p.tabg, p.imgs,
                       p.rowoff, p.ipart, (double *)p.jpart, p.quad);
    VDW_HIP(hipGetLastError());
    return VDW_OK;
}

// Instantiated variants: FP32C with n_sigma = 64 on cubic or general
// orthorhombic grids (the fast paths: without images four i-points per lane
// in 1024-thread workgroups, or eight in 512-thread ones), FP32C for any
// n_sigma, Kahan-compensated FP32C (n_sigma = 64 on cubic and square grids,
// any n_sigma elsewhere), and plain FP64 (cubic or orthorhombic; two per lane,
// 1024 threads); each with and without the adjoint sums and the image loop.
// Without images every one of them also has 256-thread workgroups with two
// i-points per lane, for work lists too short to occupy every CU.  Skew
// cells (FP64, FP32C with n_sigma = 64 or any, Kahan-compensated FP32C) have
// two i-points per lane in 1024-thread workgroups, with and without the
// adjoint and the image loop.
template <typename R, bool KAHAN, int NSIG, int GEO>
int launch_pair_v(int adj, int img, int tpb, const PairArgs &a, const PairPtrs &p, int grid, size_t lds,
                  hipStream_t s, bool attr_only)
{
    if constexpr (GEO == kSkew) {
        if (img) return adj ? launch_pair_t<R, true, true, KAHAN, NSIG, GEO, 2, 1024>(a, p, grid, lds, s, attr_only)
                            : launch_pair_t<R, false, true, KAHAN, NSIG, GEO, 2, 1024>(a, p, grid, lds, s, attr_only);
        return adj ? launch_pair_t<R, true, false, KAHAN, NSIG, GEO, 2, 1024>(a, p, grid, lds, s, attr_only)
                   : launch_pair_t<R, false, false, KAHAN, NSIG, GEO, 2, 1024>(a, p, grid, lds, s, attr_only);
    } else {
        constexpr bool FAST = sizeof(R) == 4 && !KAHAN && NSIG == 64;
        if (!img && tpb == 256)
            return adj ? launch_pair_t<R, true, false, KAHAN, NSIG, GEO, 2, 256>(a, p, grid, lds, s, attr_only)
                       : launch_pair_t<R, false, false, KAHAN, NSIG, GEO, 2, 256>(a, p, grid, lds, s, attr_only);
        if (img) return adj ? launch_pair_t<R, true, true, KAHAN, NSIG, GEO, 2, 1024>(a, p, grid, lds, s, attr_only)
                            : launch_pair_t<R, false, true, KAHAN, NSIG, GEO, 2, 1024>(a, p, grid, lds, s, attr_only);
        if constexpr (FAST) {
            if (tpb == 512)
                return adj ? launch_pair_t<R, true, false, KAHAN, NSIG, GEO, 8, 512>(a, p, grid, lds, s, attr_only)
                           : launch_pair_t<R, false, false, KAHAN, NSIG, GEO, 8, 512>(a, p, grid, lds, s, attr_only);
        }
        constexpr int W = FAST ? 4 : 2;
        return adj ? launch_pair_t<R, true, false, KAHAN, NSIG, GEO, W, 1024>(a, p, grid, lds, s, attr_only)
                   : launch_pair_t<R, false, false, KAHAN, NSIG, GEO, W, 1024>(a, p, grid, lds, s, attr_only);
    }
}

int launch_pair(int fp64, int adj, int img, int kahan, int nsig, int geo, int tpb, const PairArgs &a,
                const PairPtrs &p, int grid, size_t lds, hipStream_t s, bool attr_only)
{
    const bool cubd = a.interp == VDW_INTERP_CUBIC_D;
    if (cubd && kahan) return fail(VDW_EUNSUPPORTED, "the cubic-in-D interpolant is not offered with Kahan runs");
    if (cubd && !fp64)
        return geo == kSkew ? launch_pair_v<float, false, kCubicD, kSkew>(adj, img, tpb, a, p, grid, lds, s, attr_only)
                            : launch_pair_v<float, false, kCubicD, kOrtho>(adj, img, tpb, a, p, grid, lds, s, attr_only);
    if (geo == kSkew) {
        if (kahan) return launch_pair_v<float, true, 0, kSkew>(adj, img, tpb, a, p, grid, lds, s, attr_only);
        if (fp64)
            return cubd ? launch_pair_v<double, false, kCubicD, kSkew>(adj, img, tpb, a, p, grid, lds, s, attr_only)
                        : launch_pair_v<double, false, 0, kSkew>(adj, img, tpb, a, p, grid, lds, s, attr_only);
        if (nsig == 64) return launch_pair_v<float, false, 64, kSkew>(adj, img, tpb, a, p, grid, lds, s, attr_only);
        return launch_pair_v<float, false, 0, kSkew>(adj, img, tpb, a, p, grid, lds, s, attr_only);
    }
    if (fp64) {
        if (cubd) return launch_pair_v<double, false, kCubicD, kOrtho>(adj, img, tpb, a, p, grid, lds, s, attr_only);
        return geo == kCubic ? launch_pair_v<double, false, 0, kCubic>(adj, img, tpb, a, p, grid, lds, s, attr_only)
                             : launch_pair_v<double, false, 0, kOrtho>(adj, img, tpb, a, p, grid, lds, s, attr_only);
    }
    if (kahan) {
        if (nsig == 64 && geo == kCubic)
            return launch_pair_v<float, true, 64, kCubic>(adj, img, tpb, a, p, grid, lds, s, attr_only);
        if (nsig == 64 && geo == kSquare)
            return launch_pair_v<float, true, 64, kSquare>(adj, img, tpb, a, p, grid, lds, s, attr_only);
        return launch_pair_v<float, true, 0, kOrtho>(adj, img, tpb, a, p, grid, lds, s, attr_only);
    }
    if (nsig == 64)
        return geo == kCubic    ? launch_pair_v<float, false, 64, kCubic>(adj, img, tpb, a, p, grid, lds, s, attr_only)
               : geo == kSquare ? launch_pair_v<float, false, 64, kSquare>(adj, img, tpb, a, p, grid, lds, s, attr_only)
                                : launch_pair_v<float, false, 64, kOrtho>(adj, img, tpb, a, p, grid, lds, s, attr_only);
    return launch_pair_v<float, false, 0, kOrtho>(adj, img, tpb, a, p, grid, lds, s, attr_only);
}

// Everything an evaluation needs that does not depend on the data: the
// work layout, the launch shapes and the constant kernel arguments.
struct Exec {
    Plan P;
    int B = 0, adj = 0, fp64 = 0, kahan = 0, nsig = 0, geo = kCubic, self_term = 0, interp = 0;
    int tpb = 1024;  // pair-kernel workgroup size
    int K = 0, grid = 0;
    size_t lds = 0;
    double n_cut = 0.0, dD = 0.0, Dmax = 0.0, casym = 0.0;
    int nD = 0;
    double reach = 0.0;  // near image window: every pair closer than this is summed (smallest over the densities)
    int covered = -1;    // image_cut_covered of the window (the smallest over the densities)
    PairArgs pa;
    char *ws = nullptr;
};

constexpr double kCasym = 12.0 * (4.0 * 3.14159265358979323846 / 9.0) * (4.0 * 3.14159265358979323846 / 9.0) *
                          (4.0 * 3.14159265358979323846 / 9.0);

// Validation, layout and launch shapes (host only, no device work).
int prepare(int B, const vdw_grid *grids, const int64_t *grid_off, const vdw_table_params *tp, const vdw_opts *o,
            int adj, void *ws, size_t ws_bytes, Exec *E)
{
    int rc = validate_opts(o);
    if (rc) return rc;
    rc = validate_table(tp);
    if (rc) return rc;
    if (tp->interp == VDW_INTERP_CUBIC_D && o->kahan)
        return fail(VDW_EUNSUPPORTED, "the cubic-in-D interpolant is not offered with Kahan runs");
    if (B < 1) return fail(VDW_EINVAL, "B must be >= 1");
    if (!grids) return fail(VDW_EINVAL, "NULL argument");
    if (!ws) return fail(VDW_EINVAL, "workspace is NULL");
    DevInfo dev;
    rc = device_info(&dev);
    if (rc) return rc;
    E->B = B;
    E->adj = adj;
    E->fp64 = o->precision == VDW_FP64;
    E->kahan = o->kahan;
    E->nsig = tp->n_sigma;
    E->self_term = o->self_term;
    E->interp = tp->interp;
    E->n_cut = o->n_cut;
    rc = make_plan(B, grids, grid_off, o, plan_nsig(tp), tp->n_D, E->fp64, adj, &E->P);
    if (rc) return rc;
    const Plan &P = E->P;
    if (ws_bytes < P.L.total) return fail(VDW_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, P.L.total);
    E->reach = INFINITY;
    E->covered = 1;
    for (int b = 0; b < B; ++b) {
        const double r = image_reach(&grids[b], o->image_max);
        E->reach = fmin(E->reach, r);
        E->covered = min(E->covered, image_cut_covered(&grids[b], o, r));
    }
    E->ws = (char *)ws;
    const int S = tp->n_sigma + 1;
    if (dev.lds_per_block < (size_t)kLdsBytes)
        return fail(VDW_EUNSUPPORTED, "the pair kernel needs %d bytes of LDS per workgroup (device: %zu)", kLdsBytes,
                    dev.lds_per_block);
    // table rows that fit in the kernel's static LDS next to its reduction buffer
    E->tpb = P.tpb;
    const int cap = E->fp64 ? tab_elems<double>(E->tpb / 64) : tab_elems<float>(E->tpb / 64);
    int K = cap / S;
    if (o->table_lds_rows >= 0 && o->table_lds_rows < K) K = o->table_lds_rows;
    if (K > tp->n_D) K = tp->n_D;
    if (K < 2) K = 2;  // the kernel reads a clamped LDS row unconditionally
    if (K * S > cap) return fail(VDW_EINVAL, "n_sigma = %d is too large for the LDS table (at most %d)", tp->n_sigma,
                                 cap / 2 - 1);
    E->K = K;
    E->lds = 0;
    E->grid = o->grid_blocks > 0 ? o->grid_blocks : dev.cus;
    E->dD = tp->D_max / (tp->n_D - 1);
    E->Dmax = tp->D_max;
    E->nD = tp->n_D;
    E->casym = kCasym;
    PairArgs &pa = E->pa;
    pa.B = B;
    pa.nD = tp->n_D;
    pa.nS = tp->n_sigma;
    pa.S = S;
    pa.K = K;
    pa.JC = P.JC;
    pa.BI = P.BI;
    pa.ND = P.ND;
    pa.interp = tp->interp;
    pa.DS = P.BI / P.ND;
    pa.csig = sqrt((double)(tp->n_sigma - 1));
    pa.tDmax = (double)(tp->n_D - 1);
    pa.tSclamp = E->fp64 ? nextafter((double)(tp->n_sigma - 1), 0.0)
                         : (double)nextafterf((float)(tp->n_sigma - 1), 0.0f);
    pa.casym = kCasym / pow(2.0 * E->dD, 6);  // the asymptote in units of h_x and a = q h_x / (2 dD)
    pa.dD2 = 2.0 * E->dD;
    pa.rc2 = o->r_cut > 0.0 ? o->r_cut * o->r_cut : INFINITY;
    pa.nimg = P.nimg;
    pa.home = P.home;
    pa.NI = P.NI;
    pa.NJ = P.NJ;
    pa.istride = P.L.slots * P.BI;
    pa.jstride = P.L.slots * (int64_t)P.JC;
    // cubic grids take the exact integer form of the squared distance: its
    // partial sums stay below 12 c^2 for coordinates |c| <= c_max (image
    // shifts included), exact in FP32 while 12 c_max^2 < 2^24; skew cells
    // take the general metric
    E->geo = kCubic;
    bool square = true;
    double cmax = 0.0, cxy = 0.0;
    for (int b = 0; b < B; ++b) {
        const Seg &g = P.segs[b];
        if (!(g.hx == g.hy && g.hx == g.hz)) E->geo = kOrtho;
        if (!(g.hx == g.hy)) square = false;
        const int n3[3] = {g.nx, g.ny, g.nz};
        for (int a = 0; a < 3; ++a) cmax = fmax(cmax, (double)n3[a] * (1 + P.mimg[a]));
        for (int a = 0; a < 2; ++a) cxy = fmax(cxy, (double)n3[a] * (1 + P.mimg[a]));
    }
    // (and the ring takes -2x of the i-points and x of the j records as f16,
    // exact while |2x| <= 2048)
    if (12.0 * cmax * cmax >= 16777216.0 || cmax > 1024.0) E->geo = kOrtho;
    // square grids (h_x = h_y): the x, y part exactly in the same way, its
    // partial sums below 8 c^2 (FP32 n_sigma = 64 kernels)
    if (E->geo == kOrtho && square && !E->fp64 && E->nsig == 64 && 8.0 * cxy * cxy < 16777216.0 && cxy <= 1024.0)
        E->geo = kSquare;
    if (P.skew) E->geo = kSkew;
    PairPtrs none{};
    return launch_pair(E->fp64, adj, P.img ? 1 : 0, E->kahan, E->nsig, E->geo, E->tpb, pa, none, E->grid, E->lds, nullptr,
                       true);
}

// Copies the density descriptors and the image list into the workspace.
int upload(const Exec &E, hipStream_t s)
{
    const Layout &L = E.P.L;
    VDW_HIP(hipMemcpyAsync(E.ws + L.segs, E.P.segs.data(), E.B * sizeof(Seg), hipMemcpyHostToDevice, s));
    VDW_HIP(hipMemcpyAsync(E.ws + L.imgs, E.P.imgs.data(), E.P.imgs.size() * sizeof(int), hipMemcpyHostToDevice, s));
    return VDW_OK;
}

// The evaluation proper: kernel launches only (no copies, no host waits, no
// allocation), so that it can be recorded into a HIP graph.  `res` receives
// 4B+1 doubles: 3B energies, B retained counts, the non-finite flag.
int enqueue(const Exec &E, const double *n_d, const double *q0_d, const double *grad_d, const double *dqdn_d,
            const double *dqdg_d, const double *phi_d, const float *phi_f, double *dEdn_d, double *res, hipStream_t s,
            hipEvent_t ev0, hipEvent_t ev1, hipEvent_t evf0 = nullptr, hipEvent_t evf1 = nullptr)
{
    const Plan &P = E.P;
    const Layout &L = P.L;
    const int B = E.B;
    char *w = E.ws;
    int64_t *hdr = (int64_t *)(w + L.hdr);
    int *counter = (int *)(w + L.counter);
    int *flag = (int *)(w + L.flag);
    Seg *segs = (Seg *)(w + L.segs);
    int *imgs = (int *)(w + L.imgs);
    int64_t *counts = (int64_t *)(w + L.counts);
    void *recs = w + L.recs;
    int32_t *gidx = (int32_t *)(w + L.gidx);
    int64_t *rowoff = (int64_t *)(w + L.rowoff);
    double *ipart = (double *)(w + L.ipart);
    void *jpart = w + L.jpart;
    double *blockE = (double *)(w + L.blockE);
    double *dEdq = (double *)(w + L.dEdq);
    unsigned long long *qmin = (unsigned long long *)(w + L.qmin);

    // counter and flag live in 64-bit words right after the header
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, hdr, HDR_WORDS);
    hipLaunchKernelGGL(max_words_kernel, dim3((B + 255) / 256), dim3(256), 0, s, qmin, B);
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, (int64_t *)counter, 1);
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, (int64_t *)flag, 1);
    VDW_HIP(hipGetLastError());
    if (E.adj) {
        unsigned gb = (unsigned)((L.Gtot + 255) / 256);
        hipLaunchKernelGGL(fill_kernel, dim3(gb), dim3(256), 0, s, dEdn_d, L.Gtot);
        hipLaunchKernelGGL(fill_kernel, dim3(gb), dim3(256), 0, s, dEdq, L.Gtot);
        VDW_HIP(hipGetLastError());
    }
    // compaction
    hipLaunchKernelGGL(count_kernel, dim3((unsigned)L.nblocks), dim3(kCompactThreads), 0, s, (const Seg *)segs, B,
                       n_d, E.n_cut, counts, flag);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, counts, L.nblocks, segs, B, hdr, rowoff,
                       (int64_t)P.JC, (int64_t)P.BI, (int64_t)P.ND);
    ScatterArgs sa;
    sa.segs = segs;
    sa.B = B;
    sa.n = n_d;
    sa.q0 = q0_d;
    sa.n_cut = E.n_cut;
    sa.offs = counts;
    sa.recs = recs;
    sa.gidx = gidx;
    sa.inv2dD = 1.0 / (2.0 * E.dD);
    sa.csig = E.pa.csig;
    sa.fp64 = E.fp64;
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)L.nblocks), dim3(kCompactThreads), 0, s, sa);
    VDW_HIP(hipGetLastError());
    double *far = (double *)(w + L.far);
    if (P.far) {
        // far image shell, per density: lattice sums, then its rows (the
        // kept count and the first record come from the device descriptors)
        double *T = (double *)(w + L.fartab);
        if (evf0) VDW_HIP(hipEventRecord(evf0, s));
        for (int b = 0; b < B; ++b) {
            const Seg &sb = P.segs[b];
            int rc = launch_far_table(P.fgs[b], T + sb.far_tab_off, s);
            if (rc) return rc;
            rc = launch_far_rows(P.fgs[b], E.fp64, recs, &segs[b].N, &segs[b].p_off, sb.G, T + sb.far_tab_off,
                                 E.pa.casym, sb.hx / E.pa.dD2, sb.far_chunks, E.adj, far + sb.far_part_off, s);
            if (rc) return rc;
        }
        if (evf1) VDW_HIP(hipEventRecord(evf1, s));
    }

    // pair kernel
    PairPtrs pp;
    pp.quad = nullptr;
    if (L.quad_cells > 0) {
        float4 *quad = (float4 *)(w + L.quad);
        hipLaunchKernelGGL(quad_kernel, dim3((unsigned)((L.quad_cells + 255) / 256)), dim3(256), 0, s, phi_f, quad,
                           E.nD, E.nsig);
        VDW_HIP(hipGetLastError());
        pp.quad = quad;
    }
    pp.recs = recs;
    pp.segs = segs;
    pp.hdr = hdr;
    pp.counter = counter;
    pp.tabg = E.fp64 ? (const void *)phi_d : (const void *)phi_f;
    pp.imgs = imgs;
    pp.rowoff = rowoff;
    pp.ipart = ipart;
    pp.jpart = jpart;
    if (ev0) VDW_HIP(hipEventRecord(ev0, s));
    int rc = launch_pair(E.fp64, E.adj, P.img ? 1 : 0, E.kahan, E.nsig, E.geo, E.tpb, E.pa, pp, E.grid, E.lds, s,
                         false);
    if (rc) return rc;
    if (ev1) VDW_HIP(hipEventRecord(ev1, s));

    // finalize and reduce
    FinArgs fa;
    fa.segs = segs;
    fa.B = B;
    fa.hdr = hdr;
    fa.rowoff = rowoff;
    fa.ipart = ipart;
    fa.jpart = (const double *)jpart;
    fa.istride = E.pa.istride;
    fa.jstride = E.pa.jstride;
    fa.JC = P.JC;
    fa.BI = P.BI;
    fa.ND = P.ND;
    fa.NI = P.NI;
    fa.NJ = P.NJ;
    fa.img = P.img ? 1 : 0;
    fa.adj = E.adj;
    fa.self_term = E.self_term;
    fa.vg = kVoxelGL;
    fa.interp = E.interp;
    voxel_rule(fa.vu, fa.vw);
    fa.gidx = gidx;
    fa.n = n_d;
    fa.q0 = q0_d;
    fa.dqdn = dqdn_d;
    fa.tab = phi_d;
    fa.nD = E.nD;
    fa.nS = E.nsig;
    fa.dD = E.dD;
    fa.Dmax = E.Dmax;
    fa.casym = E.casym;
    fa.far = P.far ? far : nullptr;
    fa.blockE = blockE;
    fa.qmin = qmin;
    fa.dEdn = dEdn_d;
    fa.dEdq = dEdq;
    fa.vox = (const double *)(w + L.vox);
    if (E.self_term == 2) {
        hipLaunchKernelGGL(voxel_table_kernel, dim3((kVoxNodes + 255) / 256, B), dim3(256), 0, s, fa,
                           (double *)(w + L.vox));
        VDW_HIP(hipGetLastError());
    }
    if (L.fin_blocks > 0)
        hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)L.fin_blocks), dim3(kFinThreads), 0, s, fa);
    hipLaunchKernelGGL(seg_reduce_kernel, dim3(B), dim3(256), 0, s, (const Seg *)segs, (const double *)blockE, res, B,
                       (const int *)flag);
    VDW_HIP(hipGetLastError());
    if (E.adj) {
        AsmArgs aa;
        aa.segs = segs;
        aa.B = B;
        aa.Gtot = L.Gtot;
        aa.dEdq = dEdq;
        aa.dqdg = dqdg_d;
        aa.grad = grad_d;
        aa.dEdn = dEdn_d;
        hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)((L.Gtot + 255) / 256)), dim3(256), 0, s, aa);
        VDW_HIP(hipGetLastError());
        if (P.spec)  // the transposed Fourier derivative, per density and axis
            for (int b = 0; b < B; ++b) {
                const int64_t o = P.segs[b].grid_off;
                for (int a = 0; a < 3; ++a)
                    if (P.gds[b].spec[a]) {
                        int rc = launch_spectral_adjoint(P.gds[b], a, dEdq + o, dqdg_d + o, grad_d + 3 * o,
                                                         dEdn_d + o, s);
                        if (rc) return rc;
                    }
            }
    }
    return VDW_OK;
}

thread_local vdw_stats g_stats;
thread_local int g_timing = 0;

void set_stats(const Exec &E, const double *host, const uint64_t *qmin, float ms, float far_ms)
{
    double pairs = 0.0;
    int64_t retained = 0;
    for (int b = 0; b < E.B; ++b) {
        double Nb = host[3 * E.B + b];
        retained += (int64_t)Nb;
        pairs += Nb * Nb * E.P.nimg - Nb;
    }
    g_stats.retained = retained;
    g_stats.pairs = pairs;
    g_stats.pair_kernel_ms = ms;
    g_stats.lds_rows = E.K;
    g_stats.block_threads = E.tpb;
    g_stats.j_chunks = E.P.JC / 1024;
    g_stats.grid_blocks = E.grid;
    g_stats.diag_items = E.P.ND;
    double far_pairs = 0.0;
    if (E.P.far)
        for (int b = 0; b < E.B; ++b) far_pairs += host[3 * E.B + b] * host[3 * E.B + b];
    g_stats.far_pairs = far_pairs;
    g_stats.far_kernel_ms = far_ms;
    double q0_min = INFINITY;
    for (int b = 0; b < E.B; ++b)
        if (host[3 * E.B + b] > 0.0) q0_min = fmin(q0_min, __builtin_bit_cast(double, qmin[b]));
    g_stats.image_reach = E.reach;
    g_stats.image_cut_covered = E.covered;
    g_stats.q0_min = retained > 0 ? q0_min : 0.0;
    // far-shell pairs are at least the window's reach apart, and D >= min(q) r
    g_stats.far_D_min = (E.P.far && retained > 0) ? q0_min * E.reach : 0.0;
}

// The whole pipeline for B densities, energies read back to the host.
int run(int B, const vdw_grid *grids, const int64_t *grid_off, const double *n_d, const double *q0_d,
        const double *grad_d, const double *dqdn_d, const double *dqdg_d, const double *phi_d, const float *phi_f,
        const vdw_table_params *tp, const vdw_opts *o, void *ws, size_t ws_bytes, double *dEdn_d, double *E_out,
        hipStream_t s)
{
    const int adj = dEdn_d != nullptr;
    if (!n_d || !q0_d || !phi_d || !E_out) return fail(VDW_EINVAL, "NULL argument");
    if (o && o->precision == VDW_FP32C && !phi_f) return fail(VDW_EINVAL, "phi_f is required for VDW_FP32C");
    if (adj && (!grad_d || !dqdn_d || !dqdg_d)) return fail(VDW_EINVAL, "grad_d, dq_dn_d and dq_dg_d are required");
    Exec E;
    int rc = prepare(B, grids, grid_off, tp, o, adj, ws, ws_bytes, &E);
    if (rc) return rc;
    rc = upload(E, s);
    if (rc) return rc;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, evf0 = nullptr, evf1 = nullptr;
    if (g_timing) {
        VDW_HIP(hipEventCreate(&ev0));
        VDW_HIP(hipEventCreate(&ev1));
        if (E.P.far) {
            VDW_HIP(hipEventCreate(&evf0));
            VDW_HIP(hipEventCreate(&evf1));
        }
    }
    double *res = (double *)(E.ws + E.P.L.res);
    rc = enqueue(E, n_d, q0_d, grad_d, dqdn_d, dqdg_d, phi_d, phi_f, dEdn_d, res, s, ev0, ev1, evf0, evf1);
    std::vector<double> host(4 * B + 1);
    std::vector<uint64_t> qmin(B);
    if (!rc) {
        hipError_t e = hipMemcpyAsync(host.data(), res, host.size() * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(qmin.data(), E.ws + E.P.L.qmin, B * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = fail(VDW_EHIP, "reading the energies back: %s", hipGetErrorString(e));
    }
    float ms = 0.0f, far_ms = 0.0f;
    if (ev0) {
        if (!rc && hipEventElapsedTime(&ms, ev0, ev1) != hipSuccess) ms = 0.0f;
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }
    if (evf0) {
        if (!rc && hipEventElapsedTime(&far_ms, evf0, evf1) != hipSuccess) far_ms = 0.0f;
        (void)hipEventDestroy(evf0);
        (void)hipEventDestroy(evf1);
    }
    if (rc) return rc;
    if (host[4 * B] != 0.0) return fail(VDW_ENONFINITE, "the density holds NaN or Inf values");
    for (int k = 0; k < 3 * B; ++k) E_out[k] = host[k];
    set_stats(E, host.data(), qmin.data(), ms, far_ms);
    return VDW_OK;
}

// ---------------------------------------------------------------------------
// the entry point without allocation: its workspace is `scratch`, a static
// device array of every GPU the library runs on
// ---------------------------------------------------------------------------

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB (grids up to about 40^3 points)
constexpr int kMaxDevices = 64;

// In host code `scratch` names a host-side stand-in: kernels and copies take
// the device address that scratch_ptr() looks up per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device (set on first use)

int scratch_ptr(void **out)
{
    int dev = 0;
    VDW_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(VDW_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(VDW_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return VDW_OK;
}

// enl_potential on the static scratch.  The host-side plan is kept per
// thread, so repeated calls reuse its storage; no timing events.
int run_noalloc(const vdw_grid *grid, const double *n_d, const double *q0_d, const double *grad_d,
                const double *dqdn_d, const double *dqdg_d, const double *phi_d, const float *phi_f,
                const vdw_table_params *tp, const vdw_opts *o, double *dEdn_d, double *E_out, hipStream_t s)
{
    if (!n_d || !q0_d || !phi_d || !E_out || !dEdn_d) return fail(VDW_EINVAL, "NULL argument");
    if (o && o->precision == VDW_FP32C && !phi_f) return fail(VDW_EINVAL, "phi_f is required for VDW_FP32C");
    if (!grad_d || !dqdn_d || !dqdg_d) return fail(VDW_EINVAL, "grad_d, dq_dn_d and dq_dg_d are required");
    void *ws = nullptr;
    int rc = scratch_ptr(&ws);
    if (rc) return rc;
    static thread_local Exec E;
    rc = prepare(1, grid, nullptr, tp, o, 1, ws, kScratchBytes, &E);
    if (rc == VDW_EWORKSPACE)
        return fail(VDW_EWORKSPACE,
                    "enl_potential_noalloc: this grid and these options need %zu bytes of scratch; the library's "
                    "static scratch holds %zu (use enl_potential with a workspace)",
                    E.P.L.total, kScratchBytes);
    if (rc) return rc;
    rc = upload(E, s);
    if (rc) return rc;
    double *res = (double *)(E.ws + E.P.L.res);
    rc = enqueue(E, n_d, q0_d, grad_d, dqdn_d, dqdg_d, phi_d, phi_f, dEdn_d, res, s, nullptr, nullptr);
    if (rc) return rc;
    double host[5];
    uint64_t qmin[1];
    VDW_HIP(hipMemcpyAsync(host, res, sizeof(host), hipMemcpyDeviceToHost, s));
    VDW_HIP(hipMemcpyAsync(qmin, E.ws + E.P.L.qmin, sizeof(qmin), hipMemcpyDeviceToHost, s));
    VDW_HIP(hipStreamSynchronize(s));
    if (host[4] != 0.0) return fail(VDW_ENONFINITE, "the density holds NaN or Inf values");
    for (int k = 0; k < 3; ++k) E_out[k] = host[k];
    set_stats(E, host, qmin, 0.0f, 0.0f);
    return VDW_OK;
}

}  // namespace

}  // namespace vdw

using namespace vdw;

extern "C" size_t enl_workspace_size(const vdw_grid *grid, const vdw_table_params *tp, const vdw_opts *opts)
{
    return enl_batched_workspace_size(1, grid, tp, opts);
}

extern "C" size_t enl_batched_workspace_size(int32_t B, const vdw_grid *grids, const vdw_table_params *tp,
                                             const vdw_opts *opts)
{
    if (B < 1 || !grids || validate_opts(opts) || validate_table(tp)) return 0;
    Plan P;
    if (make_plan(B, grids, nullptr, opts, plan_nsig(tp), tp->n_D, opts->precision == VDW_FP64, 1, &P)) return 0;
    return P.L.total;
}

extern "C" int enl_energy(const vdw_grid *grid, const double *n_d, const double *q0_d, const double *phi_d,
                          const float *phi_f, const vdw_table_params *tp, const vdw_opts *opts, void *ws,
                          size_t ws_bytes, double *E_out, void *stream)
{
    return run(1, grid, nullptr, n_d, q0_d, nullptr, nullptr, nullptr, phi_d, phi_f, tp, opts, ws, ws_bytes, nullptr,
               E_out, (hipStream_t)stream);
}

extern "C" int enl_potential(const vdw_grid *grid, const double *n_d, const double *q0_d, const double *grad_d,
                             const double *dq_dn_d, const double *dq_dg_d, const double *phi_d, const float *phi_f,
                             const vdw_table_params *tp, const vdw_opts *opts, void *ws, size_t ws_bytes,
                             double *dEdn_d, double *E_out, void *stream)
{
    if (!dEdn_d) return fail(VDW_EINVAL, "dEdn_d is NULL");
    return run(1, grid, nullptr, n_d, q0_d, grad_d, dq_dn_d, dq_dg_d, phi_d, phi_f, tp, opts, ws, ws_bytes, dEdn_d,
               E_out, (hipStream_t)stream);
}

extern "C" int enl_potential_noalloc(const vdw_grid *grid, const double *n_d, const double *q0_d,
                                     const double *grad_d, const double *dq_dn_d, const double *dq_dg_d,
                                     const double *phi_d, const float *phi_f, const vdw_table_params *tp,
                                     const vdw_opts *opts, double *dEdn_d, double *E_out, void *stream)
{
    return run_noalloc(grid, n_d, q0_d, grad_d, dq_dn_d, dq_dg_d, phi_d, phi_f, tp, opts, dEdn_d, E_out,
                       (hipStream_t)stream);
}

extern "C" int enl_potential_batched(int32_t B, const vdw_grid *grids, const int64_t *grid_off, const double *n_d,
                                     const double *q0_d, const double *grad_d, const double *dq_dn_d,
                                     const double *dq_dg_d, const double *phi_d, const float *phi_f,
                                     const vdw_table_params *tp, const vdw_opts *opts, void *ws, size_t ws_bytes,
                                     double *dEdn_d, double *E_out, void *stream)
{
    if (!grid_off) return fail(VDW_EINVAL, "grid_off is NULL");
    if (grid_off[0] != 0) return fail(VDW_EINVAL, "grid_off[0] must be 0");
    if (!dEdn_d) return fail(VDW_EINVAL, "dEdn_d is NULL");
    return run(B, grids, grid_off, n_d, q0_d, grad_d, dq_dn_d, dq_dg_d, phi_d, phi_f, tp, opts, ws, ws_bytes, dEdn_d,
               E_out, (hipStream_t)stream);
}

extern "C" int vdw_last_stats(vdw_stats *out)
{
    if (!out) return fail(VDW_EINVAL, "out is NULL");
    *out = g_stats;
    return VDW_OK;
}

extern "C" void vdw_set_timing(int32_t on) { g_timing = on ? 1 : 0; }

// ---------------------------------------------------------------------------
// batch plans: descriptors uploaded once, then kernel-only evaluations that a
// HIP graph can record and replay
// ---------------------------------------------------------------------------

struct vdw_batch_plan {
    vdw::Exec E;
    std::vector<int64_t> grid_off;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" int enl_batch_plan_create(int32_t B, const vdw_grid *grids, const int64_t *grid_off,
                                     const vdw_table_params *tp, const vdw_opts *opts, int32_t potential, void *ws,
                                     size_t ws_bytes, vdw_batch_plan **plan, void *stream)
{
    if (!plan) return fail(VDW_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (!grid_off) return fail(VDW_EINVAL, "grid_off is NULL");
    if (B >= 1 && grid_off[0] != 0) return fail(VDW_EINVAL, "grid_off[0] must be 0");
    if (potential != 0 && potential != 1) return fail(VDW_EINVAL, "potential must be 0 or 1");
    vdw_batch_plan *p = new (std::nothrow) vdw_batch_plan;
    if (!p) return fail(VDW_ENOMEM, "out of host memory");
    int rc = prepare(B, grids, grid_off, tp, opts, potential, ws, ws_bytes, &p->E);
    if (!rc) rc = upload(p->E, (hipStream_t)stream);
    if (!rc) {
        hipError_t e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) rc = fail(VDW_EHIP, "uploading the plan: %s", hipGetErrorString(e));
    }
    if (rc) {
        delete p;
        return rc;
    }
    p->grid_off.assign(grid_off, grid_off + B + 1);
    *plan = p;
    return VDW_OK;
}

extern "C" int enl_batch_plan_execute(vdw_batch_plan *plan, const double *n_d, double *grad_d, double *q0_d,
                                      double *dq_dn_d, double *dq_dg_d, const double *phi_d, const float *phi_f,
                                      double *dEdn_d, double *E_d, void *stream)
{
    if (!plan) return fail(VDW_EINVAL, "plan is NULL");
    const Exec &E = plan->E;
    if (!n_d || !q0_d || !phi_d || !E_d) return fail(VDW_EINVAL, "NULL argument");
    if (!E.fp64 && !phi_f) return fail(VDW_EINVAL, "phi_f is required for VDW_FP32C");
    if (E.adj && (!grad_d || !dq_dn_d || !dq_dg_d || !dEdn_d))
        return fail(VDW_EINVAL, "a potential plan needs grad_d, dq_dn_d, dq_dg_d and dEdn_d");
    if (E.P.spec && !grad_d) return fail(VDW_EINVAL, "the spectral gradient needs grad_d");
    hipStream_t s = (hipStream_t)stream;
    const Layout &L = E.P.L;
    if (E.P.spec)
        // Fourier derivatives per grid step, staged in the densities' grad planes
        for (int b = 0; b < E.B; ++b) {
            const GridDev &g = E.P.gds[b];
            const int64_t o = E.P.segs[b].grid_off;
            for (int a = 0; a < 3; ++a)
                if (g.spec[a]) {
                    int rc = launch_spectral_lines(g, a, n_d + o, grad_d + 3 * o + a * g.G, s);
                    if (rc) return rc;
                }
        }
    hipLaunchKernelGGL(grad_q0_batched_kernel, dim3((unsigned)((L.Gtot + 255) / 256)), dim3(256), 0, s,
                       (const Seg *)(E.ws + L.segs), E.B, L.Gtot, E.n_cut, n_d, grad_d, q0_d, dq_dn_d, dq_dg_d);
    VDW_HIP(hipGetLastError());
    return enqueue(E, n_d, q0_d, grad_d, dq_dn_d, dq_dg_d, phi_d, phi_f, E.adj ? dEdn_d : nullptr, E_d, s, nullptr,
                   nullptr);
}

extern "C" int enl_batch_plan_capture(vdw_batch_plan *plan, const double *n_d, double *grad_d, double *q0_d,
                                      double *dq_dn_d, double *dq_dg_d, const double *phi_d, const float *phi_f,
                                      double *dEdn_d, double *E_d)
{
    if (!plan) return fail(VDW_EINVAL, "plan is NULL");
    if (plan->exec) {
        (void)hipGraphExecDestroy(plan->exec);
        plan->exec = nullptr;
    }
    if (plan->graph) {
        (void)hipGraphDestroy(plan->graph);
        plan->graph = nullptr;
    }
    hipStream_t cs = nullptr;
    VDW_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return fail(VDW_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    int rc = enl_batch_plan_execute(plan, n_d, grad_d, q0_d, dq_dn_d, dq_dg_d, phi_d, phi_f, dEdn_d, E_d, cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(VDW_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        plan->exec = nullptr;
        return fail(VDW_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    plan->graph = g;
    return VDW_OK;
}

extern "C" int enl_batch_plan_replay(vdw_batch_plan *plan, void *stream)
{
    if (!plan) return fail(VDW_EINVAL, "plan is NULL");
    if (!plan->exec) return fail(VDW_EINVAL, "the plan holds no captured graph");
    VDW_HIP(hipGraphLaunch(plan->exec, (hipStream_t)stream));
    return VDW_OK;
}

extern "C" int enl_batch_plan_destroy(vdw_batch_plan *plan)
{
    if (!plan) return VDW_OK;
    int rc = VDW_OK;
    if (plan->exec && hipGraphExecDestroy(plan->exec) != hipSuccess) rc = fail(VDW_EHIP, "hipGraphExecDestroy failed");
    if (plan->graph && hipGraphDestroy(plan->graph) != hipSuccess) rc = fail(VDW_EHIP, "hipGraphDestroy failed");
    delete plan;
    return rc;
}
