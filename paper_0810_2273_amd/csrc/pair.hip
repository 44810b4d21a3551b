// The O(N^2) double sum of Eq. (2) (paper, Sec. 2) over the points kept by
// the density cut-off (Sec. 3), with periodic images of the 0th cell
// (Sec. 3), the on-site term, the deterministic FP64 reductions, and the
// adjoint dE/dn through q0 and the finite-difference gradient.
//
// Pipeline of one call (all on the caller's stream, no host round trip
// before the final copy of the energies):
//   fill      zero the work counter, flags, and (potential) dE/dn buffers
//   count     brick-ordered scan of n >= n_cut, per-block counts
//   scan      one workgroup: exclusive prefix, per-density point/item offsets
//   scatter   compact the kept points into 32-byte (FP32) or 64-byte (FP64)
//             records in brick order (4x4x4 bricks, so a wavefront's 64
//             i-points are spatially compact and their table rows coherent)
//   pair      persistent workgroups pull (density, i-block, j-chunk) items
//             from an atomic counter; each lane owns one i-point, the j
//             records stream through scalar registers (wave-uniform loads),
//             the first table rows sit in LDS (row stride n_sigma + 1 so a
//             column spread over rows hits different banks), the rest is
//             read through L2; partial sums go to per-chunk slots
//   finalize  per point: fixed-order sum of the chunk partials, on-site term,
//             energy terms, and (potential) the direct part of dE/dn
//   reduce    per density: fixed-order sum of the block partials
//   assemble  (potential) transposed gradient stencil on the whole grid
#include <math.h>
#include <string.h>

#include <vector>

#include "common.h"

namespace vdw {

namespace {

constexpr int kCompactBlock = 1024;  // brick-order positions per count/scatter block
constexpr int kCompactThreads = 256;  // 4 positions (one brick row) per thread
constexpr int kPairThreads = 1024;    // i-points per item (one per lane)
constexpr int kFinThreads = 256;      // points per finalize block
constexpr int kRun = 64;              // j-terms per FP32 run before the FP64 carry

enum { HDR_ITEMS = 0, HDR_NTOTAL = 1, HDR_BLKS = 2, HDR_WORDS = 8 };

struct Seg {
    // filled on the host
    int32_t nx, ny, nz, px, py, pz;
    double hx, hy, hz, dV;
    int64_t G, grid_off;
    int32_t nbx, nby, nbz, C;
    int64_t t_off, T;  // brick-order positions: offset (multiple of kCompactBlock), padded length
    // filled on the device by scan_kernel
    int64_t N, p_off, part_off, item_off, blk_off, nIB;
};

struct alignas(32) RecF {
    float x, y, z, n, a, b, p, pad;
};
struct alignas(64) RecD {
    double x, y, z, n, a, b, p, pad;
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
                                                    Seg *__restrict__ segs, int B, int64_t *__restrict__ hdr)
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
        int64_t part_off = 0, item_off = 0, blk_off = 0;
        for (int b = 0; b < B; ++b) {
            Seg &g = segs[b];
            int64_t first = g.t_off / kCompactBlock, last = (g.t_off + g.T) / kCompactBlock;
            g.p_off = counts[first];
            g.N = counts[last] - counts[first];
            g.nIB = (g.N + kPairThreads - 1) / kPairThreads;
            g.part_off = part_off;
            g.item_off = item_off;
            g.blk_off = blk_off;
            part_off += (int64_t)g.C * g.N;
            item_off += g.nIB * g.C;
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
    double inv2dD;  // 1 / (2 dD): a = q / (2 dD) is D per unit distance in table-index units
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
    for (int u = 0; u < 4; ++u) {
        if (!keep[u]) continue;
        double nn = A.n[gi[u]], q = A.q0[gi[u]];
        double a = q * A.inv2dD;
        if (A.fp64) {
            RecD r;
            r.x = xs[u];
            r.y = ys[u];
            r.z = zs[u];
            r.n = nn;
            r.a = a;
            r.b = a * A.csig;
            r.p = q * q;
            r.pad = 0.0;
            ((RecD *)A.recs)[pos] = r;
        } else {
            RecF r;
            r.x = (float)xs[u];
            r.y = (float)ys[u];
            r.z = (float)zs[u];
            r.n = (float)nn;
            r.a = (float)a;
            r.b = (float)(a * A.csig);
            r.p = (float)(q * q);
            r.pad = 0.0f;
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
    const void *recs;
    const Seg *segs;
    int B;
    const int64_t *hdr;
    int *counter;
    const void *tabg;   // full table in global memory (float or double)
    int nD, nS, S, K;   // S: LDS row stride (n_sigma + 1); K: rows held in LDS
    double tDmax;       // n_D - 1: table branch iff t_D = D / dD < n_D - 1
    double tSclamp;     // largest value below n_sigma - 1 (sigma index clamp)
    double casym;       // C = 12 (4 pi/9)^3
    double dD2;         // 2 dD
    double rc2;         // squared distance cut (inf: none)
    const int *imgs;    // image multipliers (m_x, m_y, m_z, 0) per image
    int nimg, home;     // number of images, index of (0, 0, 0)
    double *part;       // chunk partials
    int64_t part_stride;  // doubles per accumulator array
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
__device__ inline double dsqrt(double x) { return sqrt(x); }
__device__ inline float drcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double drcp(double x) { return 1.0 / x; }
__device__ inline float dfract(float x) { return __builtin_amdgcn_fractf(x); }
__device__ inline double dfract(double x) { return x - floor(x); }

// Pointers are separate __restrict__ parameters so the compiler knows the
// records, segments and table are not written during the kernel and can
// fetch wave-uniform j records with scalar loads.
template <typename R, bool ADJ, bool IMG, bool KAHAN>
__global__ __launch_bounds__(kPairThreads) void pair_kernel(PairArgs A, const typename RecOf<R>::T *__restrict__ recs,
                                                            const Seg *__restrict__ segs,
                                                            const int64_t *__restrict__ hdr, int *__restrict__ counter,
                                                            const R *__restrict__ tabg, const int *__restrict__ imgs,
                                                            double *__restrict__ part)
{
    using Rec = typename RecOf<R>::T;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *tab = reinterpret_cast<R *>(smem_raw);
    __shared__ int s_item;

    const int S = A.S, nS = A.nS, K = A.K;

    for (int t = threadIdx.x; t < K * nS; t += kPairThreads) {
        int r = t / nS, c = t - r * nS;
        tab[r * S + c] = tabg[t];
    }
    __syncthreads();

    const int64_t total = hdr[HDR_ITEMS];
    const R tDmax = (R)A.tDmax, tSclamp = (R)A.tSclamp;
    const R casym = (R)A.casym;
    const R rc2 = (R)A.rc2;

    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= total) break;

        const int b = (A.B > 1) ? __builtin_amdgcn_readfirstlane(find_seg(segs, A.B, item, 2)) : 0;
        const Seg &sg = segs[b];
        const int N = __builtin_amdgcn_readfirstlane((int)sg.N);
        const int nIB = __builtin_amdgcn_readfirstlane((int)sg.nIB);
        const int C = sg.C;
        const int local = __builtin_amdgcn_readfirstlane((int)(item - sg.item_off));
        const int c = local / nIB;
        const int ib = local - c * nIB;
        const int len = (N + C - 1) / C;
        const int j0 = min(N, c * len), j1 = min(N, j0 + len);
        const R hx2 = (R)(sg.hx * sg.hx), hy2 = (R)(sg.hy * sg.hy), hz2 = (R)(sg.hz * sg.hz);
        const Rec *__restrict__ P = recs + sg.p_off;

        const int il = ib * kPairThreads + threadIdx.x;
        const bool active = il < N;
        const Rec I = P[active ? il : N - 1];
        const R xi = I.x, yi = I.y, zi = I.z, ai = I.a, bi = I.b, pi = I.p;
        const R c1 = (R)2 / ai;                      // asymptote, 2 dD (2 / q_i) in a-units
        const R c2 = (R)(A.dD2 * A.dD2 * 2.0) * ai;  // asymptote, 2 dD (2 q_i)

        double S0c = 0.0, S0L = 0.0, Sq = 0.0;

        const int nimg = IMG ? A.nimg : 1;
        for (int L = 0; L < nimg; ++L) {
            R sx = xi, sy = yi, sz = zi;
            bool home = true;
            if (IMG) {
                sx -= (R)(imgs[4 * L + 0] * sg.nx);
                sy -= (R)(imgs[4 * L + 1] * sg.ny);
                sz -= (R)(imgs[4 * L + 2] * sg.nz);
                home = (L == A.home);
            }
            if (j0 >= j1) continue;
            Rec Jn = P[j0];
            for (int jr = j0; jr < j1; jr += kRun) {
                const int je = min(j1, jr + kRun);
                R acc = 0, accq = 0, cmp = 0, cmpq = 0;
                for (int j = jr; j < je; ++j) {
                    const Rec J = Jn;
                    Jn = P[min(j + 1, j1 - 1)];  // prefetch the next record (wave-uniform)
                    const R dx = sx - J.x, dy = sy - J.y, dz = sz - J.z;
                    const R r2 = hx2 * (dx * dx) + hy2 * (dy * dy) + hz2 * (dz * dz);
                    R w = (r2 > (R)0) ? J.n : (R)0;
                    if (IMG) w = (r2 <= rc2) ? w : (R)0;
                    const R r = dsqrt(r2);
                    const R s = ai + J.a;
                    const R tD = s * r;
                    const R inv = drcp(s);
                    const R u = (bi - J.b) * inv;
                    R phi, dq = 0;
                    if (tD < tDmax) {
                        const R ts = (u * u < tSclamp) ? u * u : tSclamp;
                        const int k = (int)tD;
                        const int l = (int)ts;
                        const R fD = dfract(tD), fS = dfract(ts);
                        // rows below K come from LDS; the clamped LDS read is
                        // always in bounds and is replaced for rows >= K - 1
                        const int kl = min(k, K - 2);
                        const int o = (int)__umul24((unsigned)kl, (unsigned)S) + l;
                        R p00 = tab[o], p01 = tab[o + 1], p10 = tab[o + S], p11 = tab[o + S + 1];
                        // keep the LDS reads unconditional: without this the
                        // compiler folds the two sources into one FLAT load
                        asm("" : "+v"(p00), "+v"(p01), "+v"(p10), "+v"(p11));
                        if (k + 1 >= K) {
                            const R *t0 = tabg + (int64_t)k * nS + l;
                            p00 = t0[0];
                            p01 = t0[1];
                            p10 = t0[nS];
                            p11 = t0[nS + 1];
                        }
                        const R d0 = p01 - p00, d1 = p11 - p10;
                        const R lo = p00 + fS * d0, hi = p10 + fS * d1;
                        const R gD = hi - lo;
                        phi = lo + fD * gD;
                        if (ADJ) {
                            const R gS = d0 + fD * (d1 - d0);
                            // 2 dD dphi/dq_i = gD r + gS (4 csig u a_j / s^2) = gD r + gS u inv inv 4 b_j
                            dq = gD * r + gS * ((u * inv) * (inv * ((R)4 * J.b)));
                        }
                    } else {
                        const R r6 = r2 * r2 * r2;
                        const R pp = pi + J.p;
                        phi = -casym * drcp(r6 * pi * J.p * pp);
                        if (ADJ) dq = -phi * (c1 + c2 * drcp(pp));
                    }
                    if (KAHAN) {
                        R y = w * phi - cmp;
                        R t = acc + y;
                        cmp = (t - acc) - y;
                        acc = t;
                        if (ADJ) {
                            R yq = w * dq - cmpq;
                            R tq = accq + yq;
                            cmpq = (tq - accq) - yq;
                            accq = tq;
                        }
                    } else {
                        acc += w * phi;
                        if (ADJ) accq += w * dq;
                    }
                }
                if (home) S0c += (double)acc - (double)cmp;
                else S0L += (double)acc - (double)cmp;
                if (ADJ) Sq += (double)accq - (double)cmpq;
            }
        }
        if (active) {
            const int64_t slot = sg.part_off + (int64_t)c * N + il;
            part[slot] = S0c;
            if (IMG) part[A.part_stride + slot] = S0L;
            if (ADJ) part[2 * A.part_stride + slot] = Sq / A.dD2;
        }
    }
}

// ---------------------------------------------------------------------------
// finalize, reduce, assemble
// ---------------------------------------------------------------------------

struct FinArgs {
    const Seg *segs;
    int B;
    const int64_t *hdr;
    const double *part;
    int64_t part_stride;
    int img, adj, self_term;
    const int32_t *gidx;
    const double *n, *q0, *dqdn;
    const double *tab;  // FP64 table for the on-site term
    int nD, nS;
    double dD, Dmax, casym;
    double *blockE;
    double *dEdn;   // direct part scattered to the grid (potential)
    double *dEdq;   // dE/dq scattered to the grid (potential)
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
    double p0 = F.tab[(int64_t)k * F.nS], p1 = F.tab[(int64_t)(k + 1) * F.nS];
    *dphi = (p1 - p0) / F.dD;
    return p0 + fD * (p1 - p0);
}

__global__ __launch_bounds__(kFinThreads) void finalize_kernel(FinArgs F)
{
    __shared__ double r0[kFinThreads], r1[kFinThreads], r2[kFinThreads];
    const int64_t blk = blockIdx.x;
    if (blk >= F.hdr[HDR_BLKS]) return;
    const int b = find_seg(F.segs, F.B, blk, 3);
    const Seg &sg = F.segs[b];
    const int64_t lp = (blk - sg.blk_off) * kFinThreads + threadIdx.x;
    double e0 = 0.0, eL = 0.0, es = 0.0;
    if (lp < sg.N) {
        const int64_t p = sg.p_off + lp;
        double S0c = 0.0, S0L = 0.0, Sq = 0.0;
        for (int c = 0; c < sg.C; ++c) {
            int64_t slot = sg.part_off + (int64_t)c * sg.N + lp;
            S0c += F.part[slot];
            if (F.img) S0L += F.part[F.part_stride + slot];
            if (F.adj) Sq += F.part[2 * F.part_stride + slot];
        }
        const int64_t g = F.gidx[p];
        const double nn = F.n[g], q = F.q0[g];
        const double rho_s = cbrt(3.0 * sg.dV / (4.0 * 3.14159265358979323846)) * exp(-1.0 / 3.0);
        double Phi = 0.0, dPhi = 0.0;
        if (F.self_term) {
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
    __syncthreads();
    for (int st = kFinThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            r0[threadIdx.x] += r0[threadIdx.x + st];
            r1[threadIdx.x] += r1[threadIdx.x + st];
            r2[threadIdx.x] += r2[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        F.blockE[3 * blk + 0] = r0[0];
        F.blockE[3 * blk + 1] = r1[0];
        F.blockE[3 * blk + 2] = r2[0];
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

__device__ inline double bval(const AsmArgs &A, const Seg &s, int axis, int64_t gl)
{
    int64_t g = s.grid_off + gl;
    return A.dEdq[g] * A.dqdg[g] * 2.0 * A.grad[3 * s.grid_off + axis * s.G + gl];
}

__device__ inline double tstencil(const AsmArgs &A, const Seg &s, int axis, int64_t idx, int k, int N, int64_t st,
                                  int per, double h)
{
    double acc = 0.0;
    if (per) {
        int64_t up = (k + 1 == N) ? -(int64_t)(N - 1) * st : st;
        int64_t dn = (k == 0) ? (int64_t)(N - 1) * st : -st;
        acc = bval(A, s, axis, idx + dn) - bval(A, s, axis, idx + up);
    } else {
        // interior rows i = k-1 (coefficient +1 at k) and i = k+1 (coefficient -1 at k)
        if (k - 1 >= 1 && k - 1 <= N - 2) acc += bval(A, s, axis, idx - st);
        if (k + 1 >= 1 && k + 1 <= N - 2) acc -= bval(A, s, axis, idx + st);
        // face row i = 0: (-3, 4, -1) on (0, 1, 2)
        if (k <= 2) {
            const double c0[3] = {-3.0, 4.0, -1.0};
            acc += c0[k] * bval(A, s, axis, idx - (int64_t)k * st);
        }
        // face row i = N-1: (1, -4, 3) on (N-3, N-2, N-1)
        if (k >= N - 3) {
            const double c1[3] = {1.0, -4.0, 3.0};
            acc += c1[k - (N - 3)] * bval(A, s, axis, idx + (int64_t)(N - 1 - k) * st);
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
    double v = tstencil(A, s, 0, gl, ix, s.nx, 1, s.px, s.hx);
    v += tstencil(A, s, 1, gl, iy, s.ny, s.nx, s.py, s.hy);
    v += tstencil(A, s, 2, gl, iz, s.nz, (int64_t)s.nx * s.ny, s.pz, s.hz);
    A.dEdn[t] += v;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct Layout {
    size_t hdr, counter, flag, segs, imgs, counts, recs, gidx, part, blockE, res, dEdq, total;
    int64_t nblocks, part_stride, fin_blocks, Gtot;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Plan {
    std::vector<Seg> segs;
    std::vector<int> imgs;  // 4 ints per image
    int nimg = 1, home = 0;
    bool img = false;
    Layout L;
};

int chunks_for(const GridDev &g, const vdw_opts *o, int cus)
{
    if (o->j_chunks > 0) return o->j_chunks;
    // enough items to keep every CU busy several times over, and items no
    // longer than ~16k j-terms per i-block
    int64_t nib = (g.G + kPairThreads - 1) / kPairThreads;
    int64_t c1 = (8LL * cus + nib - 1) / nib;
    int64_t c2 = (g.G + 16383) / 16384;
    int64_t c = c1 > c2 ? c1 : c2;
    if (c < 1) c = 1;
    if (c > 64) c = 64;
    return (int)c;
}

int make_plan(int B, const vdw_grid *grids, const int64_t *grid_off, const vdw_opts *o, int fp64, int adj, int cus,
              Plan *P)
{
    P->segs.resize(B);
    int64_t t_off = 0, part = 0, fin = 0, Gtot = 0;
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
        s.dV = g.hx * g.hy * g.hz;
        s.G = g.G;
        s.grid_off = grid_off ? grid_off[b] : 0;
        if (grid_off && grid_off[b + 1] - grid_off[b] != g.G)
            return fail(VDW_EINVAL, "grid_off[%d+1] - grid_off[%d] != grid %d size", b, b, b);
        s.nbx = (g.nx + 3) / 4;
        s.nby = (g.ny + 3) / 4;
        s.nbz = (g.nz + 3) / 4;
        s.C = chunks_for(g, o, cus);
        int64_t T = (int64_t)s.nbx * s.nby * s.nbz * 64;
        s.T = (T + kCompactBlock - 1) / kCompactBlock * kCompactBlock;
        s.t_off = t_off;
        t_off += s.T;
        part += (int64_t)s.C * g.G;
        fin += (g.G + kFinThreads - 1) / kFinThreads;
        Gtot += g.G;
    }
    if (Gtot > ((int64_t)1 << 31) - 1) return fail(VDW_EINVAL, "total grid size exceeds 2^31 - 1");
    // images on periodic axes
    int m[3];
    for (int a = 0; a < 3; ++a) {
        int per = a == 0 ? P->segs[0].px : a == 1 ? P->segs[0].py : P->segs[0].pz;
        if (o->image_max[a] < 0) return fail(VDW_EINVAL, "image_max must be >= 0");
        m[a] = per ? o->image_max[a] : 0;
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

    Layout &L = P->L;
    L.nblocks = t_off / kCompactBlock;
    L.part_stride = part;
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
    L.recs = off;
    off = align256(off + Gtot * (fp64 ? sizeof(RecD) : sizeof(RecF)));
    L.gidx = off;
    off = align256(off + Gtot * sizeof(int32_t));
    L.part = off;
    off = align256(off + 3 * part * sizeof(double));
    L.blockE = off;
    off = align256(off + 3 * fin * sizeof(double));
    L.res = off;
    off = align256(off + (4 * B + 1) * sizeof(double));
    L.dEdq = off;
    if (adj) off = align256(off + Gtot * sizeof(double));
    L.total = off;
    return VDW_OK;
}

int validate_opts(const vdw_opts *o)
{
    if (!o) return fail(VDW_EINVAL, "opts is NULL");
    if (!(o->n_cut > 0.0) || !isfinite(o->n_cut)) return fail(VDW_EINVAL, "n_cut must be > 0");
    if (o->precision != VDW_FP64 && o->precision != VDW_FP32C) return fail(VDW_EINVAL, "precision must be 0 or 1");
    if (o->self_term != 0 && o->self_term != 1) return fail(VDW_EINVAL, "self_term must be 0 or 1");
    if (o->block_threads != 0 && o->block_threads != kPairThreads)
        return fail(VDW_EINVAL, "block_threads must be 0 or %d", kPairThreads);
    if (o->j_chunks < 0 || o->j_chunks > 64) return fail(VDW_EINVAL, "j_chunks must be in 0..64");
    if (o->grid_blocks < 0) return fail(VDW_EINVAL, "grid_blocks must be >= 0");
    if (o->kahan != 0 && o->kahan != 1) return fail(VDW_EINVAL, "kahan must be 0 or 1");
    if (!isfinite(o->r_cut)) return fail(VDW_EINVAL, "r_cut must be finite");
    return VDW_OK;
}

thread_local vdw_stats g_stats;
thread_local int g_timing = 0;

template <typename R, bool ADJ, bool IMG, bool KAHAN>
int launch_pair_t(const PairArgs &a, int grid, size_t lds, hipStream_t s)
{
    auto k = pair_kernel<R, ADJ, IMG, KAHAN>;
    if (lds > 65536) {
        // raises the dynamic-LDS limit where the runtime enforces one; a
        // failure here surfaces at the launch below
        (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    hipLaunchKernelGGL(k, dim3(grid), dim3(kPairThreads), lds, s, a, (const typename RecOf<R>::T *)a.recs, a.segs,
                       a.hdr, a.counter, (const R *)a.tabg, a.imgs, a.part);
    VDW_HIP(hipGetLastError());
    return VDW_OK;
}

int launch_pair(int fp64, int adj, int img, int kahan, const PairArgs &a, int grid, size_t lds, hipStream_t s)
{
    if (fp64) {
        if (adj) return img ? launch_pair_t<double, true, true, false>(a, grid, lds, s)
                            : launch_pair_t<double, true, false, false>(a, grid, lds, s);
        return img ? launch_pair_t<double, false, true, false>(a, grid, lds, s)
                   : launch_pair_t<double, false, false, false>(a, grid, lds, s);
    }
    if (kahan) {
        if (adj) return img ? launch_pair_t<float, true, true, true>(a, grid, lds, s)
                            : launch_pair_t<float, true, false, true>(a, grid, lds, s);
        return img ? launch_pair_t<float, false, true, true>(a, grid, lds, s)
                   : launch_pair_t<float, false, false, true>(a, grid, lds, s);
    }
    if (adj) return img ? launch_pair_t<float, true, true, false>(a, grid, lds, s)
                        : launch_pair_t<float, true, false, false>(a, grid, lds, s);
    return img ? launch_pair_t<float, false, true, false>(a, grid, lds, s)
               : launch_pair_t<float, false, false, false>(a, grid, lds, s);
}

// The whole pipeline for B densities.
int run(int B, const vdw_grid *grids, const int64_t *grid_off, const double *n_d, const double *q0_d,
        const double *grad_d, const double *dqdn_d, const double *dqdg_d, const double *phi_d, const float *phi_f,
        const vdw_table_params *tp, const vdw_opts *o, void *ws, size_t ws_bytes, double *dEdn_d, double *E_out,
        hipStream_t s)
{
    int rc = validate_opts(o);
    if (rc) return rc;
    rc = validate_table(tp);
    if (rc) return rc;
    const int adj = dEdn_d != nullptr;
    const int fp64 = o->precision == VDW_FP64;
    if (B < 1) return fail(VDW_EINVAL, "B must be >= 1");
    if (!grids || !n_d || !q0_d || !phi_d || !E_out) return fail(VDW_EINVAL, "NULL argument");
    if (!fp64 && !phi_f) return fail(VDW_EINVAL, "phi_f is required for VDW_FP32C");
    if (adj && (!grad_d || !dqdn_d || !dqdg_d)) return fail(VDW_EINVAL, "grad_d, dq_dn_d and dq_dg_d are required");
    if (!ws) return fail(VDW_EINVAL, "workspace is NULL");
    DevInfo dev;
    rc = device_info(&dev);
    if (rc) return rc;
    Plan P;
    rc = make_plan(B, grids, grid_off, o, fp64, adj, dev.cus, &P);
    if (rc) return rc;
    if (ws_bytes < P.L.total)
        return fail(VDW_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, P.L.total);
    const Layout &L = P.L;
    char *w = (char *)ws;
    int64_t *hdr = (int64_t *)(w + L.hdr);
    int *counter = (int *)(w + L.counter);
    int *flag = (int *)(w + L.flag);
    Seg *segs = (Seg *)(w + L.segs);
    int *imgs = (int *)(w + L.imgs);
    int64_t *counts = (int64_t *)(w + L.counts);
    void *recs = w + L.recs;
    int32_t *gidx = (int32_t *)(w + L.gidx);
    double *part = (double *)(w + L.part);
    double *blockE = (double *)(w + L.blockE);
    double *res = (double *)(w + L.res);
    double *dEdq = (double *)(w + L.dEdq);

    VDW_HIP(hipMemcpyAsync(segs, P.segs.data(), B * sizeof(Seg), hipMemcpyHostToDevice, s));
    VDW_HIP(hipMemcpyAsync(imgs, P.imgs.data(), P.imgs.size() * sizeof(int), hipMemcpyHostToDevice, s));
    // counter and flag live in 64-bit words right after the header
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, hdr, HDR_WORDS);
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, (int64_t *)counter, 1);
    hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(64), 0, s, (int64_t *)flag, 1);
    VDW_HIP(hipGetLastError());
    if (adj) {
        unsigned gb = (unsigned)((L.Gtot + 255) / 256);
        hipLaunchKernelGGL(fill_kernel, dim3(gb), dim3(256), 0, s, dEdn_d, L.Gtot);
        hipLaunchKernelGGL(fill_kernel, dim3(gb), dim3(256), 0, s, dEdq, L.Gtot);
        VDW_HIP(hipGetLastError());
    }
    // compaction
    hipLaunchKernelGGL(count_kernel, dim3((unsigned)L.nblocks), dim3(kCompactThreads), 0, s, (const Seg *)segs, B,
                       n_d, o->n_cut, counts, flag);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, counts, L.nblocks, segs, B, hdr);
    ScatterArgs sa;
    sa.segs = segs;
    sa.B = B;
    sa.n = n_d;
    sa.q0 = q0_d;
    sa.n_cut = o->n_cut;
    sa.offs = counts;
    sa.recs = recs;
    sa.gidx = gidx;
    const double dD = tp->D_max / (tp->n_D - 1);
    sa.inv2dD = 1.0 / (2.0 * dD);
    sa.csig = sqrt((double)(tp->n_sigma - 1));
    sa.fp64 = fp64;
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)L.nblocks), dim3(kCompactThreads), 0, s, sa);
    VDW_HIP(hipGetLastError());

    // pair kernel
    const size_t esz = fp64 ? sizeof(double) : sizeof(float);
    const int S = tp->n_sigma + 1;
    const size_t lds_cap = dev.lds_per_block > 1024 ? dev.lds_per_block - 1024 : 0;
    int K = (int)(lds_cap / (S * esz));
    if (o->table_lds_rows >= 0 && o->table_lds_rows < K) K = o->table_lds_rows;
    if (K > tp->n_D) K = tp->n_D;
    if (K < 2) K = 2;  // the kernel reads a clamped LDS row unconditionally
    PairArgs pa;
    pa.recs = recs;
    pa.segs = segs;
    pa.B = B;
    pa.hdr = hdr;
    pa.counter = counter;
    pa.tabg = fp64 ? (const void *)phi_d : (const void *)phi_f;
    pa.nD = tp->n_D;
    pa.nS = tp->n_sigma;
    pa.S = S;
    pa.K = K;
    pa.tDmax = (double)(tp->n_D - 1);
    pa.tSclamp = fp64 ? nextafter((double)(tp->n_sigma - 1), 0.0) : (double)nextafterf((float)(tp->n_sigma - 1), 0.0f);
    pa.casym = 12.0 * pow(4.0 * 3.14159265358979323846 / 9.0, 3);
    pa.dD2 = 2.0 * dD;
    pa.rc2 = o->r_cut > 0.0 ? o->r_cut * o->r_cut : INFINITY;
    pa.imgs = imgs;
    pa.nimg = P.nimg;
    pa.home = P.home;
    pa.part = part;
    pa.part_stride = L.part_stride;
    int grid = o->grid_blocks > 0 ? o->grid_blocks : dev.cus;
    size_t lds = (size_t)K * S * esz;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (g_timing) {
        VDW_HIP(hipEventCreate(&ev0));
        VDW_HIP(hipEventCreate(&ev1));
        VDW_HIP(hipEventRecord(ev0, s));
    }
    rc = launch_pair(fp64, adj, P.img ? 1 : 0, o->kahan, pa, grid, lds, s);
    if (rc) return rc;
    if (g_timing) VDW_HIP(hipEventRecord(ev1, s));

    // finalize and reduce
    FinArgs fa;
    fa.segs = segs;
    fa.B = B;
    fa.hdr = hdr;
    fa.part = part;
    fa.part_stride = L.part_stride;
    fa.img = P.img ? 1 : 0;
    fa.adj = adj;
    fa.self_term = o->self_term;
    fa.gidx = gidx;
    fa.n = n_d;
    fa.q0 = q0_d;
    fa.dqdn = dqdn_d;
    fa.tab = phi_d;
    fa.nD = tp->n_D;
    fa.nS = tp->n_sigma;
    fa.dD = dD;
    fa.Dmax = tp->D_max;
    fa.casym = pa.casym;
    fa.blockE = blockE;
    fa.dEdn = dEdn_d;
    fa.dEdq = dEdq;
    if (L.fin_blocks > 0)
        hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)L.fin_blocks), dim3(kFinThreads), 0, s, fa);
    hipLaunchKernelGGL(seg_reduce_kernel, dim3(B), dim3(256), 0, s, (const Seg *)segs, (const double *)blockE, res, B,
                       (const int *)flag);
    VDW_HIP(hipGetLastError());
    if (adj) {
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
    }
    std::vector<double> host(4 * B + 1);
    VDW_HIP(hipMemcpyAsync(host.data(), res, host.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    VDW_HIP(hipStreamSynchronize(s));
    float ms = 0.0f;
    if (g_timing) {
        VDW_HIP(hipEventElapsedTime(&ms, ev0, ev1));
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }
    if (host[4 * B] != 0.0) return fail(VDW_ENONFINITE, "the density holds NaN or Inf values");
    double pairs = 0.0;
    int64_t retained = 0;
    for (int b = 0; b < B; ++b) {
        E_out[3 * b + 0] = host[3 * b + 0];
        E_out[3 * b + 1] = host[3 * b + 1];
        E_out[3 * b + 2] = host[3 * b + 2];
        double Nb = host[3 * B + b];
        retained += (int64_t)Nb;
        pairs += Nb * Nb * P.nimg - Nb;
    }
    g_stats.retained = retained;
    g_stats.pairs = pairs;
    g_stats.pair_kernel_ms = ms;
    g_stats.lds_rows = K;
    g_stats.block_threads = kPairThreads;
    g_stats.j_chunks = P.segs[0].C;
    g_stats.grid_blocks = grid;
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
    DevInfo dev;
    int cus = 256;
    if (device_info(&dev) == VDW_OK) cus = dev.cus;
    Plan P;
    if (make_plan(B, grids, nullptr, opts, opts->precision == VDW_FP64, 1, cus, &P)) return 0;
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
