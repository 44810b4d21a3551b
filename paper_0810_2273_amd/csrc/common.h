// Internal declarations shared by the translation units of libvdwdf.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "vdwdf.h"

namespace vdw {

// Grid as the kernels see it.  Point (ix, iy, iz) sits at ix e_x + iy e_y +
// iz e_z, e_a = (lattice vector a) / n_a.  Orthorhombic cells (skew = 0)
// use h_a = |e_a| alone; skew cells also carry the step matrix E (rows e_a)
// and its inverse (grad n = E^-1 d, d_a the difference per grid step).
struct GridDev {
    int32_t nx, ny, nz;
    int32_t px, py, pz;  // periodic flags
    double hx, hy, hz;   // |e_x|, |e_y|, |e_z|
    int64_t G;
    int32_t skew;
    double E[9], Einv[9];  // row-major; E[3a + c] = component c of e_a
    double dV;             // |det E|
    int32_t spec[3];       // Fourier derivative on axis a (spectral gradient, periodic axis)
};

// Kept point as the pair kernels read it: grid coordinates (exact
// integers), n, a = q h_x / (2 dD), b = sqrt(n_sigma - 1) a, w = x^2 + y^2
// + z^2 (exact); FP32 records for VDW_FP32C, FP64 for VDW_FP64.  `off`
// holds, as raw bits, the 32-bit value x + (2 n_x - 1)(y + (2 n_y - 1) z),
// the point's term in the far-shell displacement-table index.
struct alignas(32) RecF {
    float x, y, z, n, a, b, w, off;
};
struct alignas(64) RecD {
    double x, y, z, n, a, b, w, off;
};
__host__ __device__ inline int rec_off(const RecF &r) { return (int)__builtin_bit_cast(uint32_t, r.off); }
__host__ __device__ inline int rec_off(const RecD &r)
{
    return (int)(uint32_t)__builtin_bit_cast(uint64_t, r.off);
}

// ---- far image shell (far.hip) ----
// Shell of one density: lattice vectors m with |m_a| <= hi[a], except those
// with every |m_a| <= lo[a] (hi = far_max, lo = image_max on periodic axes,
// both 0 elsewhere).  T is tabulated at every grid displacement (d_x, d_y,
// d_z), |d_a| < n_a, entry (d_x + n_x - 1) + (2 n_x - 1) ((d_y + n_y - 1) +
// (2 n_y - 1) (d_z + n_z - 1)), as sum_shell 1 / m^3 with m = |d - L|^2 /
// h_x^2 (the pair kernel's distance unit).
struct FarGeo {
    int32_t nx, ny, nz;
    int32_t lo[3], hi[3];
    double en[9];  // step vectors e_a / h_x (rows)
};
int64_t far_table_entries(const FarGeo &g);
int launch_far_table(const FarGeo &g, double *T, hipStream_t s);
// Far rows of the N kept points of one density (its records start at
// recs + *first, in compact order; N read on the device from *nkept, at
// most nmax), in `chunks` partial sums over as many
// j ranges: part[c nmax + i] = sum_j n_j phi_far(i, j) and (adj)
// part[(chunks + c) nmax + i] = qscale sum_j n_j d phi_far(i, j) / d a_i, with
// phi_far = -casym T_ij / (a_i^2 a_j^2 (a_i^2 + a_j^2)), j = i included.
// T must have fewer than 2^31 entries.
constexpr int kFarMaxChunks = 16;
int far_chunks(int64_t nmax);
int launch_far_rows(const FarGeo &g, int fp64, const void *recs, const int64_t *nkept, const int64_t *first,
                    int64_t nmax, const double *T, double casym, double qscale, int chunks, int adj, double *part,
                    hipStream_t s);

// ---- Fourier derivative along periodic axes (spectral.hip) ----
// d_a per grid step of every line along `axis` of src (x fastest), written
// to dst (same layout).
int launch_spectral_lines(const GridDev &g, int axis, const double *src, double *dst, hipStream_t s);
// Adjoint: dst[k] += sum_j D[j][k] B_a[j] along the lines of `axis`, with
// B_a[j] = dEdq dqdg 2 (E^-T grad)_a at point j (1/h_a grad_a on
// orthorhombic grids).
int launch_spectral_adjoint(const GridDev &g, int axis, const double *dEdq, const double *dqdg, const double *grad,
                            double *dst, hipStream_t s);

// Set the thread-local error message and return `code`.
int fail(int code, const char *fmt, ...);

// Check a HIP call; on error record the message and return VDW_EHIP.
#define VDW_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            return ::vdw::fail(VDW_EHIP, "%s: %s (%s:%d)", #call,                 \
                               hipGetErrorString(e_), __FILE__, __LINE__);         \
    } while (0)

int validate_grid(const vdw_grid *g, GridDev *out);
int validate_table(const vdw_table_params *tp);
double image_reach(const vdw_grid *g, const int32_t *image_max);
int image_cut_covered(const vdw_grid *g, const vdw_opts *o, double reach);

// Device properties cached per device.
struct DevInfo {
    int device;
    int cus;
    size_t lds_per_block;
};
int device_info(DevInfo *out);

// ---- table builder (table.hip) ----
void gauss_legendre_nodes(int n, double *x, double *w);  // host; ascending nodes on [-1, 1]
int launch_phi_table(const vdw_table_params *tp, double *phi_d, float *phi_f, hipStream_t s);

// ---- gradient and q0 (q0.hip) ----
int launch_grad_q0(const GridDev &g, double n_cut, const double *n, double *grad, double *q0,
                   double *dqdn, double *dqdg, int64_t grid_offset, hipStream_t s);

}  // namespace vdw
