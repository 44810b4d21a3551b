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
