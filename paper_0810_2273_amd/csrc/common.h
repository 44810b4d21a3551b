// Internal declarations shared by the translation units of libvdwdf.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "vdwdf.h"

namespace vdw {

// Orthorhombic grid as the kernels see it.
struct GridDev {
    int32_t nx, ny, nz;
    int32_t px, py, pz;  // periodic flags
    double hx, hy, hz;
    int64_t G;
};

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
int launch_phi_table(const vdw_table_params *tp, double *phi_d, float *phi_f, hipStream_t s);

// ---- gradient and q0 (q0.hip) ----
int launch_grad_q0(const GridDev &g, double n_cut, const double *n, double *grad, double *q0,
                   double *dqdn, double *dqdg, int64_t grid_offset, hipStream_t s);

}  // namespace vdw
