// Error reporting, argument validation and device queries for libvdwdf.so.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "common.h"

namespace vdw {

static thread_local char g_err[512] = "no error";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int validate_grid(const vdw_grid *g, GridDev *out)
{
    if (!g) return fail(VDW_EINVAL, "grid is NULL");
    int skew = 0;
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 3) return fail(VDW_EINVAL, "grid n[%d] = %d < 3", a, g->n[a]);
        for (int b = 0; b < 3; ++b) {
            double v = g->cell[a][b];
            if (!isfinite(v)) return fail(VDW_EINVAL, "cell[%d][%d] is not finite", a, b);
            if (a != b && v != 0.0) skew = 1;
        }
        if (g->periodic[a] != 0 && g->periodic[a] != 1)
            return fail(VDW_EINVAL, "periodic[%d] must be 0 or 1", a);
        if (g->gradient == VDW_GRAD_SPECTRAL && g->periodic[a] && g->n[a] > 4096)
            return fail(VDW_EINVAL, "spectral gradient: periodic axis %d has %d > 4096 points", a, g->n[a]);
    }
    if (g->gradient != VDW_GRAD_FD && g->gradient != VDW_GRAD_SPECTRAL)
        return fail(VDW_EINVAL, "gradient must be VDW_GRAD_FD or VDW_GRAD_SPECTRAL");
    double E[9];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) E[3 * a + c] = g->cell[a][c] / g->n[a];
    // cofactors: Einv = adj(E) / det(E)
    const double C00 = E[4] * E[8] - E[5] * E[7], C01 = E[5] * E[6] - E[3] * E[8], C02 = E[3] * E[7] - E[4] * E[6];
    const double det = E[0] * C00 + E[1] * C01 + E[2] * C02;
    if (!skew) {
        for (int a = 0; a < 3; ++a)
            if (!(g->cell[a][a] > 0.0)) return fail(VDW_EINVAL, "cell[%d][%d] must be > 0", a, a);
    } else {
        const double la = sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]);
        const double lb = sqrt(E[3] * E[3] + E[4] * E[4] + E[5] * E[5]);
        const double lc = sqrt(E[6] * E[6] + E[7] * E[7] + E[8] * E[8]);
        if (!(fabs(det) > 1e-6 * la * lb * lc)) return fail(VDW_EINVAL, "degenerate cell (|det| = %g)", fabs(det));
    }
    int64_t G = (int64_t)g->n[0] * g->n[1] * g->n[2];
    if (G > (int64_t)1 << 31) return fail(VDW_EINVAL, "grid too large (%lld points)", (long long)G);
    if (out) {
        out->nx = g->n[0];
        out->ny = g->n[1];
        out->nz = g->n[2];
        out->px = g->periodic[0];
        out->py = g->periodic[1];
        out->pz = g->periodic[2];
        out->G = G;
        out->skew = skew;
        for (int a = 0; a < 3; ++a) out->spec[a] = g->gradient == VDW_GRAD_SPECTRAL && g->periodic[a];
        for (int k = 0; k < 9; ++k) out->E[k] = E[k];
        if (!skew) {
            out->hx = g->cell[0][0] / g->n[0];
            out->hy = g->cell[1][1] / g->n[1];
            out->hz = g->cell[2][2] / g->n[2];
            out->dV = out->hx * out->hy * out->hz;
            for (int k = 0; k < 9; ++k) out->Einv[k] = 0.0;
            out->Einv[0] = 1.0 / out->hx;
            out->Einv[4] = 1.0 / out->hy;
            out->Einv[8] = 1.0 / out->hz;
        } else {
            out->hx = sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]);
            out->hy = sqrt(E[3] * E[3] + E[4] * E[4] + E[5] * E[5]);
            out->hz = sqrt(E[6] * E[6] + E[7] * E[7] + E[8] * E[8]);
            out->dV = fabs(det);
            const double id = 1.0 / det;
            out->Einv[0] = C00 * id;
            out->Einv[3] = C01 * id;
            out->Einv[6] = C02 * id;
            out->Einv[1] = (E[2] * E[7] - E[1] * E[8]) * id;
            out->Einv[4] = (E[0] * E[8] - E[2] * E[6]) * id;
            out->Einv[7] = (E[1] * E[6] - E[0] * E[7]) * id;
            out->Einv[2] = (E[1] * E[5] - E[2] * E[4]) * id;
            out->Einv[5] = (E[2] * E[3] - E[0] * E[5]) * id;
            out->Einv[8] = (E[0] * E[4] - E[1] * E[3]) * id;
        }
    }
    return VDW_OK;
}

// Reach of the near image window: every pair (i, j, L) whose distance is below
// it has its L inside |m_a| <= image_max[a] (periodic axes).  A lattice vector
// outside the window has |m_a| >= image_max[a] + 1 on some periodic axis a,
// while two grid points of the cell differ by at most (n_a - 1)/n_a in the
// fractional coordinate along a, so the pair's separation has a fractional
// component of at least image_max[a] + 1/n_a there, i.e. a length of at least
// (image_max[a] + 1/n_a) times the spacing of the lattice planes along a,
// |det(cell)| / |cell[b] x cell[c]|.  Exact on orthorhombic cells.  +inf
// without periodic axes.
double image_reach(const vdw_grid *g, const int32_t *image_max)
{
    double reach = INFINITY;
    const double(*c)[3] = g->cell;
    const double det = c[0][0] * (c[1][1] * c[2][2] - c[1][2] * c[2][1]) -
                       c[0][1] * (c[1][0] * c[2][2] - c[1][2] * c[2][0]) +
                       c[0][2] * (c[1][0] * c[2][1] - c[1][1] * c[2][0]);
    for (int a = 0; a < 3; ++a) {
        if (!g->periodic[a]) continue;
        const double *u = c[(a + 1) % 3], *v = c[(a + 2) % 3];
        const double x = u[1] * v[2] - u[2] * v[1], y = u[2] * v[0] - u[0] * v[2], z = u[0] * v[1] - u[1] * v[0];
        const double height = fabs(det) / sqrt(x * x + y * y + z * z);
        reach = fmin(reach, (image_max[a] + 1.0 / g->n[a]) * height);
    }
    return reach;
}

// 1: the near images hold every pair closer than opts->r_cut (> 0); 0: the
// window leaves out some pair inside the cut, or there is no cut on a
// periodic grid (the window then truncates the sum); -1: no periodic axis.
int image_cut_covered(const vdw_grid *g, const vdw_opts *o, double reach)
{
    if (!g->periodic[0] && !g->periodic[1] && !g->periodic[2]) return -1;
    return (o->r_cut > 0.0 && reach > o->r_cut) ? 1 : 0;
}

int validate_table(const vdw_table_params *tp)
{
    if (!tp) return fail(VDW_EINVAL, "table params are NULL");
    if (tp->n_D < 3) return fail(VDW_EINVAL, "n_D = %d < 3", tp->n_D);
    if (tp->n_sigma < 2) return fail(VDW_EINVAL, "n_sigma = %d < 2", tp->n_sigma);
    if ((int64_t)tp->n_D * tp->n_sigma > (int64_t)1 << 26) return fail(VDW_EINVAL, "table too large");
    if (!(tp->D_max > 0.0) || !isfinite(tp->D_max)) return fail(VDW_EINVAL, "D_max must be > 0");
    if (tp->gl_points < 2 || tp->gl_points > 32) return fail(VDW_EINVAL, "gl_points must be in 2..32");
    if (tp->graded_levels < 0 || tp->graded_levels > 40) return fail(VDW_EINVAL, "graded_levels must be in 0..40");
    if (!(tp->kappa > 0.0) || !(tp->A0 > 0.0) || !isfinite(tp->kappa) || !isfinite(tp->A0))
        return fail(VDW_EINVAL, "kappa and A0 must be > 0");
    if (tp->interp != VDW_INTERP_BILINEAR && tp->interp != VDW_INTERP_CUBIC_D)
        return fail(VDW_EINVAL, "interp must be VDW_INTERP_BILINEAR or VDW_INTERP_CUBIC_D");
    return VDW_OK;
}

int device_info(DevInfo *out)
{
    static thread_local int cached_dev = -1;
    static thread_local DevInfo cached;
    int dev = 0;
    VDW_HIP(hipGetDevice(&dev));
    if (dev != cached_dev) {
        hipDeviceProp_t p;
        VDW_HIP(hipGetDeviceProperties(&p, dev));
        cached.device = dev;
        cached.cus = p.multiProcessorCount;
        cached.lds_per_block = p.sharedMemPerBlock;
        cached_dev = dev;
    }
    *out = cached;
    return VDW_OK;
}

}  // namespace vdw

extern "C" const char *vdw_last_error(void) { return vdw::g_err; }

extern "C" const char *vdw_version(void) { return "vdwdf-mi355x 0.3 (gfx950)"; }

extern "C" int vdw_image_window(const vdw_grid *grid, const vdw_opts *opts, double *reach, int32_t *covers)
{
    int rc = vdw::validate_grid(grid, nullptr);
    if (rc) return rc;
    if (!opts) return vdw::fail(VDW_EINVAL, "opts is NULL");
    if (!reach && !covers) return vdw::fail(VDW_EINVAL, "reach and covers are both NULL");
    for (int a = 0; a < 3; ++a)
        if (opts->image_max[a] < 0) return vdw::fail(VDW_EINVAL, "image_max must be >= 0");
    const double r = vdw::image_reach(grid, opts->image_max);
    if (reach) *reach = r;
    if (covers) *covers = vdw::image_cut_covered(grid, opts, r);
    return VDW_OK;
}
