/*
 * enl_from_c.c -- a plain C99 caller of libvdwdf.so (test infrastructure).
 *
 * It uses nothing but vdwdf.h and the C API of the HIP runtime: no C++, no
 * PyTorch.  vdw_c_demo() evaluates E_c^nl and dE/dn of one density on an
 * orthorhombic grid the way an application would: it sizes and allocates
 * the device buffers and the workspace itself, builds the kernel table,
 * computes the gradient and q0, runs enl_potential on the default stream,
 * copies the results back and frees everything.
 */
#include <hip/hip_runtime_api.h>
#include <string.h>

#include "vdwdf.h"

/* The kernel table of the demo: 256 x 16 nodes on D <= 16, a light
 * quadrature rule (6 points per panel, 8 graded levels, kappa 2, A0 20). */
void vdw_c_demo_table(vdw_table_params *tp)
{
    tp->n_D = 256;
    tp->n_sigma = 16;
    tp->D_max = 16.0;
    tp->gl_points = 6;
    tp->graded_levels = 8;
    tp->kappa = 2.0;
    tp->A0 = 20.0;
    tp->interp = VDW_INTERP_BILINEAR;
}

/* n3, h: grid points and spacings per axis; periodic, image_max: as in
 * vdw_grid / vdw_opts; n: host density (x fastest); E: host, 3 doubles;
 * dEdn: host, n3[0] n3[1] n3[2] doubles.  Returns VDW_OK or the first
 * failing status (a failed HIP allocation or copy as VDW_EHIP). */
int vdw_c_demo(const int32_t n3[3], const double h[3], const int32_t periodic[3], const int32_t image_max[3],
               double n_cut, int32_t precision, const double *n, double *E, double *dEdn)
{
    vdw_grid g;
    vdw_table_params tp;
    vdw_opts o;
    double *phi_d = NULL, *n_d = NULL, *grad_d = NULL, *q0_d = NULL, *dqdn_d = NULL, *dqdg_d = NULL;
    double *dEdn_d = NULL;
    float *phi_f = NULL;
    void *ws = NULL;
    size_t G, wsb, ntab;
    int a, rc = VDW_OK;

    memset(&g, 0, sizeof g);
    memset(&o, 0, sizeof o);
    for (a = 0; a < 3; ++a) {
        g.n[a] = n3[a];
        g.cell[a][a] = h[a] * n3[a];
        g.periodic[a] = periodic[a];
        o.image_max[a] = image_max[a];
    }
    g.gradient = VDW_GRAD_FD;
    o.n_cut = n_cut;
    o.precision = precision;
    o.self_term = 1;
    o.table_lds_rows = -1;
    vdw_c_demo_table(&tp);

    G = (size_t)n3[0] * (size_t)n3[1] * (size_t)n3[2];
    ntab = (size_t)tp.n_D * (size_t)tp.n_sigma;
    wsb = enl_workspace_size(&g, &tp, &o);
    if (wsb == 0) return VDW_EINVAL;
    if (hipMalloc((void **)&phi_d, ntab * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&phi_f, ntab * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&n_d, G * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&grad_d, 3 * G * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&q0_d, G * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&dqdn_d, G * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&dqdg_d, G * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&dEdn_d, G * sizeof(double)) != hipSuccess || hipMalloc(&ws, wsb) != hipSuccess) {
        rc = VDW_EHIP;
        goto out;
    }
    if (hipMemcpy(n_d, n, G * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        rc = VDW_EHIP;
        goto out;
    }
    rc = build_phi_table(&tp, phi_d, phi_f, NULL);
    if (rc) goto out;
    rc = compute_q0(&g, n_cut, n_d, grad_d, q0_d, dqdn_d, dqdg_d, NULL);
    if (rc) goto out;
    rc = enl_potential(&g, n_d, q0_d, grad_d, dqdn_d, dqdg_d, phi_d, phi_f, &tp, &o, ws, wsb, dEdn_d, E, NULL);
    if (rc) goto out;
    if (hipMemcpy(dEdn, dEdn_d, G * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) rc = VDW_EHIP;
out:
    (void)hipFree(ws);
    (void)hipFree(dEdn_d);
    (void)hipFree(dqdg_d);
    (void)hipFree(dqdn_d);
    (void)hipFree(q0_d);
    (void)hipFree(grad_d);
    (void)hipFree(n_d);
    (void)hipFree(phi_f);
    (void)hipFree(phi_d);
    return rc;
}
