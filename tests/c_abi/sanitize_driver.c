/*
 * sanitize_driver.c -- test infrastructure: a CPU-only driver that runs the
 * C parts of the test oracle (oracle/vdw_oracle.c, compiled into the same
 * executable) and, when built with -DWITH_LIBVDWDF, the host-only entry
 * points of libvdwdf.so through the plain C caller of tests/c_abi, on small
 * inputs, so that an AddressSanitizer / UndefinedBehaviorSanitizer build
 * exercises their loops and index arithmetic.  No device work: nothing here
 * launches a kernel.  Prints "sanitize driver ok" and returns 0 when every
 * call returned the expected status.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n_D, n_sigma;
    double D_max;
    int32_t gl_points, graded_levels;
    double kappa, A0;
    int32_t interp;
} vo_table_params;

void vo_gauss_legendre(int n, double *x, double *w);
int vo_build_table(const vo_table_params *p, double *phi);
int vo_table_nodes(const vo_table_params *p, long count, const int32_t *k, const int32_t *l, double *out);
int vo_phi_many(long count, const double *D, const double *sigma, const vo_table_params *p, double *out);
double vo_table_interp(const double *tab, const vo_table_params *p, double D, double sigma, double *dD, double *dS);
double vo_self_voxel(double q, const double E[9], int g, const double *tab, const vo_table_params *p, double *dq);
int vo_pair_rows(long npts, const int32_t *ix, const int32_t *iy, const int32_t *iz, const double *n, const double *q,
                 const double h[3], const int32_t gdim[3], const int32_t periodic[3], const int32_t image_max[3],
                 double r_cut, const double *tab, const vo_table_params *p, long nrows, const int64_t *rows,
                 double *S0_cell, double *S0_img, double *Sq);
int vo_pair_rows_cell(long npts, const int32_t *ix, const int32_t *iy, const int32_t *iz, const double *n,
                      const double *q, const double E[9], const int32_t gdim[3], const int32_t periodic[3],
                      const int32_t image_max[3], double r_cut, const double *tab, const vo_table_params *p,
                      long nrows, const int64_t *rows, double *S0_cell, double *S0_img, double *Sq);
double vo_image_pair_sum(long npts, const int32_t *ix, const int32_t *iy, const int32_t *iz, const double *n,
                         const double *q, const double h[3], const int32_t gdim[3], const int32_t m[3], double r_cut,
                         const double *tab, const vo_table_params *p);
double vo_block_sum(long na, const int32_t *ia, long nb, const int32_t *ib, const int32_t *ix, const int32_t *iy,
                    const int32_t *iz, const double *n, const double *q, const double h[3], const int32_t gdim[3],
                    const int32_t periodic[3], const int32_t image_max[3], double r_cut, const double *tab,
                    const vo_table_params *p);
int vo_far_rows(long npts, const int32_t *ix, const int32_t *iy, const int32_t *iz, const double *n, const double *q,
                const double E[9], const int32_t gdim[3], const int32_t periodic[3], const int32_t image_max[3],
                const int32_t far_max[3], long nrows, const int64_t *rows, double *F0, double *Fq);

#ifdef WITH_LIBVDWDF
#include "vdwdf.h"
void vdw_c_demo_table(vdw_table_params *tp);
#endif

static int fails = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++fails;                                                          \
        }                                                                     \
    } while (0)

int main(void)
{
    /* Gauss-Legendre rule and a small table with the cubic interpolant */
    double x[16], w[16];
    vo_gauss_legendre(16, x, w);
    double ws = 0.0;
    for (int i = 0; i < 16; ++i) ws += w[i];
    CHECK(fabs(ws - 2.0) < 1e-13);
    vo_table_params tp = {24, 5, 6.0, 4, 6, 2.0, 16.0, 1};
    double *tab = (double *)malloc(sizeof(double) * 24 * 5);
    CHECK(vo_build_table(&tp, tab) == 0);
    int32_t kk[3] = {0, 11, 23}, ll[3] = {4, 2, 0};
    double nodes[3], Ds[2] = {0.3, 5.9}, Ss[2] = {0.0, 1.0}, ph[2];
    CHECK(vo_table_nodes(&tp, 3, kk, ll, nodes) == 0);
    CHECK(vo_phi_many(2, Ds, Ss, &tp, ph) == 0);
    double dD, dS;
    CHECK(isfinite(vo_table_interp(tab, &tp, 5.99, 0.999, &dD, &dS)));
    const double E[9] = {0.4, 0, 0, 0.1, 0.45, 0, 0, 0.05, 0.5};
    double dq;
    CHECK(isfinite(vo_self_voxel(1.3, E, 4, tab, &tp, &dq)));

    /* a 4 x 3 x 5 grid, every point kept, periodic in x and y */
    enum { NX = 4, NY = 3, NZ = 5, N = NX * NY * NZ };
    int32_t ix[N], iy[N], iz[N];
    double n[N], q[N];
    for (int t = 0; t < N; ++t) {
        ix[t] = t % NX;
        iy[t] = (t / NX) % NY;
        iz[t] = t / (NX * NY);
        n[t] = 0.01 + 0.003 * (t % 7);
        q[t] = 0.4 + 0.05 * (t % 11);
    }
    const double h[3] = {0.4, 0.45, 0.5};
    const int32_t gd[3] = {NX, NY, NZ}, per[3] = {1, 1, 0}, im[3] = {1, 2, 0}, far[3] = {3, 3, 0};
    int64_t rows[5] = {0, 7, 19, 42, N - 1};
    double S0c[N], S0i[N], Sq[N], F0[N], Fq[N];
    CHECK(vo_pair_rows(N, ix, iy, iz, n, q, h, gd, per, im, 1.6, tab, &tp, N, NULL, S0c, S0i, Sq) == 0);
    CHECK(vo_pair_rows(N, ix, iy, iz, n, q, h, gd, per, im, 0.0, tab, &tp, 5, rows, S0c, S0i, Sq) == 0);
    CHECK(vo_pair_rows_cell(N, ix, iy, iz, n, q, E, gd, per, im, 2.0, tab, &tp, 5, rows, S0c, S0i, Sq) == 0);
    const int32_t m0[3] = {0, 0, 0}, m1[3] = {1, -2, 0};
    CHECK(isfinite(vo_image_pair_sum(N, ix, iy, iz, n, q, h, gd, m0, 1.6, tab, &tp)));
    CHECK(isfinite(vo_image_pair_sum(N, ix, iy, iz, n, q, h, gd, m1, 0.0, tab, &tp)));
    int32_t ia[3] = {0, 5, 9}, ib[4] = {1, 2, 30, 59};
    CHECK(isfinite(vo_block_sum(3, ia, 4, ib, ix, iy, iz, n, q, h, gd, per, im, 0.0, tab, &tp)));
    const double Eo[9] = {0.4, 0, 0, 0, 0.45, 0, 0, 0, 0.5};
    CHECK(vo_far_rows(N, ix, iy, iz, n, q, Eo, gd, per, im, far, 5, rows, F0, Fq) == 0);
    free(tab);

#ifdef WITH_LIBVDWDF
    /* host-only paths of the library through its C ABI */
    vdw_table_params t;
    vdw_c_demo_table(&t);
    vdw_grid g;
    vdw_opts o;
    memset(&g, 0, sizeof g);
    memset(&o, 0, sizeof o);
    for (int a = 0; a < 3; ++a) {
        g.n[a] = 12;
        g.cell[a][a] = 4.8;
    }
    g.periodic[0] = 1;
    o.n_cut = 1e-5;
    o.precision = VDW_FP32C;
    o.image_max[0] = 2;
    o.r_cut = 3.0;
    o.table_lds_rows = -1;
    CHECK(enl_workspace_size(&g, &t, &o) > 0);
    double reach = 0.0;
    int32_t covers = 7;
    CHECK(vdw_image_window(&g, &o, &reach, &covers) == VDW_OK && covers == 1 && reach > 3.0);
    CHECK(compute_q0(NULL, 1e-5, NULL, NULL, NULL, NULL, NULL, NULL) == VDW_EINVAL);
    CHECK(strlen(vdw_last_error()) > 0);
    o.precision = 7;
    CHECK(enl_workspace_size(&g, &t, &o) == 0);
    CHECK(strlen(vdw_version()) > 0);
#endif
    if (fails) return 1;
    printf("sanitize driver ok\n");
    return 0;
}
