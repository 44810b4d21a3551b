/*
 * vdwdf.h -- C ABI of libvdwdf.so, the MI355X (gfx950) implementation of the
 * vdW-DF nonlocal correlation energy and its potential.
 *
 * The method is the one of Lazic et al., "JuNoLo - Julich Non Local code for
 * parallel calculation of vdW-DF nonlocal density functional theory"
 * (arXiv:0810.2273):
 *   - Sec. 2, Eq. (1): E_c^nl = 1/2 int int n(r) phi(r, r') n(r') d^3r d^3r';
 *     the kernel depends on D >= 0 and |delta| < 1 and is the double integral
 *     of Dion et al. (their Eq. 14), with their large-D asymptote (Eq. 17).
 *   - Sec. 2, Eq. (2): on the density grid the integral is the double sum
 *     E = 1/2 sum_i sum_j n_i phi_ij n_j (times dV^2, the volume elements).
 *   - Sec. 3: the gradient of n (finite differences, or the Fourier
 *     derivative the paper's code takes by FFT), a density cut-off below
 *     which points are dropped, the sum over the 0th cell, then over
 *     periodic repetitions of it.
 *   - Eq. (3): the recombination with the LDA and GGA exchange-correlation
 *     energies, which the paper's code also evaluates.
 *
 * Conventions for every entry point:
 *   - Units are Hartree atomic units (bohr, Hartree, electrons/bohr^3).
 *   - Grid arrays are FP64, x fastest: index = ix + nx (iy + ny iz).
 *   - Pointers named *_d are DEVICE pointers (HIP global memory on the
 *     current device); E_out is HOST memory.  The caller owns every buffer;
 *     the library allocates nothing on these paths.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Work is enqueued asynchronously on it; the entry points that
 *     write E_out synchronise that stream before returning.
 *   - Every function returns VDW_OK (0) or a negative status; inputs are
 *     validated on the host before anything is launched, and a failed call
 *     leaves output buffers unspecified.  vdw_last_error() returns a
 *     thread-local message describing the last failure.
 *   - Calls on one stream are ordered; concurrent calls on different
 *     streams must use different workspaces.
 */
#ifndef VDWDF_H
#define VDWDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VDW_OK = 0,
    VDW_EINVAL = -1,        /* bad argument: null pointer, size, parameter range  */
    VDW_ENOMEM = -2,        /* host allocation failed (batch plan object)         */
    VDW_EHIP = -3,          /* a HIP runtime call failed                          */
    VDW_EUNSUPPORTED = -4,  /* valid but not offered (e.g. the cubic-in-D table with Kahan runs) */
    VDW_EWORKSPACE = -5,    /* workspace smaller than enl_workspace_size()        */
    VDW_ENONFINITE = -6     /* NaN or Inf found in the density                    */
};

enum { VDW_FP64 = 0, VDW_FP32C = 1 };

/* Equidistant grid (Sec. 2).  cell[a] is the a-th cell vector (bohr); grid
 * point (i, j, k) sits at i e_0 + j e_1 + k e_2, e_a = cell[a] / n[a].  Any
 * non-degenerate cell is accepted: orthorhombic (cell[a][b] = 0 for a != b,
 * cell[a][a] > 0) or skew, like the hexagonal cell of the sample run
 * (App. A).  On skew cells the finite differences are taken along the grid
 * axes and mapped to Cartesian components by the inverse of the step
 * matrix, and pair distances use the full metric e_a . e_b.  periodic[a] = 1
 * marks a periodic axis (the input's perx/pery/perz, App. A); images are
 * whole cell translations.  Every n[a] must be >= 3.
 * gradient selects the derivative along periodic axes: VDW_GRAD_FD (0,
 * second-order differences everywhere) or VDW_GRAD_SPECTRAL (1, the
 * Fourier derivative, i.e. the FFT gradient of the paper's code, on
 * periodic axes of at most 4096 points; open axes keep the differences).
 * Every entry point that takes grids accepts the spectral form (batch
 * plans then need grad_d, where the derivatives are staged). */
enum { VDW_GRAD_FD = 0, VDW_GRAD_SPECTRAL = 1 };

typedef struct {
    int32_t n[3];
    double  cell[3][3];
    int32_t periodic[3];
    int32_t gradient;
} vdw_grid;

/* The kernel table (Sec. 2; node counts and limits are free parameters,
 * Sec. 7).  Nodes D_k = k D_max/(n_D-1), sigma_l = l/(n_sigma-1) with
 * sigma = delta^2; row-major phi[k * n_sigma + l].  The quadrature rule that
 * fills it (the same rule the test oracle implements):
 *   phi(d1,d2) = 2/pi^2 sum_i sum_j w_i w_j a_i^2 a_j^2 W(a_i,a_j)
 *                T(nu(a_i), nu(a_j), nu'(a_i), nu'(a_j)),
 *   d1 = D(1+delta), d2 = D(1-delta); nodes: gl_points Gauss-Legendre points
 *   on each panel [0, w 2^-K], [w 2^-(j+1), w 2^-j] (j = K-1..0), then
 *   [t w, (t+1) w] up to A, with w = pi/2, K = graded_levels, and A the
 *   smallest odd multiple of w with A >= max(A0, kappa max(d1, d2)).
 * Row 0 (D = 0, where phi diverges like -ln D) is the linear extrapolation
 * 2 phi(D_1) - phi(D_2).  Defaults: gl_points 8, graded_levels 12,
 * kappa 16, A0 512: doubling kappa, A0 and gl_points moves no node of a
 * 48-bohr table by more than 1e-7 relative (away from the zero crossing of
 * phi near D = 2), the refinement test of Sec. 7.  The builder needs about
 * 1.1e12 integrand evaluations for 2048 x 64 nodes on [0, 48]; the rule may
 * not need more than 2^20 points per axis at D_max (VDW_EINVAL). */
typedef struct {
    int32_t n_D;
    int32_t n_sigma;
    double  D_max;
    int32_t gl_points;      /* 2..32 */
    int32_t graded_levels;  /* 0..40 */
    double  kappa;          /* > 0   */
    double  A0;             /* > 0   */
    int32_t interp;         /* VDW_INTERP_BILINEAR (0) or VDW_INTERP_CUBIC_D (1):
                               the pair and on-site terms read the table
                               bilinearly, or cubic in D (Catmull-Rom form of
                               each sigma column, rows beyond the ends
                               extrapolated linearly; C1 in D) and linear in
                               sigma, in either precision (not with Kahan
                               runs: VDW_EUNSUPPORTED). */
} vdw_table_params;

enum { VDW_INTERP_BILINEAR = 0, VDW_INTERP_CUBIC_D = 1 };

/* Options of the energy / potential evaluation. */
typedef struct {
    double  n_cut;          /* points with n < n_cut are dropped (Sec. 3); > 0    */
    double  r_cut;          /* pair distance cut (bohr) applied to every (i,j,L);
                               <= 0: none                                          */
    int32_t image_max[3];   /* images |m_a| <= image_max[a] on periodic axes      */
    int32_t precision;      /* VDW_FP64 or VDW_FP32C (FP32 pair terms with
                               compensated FP32 runs carried in FP64)             */
    int32_t self_term;      /* on-site term E_self (below): 1 the sphere form,
                               2 the voxel double average, 0 none             */
    int32_t table_lds_rows; /* rows of the table kept in LDS; -1: as many as fit  */
    int32_t block_threads;  /* pair-kernel workgroup size: 1024 (row blocks of
                               4096 points for FP32C with n_sigma = 64 and no
                               images, else 2048); 512 (eight i-points per
                               lane, the same blocks; FP32C with n_sigma = 64
                               and no images, else 1024); 256 (blocks of 512;
                               no images, else 1024); 0: auto (256 when, with
                               every grid point kept, the 1024-thread work
                               list at 1024-point chunks has fewer than 128
                               items and there are no images; else 1024).
                               Skew cells: always 1024 threads with blocks
                               of 2048.                                       */
    int32_t j_chunks;       /* j-points per off-diagonal work item, in units of
                               1024 (1..64); 0: auto (the longest of 8, 4, 2,
                               1 whose work list, with every grid point kept,
                               has at least 4096 items; else 1).  Chunks
                               shorter than a row block split its diagonal
                               work into (block / chunk) items.               */
    int32_t grid_blocks;    /* persistent workgroups; 0: auto (all CUs)           */
    int32_t kahan;          /* 1: Kahan-compensate the FP32 runs (FP32C only)     */
    int32_t far_max[3];     /* far image shell (Sec. 7: the large-D form of the
                               kernel for the far repeated cells): the images
                               with |m_a| <= far_max[a] on periodic axes that
                               are not near images (image_max) enter with the
                               asymptote -C/(d1^2 d2^2 (d1^2 + d2^2)) whatever
                               D; all 0 (or 0 on every periodic axis): none.
                               With a shell: r_cut <= 0, far_max[a] >=
                               image_max[a] on every periodic axis, at most
                               2^22 lattice vectors.  The asymptote is meant
                               for distant cells: with two near rings it
                               moves a Xe monolayer's E_pairL by 1e-6 of
                               itself, with one ring by 2e-4, with none it
                               replaces the nearest neighbours' kernel.       */
} vdw_opts;

/* Thread-local description of the last error (never NULL). */
const char *vdw_last_error(void);

/* Library version string.  0.2: vdw_opts.far_max and the far-shell fields
 * of vdw_stats; 0.3: the image-window fields of vdw_stats (the structs grew
 * at their ends). */
const char *vdw_version(void);

/* ---------------------------------------------------------------------
 * build_phi_table -- fill the kernel table on the device (Sec. 2, the
 * double integral of Dion et al.), in FP64.
 *   phi_d: device, n_D * n_sigma doubles (written).
 *   phi_f: device, n_D * n_sigma floats, or NULL (FP32 copy for the
 *          VDW_FP32C pair kernel).
 * The Gauss-Legendre points of one panel are computed on the host and
 * passed as kernel arguments, so nothing is allocated; synchronises
 * `stream`.
 * Errors: VDW_EINVAL (null phi_d, n_D < 3, n_sigma < 2, D_max <= 0,
 * quadrature parameters out of range), VDW_EHIP.
 * ------------------------------------------------------------------- */
int build_phi_table(const vdw_table_params *tp, double *phi_d, float *phi_f, void *stream);

/* ---------------------------------------------------------------------
 * compute_q0 -- density gradient and q0 on every grid point (Sec. 3; q0 of
 * Dion et al. from the LDA exchange and Perdew-Wang 1992 correlation plus
 * the gradient term):
 *   grad n:  along each grid axis second-order central differences with
 *            periodic wrap on periodic axes and second-order one-sided
 *            differences at the faces of non-periodic axes, or the Fourier
 *            derivative on periodic axes (grid->gradient); divided by the
 *            spacing on orthorhombic cells, mapped by the inverse step
 *            matrix on skew cells (Cartesian components);
 *   q0 = k_F - (4 pi/3) eps_c^PW92(r_s) - (Z_ab/36) |grad n|^2 / (k_F n^2),
 *        Z_ab = -0.8491, where n >= n_cut; 0 elsewhere.
 *   n_d:     device, G doubles (read).
 *   grad_d:  device, 3G doubles (planes d/dx, d/dy, d/dz), or NULL (not
 *            with the spectral gradient, which stages its derivatives
 *            there).
 *   q0_d:    device, G doubles (written).
 *   dq_dn_d: device, G doubles, or NULL: dq0/dn at fixed |grad n|^2.
 *   dq_dg_d: device, G doubles, or NULL: dq0/d(|grad n|^2).
 * Errors: VDW_EINVAL (null pointers, n_cut <= 0, n[a] < 3, degenerate
 * cell), VDW_EHIP.
 * ------------------------------------------------------------------- */
int compute_q0(const vdw_grid *grid, double n_cut, const double *n_d, double *grad_d, double *q0_d,
               double *dq_dn_d, double *dq_dg_d, void *stream);

/* ---------------------------------------------------------------------
 * xc_energies -- the local and semilocal exchange-correlation energies that
 * the recombination of Eq. (3) needs (the paper's code evaluates them from
 * the same density, Sec. 3), spin-unpolarised, in Hartree:
 *   E[0] E_x^LDA     = dV sum n eps_x,           eps_x = -3 k_F / (4 pi)
 *   E[1] E_c^LDA     = dV sum n eps_c^PW92(r_s)
 *   E[2] E_x^PBE     = dV sum n eps_x F_x(s),    F_x = 1 + k - k / (1 + mu s^2 / k),
 *                      k = 0.804, mu = beta pi^2 / 3, s = |grad n| / (2 k_F n)
 *   E[3] E_c^PBE     = dV sum n (eps_c^PW92 + H(r_s, t)),
 *                      H = gamma ln(1 + (beta/gamma) t^2 (1 + A t^2) / (1 + A t^2 + A^2 t^4)),
 *                      A = (beta/gamma) / (exp(-eps_c/gamma) - 1), t = |grad n| / (2 k_s n),
 *                      k_s = sqrt(4 k_F / pi), beta = 0.06672455060314922, gamma = (1 - ln 2) / pi^2
 *   E[4] E_x^revPBE  = E_x^PBE with k = 1.245
 * over the grid points with n > n_floor (others, negative densities
 * included, add nothing); grad n as in compute_q0.
 *   n_d:     device, G doubles (read).
 *   n_floor: finite, >= 0 (1e-12 is a safe choice: near n = 0 the gradient
 *            terms overflow).
 *   ws:      device workspace of xc_workspace_size(grid) bytes.
 *   E:       host, 5 doubles, written after `stream` has been synchronised.
 * Errors: VDW_EINVAL (null pointers, n_floor < 0 or not finite, bad grid),
 * VDW_EWORKSPACE, VDW_ENONFINITE
 * (an energy is not finite; E is still written), VDW_EHIP.
 * ------------------------------------------------------------------- */
size_t xc_workspace_size(const vdw_grid *grid);
int xc_energies(const vdw_grid *grid, const double *n_d, double n_floor, void *ws, size_t ws_bytes, double *E,
                void *stream);

/* Eq. (3): E_tot^NL = E_tot^DFT - E_x^PBE - E_c^PBE + (E_x + E_c^LDA + E_c^NL),
 * with E_x = E_x^PBE (exchange = 0) or E_x^revPBE (exchange = 1), E_xc the
 * five energies of xc_energies and E_nl = E_pair0 + E_pairL + E_self.  With
 * E_dft = 0 this is the correction to add to a PBE total energy.  NaN for a
 * NULL E_xc or another exchange value. */
double vdw_recombine(const double *E_xc, double E_nl, double E_dft, int32_t exchange);

/* Bytes of device workspace enl_energy / enl_potential need for this grid
 * and these options (an upper bound that holds for any density). */
size_t enl_workspace_size(const vdw_grid *grid, const vdw_table_params *tp, const vdw_opts *opts);

/* ---------------------------------------------------------------------
 * enl_energy -- E_c^nl of Eq. (2) over the retained points S = {n >= n_cut}
 * (Sec. 3), with phi~ the table interpolant (bilinear in (D, sigma)) for
 * D < D_max and -C/(d1^2 d2^2 (d1^2 + d2^2)), C = 12 (4 pi/9)^3, beyond:
 *   E_pair0 = 1/2 dV^2 sum_{i != j in S} n_i n_j phi~(q_i, q_j, |r_i - r_j|)
 *   E_pairL = 1/2 dV^2 sum_{i, j in S} sum_{L != 0} n_i n_j phi~(.., |r_i - r_j - L|)
 *   E_self  = 1/2 dV^2 sum_{i in S} n_i^2 Phi(q_i), with (opts->self_term)
 *     1: Phi(q) = phi~(q rho_s, 0), rho_s = (3 dV / 4 pi)^(1/3) e^(-1/3)
 *        (the log kernel averaged over the sphere of volume dV);
 *     2: Phi(q) = int_{[-1,1]^3} phi~(q |sum_a t_a e_a|, 0) prod_a (1 - |t_a|) dt,
 *        the double average over the grid cell (e_a its step vectors), by
 *        8 octants with t_a = +-u^2 at 8 Gauss-Legendre nodes u of [0, 1]
 *        (4096 kernel values per kept point; a reading of the paper's phi0
 *        step, App. A);
 *     0: none.
 * L runs over the images selected by opts->image_max on periodic axes
 * (Sec. 3, periodic problems), and every (i, j, L) with a distance above
 * opts->r_cut (if > 0) is dropped.  With a far image shell
 * (opts->far_max) E_pairL also holds
 *   1/2 dV^2 sum_{i, j in S} n_i n_j (-C) T(r_i - r_j) / (q_i^2 q_j^2 (q_i^2 + q_j^2)),
 *   T(d) = sum_{L in shell} |d - L|^-6  (i = j included),
 * the asymptote summed over the shell's images (one O(N^2) pass over a
 * table of T at every grid displacement, whatever the shell's size).  dV = |det(cell)| / G (hx hy hz on
 * orthorhombic cells).
 *   n_d, q0_d: device, G doubles (q0 from compute_q0).
 *   phi_d:     device FP64 table (always required: the on-site term and the
 *              VDW_FP64 pair kernel read it).
 *   phi_f:     device FP32 table (required for VDW_FP32C, else ignored).
 *   ws, ws_bytes: device workspace of at least enl_workspace_size() bytes.
 *   E_out:     host, 3 doubles: {E_pair0, E_pairL, E_self} (Hartree).
 * Errors: VDW_EINVAL, VDW_EUNSUPPORTED (the cubic-in-D table with
 * Kahan runs), VDW_EWORKSPACE, VDW_EHIP.
 * ------------------------------------------------------------------- */
int enl_energy(const vdw_grid *grid, const double *n_d, const double *q0_d, const double *phi_d,
               const float *phi_f, const vdw_table_params *tp, const vdw_opts *opts, void *ws,
               size_t ws_bytes, double *E_out, void *stream);

/* ---------------------------------------------------------------------
 * enl_potential -- the energy of enl_energy and its derivative
 *   dEdn_d[k] = dE / dn_k  at every grid point k,
 * through n directly, through q0(n, |grad n|^2) and through the gradient
 * stencil (dropped points pick up their share via the transposed stencil).
 * The potential is v_nl = dEdn / dV.
 *   grad_d, dq_dn_d, dq_dg_d: device, from compute_q0 on the same density.
 *   dEdn_d: device, G doubles (written).
 * Other arguments and errors as enl_energy.
 * ------------------------------------------------------------------- */
int enl_potential(const vdw_grid *grid, const double *n_d, const double *q0_d, const double *grad_d,
                  const double *dq_dn_d, const double *dq_dg_d, const double *phi_d, const float *phi_f,
                  const vdw_table_params *tp, const vdw_opts *opts, void *ws, size_t ws_bytes,
                  double *dEdn_d, double *E_out, void *stream);

/* ---------------------------------------------------------------------
 * enl_potential_noalloc -- enl_potential for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same kernels and results, with
 * the workspace taken from a static device array of the library instead of
 * the caller (64 MiB on every GPU the library runs on, held until the
 * process ends; enough for grids of about 40^3 points in either precision).
 * Nothing is allocated on the device; the first call on a device looks up
 * that device's copy of the array.  Every call on one GPU shares the array:
 * calls that overlap on one GPU (other host threads, other streams) race and
 * give wrong results, so the caller serialises them.  The array keeps the
 * last call's contents; each call clears what it needs.
 *   Arguments as enl_potential, without ws and ws_bytes.
 * Errors as enl_potential; VDW_EWORKSPACE when the grid and options need
 * more than the static array (enl_workspace_size() > 64 MiB).
 * ------------------------------------------------------------------- */
int enl_potential_noalloc(const vdw_grid *grid, const double *n_d, const double *q0_d, const double *grad_d,
                          const double *dq_dn_d, const double *dq_dg_d, const double *phi_d, const float *phi_f,
                          const vdw_table_params *tp, const vdw_opts *opts, double *dEdn_d, double *E_out,
                          void *stream);

/* Bytes of workspace enl_potential_batched needs for these B grids. */
size_t enl_batched_workspace_size(int32_t B, const vdw_grid *grids, const vdw_table_params *tp,
                                  const vdw_opts *opts);

/* ---------------------------------------------------------------------
 * enl_potential_batched -- enl_potential for B independent densities of
 * uneven sizes in one pass: one compaction over the packed grids, then one
 * persistent pair-kernel launch that takes (density, i-block, j-chunk)
 * work items from a shared list, then per-density reductions.
 *   grids:    host, B grid descriptors (each non-periodic or periodic as
 *             for enl_potential; opts apply to all).
 *   grid_off: host, B+1 offsets: density b occupies elements
 *             [grid_off[b], grid_off[b+1]) of the packed n/q0/dq/dEdn
 *             arrays, and 3 planes of that size in grad_d at offset
 *             3*grid_off[b].
 *   E_out:    host, 3B doubles, {E_pair0, E_pairL, E_self} per density.
 * Errors as enl_potential; VDW_EINVAL when offsets do not match the grids.
 * ------------------------------------------------------------------- */
int enl_potential_batched(int32_t B, const vdw_grid *grids, const int64_t *grid_off, const double *n_d,
                          const double *q0_d, const double *grad_d, const double *dq_dn_d,
                          const double *dq_dg_d, const double *phi_d, const float *phi_f,
                          const vdw_table_params *tp, const vdw_opts *opts, void *ws, size_t ws_bytes,
                          double *dEdn_d, double *E_out, void *stream);

/* ---------------------------------------------------------------------
 * Batch plans -- the batched evaluation of enl_potential_batched split into
 * a set-up step and a step that only launches kernels, so that a whole
 * evaluation (gradient and q0 of every density, compaction, the persistent
 * pair kernel over the shared work list, reductions, adjoint assembly; the
 * same kernels and results as enl_potential_batched) can be recorded into
 * a HIP graph and replayed, e.g. once per iteration of a self-consistent
 * loop whose density buffer is rewritten in place.
 *
 * enl_batch_plan_create: validates the arguments, lays out the work for
 *   these B grids (grid_off as for enl_potential_batched, always required;
 *   potential = 1 for energy + dEdn, 0 for the energy only) and copies the
 *   descriptors into the workspace `ws` (enl_batched_workspace_size bytes),
 *   synchronising `stream`.  *plan receives a host object that keeps
 *   pointing at `ws`: the workspace must outlive the plan and may not be
 *   used by any other call meanwhile.
 * enl_batch_plan_execute: enqueues one evaluation on `stream`: kernel
 *   launches only (no copies, host waits or allocation).  It computes
 *   grad_d (3 planes per density, as compute_q0), q0_d, dq_dn_d, dq_dg_d
 *   (device, packed like n_d; grad_d, dq_dn_d, dq_dg_d and dEdn_d may be
 *   NULL for an energy-only plan, grad_d only if no grid takes the
 *   spectral gradient) and writes
 *     E_d: device, 4B+1 doubles: {E_pair0, E_pairL, E_self} for each
 *          density, then the B retained-point counts, then a flag that is
 *          non-zero when the density held NaN or Inf values.
 *   Nothing is read back: the caller checks the flag.
 * enl_batch_plan_capture: records one execute with these buffers into a
 *   graph held by the plan (on a private stream; any earlier graph is
 *   dropped).  The graph keeps the buffer addresses; new inputs go into
 *   the same buffers.
 * enl_batch_plan_replay: launches the recorded graph on `stream`.
 *   Replays, executes and other calls on the same workspace are ordered
 *   only by their streams; overlapping ones race.
 * enl_batch_plan_destroy: frees the plan and its graph (NULL is a no-op).
 * Errors: as enl_potential_batched; VDW_EINVAL for a NULL plan, a replay
 * without a capture or missing buffers; VDW_EHIP for failed graph calls.
 * ------------------------------------------------------------------- */
typedef struct vdw_batch_plan vdw_batch_plan;

int enl_batch_plan_create(int32_t B, const vdw_grid *grids, const int64_t *grid_off, const vdw_table_params *tp,
                          const vdw_opts *opts, int32_t potential, void *ws, size_t ws_bytes,
                          vdw_batch_plan **plan, void *stream);
int enl_batch_plan_execute(vdw_batch_plan *plan, const double *n_d, double *grad_d, double *q0_d,
                           double *dq_dn_d, double *dq_dg_d, const double *phi_d, const float *phi_f,
                           double *dEdn_d, double *E_d, void *stream);
int enl_batch_plan_capture(vdw_batch_plan *plan, const double *n_d, double *grad_d, double *q0_d,
                           double *dq_dn_d, double *dq_dg_d, const double *phi_d, const float *phi_f,
                           double *dEdn_d, double *E_d);
int enl_batch_plan_replay(vdw_batch_plan *plan, void *stream);
int enl_batch_plan_destroy(vdw_batch_plan *plan);

/* ---------------------------------------------------------------------
 * Diagnostics of the last enl_* call on this host thread (after it
 * returned VDW_OK): retained points, logical pairs (ordered (i, j, L),
 * self pair excluded, before the distance cut), and kernel times of the
 * pair kernel and of the far-shell kernels in milliseconds measured with
 * HIP events on `stream` (0 unless timing was enabled with
 * vdw_set_timing(1)).
 * ------------------------------------------------------------------- */
typedef struct {
    int64_t retained;
    double  pairs;
    float   pair_kernel_ms;
    int32_t lds_rows;
    int32_t block_threads;
    int32_t j_chunks;
    int32_t grid_blocks;
    int32_t diag_items;     /* diagonal work items per row block */
    double  far_pairs;      /* ordered pairs (i, j) of the far-shell pass (N^2), or 0 */
    float   far_kernel_ms;  /* far-shell table and row kernels (timing on), or 0 */
    /* since 0.3: how far the near images reach and how far the far shell is
     * from the table (Sec. 3 periodic repetition; Sec. 7 asymptote) */
    double  image_reach;    /* every pair (i, j, L) closer than this (bohr) is
                               summed by the near images (vdw_image_window);
                               +inf without periodic axes */
    int32_t image_cut_covered; /* 1: image_reach > r_cut, every pair inside
                               the cut is summed; 0: the image window leaves
                               out pairs inside the cut (or truncates the sum
                               when there is no cut); -1: no periodic axis */
    double  q0_min;         /* smallest q0 over the kept points (1/bohr) */
    double  far_D_min;      /* a lower bound on D = (q_i + q_j) r / 2 over the
                               far-shell pairs, q0_min * image_reach (0 without
                               a far shell): the shell's asymptote is exact only
                               where D >= D_max, so far_D_min < D_max marks the
                               shell as an approximation */
} vdw_stats;

int vdw_last_stats(vdw_stats *out);

/* The near image window of a grid and options, from the geometry alone
 * (Sec. 3, periodic repetition): *reach (bohr, may be NULL) is a distance
 * below which every pair (i, j, L) has its image L inside |m_a| <=
 * image_max[a] on the periodic axes: min over periodic axes of
 * (image_max[a] + 1/n[a]) times the spacing of the lattice planes along a
 * (|det(cell)| / |cell[b] x cell[c]|; exact on orthorhombic cells), +inf
 * without periodic axes.  *covers (may be NULL) is image_cut_covered of
 * vdw_stats.  Host only; no device work.
 * Errors: VDW_EINVAL (bad grid, NULL opts, negative image_max, both outputs
 * NULL). */
int vdw_image_window(const vdw_grid *grid, const vdw_opts *opts, double *reach, int32_t *covers);
void vdw_set_timing(int32_t on);

#ifdef __cplusplus
}
#endif

#endif /* VDWDF_H */
