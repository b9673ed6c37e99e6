/*
 * twmg -- tweed / wireframe geometric multigrid for the nonuniform-grid Poisson
 * equation on MI355X (gfx950).  C ABI of libtwmg.so.
 *
 * The problem (arXiv 2110.08389, Section 2, problem (CP)/(DP)): on a stretched
 * tensor grid with (n_x+1) x (n_y+1) [x (n_z+1)] nodes, find u with
 *     W_i u_{i-1,j} + E_i u_{i+1,j} + S_j u_{i,j-1} + N_j u_{i,j+1} [+ B_l, T_l] + C u_{i,j} = f_{i,j}
 * at every interior node and u = g on the boundary nodes, where
 * W_i = 1/(dx_i dx_{i-1/2}), E_i = 1/(dx_i dx_{i+1/2}) (likewise S, N, B, T) and C is
 * minus the sum of the others.  The solver is the multigrid cycle of Section 4
 * (V-cycle, gamma = 2 for a W-cycle) with full-weighting restriction and
 * bilinear (trilinear) prolongation, smoothed by the block relaxations of
 * Section 3 (tweed, wireframe, checkerboard, zebra, alternating schemes) and
 * Section 7 (3D tweed).
 *
 * Arrays.  Every array argument is a DEVICE pointer to a full node array
 * (boundary nodes included), row-major with x fastest:
 *     index = ((b*(n_z+1) + l)*(n_y+1) + j)*(n_x+1) + i,
 * b = batch index (the batch problems share one grid).  n_z = 0 in 2D.  All
 * element types are double unless a name says f32.  The caller owns all
 * arrays it passes; the library never frees them.
 *
 * Streams.  All device work is enqueued on the stream given to mg_setup (or
 * mg_set_stream); a handle must not be used from two host threads at once.
 * mg_solve and mg_solve_adjoint synchronise that stream once per cycle to read
 * the defect norm; the other calls are asynchronous.
 *
 * Errors.  Every int-returning call returns MG_OK (0) or one of the MG_E*
 * codes below; mg_strerror gives a message.  No exception crosses the ABI.
 */
#ifndef TWMG_H
#define TWMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MG_OK = 0,
    MG_EINVAL = 1,     /* bad argument: sizes, kinds, null pointers           */
    MG_ENOMEM = 2,     /* device or host allocation failed / workspace short  */
    MG_EHIP = 3,       /* a HIP runtime call or kernel launch failed          */
    MG_ENOTCONV = 4,   /* tolerance not met within max_cycles (u is valid)    */
    MG_EDIVERGED = 5,  /* NaN/Inf or defect above 1e6 times the initial one   */
    MG_EUNSUPPORTED = 6 /* valid request this build does not provide          */
};

/* Grid stretching (Section 5).  MG_TANH_WALL: eq. (tanh), clustering at both
 * walls; MG_TANH_CENTRE: eq. (tanh_inv), clustering at the centre;
 * MG_SINH_CENTRE: x = L(1/2 + sinh(b(2i/n-1))/(2 sinh b)); MG_EXPLICIT: node
 * coordinates given by the caller (host array of n+1 increasing values). */
typedef enum { MG_UNIFORM = 0, MG_TANH_WALL = 1, MG_TANH_CENTRE = 2, MG_SINH_CENTRE = 3, MG_EXPLICIT = 4 } mg_stretch_kind;

/* Smoothers (Section 3; Section 7 for 3D tweed).  MG_ADZ is alternating-
 * direction zebra (x then y [then z] line sweeps); MG_ALT_TW alternates a tweed
 * and a wireframe sweep.  For these two, one relaxation (one count of nu) is
 * the whole group of sweeps, as in the paper's tables. */
typedef enum {
    MG_TWEED = 0, MG_WIREFRAME = 1, MG_CHECKERBOARD = 2, MG_ZEBRA_X = 3, MG_ZEBRA_Y = 4, MG_ZEBRA_Z = 5,
    MG_ADZ = 6, MG_ALT_TW = 7
} mg_smoother;

enum { MG_FP64 = 0, MG_FP32_IR = 1 };          /* mg_options.precision */
enum { MG_INITIAL_GUESS = 1u };                /* mg_options.flags     */

typedef struct {
    int dim;          /* 2 or 3                                                      */
    int n[3];         /* cells per axis: even, n = 2^p * a; n[2] ignored in 2D        */
    double L[3];      /* domain lengths                                               */
    int batch;        /* independent problems sharing the grid (>= 1)                 */
} mg_grid;

/* Grid and medium.  sigma[a] (optional, host, n[a] positive finite values)
 * is the conductivity along axis a, one value per cell [x_k, x_{k+1}]: the
 * axis-wise heterogeneous, anisotropic form of problem (CP) of Section 2
 * with sigma_ij = diag(s_x(x), s_y(y)[, s_z(z)]) (no cross terms), discretised
 * in flux form, W_i = s_{i-1/2}/(dx_i dx_{i-1/2}), E_i = s_{i+1/2}/(dx_i
 * dx_{i+1/2}); a coarse cell takes the series conductance of its two fine
 * cells, (h0 + h1)/(h0/s0 + h1/s1).  NULL means s = 1 (problem (DP)). */
typedef struct {
    int kind[3];            /* mg_stretch_kind per axis                              */
    double param[3];        /* c (tanh) or b (sinh) per axis                         */
    const double *coords[3];/* MG_EXPLICIT: host arrays of n[a]+1 coordinates        */
    const double *sigma[3]; /* optional: host arrays of n[a] cell conductivities     */
} mg_stretching;

typedef struct {
    int smoother;     /* mg_smoother                                                  */
    int nu1, nu2;     /* pre/post relaxations                                         */
    int gamma;        /* 1 = V-cycle, 2 = W-cycle                                     */
    int precision;    /* MG_FP64, or MG_FP32_IR: FP32 cycles inside FP64 refinement    */
    int max_cycles;   /* cap on cycles (or refinement steps) per solve                */
    unsigned flags;   /* MG_INITIAL_GUESS: keep u's interior as the start             */
} mg_options;

typedef struct {
    int cycles;       /* cycles (refinement steps) done                               */
    int status;       /* MG_OK, MG_ENOTCONV or MG_EDIVERGED                           */
    double rel_res;   /* final ||f - L u||_inf / ||f - L u_0||_inf (interior nodes;   *
                       * each problem against its own, the largest over the batch)   */
    double res0;      /* ||f - L u_0||_inf (largest over the batch)                   */
    double *history;  /* optional host array: rel_res after each cycle                */
    int history_cap;  /* its capacity                                                 */
    double ms;        /* wall time of the solve, milliseconds                         */
} mg_stats;

typedef struct mg_handle mg_handle;

/* Builds the grid hierarchy (Section 4: coarse nodes are every other fine node,
 * down to 3 nodes on some axis or an odd cell count), the coefficients of
 * every level in FP64 and FP32 for the operator and its transpose, the
 * smoother block tables (Section 3 motifs), and uploads them.  stream is a
 * hipStream_t (NULL = default stream).  Returns MG_EINVAL for odd or too small
 * n (or n above 32000), unknown kinds, dim not 2/3, batch < 1;
 * MG_EUNSUPPORTED when one problem's array (in the device layout, which holds
 * up to twice the nodes) would reach 2^31 entries -- the kernels address a
 * problem with 32-bit offsets -- or for a smoother this build does not
 * provide in that dimension; *out is set only on success. */
int mg_setup(const mg_grid *grid, const mg_stretching *stretch, const mg_options *opt, void *stream,
             mg_handle **out);
void mg_destroy(mg_handle *h);
int mg_set_stream(mg_handle *h, void *stream);
/* Replaces the cycle options (smoother must use motifs built at setup:
 * the same smoother, or checkerboard). */
int mg_set_options(mg_handle *h, const mg_options *opt);

/* Device workspace for the coarse levels and the FP32 copies (bytes).  Bind
 * caller-owned device memory of at least this size (256-byte aligned) before
 * the first solve; otherwise the library allocates it on first use.  The
 * bound memory must outlive the handle. */
size_t mg_workspace_bytes(const mg_handle *h);
int mg_bind_workspace(mg_handle *h, void *dev_ptr, size_t bytes);

/* Level introspection: n[3] cells of level lv (0 = finest); nlevels count. */
int mg_levels(const mg_handle *h, int *nlevels);
int mg_level_shape(const mg_handle *h, int lv, int *n);
/* Host copies of level lv's node coordinates and W/E (S/N, B/T) coefficients
 * along axis a (n+1 values each; coefficient entries 0 and n are 0). */
int mg_level_coefs(const mg_handle *h, int lv, int axis, double *x, double *lo, double *hi);

/* One gamma-cycle (Section 4, steps (2)-(6)) in place on u at the finest level;
 * u's boundary nodes hold the Dirichlet data and are not written. */
int mg_vcycle(mg_handle *h, double *u, const double *f);

/* Solve: u's boundary nodes are set from bc (if bc != NULL; else u's own
 * boundary values are used), its interior set to 0 (unless MG_INITIAL_GUESS),
 * then cycles run until ||f_b - L u_b||_inf / ||f_b - L u_b,0||_inf < tol for
 * every batch problem b (Section 4 stopping rule, each problem measured
 * against its own initial defect; a problem whose initial defect is zero is
 * already solved and is left out).  stats->rel_res is the largest of these
 * ratios and stats->res0 the largest initial defect.
 * With precision MG_FP32_IR each step is r = f - A u in FP64, one FP32 cycle
 * on A e = r from e = 0, u += e in FP64.  Returns MG_OK, MG_ENOTCONV (u holds
 * the last iterate) or MG_EDIVERGED.  stats may be NULL. */
int mg_solve(mg_handle *h, double *u, const double *f, const double *bc, double tol, mg_stats *stats);

/* Adjoint solve A_II^T lam = w_I (interior), lam = 0 on the boundary, by the
 * same cycle applied to the transposed operator with the colour order of every
 * block sweep reversed, so that the adjoint cycle is the transpose of the
 * forward one.  w is a full node array; only its interior is read.  An
 * extension of the method for differentiation: the paper defines no adjoint,
 * so no passage is cited (A is the operator of problem (DP), Section 2).  The
 * stopping rule and return codes are those of mg_solve. */
int mg_solve_adjoint(mg_handle *h, double *lam, const double *w, double tol, mg_stats *stats);

/* Gradient of L = sum(w * u) with respect to the Dirichlet data g, given the
 * adjoint solution lam:  grad_g = w_B - A_IB^T lam on boundary nodes, 0 on
 * interior nodes (the gradient with respect to f is lam itself).  An extension
 * for differentiation with no passage in the paper: A_IB is the part of the
 * operator of problem (DP), Section 2, that couples interior nodes to the
 * boundary data.  Asynchronous; lam, w and grad_bc are full node arrays
 * (grad_bc is written at every node). */
int mg_bc_grad(mg_handle *h, const double *lam, const double *w, double *grad_bc);

/* ||f - L u||_inf over interior nodes, the defect norm of the stopping rule of
 * Section 4 (the maximum over the batch problems); synchronous, *out_inf is a
 * host pointer. */
int mg_residual_norm(mg_handle *h, const double *u, const double *f, double *out_inf);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): mg_residual_norm without
 * any allocation or synchronisation.  Enqueues on the handle's stream the
 * computation of the maximum over the batch of ||f - L u||_inf (interior
 * nodes, row-major u and f as for mg_residual_norm) and writes it to
 * out_dev[0], a DEVICE pointer to one double owned by the caller.  The partial
 * maxima live in a library-wide device array of 16384 doubles (128 KiB, one
 * per GPU, resolved at mg_setup and held until the process ends) that every
 * call on a GPU shares: calls that overlap on one GPU (different streams or
 * host threads) race and must be ordered by the caller.  Nothing in the array
 * needs clearing between calls.  Returns MG_EINVAL for null pointers, a
 * host-only handle, or a batch above 16384 (the array's capacity);
 * MG_EHIP if the launch fails or the array was never resolved.  Calls no
 * hipMalloc, hipFree or allocating library routine. */
int mg_residual_norm_noalloc(mg_handle *h, const double *u, const double *f, double *out_dev);

/* Kernel-level entry points on level lv (arrays of that level's shape):
 * mg_smooth: nu relaxations of the configured smoother (Section 3).
 * mg_residual: d = f - L u at interior nodes, 0 at boundary nodes.
 * mg_residual_restrict: f_c = R (f - L u) by full weighting onto level lv+1
 *   (Section 4, fused steps (3)); the coarse interior of u_c is zeroed.
 * mg_prolong_add: u += P e_c, bilinear/trilinear in index space (Section 4,
 *   fused step (5)); e_c is a level lv+1 array with zero boundary.
 * adjoint != 0 selects the transposed operator (and reversed colours). */
int mg_smooth(mg_handle *h, int lv, double *u, const double *f, int nu, int adjoint);
int mg_residual(mg_handle *h, int lv, const double *u, const double *f, double *d, int adjoint);
int mg_residual_restrict(mg_handle *h, int lv, const double *u, const double *f, double *fc, double *uc, int adjoint);
int mg_prolong_add(mg_handle *h, int lv, const double *ec, double *u);
/* FP32 version of mg_smooth (the smoother used inside refinement cycles; u and f are FP32 node arrays). */
int mg_smooth_f32(mg_handle *h, int lv, float *u, const float *f, int nu, int adjoint);

/* Device layout.  Internally each level keeps its arrays in a layout chosen
 * for its smoother: on the large 2D levels of the tweed, wireframe and
 * y-zebra smoothers, the nodes whose block lines run along y (Section 3: the
 * lines are orthogonal to the nearest wall for tweed, parallel to it for
 * wireframe) sit in a second, column-major plane, so that every line is
 * contiguous; elsewhere the layout is the row-major one above.  The calls
 * above convert on entry and exit.  A caller that keeps data in the device
 * layout between calls uses these:
 * mg_level_array_len: number of elements of one problem's array of level lv
 *   in the device layout (the batch stride); *len is a host pointer.
 * mg_to_layout / mg_from_layout: row-major <-> device layout (all problems of
 *   the batch); src and dst must not overlap.
 * mg_half_sweep: one half-sweep -- every block of one colour (0 red, 1 black)
 *   of motif slot `slot` (0; 1 and 2 for the second and third sweeps of an
 *   alternating smoother) solved exactly with the other colour frozen -- on arrays in the
 *   device layout.  MG_EINVAL for the checkerboard smoother or a slot the
 *   smoother does not have. */
int mg_level_array_len(const mg_handle *h, int lv, long long *len);
int mg_to_layout(mg_handle *h, int lv, const double *src, double *dst);
int mg_from_layout(mg_handle *h, int lv, const double *src, double *dst);
int mg_half_sweep(mg_handle *h, int lv, double *u, const double *f, int slot, int colour, int adjoint);

const char *mg_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* TWMG_H */
