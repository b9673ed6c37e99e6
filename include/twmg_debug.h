/*
 * twmg test hooks.  Not part of the solver: nothing in the library calls
 * these, and they exist so that the CPU test suite can check the block tables
 * of the relaxation motifs (Section 3 of arXiv 2110.08389) without a GPU.
 */
#ifndef TWMG_DEBUG_H
#define TWMG_DEBUG_H

#include "twmg.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Statistics of the block table of level lv, motif slot (0; 1 and 2 for the
 * later sweeps of an alternating smoother) and colour (0 red, 1 black):
 * info[0] workgroups, [1] chunks, [2] blocks, [3] max chunks in a workgroup,
 * [4] max blocks in a workgroup, [5] points covered.  Host memory. */
int mg_debug_table_info(const mg_handle *h, int lv, int slot, int colour, int *info);

/* Builds a handle with the host-side structures only (hierarchy,
 * coefficients, block tables; no device allocation, no HIP call).  Only the
 * mg_debug_* calls, mg_levels, mg_level_shape, mg_level_coefs and mg_destroy
 * accept such a handle. */
int mg_debug_setup_host(const mg_grid *grid, const mg_stretching *stretch, const mg_options *opt, mg_handle **out);

/* Runs nu relaxations of the configured block smoother on HOST arrays u, f
 * (FP64, level lv shape, batch included) by executing the device kernel's
 * per-lane steps sequentially, workgroup by workgroup.  A test hook for the
 * table construction only; the solver never uses it.  MG_EUNSUPPORTED for the
 * checkerboard smoother (it has no tables). */
int mg_debug_host_smooth(mg_handle *h, int lv, double *u, const double *f, int nu, int adjoint);

/* As mg_debug_host_smooth, but the per-lane steps address the arrays in the
 * level's own device layout (for the large levels of the tweed, wireframe and
 * y-zebra smoothers, two planes: the points of lines along x row-major, those
 * of lines along y column-major).  u and f are given and returned row-major;
 * the hook converts them on the host. */
int mg_debug_host_smooth_layout(mg_handle *h, int lv, double *u, const double *f, int nu, int adjoint);

#ifdef __cplusplus
}
#endif
#endif /* TWMG_DEBUG_H */
