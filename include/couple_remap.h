/*
 * couple_remap.h -- C ABI of the grid-to-grid transfer between grids that need
 * not be nested.
 *
 * The coupling step of couple.h uses nested grids (fine cells split every bulk
 * cell r x r x r).  In general the fine CFD grid and the bulk grid are not
 * aligned, and the exchange between them is an interpolation from a "sender"
 * grid to a "receiver" grid through a map that, for non-deforming grids, is
 * computed once per simulation (Sec. 2.3).  This interface provides that
 * transfer for rectilinear, cell-centred grids over the same box:
 *
 *     dst_c = (sum_f |f intersect c| src_f) / |c|,
 *
 * the volume-weighted average of the sender cells f that overlap receiver cell
 * c.  It copies twin cells of identical grids, averages the children of a
 * nested coarse cell, preserves constants and conserves the integral
 * sum_c dst_c |c| = sum_f src_f |f|, in either direction (coarse -> fine or fine
 * -> coarse).
 *
 * The overlap map is a sparse matrix whose entries factor over the axes,
 * |f intersect c| / |c| = w_x(c_x, f_x) w_y(c_y, f_y) w_z(c_z, f_z); it is stored
 * as its three 1-D factors (per receiver index along an axis: the first
 * overlapping sender index, the count and the weights), built on the host in
 * FP64 by couple_remap_init() and kept on the device.
 *
 * Grids: axis a has n[a] >= 1 cells between nodes x_a[0] < x_a[1] < ... <
 * x_a[n[a]] (finite); `nodes` holds the three axes' node coordinates one after
 * the other (n[0] + 1 + n[1] + 1 + n[2] + 1 doubles, host memory).  Both grids
 * must span the same interval on every axis (end nodes equal to within 1e-12
 * relative).  Fields are [nz][ny][nx], x fastest; `nfields` fields are stored
 * back to back (a vector field is nfields = 3).
 *
 * Memory and errors follow couple.h: device pointers owned by the caller,
 * enqueue on the given stream, negative status codes detected before any launch.
 */
#ifndef COUPLE_REMAP_H
#define COUPLE_REMAP_H

#include <stdint.h>

#include "couple.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct couple_remap couple_remap;

/* Build the map from the sender grid (src_n, src_nodes) to the receiver grid
 * (dst_n, dst_nodes) for fields of the given precision (COUPLE_FP64: double
 * fields and weights; COUPLE_FP32_WIDE / COUPLE_FP32_KAHAN / COUPLE_FP32_NAIVE:
 * float fields, sums in FP64 registers, Kahan-compensated in FP32, or plain).  Each grid: cells per axis >= 1, fewer than 2^31
 * cells in all.  On success *out receives the map (a few device arrays of the
 * size of the receiver's axes). */
int couple_remap_init(const int32_t src_n[3], const double *src_nodes, const int32_t dst_n[3],
                      const double *dst_nodes, int32_t precision, couple_remap **out);

/* dst [nfields][receiver cells] from src [nfields][sender cells] (device);
 * 1 <= nfields <= 64.  src and dst must not overlap. */
int couple_remap_apply(couple_remap *r, const void *src, void *dst, int32_t nfields, void *stream);

/* Nonzeros of the three 1-D factors and of the full 3-D map they define. */
int couple_remap_info(const couple_remap *r, int64_t nnz_axis[3], int64_t *nnz_total);

int couple_remap_free(couple_remap *r);            /* NULL is accepted */
const char *couple_remap_last_error(const couple_remap *r);

#ifdef __cplusplus
}
#endif
#endif /* COUPLE_REMAP_H */
