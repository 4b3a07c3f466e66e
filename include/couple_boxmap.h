/*
 * couple_boxmap.h -- C ABI of the grid-to-grid transfer between grids made of
 * arbitrary axis-aligned cells: locally refined, non-uniform grids that are not
 * nested in each other.
 *
 * The fine CFD grid of the dual-grid coupling may be non-uniform and locally
 * refined, and the bulk grid is in general not nested in it (Sec. 2.1); the
 * exchange between them goes through a static sender -> receiver map computed
 * once per simulation for non-deforming grids (Sec. 2.3).  This interface builds
 * that map for any two grids given as lists of boxes and applies it on the
 * device:
 *
 *     dst_r = (sum_s |r intersect s| src_s) / |r|,
 *
 * the volume-weighted average of the sender cells s that overlap receiver cell
 * r.  It copies twin cells, averages the children of a refined cell into their
 * parent, preserves constants and conserves the integral sum_r dst_r |r| =
 * sum_s src_s |s| when both grids tile the same region, in either direction.
 * (couple_remap.h does the same for rectilinear grids, whose map factors over
 * the axes and needs no stored matrix.)
 *
 * Grids: cell c is the box [b[6c], b[6c+1]] x [b[6c+2], b[6c+3]] x [b[6c+4],
 * b[6c+5]] (host memory, FP64, finite, lower < upper on every axis); the cells
 * of one grid should not overlap each other.  A receiver cell that overlaps no
 * sender cell receives 0.  Fields are [nfields][cells] in the grids' cell
 * order.
 *
 * The map: a CSR matrix with one row per receiver cell (columns ascending), its
 * weights |r intersect s| / |r| computed in FP64 on the host by
 * couple_boxmap_init() (candidate senders from a uniform bucket grid over the
 * sender cells, overlaps as products of the three 1-D overlaps) and stored on
 * the device as int64 row offsets, int32 columns and weights of the field
 * precision.
 *
 * Memory and errors follow couple.h: device pointers owned by the caller,
 * enqueue on the given stream, negative status codes detected before any launch.
 */
#ifndef COUPLE_BOXMAP_H
#define COUPLE_BOXMAP_H

#include <stdint.h>

#include "couple.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct couple_boxmap couple_boxmap;

/* Build the map from the sender grid (ns cells, sender_boxes [ns][6]) to the
 * receiver grid (nr cells, receiver_boxes [nr][6]) for fields of the given
 * precision (COUPLE_FP64: double fields and weights, FP64 sums; the FP32
 * precisions: float fields and weights, FP64 register sums for
 * COUPLE_FP32_WIDE, Kahan-compensated FP32 sums for COUPLE_FP32_KAHAN, plain
 * FP32 sums for COUPLE_FP32_NAIVE).  1 <= ns, nr <
 * 2^31; the map may hold at most 2^31 - 1 nonzeros.  Synchronous. */
int couple_boxmap_init(int64_t ns, const double *sender_boxes, int64_t nr, const double *receiver_boxes,
                       int32_t precision, couple_boxmap **out);

/* dst [nfields][nr] from src [nfields][ns] (device); 1 <= nfields <= 64; src
 * and dst must not overlap. */
int couple_boxmap_apply(couple_boxmap *m, const void *src, void *dst, int32_t nfields, void *stream);

/* Nonzeros of the map and the longest row. */
int couple_boxmap_info(const couple_boxmap *m, int64_t *nnz, int64_t *max_row);

int couple_boxmap_free(couple_boxmap *m);            /* NULL is accepted */
const char *couple_boxmap_last_error(const couple_boxmap *m);

#ifdef __cplusplus
}
#endif
#endif /* COUPLE_BOXMAP_H */
