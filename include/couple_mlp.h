/*
 * couple_mlp.h -- C ABI of the learned velocity surrogate of the coupling library.
 *
 * The coupling step needs the fluid velocity at every particle ("cell values or
 * locally interpolated values", Sec. 1).  With vel_source = COUPLE_VEL_MLP it
 * takes it from a small network instead of the fine-grid lookup:
 *
 *     u_f = u_bulk + s * y,    y = MLP(standardised features),
 *
 * u_bulk being the trilinear interpolation of the restricted bulk velocity and
 * s the per-component scale of the residual u_fine - u_bulk on the training set
 * (the surrogate is not part of the paper; it replaces the fine lookup that the
 * dual-grid exchange of Sec. 2.1 and Fig. 1 performs).
 *
 * Features (COUPLE_MLP_NFEAT = 193, in this order): for the 27 bulk cells around
 * the particle's cell (dz, dy, dx in -1..1, dx fastest, indices clamped at the
 * walls) the seven values (eps = 1 - phi, U_x, U_y, U_z, G_x, G_y, G_z), where
 * every neighbour enters as its difference from the centre cell and the centre
 * cell as its own values; then the in-cell offsets x n_x / L_x - i (three); then
 * d n_x / L_x.  Each feature is standardised with a mean and standard deviation
 * fitted on the training set.
 *
 * Network: 193 -> 128 -> 128 -> 128 -> 3, tanh-form GELU after the hidden
 * layers.  Products run on the matrix cores with BF16 operands (weights and
 * every layer input rounded to nearest even) and FP32 accumulation; the master
 * parameters and the Adam moments are FP32.  Parameter vector
 * (COUPLE_MLP_NPARAM = 58243 floats), layer by layer: W_l as [fan_in][fan_out]
 * row-major, then b_l.  Training loss: mean over the batch of 1/2 |y - t|^2 with
 * t = (u_fine - u_bulk) / s.  Adam with bias correction.
 *
 * In the step the network's velocity is checked on a deterministic sample: every
 * particle with id mod mlp_period = step mod mlp_period is also looked up on the
 * fine grid, per brick of 8x8x8 bulk cells.  Where the sampled relative L2 error
 * of a brick exceeds mlp_tol, every particle of that brick takes the fine lookup
 * instead (diag[COUPLE_DIAG_N_FALLBACK] counts them).  The sampled squared error
 * and reference are reported in diag[COUPLE_DIAG_MLP_ERR2 / _REF2].
 *
 * Memory: pointers named "device" are device memory owned by the caller; "host"
 * pointers are host memory.  The handle owns its parameters, Adam moments and
 * batch buffers (sized by max_batch), allocated by couple_mlp_init().
 * Streams and errors follow couple.h: enqueue on the given stream, return a
 * couple_status, detect argument errors before any launch.  Forward, gradient
 * and training calls on one handle share its batch buffers: such calls that
 * overlap (different streams or threads) race; calls in order on one stream
 * do not.
 */
#ifndef COUPLE_MLP_H
#define COUPLE_MLP_H

#include <stdint.h>

#include "couple.h"

#ifdef __cplusplus
extern "C" {
#endif

#define COUPLE_MLP_NFEAT 193
#define COUPLE_MLP_NPARAM 58243

typedef struct couple_mlp couple_mlp;

typedef struct couple_mlp_config {
    int64_t max_batch;   /* largest batch of couple_mlp_forward/grads/train_step, 32 <= max_batch < 2^26 */
    double  lr;          /* Adam step size (> 0)                                                        */
    double  beta1;       /* Adam first-moment decay, in [0, 1)                                          */
    double  beta2;       /* Adam second-moment decay, in [0, 1)                                         */
    double  eps;         /* Adam denominator guard (> 0)                                                */
} couple_mlp_config;

/* Allocate a network (parameters zero, standardisation identity, scale 1). */
int couple_mlp_init(const couple_mlp_config *cfg, couple_mlp **out);
int couple_mlp_free(couple_mlp *m);
const char *couple_mlp_last_error(const couple_mlp *m);

/* Parameters from host memory [COUPLE_MLP_NPARAM]; resets Adam (step 0, zero
 * moments).  Synchronous. */
int couple_mlp_set_params(couple_mlp *m, const float *params);

/* Standardisation (host, FP64): feature mean and std [193] (std > 0) and the
 * residual scale [3] (> 0).  Synchronous. */
int couple_mlp_set_norm(couple_mlp *m, const double *mean, const double *std, const double *scale);

/* Fit the standardisation on n >= 1 training rows: feat [n][193] and resid
 * [n][3] (device).  Mean and population standard deviation per column in FP64
 * (two passes, fixed order).  A neighbour-difference feature's std is raised to
 * at least 1e-4 times the std of the centre cell's value of the same channel
 * (differences of a field that does not vary in that direction are rounding
 * only); then a feature with std below 1e-12 gets std 1.  A residual component
 * with no spread gets the largest of the others (1 if all are zero).
 * Synchronises `stream`. */
int couple_mlp_fit_norm(couple_mlp *m, const float *feat, const float *resid, int64_t n, void *stream);

/* Full state to / from host memory (checkpoint and resume): params, Adam
 * moments m, v [COUPLE_MLP_NPARAM], Adam step count, feature mean/std [193],
 * scale [3].  Any output pointer may be NULL.  Synchronous. */
int couple_mlp_get_state(couple_mlp *m, float *params, float *adam_m, float *adam_v, int64_t *step,
                         double *mean, double *std, double *scale);
int couple_mlp_set_state(couple_mlp *m, const float *params, const float *adam_m, const float *adam_v,
                         int64_t step, const double *mean, const double *std, const double *scale);

/* Network output y [n][3] (device, unscaled) of raw features feat [n][193]
 * (device), 0 <= n <= max_batch. */
int couple_mlp_forward(couple_mlp *m, const float *feat, int64_t n, float *y, void *stream);

/* Loss and gradient of one batch: rows idx[0..B) (device int32, each in
 * [0, nrows); NULL = rows 0..B-1) of feat [nrows][193] and resid [nrows][3]
 * (device).  An index outside [0, nrows) is not detected (the indices stay on
 * the device); the kernels read row 0 for it, so every access stays in bounds.  B is a multiple of 32, 32 <= B <= max_batch.  grads
 * [COUPLE_MLP_NPARAM] and loss [1] are device FP32 outputs (loss may be NULL).
 * The parameters are not changed. */
int couple_mlp_grads(couple_mlp *m, const float *feat, const float *resid, int64_t nrows, const int32_t *idx,
                     int64_t B, float *grads, float *loss, void *stream);

/* One Adam step with the given gradient (device [COUPLE_MLP_NPARAM]). */
int couple_mlp_adam(couple_mlp *m, const float *grads, void *stream);

/* couple_mlp_grads followed by couple_mlp_adam (gradient kept in the handle). */
int couple_mlp_train_step(couple_mlp *m, const float *feat, const float *resid, int64_t nrows, const int32_t *idx,
                          int64_t B, float *loss, void *stream);

/* Training pairs from the bulk fields of a coupling step (FP32 configurations):
 * for particles sel[0..nsel) (device int32 ids in [0, n); NULL = 0..nsel-1) the
 * raw features feat [nsel][193], optionally the bulk trilinear velocity
 * u_bulk [nsel][3] and, given the fine-grid velocity at the particles u_fine
 * [n][3] (couple_outputs.uf of a COUPLE_VEL_FINE step), the residual
 * resid [nsel][3] = u_fine - u_bulk.  pos [n][3], diam [n], bulk_phi [Nb],
 * bulk_U [3][Nb], bulk_G [3][Nb] are device arrays laid out as in couple.h. */
int couple_mlp_features(const couple_config *cfg, int64_t n, const float *pos, const float *diam,
                        const float *bulk_phi, const float *bulk_U, const float *bulk_G, const float *u_fine,
                        const int32_t *sel, int64_t nsel, float *feat, float *u_bulk, float *resid, void *stream);

/* Use network m in the COUPLE_VEL_MLP steps of h (NULL detaches).  The network
 * must outlive its use; its parameters are read when each step runs. */
int couple_set_mlp(couple_handle *h, const couple_mlp *m);

#ifdef __cplusplus
}
#endif
#endif /* COUPLE_MLP_H */
