/*
 * couple.h -- C ABI of the MI355X (gfx950) dual-grid coupling exchange.
 *
 * One call of couple_step() performs the per-timestep exchange between
 * Lagrangian particles, the coarse "bulk" grid on which the fluid-particle
 * interaction is resolved and the fine grid on which the fluid equations are
 * discretised (dual-grid multiscale coupling, Sec. 2.1 and Fig. 1):
 *
 *   1. bin      containing bulk cell of every particle and the canonical
 *               (cell, id) order, rebuilt every coupling step (Sec. 2.2);
 *   2. deposit  bulk solid fraction phi = sum_p w_pc V_p / V_b; porosity
 *               eps = 1 - phi (Table 1 and the porosity definition of Sec. 2.4);
 *   3. restrict fine fluid velocity and pressure averaged over the fine children
 *               of every bulk cell ("fluid solution" arrow of Fig. 1), plus the
 *               bulk pressure gradient;
 *   4. gather   fluid velocity and void fraction at each particle ("cell values
 *               or locally interpolated values", Sec. 1), or the learned
 *               surrogate of that velocity (couple_mlp.h);
 *   5. drag     F_p = beta (u_f - u_p), Eq. DragLaw of Sec. 2.4, with beta from
 *               the Di Felice voidage correlation; with vof = 1 the fluid density
 *               and viscosity at the particle are those of the two-fluid (VOF)
 *               mixture, rho_f = rho_1 alpha + rho_2 (1 - alpha) and likewise mu_f
 *               (Sec. 2.5), alpha being the liquid volume fraction restricted to
 *               the bulk grid (its volume average) and interpolated trilinearly
 *               to the particle;
 *   6. source   momentum source F_fpi,c = -(1/V_b) sum_p w_pc F_p, the counterpart
 *               of the drag in Eq. UFP (Sec. 2.5); with semi_implicit = 1 also its
 *               semi-implicit split (the drag term of Eq. UFP is treated
 *               semi-implicitly in the fluid solve, Sec. 2.5):
 *                 K_c  = (1/V_b) sum_p w_pc beta_p        implicit coefficient,
 *                 KU_c = (1/V_b) sum_p w_pc beta_p u_p    explicit part,
 *               so that F_fpi = -K u_f + KU wherever u_f is uniform over the
 *               deposition stencil (u_p: the velocity before advection);
 *   7. prolong  eps and F_fpi (and K, KU) transferred to the fine grid ("particle
 *               related fields" arrow of Fig. 1) by a conservative trilinear
 *               prolongation;
 *   8. sums     FP64 conservation diagnostics;
 *   9. advect   optional explicit Euler step of Eq. DEM_EQUATIONS with the drag
 *               as the only force.
 *
 * Grids: uniform, nested, cell-centred.  The box is [0,Lx]x[0,Ly]x[0,Lz]; the bulk
 * grid has nb[0] x nb[1] x nb[2] cells; the fine grid has `ratio` fine cells per
 * bulk cell along each axis.  Every grid array is stored z-major with x fastest
 * ([nz][ny][nx]); a vector grid field is its three components back to back
 * ([3][nz][ny][nx]).  Particle vectors are [n][3] (x, y, z interleaved).
 *
 * Memory: every pointer in couple_inputs / couple_outputs is a DEVICE pointer
 * owned by the caller (for example a torch tensor's data_ptr()), C-contiguous and
 * aligned to at least 16 bytes.  Floating-point arrays are `double` when the
 * handle's precision is COUPLE_FP64 and `float` otherwise.  The library owns only
 * its scratch, allocated by couple_init() and released by couple_free().
 *
 * Streams: couple_step() enqueues its kernels on the given HIP stream (a
 * hipStream_t passed as void*; NULL is the null stream) and returns without
 * synchronising.  Outputs, including diag, are valid once the stream has reached
 * that point.  It allocates nothing.
 *
 * Errors: every function returns a couple_status (0 or negative) and never throws
 * across the ABI.  Argument and state errors are detected before any launch and
 * leave all outputs untouched; couple_last_error() then describes the failure.
 * Particles outside the box (or with a non-finite coordinate) are not an error:
 * they are clamped into the box and counted in diag[COUPLE_DIAG_N_OUTSIDE].
 *
 * Threading: a handle is not thread-safe; distinct handles are independent.
 */
#ifndef COUPLE_H
#define COUPLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct couple_handle couple_handle;

typedef enum {
    COUPLE_OK = 0,
    COUPLE_EINVAL = -1,     /* invalid configuration or argument (NULL pointer, n < 0) */
    COUPLE_ENOMEM = -2,     /* device allocation failed in couple_init                  */
    COUPLE_EHIP = -3,       /* a HIP runtime call or kernel launch failed               */
    COUPLE_ECAPACITY = -4,  /* n > max_particles                                        */
    COUPLE_ESTATE = -6      /* call not valid in the handle's state                     */
} couple_status;

enum { COUPLE_NGP = 0, COUPLE_CIC = 1 };                  /* deposition weights            */
/* Precision: the data type and how per-cell sums (restriction children,
 * deposition terms, transfer overlaps) accumulate; the global diagnostics are
 * FP64 sums in every mode.
 *   COUPLE_FP64        FP64 data, plain FP64 sums.
 *   COUPLE_FP32_WIDE   FP32 data; per-cell sums accumulated in FP64 registers and
 *                      rounded to FP32 once per cell (the pressure keeps an FP32
 *                      low word for its gradient).  The default FP32 mode.
 *   COUPLE_FP32_NAIVE  FP32 data, plain FP32 sums (the uncompensated baseline).
 *   COUPLE_FP32_KAHAN  FP32 data, Kahan-compensated FP32 per-cell sums (the
 *                      pressure's low word is the negated compensation). */
enum { COUPLE_FP64 = 0, COUPLE_FP32_WIDE = 1, COUPLE_FP32_NAIVE = 2, COUPLE_FP32_KAHAN = 3 };  /* precision */
enum { COUPLE_VEL_FINE = 0, COUPLE_VEL_BULK = 1, COUPLE_VEL_GIVEN = 2, COUPLE_VEL_MLP = 3 }; /* u_f */

/* Indices into the FP64 diagnostics vector (length COUPLE_DIAG_LEN). */
enum {
    COUPLE_DIAG_V_TOT = 0,      /* sum_p V_p, V_p = pi d^3 / 6                              */
    COUPLE_DIAG_V_DEP = 1,      /* sum_c phi_c V_b (equals V_TOT: volume is conserved)     */
    COUPLE_DIAG_SUM_FP = 2,     /* [2..4]  sum_p F_p (drag on the particles)               */
    COUPLE_DIAG_S_B = 5,        /* [5..7]  sum_c F_fpi,c V_b  (equals -sum_p F_p)          */
    COUPLE_DIAG_S_F = 8,        /* [8..10] sum_f F_f V_f on the fine grid (equals S_B)     */
    COUPLE_DIAG_E_F = 11,       /* sum_f eps_f V_f, fluid volume on the fine grid          */
    COUPLE_DIAG_N_CLAMPED = 12, /* particles whose void fraction was raised to eps_min     */
    COUPLE_DIAG_N_OUTSIDE = 13, /* particles with a coordinate outside [0,L] or not finite */
    COUPLE_DIAG_MAX_PHI = 14,   /* max_c phi_c                                              */
    COUPLE_DIAG_N_FALLBACK = 15,/* VEL_MLP: particles that took the fine-grid fallback       */
    COUPLE_DIAG_MLP_ERR2 = 16,  /* VEL_MLP: sum over the checked sample of |u_mlp - u_fine|^2 */
    COUPLE_DIAG_MLP_REF2 = 17,  /* VEL_MLP: sum over the checked sample of |u_fine|^2         */
    COUPLE_DIAG_MLP_NSAMP = 18, /* VEL_MLP: particles in the checked sample                   */
    COUPLE_DIAG_K_P = 19,       /* semi_implicit: sum_p beta_p                                */
    COUPLE_DIAG_KU_P = 20,      /* [20..22] semi_implicit: sum_p beta_p u_p                   */
    COUPLE_DIAG_K_B = 23,       /* sum_c K_c V_b (equals K_P)                                 */
    COUPLE_DIAG_KU_B = 24,      /* [24..26] sum_c KU_c V_b (equals KU_P)                      */
    COUPLE_DIAG_K_F = 27,       /* sum_f K_f V_f on the fine grid (equals K_B)                */
    COUPLE_DIAG_KU_F = 28,      /* [28..30] sum_f KU_f V_f (equals KU_B)                      */
    COUPLE_DIAG_LEN = 31
};

typedef struct couple_config {
    double  box[3];          /* Lx, Ly, Lz > 0                                              */
    int32_t nb[3];           /* bulk cells per axis, >= 1, nb[0] <= 32767, product < 2^31    */
    int32_t ratio;           /* fine cells per bulk cell per axis: 1, 2 or 4                  */
    double  rho_f, mu_f;     /* fluid density and viscosity (> 0)                            */
    double  rho_p;           /* particle density (> 0), used by the advection                */
    double  eps_min;         /* drag uses max(eps_p, eps_min), 0 <= eps_min < 1              */
    double  phi_fp64;        /* particle solid fraction above which the FP32 modes evaluate
                                eps_p and the voidage factor in FP64 (near close packing)     */
    int32_t deposit;         /* COUPLE_NGP or COUPLE_CIC                                      */
    int32_t precision;       /* COUPLE_FP64, COUPLE_FP32_WIDE, _NAIVE or _KAHAN               */
    int32_t vel_source;      /* COUPLE_VEL_FINE (trilinear on the fine grid), COUPLE_VEL_BULK
                                (trilinear on the restricted bulk velocity),
                                COUPLE_VEL_GIVEN (couple_inputs.uf_given) or COUPLE_VEL_MLP
                                (learned surrogate with fine fallback, FP32 precisions only,
                                network attached with couple_set_mlp)                         */
    int32_t advect;          /* 1: explicit Euler update of pos and vel in place              */
    double  dt;              /* advection time step                                           */
    int64_t max_particles;   /* capacity of the scratch; n > max_particles is an error        */
    double  mlp_tol;         /* VEL_MLP: relative L2 error of a brick's checked sample above
                                which the brick takes the fine lookup (>= 0)                  */
    int32_t mlp_period;      /* VEL_MLP: one particle in mlp_period is checked (>= 1)          */
    int32_t semi_implicit;   /* 1: also deposit and prolong K and KU (step 6); 0 or 1          */
    int32_t vof;             /* 1: two-fluid drag (step 5); rho_f, mu_f are fluid 1's; 0 or 1 */
    double  rho_f2, mu_f2;   /* vof: density and viscosity of fluid 2 (> 0)                   */
} couple_config;

typedef struct couple_inputs {
    int64_t     n;           /* number of particles, 0 <= n <= max_particles                  */
    void       *pos;         /* [n][3] positions; updated in place when advect = 1           */
    void       *vel;         /* [n][3] velocities; updated in place when advect = 1          */
    const void *diam;        /* [n] diameters                                                 */
    const void *fine_u;      /* [nfz][nfy][nfx] fine fluid velocity, x component              */
    const void *fine_v;      /*   y component                                                 */
    const void *fine_w;      /*   z component                                                 */
    const void *fine_p;      /* [nfz][nfy][nfx] fine pressure                                 */
    const void *uf_given;    /* [n][3] fluid velocity at each particle (VEL_GIVEN only)       */
    int64_t     step;        /* caller's step index; VEL_MLP checks ids = step mod mlp_period */
    const void *fine_alpha;  /* [nfz][nfy][nfx] liquid volume fraction in [0, 1] (vof only)     */
} couple_inputs;

typedef struct couple_outputs {
    void    *drag;           /* [n][3] F_p, drag on each particle (input order)               */
    void    *beta;           /* [n] drag factor beta, or NULL if not wanted                   */
    int32_t *cell;           /* [n] containing bulk cell (linear index) per particle          */
    int32_t *perm;           /* [n] particle ids in ascending (cell, id) order                */
    int32_t *count;          /* [Nb] particles per bulk cell                                  */
    int32_t *start;          /* [Nb+1] exclusive prefix sum of count                          */
    void    *bulk_phi;       /* [Nb] solid volume fraction                                    */
    void    *bulk_F;         /* [3][Nb] momentum source F_fpi                                 */
    void    *bulk_U;         /* [3][Nb] restricted fluid velocity                             */
    void    *bulk_P;         /* [Nb] restricted pressure                                      */
    void    *bulk_G;         /* [3][Nb] bulk pressure gradient                                */
    void    *fine_eps;       /* [Nf] porosity prolonged to the fine grid                      */
    void    *fine_F;         /* [3][Nf] momentum source prolonged to the fine grid            */
    double  *diag;           /* [COUPLE_DIAG_LEN] FP64 diagnostics (device memory)            */
    void    *uf;             /* [n][3] fluid velocity used by the drag, or NULL if not wanted */
    void    *bulk_K;         /* [Nb] semi-implicit drag coefficient K (semi_implicit only)    */
    void    *bulk_KU;        /* [3][Nb] semi-implicit explicit part KU (semi_implicit only)   */
    void    *fine_K;         /* [Nf] K prolonged to the fine grid (semi_implicit only)        */
    void    *fine_KU;        /* [3][Nf] KU prolonged to the fine grid (semi_implicit only)    */
    void    *bulk_alpha;     /* [Nb] restricted liquid volume fraction (vof only)             */
} couple_outputs;

/* Validate the configuration and allocate the scratch (about 48 * max_particles
 * bytes plus a few bytes per bulk cell; 32 more bytes per bulk cell for
 * VEL_MLP, 9 more values per bulk cell for semi_implicit with CIC).  On success
 * *out receives a handle. */
int couple_init(const couple_config *cfg, couple_handle **out);

/* Enqueue one coupling step (stages 1-9 above) on `stream`.  Every pointer of
 * `in` and `out` except out->beta and out->uf (and in->uf_given unless
 * VEL_GIVEN) must be non-NULL when n > 0; the grid outputs are always required,
 * the four K/KU outputs when semi_implicit = 1 (ignored otherwise), in->fine_alpha
 * and out->bulk_alpha when vof = 1 (ignored otherwise).
 * VEL_MLP without an attached network is COUPLE_ESTATE. */
int couple_step(couple_handle *h, const couple_inputs *in, couple_outputs *out, void *stream);

/* Release the scratch and the handle.  NULL is accepted. */
int couple_free(couple_handle *h);

/* Text of the last error on this handle (or, when h is NULL, of the calling
 * thread's last couple_init or couple_step_noalloc failure).  The pointer stays
 * valid until the next call on the same handle (or thread). */
const char *couple_last_error(const couple_handle *h);

/* ---- per-kernel timing (profiling aid, not part of the coupling method) -----
 * couple_timing_begin() starts recording: every following couple_step() records
 * a HIP event on its stream before each kernel launch and after the last one,
 * for at most `max_steps` steps (the event pool is created here).
 * couple_timing_end() waits for the recorded events, stops recording and
 * writes, per kernel name in launch order, the number of launches and the summed
 * event-to-event milliseconds into stats[0..max_stats); *n_stats receives the
 * number of names.  Names are static strings owned by the library. */
typedef struct couple_kernel_stat {
    const char *name;
    int64_t     launches;
    double      total_ms;
} couple_kernel_stat;

int couple_timing_begin(couple_handle *h, int32_t max_steps);
int couple_timing_end(couple_handle *h, couple_kernel_stat *stats, int32_t max_stats, int32_t *n_stats);

/* ---- partitioned step (partition-equivalence emulation on one device) ---------
 * The paper runs the coupling on many processes: each owns a partition of the
 * bulk grid together with the particles whose containing bulk cell it owns and
 * the fine cells nested in it (co-located partitions, Sec. 2.2), and the
 * partitions exchange the data their neighbours need through a static, sparse
 * process-to-process communication matrix, executed either through a master
 * process ("gather-scatter") or directly between neighbours ("distributed",
 * Sec. 2.3); the partitioned run must give the results of the sequential one
 * (Sec. 3.1).  couple_part_step() does this on one device with nparts z-slabs:
 * slab k owns bulk layers [z_k, z_{k+1}) (as equal as possible) and keeps, in
 * buffers of its own, the particles binned there, its fine slab and one ghost
 * bulk layer towards each neighbour.  Per step it exchanges (i) the fine cells of
 * the boundary bulk layer (for the lookups and the pressure gradient next to the
 * slab face), (ii) the ghost-layer partial sums of the volume deposition, added
 * into the owner (reverse halo add), then the completed boundary layer back into
 * the ghost layer, (iii) the same for the momentum source (and K, KU).  Only
 * neighbouring slabs communicate: the matrix has the nonzero blocks (k, k +- 1).
 *   exchange = COUPLE_EXCHANGE_DISTRIBUTED: each block is copied (or added)
 *   directly from the sender's buffer into the receiver's;
 *   COUPLE_EXCHANGE_GATHER_SCATTER: every block goes to a root buffer first and
 *   from there to its receiver (two transfers).
 * Results: cell, perm, count and start equal couple_step()'s bit for bit; the
 * fields differ from it by the order of the summations split across owners
 * (rounding only); the FP64 sums are the partitions' sums added in order.
 * Scope: velocity source FINE or BULK; no two-fluid drag; the bulk spacing
 * L_z / nb[2] must be a power of two (so that shifting positions into a slab's
 * frame is exact); with advection, particles are assumed to move less than one
 * bulk layer per step (the halo is one layer deep).  The call synchronises the
 * stream once (to read the partition sizes).  Outputs and inputs as couple_step. */
enum { COUPLE_EXCHANGE_DISTRIBUTED = 0, COUPLE_EXCHANGE_GATHER_SCATTER = 1 };
typedef struct couple_part couple_part;

/* nparts in [1, min(64, nb[2])]; allocates each slab's scratch and buffers
 * (about nparts handles of couple_init, plus one copy of the fine inputs and
 * outputs). */
int couple_part_init(const couple_config *cfg, int32_t nparts, couple_part **out);
int couple_part_step(couple_part *p, const couple_inputs *in, couple_outputs *out, int32_t exchange, void *stream);
/* bytes[i * nparts + j]: bytes slab j sends to slab i in one step (the static
 * communication matrix; zero unless |i - j| = 1). */
int couple_part_comm_matrix(const couple_part *p, int64_t *bytes);
int couple_part_free(couple_part *p);                     /* NULL is accepted */
const char *couple_part_last_error(const couple_part *p);

/* ---- the step without allocation ----------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  couple_step_noalloc()
 * runs the same kernels as couple_step() (same results, bit for bit) without a
 * handle: it validates *cfg as couple_init() does and takes its scratch from a
 * static device array of COUPLE_NOALLOC_SCRATCH_BYTES, one per device (each
 * device that loads the library holds it until the process ends).  It calls no
 * hipMalloc/hipFree and no allocating routine.
 *   Capacity: the scratch a call needs grows with n and the bulk cell count
 *   (about 48 bytes per particle plus 52 per bulk cell in FP32 with CIC); a call
 *   that needs more than the array holds returns COUPLE_ECAPACITY before any
 *   launch.  cfg->max_particles is not used (the capacity is the array).
 *   Not supported: vel_source = COUPLE_VEL_MLP (the network lives in a handle);
 *   COUPLE_EINVAL.
 *   Concurrency: every call on a device uses that device's one array, which
 *   keeps the last call's contents; calls that overlap on one device (other
 *   streams or threads) race and give wrong results.  Calls in order on one
 *   stream are safe.
 * Errors as couple_step(); couple_last_error(NULL) describes the last failure of
 * the calling thread. */
#define COUPLE_NOALLOC_SCRATCH_BYTES (64ll << 20)
int couple_step_noalloc(const couple_config *cfg, const couple_inputs *in, couple_outputs *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* COUPLE_H */
