// launch.hpp -- host-side launchers of the coupling kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace cpl {

// Optional per-kernel event recording (profiling): mark(name) records an event
// on the stream just before the kernel `name` is launched; mark(nullptr) closes
// the step.  A no-op when `on` is false or the pool is full.
struct Marker {
    bool on = false;
    hipEvent_t *events = nullptr;
    const char **names = nullptr;
    int cap = 0, used = 0;
    void mark(const char *name, hipStream_t st) {
        if (!on || used >= cap) return;
        if (hipEventRecord(events[used], st) != hipSuccess) {
            (void)hipGetLastError();
            on = false;
            return;
        }
        names[used++] = name;
    }
};

// Scratch of the radix sort, owned by the handle.
struct SortScratch {
    uint32_t *keys_a, *keys_b;   // [max_particles]
    uint32_t *vals_a, *vals_b;   // [max_particles]
    uint32_t *hist;              // [256 * max_tiles]
    uint32_t *totals;            // [256]
};

int sort_tiles(int64_t n);

// One stable radix pass over keys < 2^bits (1 <= bits <= 8) from the identity
// order: keys_out / ids_out in ascending key, ties by id; s.totals[d] receives
// the number of keys equal to d.
hipError_t launch_stable_partition(const uint32_t *keys, int64_t n, int bits, const SortScratch &s, uint32_t *keys_out,
                                   uint32_t *ids_out, hipStream_t st);

// Bin particles, sort (cell, id), and build start/count.
template <typename T>
hipError_t launch_bin_sort(const T *pos, const T *diam, int64_t n, const Geo<T> &g, int32_t *cell, vec4<T> *pk,
                           int32_t *perm, int32_t *start, int32_t *count, const SortScratch &s, double *part_nout,
                           const uint32_t **sorted_keys, Marker *mk, hipStream_t st);

// Device state of the learned surrogate as the step kernels read it.
struct MlpNet {
    const uint16_t *wt[4];   // BF16 W^T of each layer, [padded fan-out][padded fan-in]
    const float *params;     // FP32 master parameters (biases are read from here)
    const float *mean_inv;   // [2][224] feature mean, then 1/std (0 in the padding)
    float scale[3];          // per-component scale of the residual
};

// Everything the stage kernels need for one step.
template <typename T> struct StepArgs {
    Geo<T> g;
    int64_t n;
    int ratio;
    int cic;           // deposition / gather weights: 1 = CIC, 0 = NGP
    int sum_mode;      // SumMode of the per-cell sums (FP32 modes)
    int vel_source;    // 0 fine, 1 bulk, 2 given, 3 learned surrogate (+ fine fallback)
    int advect;
    int semi;          // semi-implicit source fields K, KU
    int vof;           // two-fluid drag: (rho_f, mu_f) mixed with (rho_f2, mu_f2) by alpha
    T dt, rho_f, mu_f, rho_p, eps_min;
    T rho_f2, mu_f2;
    float phi_fp64;    // FP32 modes: FP64 void fraction above this particle solid fraction
    // inputs
    T *pos, *vel;
    const T *diam;
    const T *fine[4];      // u, v, w, p
    const T *uf_given;     // [n][3]
    const T *fine_alpha;   // [nfine] liquid volume fraction (vof)
    // outputs
    T *drag, *beta;
    const int32_t *perm, *start;
    T *phi, *F, *U, *P, *G;  // bulk
    T *fine_eps, *fine_F;    // fine
    T *K, *KU;               // bulk semi-implicit coefficient [ncell] and beta u_p source [3][ncell]
    T *alpha;                // bulk liquid volume fraction [ncell] (vof)
    T *alpha8;               // [ncell][8] bulk alpha at cell + {0,1}^3 (clamped): one stencil record per cell (vof)
    T *fine_K, *fine_KU;     // the same prolonged to the fine grid
    double *diag;
    // scratch
    vec4<T> *sp;     // sorted particles (x, y, z, d)
    vec4<T> *uf4;    // per particle (input order): packed (x, y, z, d) from binning until the
                     // gather has read it, then fluid velocity and void fraction until the
                     // drag has read it, then (beta, beta u_p) when semi
    T *Plo;          // [ncell] low word of the restricted pressure (Kahan compensation)
    T *dep_partial;  // [4][nc][ncell] per-source-group partial sums of the CIC deposition (nc <= 4)
    double *part;    // [SL_COUNT][max_blocks]
    int64_t part_stride;
    Marker *mk;      // per-kernel event recording (never null)
    // optional output: fluid velocity used by the drag, [n][3] (input order)
    T *uf_out;
    // learned surrogate (vel_source 3)
    const uint32_t *keys;        // containing cell of each particle in the sorted order
    MlpNet net;                  // device state of the network
    float4 *fgrid;               // [ncell][2] packed bulk features (eps, U, G)
    int64_t step;                // caller's step index: selects the checked sample
    int mlp_period;              // one particle in mlp_period is checked (id mod period)
    float mlp_tol;               // brick falls back to the fine lookup above this error
    int64_t n_bricks;            // 8x8x8-cell bricks of the bulk grid
    int64_t own_c0, own_c1;      // bulk cells whose fine cells enter the fine-grid sums (all, except in a
                                 // partition of the partitioned step: its owned layers)
};

// Stage launchers: the phases of a step after binning and sorting: the sorted
// copy and the volume deposition; the velocity at the particles and the drag;
// the momentum-source deposition (and K, KU); the prolongations; the FP64 sums.
// A whole step runs them all (kPhaseAll); the partitioned step runs them one at
// a time with halo exchanges in between.
enum { kPhaseDeposit = 1, kPhaseVelocity = 2, kPhaseSource = 4, kPhaseProlong = 8, kPhaseDiag = 16, kPhaseAll = 31 };
template <typename T> hipError_t launch_stages(const StepArgs<T> &a, hipStream_t st, int phases = kPhaseAll);

// Learned-surrogate stages of the step (mlp.hip): packed features and pressure
// gradient, inference, sampled check with fine fallback.  Each check workgroup
// writes one partial per MLP diagnostic slot; mlp_check_blocks() is their number.
void launch_mlp_pack(const StepArgs<float> &a, hipStream_t st);
void launch_mlp_infer(const StepArgs<float> &a, hipStream_t st);
void launch_mlp_check(const StepArgs<float> &a, hipStream_t st);
int64_t mlp_check_blocks(int64_t n_bricks);
int64_t bricks_of(const int nb[3]);

// Deposition (deposit.hip); each returns the number of workgroups launched
// (one FP64 partial per workgroup and diagnostic slot).
template <typename T, int SM> int launch_deposit_phi(const StepArgs<T> &a, hipStream_t st);
template <typename T, int SM> int launch_deposit_force(const StepArgs<T> &a, hipStream_t st);
template <typename T, int SM> int launch_deposit_semi(const StepArgs<T> &a, hipStream_t st);
int deposit_blocks(const int nb[3], int64_t ncell, int cic);
// Source rows per group of the CIC row pass (1 or 2 in y and z): the partial
// buffer holds (G == 1 ? 9 : 4) slots per cell and component.
int deposit_group(const int nb[3]);

// Workgroups of a prolongation launch (stages.hip), one FP64 partial each per
// prolonged field.
int64_t prolong_tiles(const int nb[3]);

}  // namespace cpl
