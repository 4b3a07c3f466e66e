// handle.hpp -- the coupling handle and the phase-level step (internal; shared by
// the C ABI in api.hip and the partitioned step in part.hip).
#pragma once
#include <string>
#include <vector>

#include "couple.h"
#include "launch.hpp"

struct couple_mlp;

struct couple_handle {
    couple_config cfg;
    std::string err;
    int64_t ncell = 0, nfine = 0;
    int64_t part_stride = 0;
    cpl::SortScratch sort{};
    void *sp = nullptr, *uf4 = nullptr, *plo = nullptr, *dep = nullptr;
    void *alpha8 = nullptr;         // vof: packed stencil records of the bulk alpha
    float4 *fgrid = nullptr;        // VEL_MLP: packed bulk features
    const couple_mlp *mlp = nullptr;
    double *part = nullptr;
    const uint32_t *skeys = nullptr;  // sorted keys of the last binning (the learned source reads them)
    // per-kernel timing
    cpl::Marker mk;
    std::vector<hipEvent_t> events;
    std::vector<const char *> names;
};

namespace cpl {

// Grid geometry of a configuration (spacings, scales and volumes in the
// precision of the step).
template <typename T> inline Geo<T> make_geo(const couple_config &c) {
    Geo<T> g;
    for (int a = 0; a < 3; ++a) {
        g.nb[a] = c.nb[a];
        g.nf[a] = c.nb[a] * c.ratio;
        g.L[a] = (T)c.box[a];
        g.sb[a] = (T)((double)c.nb[a] / c.box[a]);
        g.sf[a] = (T)((double)g.nf[a] / c.box[a]);
        g.hb[a] = (T)(c.box[a] / (double)c.nb[a]);
    }
    g.ncell = (int64_t)c.nb[0] * c.nb[1] * c.nb[2];
    g.nfine = g.ncell * c.ratio * c.ratio * c.ratio;
    g.vb = (c.box[0] / c.nb[0]) * (c.box[1] / c.nb[1]) * (c.box[2] / c.nb[2]);
    g.vf = g.vb / ((double)c.ratio * c.ratio * c.ratio);
    g.inv_vb = (T)(1.0 / g.vb);
    return g;
}

// Enqueue the phases `phases` (kPhase* of launch.hpp; kPhaseDeposit includes the
// binning and sort before it) of one step with the handle's scratch.  Fine-grid
// sums (the prolongations' diagnostic partials) count the bulk cells [own_c0,
// own_c1) only.  On a launch failure returns COUPLE_EHIP with a static text in
// *what and the HIP error in *herr.  Allocates nothing.
int step_phases(couple_handle *h, const couple_inputs *in, couple_outputs *out, hipStream_t st, int phases,
                int64_t own_c0, int64_t own_c1, const char **what, hipError_t *herr);
}  // namespace cpl
