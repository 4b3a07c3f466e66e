// mlp_state.hpp -- host-side state of a couple_mlp handle (internal).
#pragma once
#include <string>

#include "couple_mlp.h"
#include "mlp.hpp"

struct couple_mlp {
    couple_mlp_config cfg;
    std::string err;
    cpl::mlp::NetBufs net;
    cpl::mlp::TrainBufs tb;
    int64_t t = 0;                           // Adam steps taken
    double mean[cpl::mlp::kFeat];            // feature standardisation
    double std[cpl::mlp::kFeat];
    double scale[3];                         // residual scale
    double *stats = nullptr;                 // fit_norm scratch: partials, then mean/std
    int64_t stats_chunks = 0;
};
