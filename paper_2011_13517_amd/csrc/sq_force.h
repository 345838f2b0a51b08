// Nonlocal force by the Clenshaw-Curtis quadrature: launch interface of the
// force kernel (sq_force.hip) for the API.
#pragma once

#include "sq_internal.h"

namespace sqk {

struct ForceParams {
    double grad[3][MAX_R + 1];   // first-derivative weights / h_a, per axis and distance
    const double *cp;            // [K+1] Fermi-function coefficients, c_0 halved
    double *force;               // [n_atoms][3] FP64, accumulated
};

// whether the force kernel exists for this precision and edge bucket (the
// column projector path must fit the LDS next to the box)
bool cc_force_supported(int prec, int E);
hipError_t launch_cc_force(int prec, int E, int R, bool maskz, const void *args,
                           const ForceParams &fp, int grid, hipStream_t s);
int cc_force_blocks_per_cu(int prec, int E, int R, bool maskz);

}  // namespace sqk
