// FP64 adjoint for the edge-27 bucket (sq_adjoint64.h), all FD radii.
#include "sq_adjoint64.h"

namespace sqk {

namespace {
hipError_t a64_dispatch(int R, const void *args, int grid, hipStream_t s, int *occ) {
    switch (R) {
        case 1: return a64_launch_one<1>(args, grid, s, occ);
        case 2: return a64_launch_one<2>(args, grid, s, occ);
        case 3: return a64_launch_one<3>(args, grid, s, occ);
        case 4: return a64_launch_one<4>(args, grid, s, occ);
        case 5: return a64_launch_one<5>(args, grid, s, occ);
        case 6: return a64_launch_one<6>(args, grid, s, occ);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

bool adjoint64_edge(int prec, int E) { return prec == SQ_FP64 && E == A64_EDGE; }

int64_t adjoint64_slot_elems(int K, int E) { return a64_slot_elems(K, E); }

int64_t adjoint64_max_grid() { return A64_MAX_GRID; }

hipError_t launch_adjoint64(int E, int R, bool grad, const void *args, int grid, hipStream_t s) {
    if (E != A64_EDGE) return hipErrorInvalidValue;
    (void)grad;   // dR is formed in the final pass when requested
    return a64_dispatch(R, args, grid, s, nullptr);
}

int adjoint64_blocks_per_cu(int E, int R, bool grad) {
    int occ = 1;
    (void)grad;
    if (E == A64_EDGE) (void)a64_dispatch(R, nullptr, 0, nullptr, &occ);
    return occ;
}

}  // namespace sqk
