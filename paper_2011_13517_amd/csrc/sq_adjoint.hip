// Adjoint dispatch over the FD radius; the kernels live in sq_adjoint_kernel.h
// and are instantiated per radius in sq_adjoint_r<R>.hip.
#include "sq_internal.h"

namespace sqk {

template <int R>
hipError_t adjoint_dispatch_r(int prec, int E, bool M, bool G, const void *args, int grid,
                              hipStream_t s, int *occ);

static hipError_t dispatch(int prec, int E, int R, bool M, bool G, const void *args, int grid,
                           hipStream_t s, int *occ) {
    switch (R) {
        case 1: return adjoint_dispatch_r<1>(prec, E, M, G, args, grid, s, occ);
        case 2: return adjoint_dispatch_r<2>(prec, E, M, G, args, grid, s, occ);
        case 3: return adjoint_dispatch_r<3>(prec, E, M, G, args, grid, s, occ);
        case 4: return adjoint_dispatch_r<4>(prec, E, M, G, args, grid, s, occ);
        case 5: return adjoint_dispatch_r<5>(prec, E, M, G, args, grid, s, occ);
        case 6: return adjoint_dispatch_r<6>(prec, E, M, G, args, grid, s, occ);
        default: return hipErrorInvalidValue;
    }
}

// Edge 27 in FP64 runs its own kernel (sq_adjoint64.hip); the kernels here
// cover FP64 up to edge 21 and FP32 up to edge 27.
int adjoint_max_edge(int prec) { return 27; }

hipError_t launch_adjoint(int prec, int E, int R, bool storeall, bool grad, const void *args,
                          int grid, hipStream_t s) {
    return dispatch(prec, E, R, storeall, grad, args, grid, s, nullptr);
}

int adjoint_blocks_per_cu(int prec, int E, int R, bool storeall, bool grad) {
    int occ = 1;
    dispatch(prec, E, R, storeall, grad, nullptr, 0, nullptr, &occ);
    return occ;
}

}  // namespace sqk
