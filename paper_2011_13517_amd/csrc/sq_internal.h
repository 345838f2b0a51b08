// Internal declarations shared by the HIP sources of libsq (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sq.h"

namespace sqk {

constexpr int NP = 4;          // projector slots per atom (n_proj <= 4, zero padded)
constexpr int MAX_R = 6;       // largest FD radius supported (order 12)
constexpr int LDS_BYTES = 163840;   // gfx950: 160 KiB of LDS per workgroup
constexpr int MAX_REGION_ATOMS = 128;  // cap on the atom list of one region box
// store-all adjoint slot: v_0..v_{K-1} ([k][z][pencil]), then the projections
// (chi . v_k, and dchi/dR . v_k where formed) of every atom of the box
// ([k][atom][4 NP]), then the dR row accumulators W
constexpr int64_t storeall_proj_elems(int K) { return (int64_t)K * MAX_REGION_ATOMS * 4 * NP; }
constexpr int MAXC = 4;    // atom supports crossing one pencil of a box
// dR accumulators W of the store-all adjoint: [row][thread][NP] (a thread's rows
// numbered densely over its column pieces, at most MAXC * E),
// NP-vector aligned (the slot stride and the W offset are multiples of NP)
constexpr int64_t storeall_w_elems(int E) {
    return (int64_t)MAXC * E * NP * ((E * E + 63) / 64 * 64);
}
constexpr int64_t round_np(int64_t n) { return (n + NP - 1) / NP * NP; }
constexpr int64_t storeall_w_offset(int K, int E) {
    return round_np((int64_t)K * E * E * E + storeall_proj_elems(K));
}
constexpr int64_t storeall_slot_elems(int K, int E) {
    return storeall_w_offset(K, E) + storeall_w_elems(E);
}
constexpr int SCAN_BLOCK = 256;

// One region of influence: box origin in V-grid coordinates (periodic boxes
// are unwrapped and may start below 0), extent, node position in the box and
// the output row of the node.
struct Item {
    int32_t lo[3];
    int32_t dim[3];
    int32_t ctr[3];
    int32_t out;
};

// Support of one atom: unwrapped bounding box (V-grid coordinates) of its
// support points and the rows of the per-point tables.
struct AtomDev {
    int32_t lo[3];
    int32_t dim[3];
    int32_t start;      // first row of the region tables (column-major support)
    int32_t count;
    int32_t col_start;  // first column of the atom in the column index
    int32_t pad_;
};

// Device-resident scalars of a context (all FP64 unless integer).
struct Scalars {
    double omega, tau;      // scaling of Section 2.2
    double lmin, lmax;      // spectral bounds in use
    double lambda_f;        // Fermi level of the last solve
    double lo, hi, mid;     // bisection bracket
    double ne_lo, ne_hi, ne_mid;
    double ne_target, tol;
    int32_t done;           // bisection finished
    int32_t iters;
    int32_t status;         // SQ_OK or SQ_ERR_* found on the device
    int32_t nq_log2;        // Chebyshev-Gauss points N_q = 2^nq_log2
    int32_t max_iter;
    int32_t pad_;
};

// Region-kernel arguments (forward and adjoint share the geometry part).
template <typename T>
struct RegionArgs {
    const Item *items;
    int32_t n_items;
    int32_t *counter;          // persistent work counter (reset before launch)
    const T *D;                // scaled diagonal 2 (V + kin - omega) / tau on the V grid
    int32_t N[3];              // V grid
    int32_t periodic;
    const Scalars *scal;
    double w[MAX_R + 1];       // FD weights
    double ih2[3];             // 1 / h_a^2
    double h3;                 // h0 h1 h2
    int32_t K;
    double *moments;           // [n_nodes][K+1]
    // projectors
    int32_t n_atoms;
    const AtomDev *atoms;
    const int32_t *sup_pack;   // packed (x | y << 10 | z << 20) offsets in the atom box
    const int32_t *colidx;     // per atom column (x, y) of its box: {first row, zoff | n << 16}
    const T *chi;              // [nnz][NP]
    const T *dchi;             // [nnz][NP][3]
    const double *cJ;          // [n_atoms][NP]
    int32_t *status;
};

// Adjoint-only arguments.
template <typename T>
struct AdjointArgs {
    RegionArgs<T> g;
    const double *coef_c;      // [K+1] c'_k (c_0 halved)
    const double *coef_d;      // [K+1] d'_k
    const double *g_rho;       // [n_nodes] or null
    const double *g_u;         // [n_nodes] or null
    double *dV;                // V grid, accumulated, or null
    double *dR;                // [n_atoms][3], accumulated, or null
    T *ckpt;                   // per workgroup: [n_ckpt][2][E^3] pairs, or [K][E^3] (store-all)
    int32_t ckpt_every;
    int32_t n_ckpt;
    int64_t ckpt_stride;       // elements per workgroup slot
};

// Launchers implemented in sq_forward.hip / sq_adjoint.hip.  They return
// hipSuccess or the launch error; `E` is the region-edge bucket.
hipError_t launch_forward(int prec, int E, int R, bool maskz, const void *args, int grid,
                          hipStream_t s);
int forward_blocks_per_cu(int prec, int E, int R, bool maskz);
// Lanczos sweep of the Gauss quadrature: alpha, beta [n_nodes][K] (FP64)
hipError_t launch_gauss_lanczos(int prec, int E, int R, bool maskz, const void *args,
                                double *alpha, double *beta, int grid, hipStream_t s);
int gauss_lanczos_blocks_per_cu(int prec, int E, int R, bool maskz);
// storeall: the forward pass keeps every v_k (checkpoint stride 1) instead
// of checkpoints every ckpt_every steps plus the reverse rebuild.
hipError_t launch_adjoint(int prec, int E, int R, bool storeall, bool grad, const void *args,
                          int grid, hipStream_t s);
int adjoint_blocks_per_cu(int prec, int E, int R, bool storeall, bool grad);
int adjoint_max_edge(int prec);
// FP64 adjoint for the largest bucket (edge 27: the FP64 box fills the LDS);
// its slot per workgroup holds v_k, vt_{k+1}, the forward and reverse
// projections, the atom list and the column entries (doubles).  Its 32-bit
// stream offsets bound the V grid to adjoint64_max_grid() points.
bool adjoint64_edge(int prec, int E);
int64_t adjoint64_max_grid();
int64_t adjoint64_slot_elems(int K, int E);
hipError_t launch_adjoint64(int E, int R, bool grad, const void *args, int grid, hipStream_t s);
int adjoint64_blocks_per_cu(int E, int R, bool grad);

// Sets the thread-local message returned by sq_last_error and returns st.
sq_status set_error(sq_status st, const char *msg);

// Region-edge buckets with a compiled kernel (the largest edge of every box
// must not exceed the bucket).
constexpr int EDGE_BUCKETS[] = {9, 13, 17, 21, 27, 32};
inline int edge_bucket(int e) {
    for (int b : EDGE_BUCKETS)
        if (e <= b) return b;
    return -1;
}
// FP64 regions are limited by LDS (one pencil array of the whole box).
inline int max_edge(int prec) { return prec == SQ_FP64 ? 27 : 32; }

// Stride of a pencil in LDS, in elements: z-contiguous pencils padded so that
// 16-byte vector reads of neighbouring pencils fall in distinct bank groups
// (stride = 4 mod 8 words), when that still fits.
template <typename T, int E>
constexpr int pencil_stride() {
    if (sizeof(T) == 4) {
        int s = (E + 3) / 4 * 4;
        if (s % 8 == 0) s += 4;
        return s;
    }
    // FP64: an even stride keeps 16-byte pairs aligned; fall back to E when
    // the padded box would not leave room for the atom tables.
    if (E % 2 == 0) return E;
    return (E * E + 1) * (E + 1) * 8 <= LDS_BYTES - 4096 ? E + 1 : E;
}
template <typename T, int E>
constexpr int region_lds_elems() {
    return (E * E + 1) * pencil_stride<T, E>();
}
template <typename T, int E>
constexpr int fits_lds() {
    return region_lds_elems<T, E>() * (int)sizeof(T) <= LDS_BYTES - 4096;
}

}  // namespace sqk
