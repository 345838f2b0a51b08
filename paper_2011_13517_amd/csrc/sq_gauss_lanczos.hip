// Per-node Lanczos iteration over node regions (gfx950), the first half of the
// spectral Gauss quadrature (LSSGQ) of Section 2.2.
//
// For every node q of the work list this runs Eq. (Lanczos) on the scaled node
// Hamiltonian Hs_q = (H_q - omega)/tau, started at v_0 = e_q with b_0 = 0:
//   u = Hs v_k - b_k v_{k-1},  a_{k+1} = v_k . u,  w = u - a_{k+1} v_k,
//   b_{k+1} = |w|,  v_{k+1} = w / b_{k+1},
// and writes the Jacobi matrix entries a_1..a_K (alpha) and b_1..b_{K-1} (beta)
// of the node.  Subtracting b_k v_{k-1} before the inner product (the modified
// Gram-Schmidt order) equals the textbook a = v_k . Hs v_k in exact arithmetic
// and is the better-conditioned form in floating point.  A Krylov space that
// closes early (b_{k+1} <= 1e-14) ends the node with beta = 0 at that step;
// beta at the last step is 0 as well, so the rule of a node has
// 1 + (index of its first zero beta) points.
//
// MI355X design: the same region-resident layout as the Chebyshev kernel (one
// workgroup per region, persistent work counter, the z-pencil of each thread
// in VGPRs, the box in LDS), and the same fused step: with prev = 2 b_k v_{k-1}
// and the halving of the first Chebyshev step, one region step returns
// Hs v_k - b_k v_{k-1} in place.  The two inner products of a step are FP64
// block reductions (wave butterflies, then one LDS slot per wave that every
// thread sums in wave order, so all threads hold the same bits and the
// early-exit test is uniform across the block).
#include "sq_region.h"

namespace sqk {

// sum of x over the block, identical in every thread (NW waves, sh[NW])
template <int NW>
__device__ __forceinline__ double block_allsum(double x, double *sh) {
    x = wave_sum(x);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) t += sh[i];
    return t;
}

// One Lanczos step: on entry cur = v_k and prev = 2 b_k v_{k-1}; on a
// continuing exit cur = 2 b_{k+1} v_k and prev = v_{k+1}.  Writes a_{k+1} and
// b_{k+1} (0 when the rule ends here) and returns true when the node's rule is
// complete.
template <typename T, int E, int R, int ZS, int NW, int BLOCK, bool MASKZ, bool DREG, bool COLNL>
__device__ __forceinline__ bool lanczos_step(const RegionArgs<T> &a, const StepCtx<T, E, R> &c,
                                             const T (&d)[DREG ? E : 1], int64_t col,
                                             int64_t plane, int gz0, int n2, T (&cur)[E],
                                             T (&prev)[E], T *lds, ColNL<T> &nl,
                                             const Slot *slots, T (*pfac)[NP], double (*red)[NW],
                                             double tau, int k, double *al, double *be) {
    if constexpr (COLNL)
        region_step_col<T, E, R, ZS, BLOCK, MASKZ, DREG, false>(a, c, d, col, plane, gz0, n2, cur,
                                                                prev, lds, nl, true);
    else
        region_step<T, E, R, ZS, NW, MASKZ, DREG>(a, c, d, col, plane, gz0, n2, cur, prev, lds,
                                                  slots, pfac, true, tau);
    double pa = 0.0;
#pragma unroll
    for (int z = 0; z < E; ++z) pa += (double)cur[z] * (double)prev[z];
    const double ak = block_allsum<NW>(pa, red[0]);
    const T ta = (T)ak;
    double pb = 0.0;
#pragma unroll
    for (int z = 0; z < E; ++z) {
        prev[z] -= ta * cur[z];
        pb += (double)prev[z] * (double)prev[z];
    }
    const double bn = sqrt(block_allsum<NW>(pb, red[1]));
    const bool done = k == a.K - 1 || !(bn > 1e-14);
    if (threadIdx.x == 0) {
        al[k] = ak;
        be[k] = done ? 0.0 : bn;
    }
    if (done) return true;
    const T t2b = (T)(2.0 * bn), tinv = (T)(1.0 / bn);
#pragma unroll
    for (int z = 0; z < E; ++z) {
        cur[z] *= t2b;
        prev[z] *= tinv;
    }
    return false;
}

template <typename T, int E, int R, bool MASKZ>
__global__ void __launch_bounds__(((E * E + 63) / 64) * 64)
gauss_lanczos_kernel(const RegionArgs<T> a, double *alpha, double *beta) {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    constexpr int ZS = pencil_stride<T, E>();
    constexpr int NW = BLOCK / 64;
    constexpr int COLBYTES = BLOCK * MAXC * (int)sizeof(ColEntry);
    constexpr int RED = 2 * NW * (int)sizeof(double);
    constexpr bool COLNL =
        max_atoms_in_region<T, E, 2 * NP * (int)sizeof(T), COLBYTES + RED>() >= 32;
    constexpr int MAXAT = COLNL ? max_atoms_in_region<T, E, 2 * NP * (int)sizeof(T), COLBYTES + RED>()
                                : max_atoms_in_region<T, E, 0, RED>();
    constexpr int AT = MAXAT > 0 ? MAXAT : 1;
    constexpr bool DREG = sizeof(T) == 4 || E <= 17;

    __shared__ __align__(16) T lds[region_lds_elems<T, E>()];
    __shared__ Slot slots[AT];
    __shared__ T pfac[AT][NP];
    __shared__ T pacc[COLNL ? 2 : 1][COLNL ? AT : 1][NP];
    __shared__ ColEntry colbuf[COLNL ? BLOCK * MAXC : 1];
    __shared__ double red[2][NW];
    __shared__ int s_item, s_nat;

    const int tid = threadIdx.x;
    const double tau = a.scal->tau;
    const int K = a.K;
    StepCtx<T, E, R> c;
#pragma unroll
    for (int p = 1; p <= R; ++p) {
        c.cx[p] = (T)(-a.w[p] * a.ih2[0] / tau);
        c.cy[p] = (T)(-a.w[p] * a.ih2[1] / tau);
        c.cz[p] = (T)(-a.w[p] * a.ih2[2] / tau);
    }

    for (;;) {
        if (tid == 0) {
            s_item = atomicAdd(a.counter, 1);
            s_nat = 0;
        }
        __syncthreads();
        const int itn = s_item;
        if (itn >= a.n_items) break;
        const Item it = a.items[itn];
        c.dx = it.dim[0];
        c.dy = it.dim[1];
        c.dz = it.dim[2];
        const int npen = c.dx * c.dy;
        c.active = tid < npen;
        const int px = c.active ? tid % c.dx : 0, py = c.active ? tid / c.dx : 0;

        for (int i = tid; i < (npen + 1) * ZS; i += BLOCK) lds[i] = (T)0;
        if (a.n_atoms) gather_atoms<T, MAXAT, BLOCK>(a, it, slots, &s_nat);

        int gx = it.lo[0] + px, gy = it.lo[1] + py;
        if (a.periodic) {
            gx = wrap(gx, a.N[0]);
            gy = wrap(gy, a.N[1]);
        }
        const int64_t col = (int64_t)gx + (int64_t)a.N[0] * gy;
        const int64_t plane = (int64_t)a.N[0] * a.N[1];
        const int gz0 = a.periodic ? wrap(it.lo[2], a.N[2]) : it.lo[2];
        const int n2 = a.periodic ? a.N[2] : (1 << 30);
        T d[DREG ? E : 1];
        if constexpr (DREG) {
#pragma unroll
            for (int z = 0; z < E; ++z) {
                int gz = gz0 + z;
                gz = gz >= n2 ? gz - n2 : gz;
                d[z] = (c.active && z < c.dz) ? a.D[col + plane * gz] : (T)0;
            }
        }

        // v_0 = e_q; the partner array holds 2 b_0 v_{-1} = 0
        const bool is_ctr = c.active && px == it.ctr[0] && py == it.ctr[1];
        const int cz0 = it.ctr[2];
        T v[E], w[E];
#pragma unroll
        for (int z = 0; z < E; ++z) {
            v[z] = (is_ctr && z == cz0) ? (T)1 : (T)0;
            w[z] = (T)0;
        }
        double *al = alpha + (int64_t)it.out * K;
        double *be = beta + (int64_t)it.out * K;

#pragma unroll
        for (int p = 1; p <= R; ++p) {
            c.nb[4 * (p - 1) + 0] = (c.active && px + p < c.dx) ? tid + p : npen;
            c.nb[4 * (p - 1) + 1] = (c.active && px - p >= 0) ? tid - p : npen;
            c.nb[4 * (p - 1) + 2] = (c.active && py + p < c.dy) ? tid + p * c.dx : npen;
            c.nb[4 * (p - 1) + 3] = (c.active && py - p >= 0) ? tid - p * c.dx : npen;
        }
        c.mine = lds + tid * ZS;
        c.px = px;
        c.py = py;
        c.npen = npen;
        __syncthreads();
        c.nat = min(s_nat, MAXAT);
        if (tid == 0 && s_nat > MAXAT) atomicOr(a.status, 1);

        ColNL<T> nl{};
        if constexpr (COLNL) {
            for (int j = tid; j < c.nat; j += BLOCK) {
                const double f = 2.0 * a.h3 / tau;
                const double *cj = a.cJ + (int64_t)slots[j].atom * NP;
#pragma unroll
                for (int l = 0; l < NP; ++l) {
                    pfac[j][l] = (T)(f * cj[l]);
                    pacc[0][j][l] = (T)0;
                    pacc[1][j][l] = (T)0;
                }
            }
            int ncol = build_columns<T>(a, slots, c.nat, c.active, px, py, c.dz, colbuf + tid * MAXC);
            if (ncol > MAXC) {
                atomicOr(a.status, 2);
                ncol = MAXC;
            }
            nl.cols = colbuf + tid * MAXC;
            nl.ncol = ncol;
            nl.pacc = &pacc[0][0][0];
            nl.scale = &pfac[0][0];
            nl.maxat = AT;
            __syncthreads();
        }

        for (int k = 0; k < K; k += 2) {
            if (lanczos_step<T, E, R, ZS, NW, BLOCK, MASKZ, DREG, COLNL>(
                    a, c, d, col, plane, gz0, n2, v, w, lds, nl, slots, pfac, red, tau, k, al, be))
                break;
            if (lanczos_step<T, E, R, ZS, NW, BLOCK, MASKZ, DREG, COLNL>(
                    a, c, d, col, plane, gz0, n2, w, v, lds, nl, slots, pfac, red, tau, k + 1, al, be))
                break;
        }
        __syncthreads();
    }
}

template <typename T, int E, int R, bool M>
static hipError_t launch_one(const void *args, double *alpha, double *beta, int grid,
                             hipStream_t s) {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    hipLaunchKernelGGL((gauss_lanczos_kernel<T, E, R, M>), dim3(grid), dim3(BLOCK), 0, s,
                       *static_cast<const RegionArgs<T> *>(args), alpha, beta);
    return hipGetLastError();
}

template <typename T, int E, int R, bool M>
static int occ_one() {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gauss_lanczos_kernel<T, E, R, M>, BLOCK,
                                                     0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <typename T, int E>
static hipError_t by_r(int R, bool M, const void *args, double *al, double *be, int grid,
                       hipStream_t s, int *occ) {
#define SQ_CASE(RR)                                                                 \
    case RR:                                                                        \
        if (occ) {                                                                  \
            *occ = M ? occ_one<T, E, RR, true>() : occ_one<T, E, RR, false>();      \
            return hipSuccess;                                                      \
        }                                                                           \
        return M ? launch_one<T, E, RR, true>(args, al, be, grid, s)                \
                 : launch_one<T, E, RR, false>(args, al, be, grid, s);
    switch (R) {
        SQ_CASE(1)
        SQ_CASE(2)
        SQ_CASE(3)
        SQ_CASE(4)
        SQ_CASE(5)
        SQ_CASE(6)
        default:
            return hipErrorInvalidValue;
    }
#undef SQ_CASE
}

template <typename T>
static hipError_t by_e(int E, int R, bool M, const void *args, double *al, double *be, int grid,
                       hipStream_t s, int *occ) {
    switch (E) {
        case 9: return by_r<T, 9>(R, M, args, al, be, grid, s, occ);
        case 13: return by_r<T, 13>(R, M, args, al, be, grid, s, occ);
        case 17: return by_r<T, 17>(R, M, args, al, be, grid, s, occ);
        case 21: return by_r<T, 21>(R, M, args, al, be, grid, s, occ);
        case 27: return by_r<T, 27>(R, M, args, al, be, grid, s, occ);
        case 32:
            if constexpr (sizeof(T) == 4) return by_r<T, 32>(R, M, args, al, be, grid, s, occ);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gauss_lanczos(int prec, int E, int R, bool maskz, const void *args,
                                double *alpha, double *beta, int grid, hipStream_t s) {
    if (prec == SQ_FP64) return by_e<double>(E, R, maskz, args, alpha, beta, grid, s, nullptr);
    return by_e<float>(E, R, maskz, args, alpha, beta, grid, s, nullptr);
}

int gauss_lanczos_blocks_per_cu(int prec, int E, int R, bool maskz) {
    int occ = 1;
    if (prec == SQ_FP64) by_e<double>(E, R, maskz, nullptr, nullptr, nullptr, 0, nullptr, &occ);
    else by_e<float>(E, R, maskz, nullptr, nullptr, nullptr, 0, nullptr, &occ);
    return occ;
}

}  // namespace sqk
