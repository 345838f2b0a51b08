// Forward Chebyshev recurrence over node regions (gfx950).
//
// Computes, for every node q of the work list, the moments
//   mu_k^q = e_q^T T_k(Hs_q) e_q,  k = 0..K,
// of the scaled node Hamiltonian Hs_q = (H_q - omega)/tau (Section 2.2), where
// H_q is the Kohn-Sham Hamiltonian -1/2 Lap_h + V + V_nl restricted to the
// node's region of influence (Section 3), by the three-term recurrence of
// Eq. (Chebyshev): v_0 = e_q, v_1 = Hs v_0, v_{k+1} = 2 Hs v_k - v_{k-1}.
//
// MI355X design: one workgroup owns one region at a time (persistent, work
// counter in HBM).  Thread t owns the z-pencil (x, y) = (t mod dx, t / dx) of
// the box and keeps v_k, v_{k-1} and the scaled diagonal of its pencil in
// VGPRs, so the recurrence state never leaves the CU.  Each step publishes v_k
// to an LDS copy of the box laid out pencil-major (z contiguous, stride padded
// for conflict-free 16-byte reads, plus one all-zero pencil standing in for
// every out-of-box neighbour), then every thread forms
//   2 Hs v_k = D v_k + sum_p a_{p,x}(v[x+p] + v[x-p]) + ... (LDS for x and y,
//              registers for z) + 2 (h^3/tau) sum_J sum_lm c_Jl chi (chi . v_k)
// and v_{k+1} = 2 Hs v_k - v_{k-1} stays in its registers.  The nonlocal
// projector block works per pencil: each thread projects its own pencil (read
// back from LDS) onto the pieces of atom supports that cross it, the four dot
// products chi_Jlm . v_k of every atom are reduced over the box with LDS
// atomics, and after the step's second barrier each thread adds the rank-4
// term to its own pencil (no atomics, no extra pass, no extra barrier).  The
// projector tables are stored column-major per atom with a column index, so a
// pencil's piece of a support is one contiguous run of rows.  When the box
// and the column tables do not fit the LDS (FP64 at edge 27), a wave-per-atom
// two-pass variant is used instead.
#include "sq_region.h"

namespace sqk {

template <typename T, int E, int R, bool MASKZ>
__global__ void __launch_bounds__(((E * E + 63) / 64) * 64)
cheb_forward_kernel(const RegionArgs<T> a) {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    constexpr int ZS = pencil_stride<T, E>();
    constexpr int NW = BLOCK / 64;
    constexpr int COLBYTES = BLOCK * MAXC * (int)sizeof(ColEntry);
    constexpr bool COLNL = max_atoms_in_region<T, E, 2 * NP * (int)sizeof(T), COLBYTES>() >= 32;
    constexpr int MAXAT = COLNL ? max_atoms_in_region<T, E, 2 * NP * (int)sizeof(T), COLBYTES>()
                                : max_atoms_in_region<T, E>();
    constexpr int AT = MAXAT > 0 ? MAXAT : 1;
    constexpr bool DREG = sizeof(T) == 4 || E <= 17;   // keep D in VGPRs when it fits

    __shared__ __align__(16) T lds[region_lds_elems<T, E>()];
    __shared__ Slot slots[AT];
    __shared__ T pfac[AT][NP];                       // column path: 2 h^3 c / tau
    __shared__ T pacc[COLNL ? 2 : 1][COLNL ? AT : 1][NP];
    __shared__ ColEntry colbuf[COLNL ? BLOCK * MAXC : 1];
    __shared__ int s_item, s_nat;

    const int tid = threadIdx.x;
    const double tau = a.scal->tau;
    const int K = a.K;
    StepCtx<T, E, R> c;
    // off-diagonal weights of 2 Hs: -w_p / (tau h_a^2)
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

        // scaled diagonal of this pencil
        int gx = it.lo[0] + px, gy = it.lo[1] + py;
        if (a.periodic) {
            gx = wrap(gx, a.N[0]);
            gy = wrap(gy, a.N[1]);
        }
        const int64_t col = (int64_t)gx + (int64_t)a.N[0] * gy;
        const int64_t plane = (int64_t)a.N[0] * a.N[1];
        // z coordinates of the pencil are gz0, gz0 + 1, ... wrapped once at n2
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

        // v_0 = e_q
        const bool is_ctr = c.active && px == it.ctr[0] && py == it.ctr[1];
        const int cz0 = it.ctr[2];
        T v[E], w[E];
#pragma unroll
        for (int z = 0; z < E; ++z) {
            v[z] = (is_ctr && z == cz0) ? (T)1 : (T)0;
            w[z] = (T)0;
        }
        double *mu = a.moments + (int64_t)it.out * (K + 1);
        if (tid == 0) mu[0] = 1.0;

        // neighbour pencils (the zero pencil npen stands for outside the box)
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
            for (int k = 0; k < K; k += 2) {
                region_step_col<T, E, R, ZS, BLOCK, MASKZ, DREG, false>(a, c, d, col, plane, gz0, n2,
                                                                        v, w, lds, nl, k == 0);
                if (is_ctr) mu[k + 1] = pick(w, cz0);
                if (k + 1 < K) {
                    region_step_col<T, E, R, ZS, BLOCK, MASKZ, DREG, false>(a, c, d, col, plane, gz0,
                                                                            n2, w, v, lds, nl, false);
                    if (is_ctr) mu[k + 2] = pick(v, cz0);
                }
            }
        } else {
        // ping-pong: the newest vector alternates between v and w
        for (int k = 0; k < K; k += 2) {
            region_step<T, E, R, ZS, NW, MASKZ, DREG>(a, c, d, col, plane, gz0, n2, v, w, lds, slots, pfac,
                                                      k == 0, tau);
            if (is_ctr) mu[k + 1] = pick(w, cz0);
            if (k + 1 < K) {
                region_step<T, E, R, ZS, NW, MASKZ, DREG>(a, c, d, col, plane, gz0, n2, w, v, lds, slots, pfac,
                                                          false, tau);
                if (is_ctr) mu[k + 2] = pick(v, cz0);
            }
        }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------- //
// dispatch over (precision, edge bucket, radius, z masking)
// ------------------------------------------------------------------------- //
template <typename T, int E, int R, bool M>
static hipError_t launch_one(const void *args, int grid, hipStream_t s) {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    hipLaunchKernelGGL((cheb_forward_kernel<T, E, R, M>), dim3(grid), dim3(BLOCK), 0, s,
                       *static_cast<const RegionArgs<T> *>(args));
    return hipGetLastError();
}

template <typename T, int E, int R, bool M>
static int occ_one() {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cheb_forward_kernel<T, E, R, M>, BLOCK,
                                                     0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <typename T, int E>
static hipError_t by_r(int R, bool M, const void *args, int grid, hipStream_t s, int *occ) {
#define SQ_CASE(RR)                                                                 \
    case RR:                                                                        \
        if (occ) {                                                                  \
            *occ = M ? occ_one<T, E, RR, true>() : occ_one<T, E, RR, false>();      \
            return hipSuccess;                                                      \
        }                                                                           \
        return M ? launch_one<T, E, RR, true>(args, grid, s)                        \
                 : launch_one<T, E, RR, false>(args, grid, s);
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
static hipError_t by_e(int E, int R, bool M, const void *args, int grid, hipStream_t s,
                       int *occ) {
    switch (E) {
        case 9: return by_r<T, 9>(R, M, args, grid, s, occ);
        case 13: return by_r<T, 13>(R, M, args, grid, s, occ);
        case 17: return by_r<T, 17>(R, M, args, grid, s, occ);
        case 21: return by_r<T, 21>(R, M, args, grid, s, occ);
        case 27: return by_r<T, 27>(R, M, args, grid, s, occ);
        case 32:
            if constexpr (sizeof(T) == 4) return by_r<T, 32>(R, M, args, grid, s, occ);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forward(int prec, int E, int R, bool maskz, const void *args, int grid,
                          hipStream_t s) {
    if (prec == SQ_FP64) return by_e<double>(E, R, maskz, args, grid, s, nullptr);
    return by_e<float>(E, R, maskz, args, grid, s, nullptr);
}

int forward_blocks_per_cu(int prec, int E, int R, bool maskz) {
    int occ = 1;
    if (prec == SQ_FP64) by_e<double>(E, R, maskz, nullptr, 0, nullptr, &occ);
    else by_e<float>(E, R, maskz, nullptr, 0, nullptr, &occ);
    return occ;
}

}  // namespace sqk
