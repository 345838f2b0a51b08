// Nonlocal atomic force by the spectral Clenshaw-Curtis quadrature (Section
// 2.2, Eq. (NLforceSQ), and its discrete form in Section 3):
//   f_J,nl = -4 sum_q e_q^T V_J^q grad_h gamma_q,  gamma_q = sum'_k c_k v_k^q,
// with v_k^q the Chebyshev vectors of Eq. (Chebyshev) on the node's region,
// c_k the Fermi-function coefficients of Eq. (ChebyshevWeights) at the solved
// Fermi level (c_0 halved), grad_h the central first-derivative stencil of
// radius r on the region box (zero outside it, like the truncated
// Hamiltonian), and V_J^q the nonlocal operator of atom J on the box:
//   e_q^T V_J^q f = h^3 sum_lm c_Jl chi_Jlm(q) (chi_Jlm . f).
// Only nodes inside some atom's support contribute (chi_Jlm(q) != 0); the
// work list of this kernel holds just those.
//
// MI355X design: the region-resident Chebyshev kernel with the column
// projector path, plus gamma accumulated in VGPRs during the sweep.  After the
// sweep, per axis: gamma goes to the LDS copy of the box, each thread forms
// the derivative of its pencil (x, y from LDS, z from registers), publishes
// it, the column path projects it onto every atom of the box (LDS atomics),
// and the node's thread contracts the projections with the projector values
// at the node and adds -4 h^3 c_Jl chi_Jlm(q) (chi_Jlm . d_a gamma) to the
// atom's force with one FP64 atomic per atom and axis.  Where the column
// tables do not fit the LDS beside the box (FP64 at edge 27), the sweep and the
// projections take the wave-per-atom path, and the lane that holds the node's
// support row adds the node's term.
#include "sq_force.h"
#include "sq_region.h"

namespace sqk {

// the column path fits the LDS for this precision and edge
template <typename T, int E>
constexpr bool force_colnl() {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    constexpr int COLBYTES = BLOCK * MAXC * (int)sizeof(ColEntry);
    return max_atoms_in_region<T, E, 2 * NP * (int)sizeof(T), COLBYTES>() >= 32;
}

// the kernel exists: column path, or the wave-per-atom path with room for atoms
template <typename T, int E>
constexpr bool force_supported() {
    return force_colnl<T, E>() || max_atoms_in_region<T, E, NP * (int)sizeof(T)>() > 0;
}

template <typename T, int E, int R, bool MASKZ>
__global__ void __launch_bounds__(((E * E + 63) / 64) * 64)
cc_force_kernel(const RegionArgs<T> a, const ForceParams fp) {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    constexpr int ZS = pencil_stride<T, E>();
    constexpr int NW = BLOCK / 64;
    constexpr int COLBYTES = BLOCK * MAXC * (int)sizeof(ColEntry);
    constexpr bool COLNL = force_colnl<T, E>();
    constexpr int MAXAT = COLNL ? max_atoms_in_region<T, E, 2 * NP * (int)sizeof(T), COLBYTES>()
                                : max_atoms_in_region<T, E, NP * (int)sizeof(T)>();
    constexpr int AT = MAXAT > 0 ? MAXAT : 1;
    // gamma takes E more VGPRs than the forward sweep: the diagonal is re-read
    // from L2 at the largest FP32 edge, and the stencil recomputes its neighbour
    // offsets per step (low-register variant), instead of spilling
    constexpr bool DREG = (sizeof(T) == 4 && E <= 21) || E <= 17;
    constexpr bool LOWREG = E >= 27 && COLNL;
    if constexpr (!force_supported<T, E>()) {
        return;
    } else {
    __shared__ __align__(16) T lds[region_lds_elems<T, E>()];
    __shared__ Slot slots[AT];
    __shared__ T pfac[AT][NP];
    __shared__ T pacc[COLNL ? 2 : 1][COLNL ? AT : 1][NP];
    __shared__ ColEntry colbuf[COLNL ? BLOCK * MAXC : 1];
    __shared__ T dots[COLNL ? 1 : AT][NP];   // wave-per-atom path: raw projections
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
        gather_atoms<T, MAXAT, BLOCK>(a, it, slots, &s_nat);

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

        const bool is_ctr = c.active && px == it.ctr[0] && py == it.ctr[1];
        const int cz0 = it.ctr[2];
        T v[E], w[E], g[E];
        const T c0 = (T)fp.cp[0];
#pragma unroll
        for (int z = 0; z < E; ++z) {
            v[z] = (is_ctr && z == cz0) ? (T)1 : (T)0;
            w[z] = (T)0;
            g[z] = c0 * v[z];
        }
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
            int ncol = build_columns<T>(a, slots, c.nat, c.active, px, py, c.dz,
                                        colbuf + tid * MAXC);
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

        // Chebyshev sweep (the newest vector alternates between v and w),
        // gamma += c'_k v_k after every step
        for (int k = 0; k < K; k += 2) {
            if constexpr (COLNL)
                region_step_col<T, E, R, ZS, BLOCK, MASKZ, DREG, false, LOWREG>(
                    a, c, d, col, plane, gz0, n2, v, w, lds, nl, k == 0);
            else
                region_step<T, E, R, ZS, NW, MASKZ, DREG>(a, c, d, col, plane, gz0, n2, v, w, lds,
                                                          slots, pfac, k == 0, tau);
            {
                const T ck = (T)fp.cp[k + 1];
#pragma unroll
                for (int z = 0; z < E; ++z) g[z] += ck * w[z];
            }
            if (k + 1 < K) {
                if constexpr (COLNL)
                    region_step_col<T, E, R, ZS, BLOCK, MASKZ, DREG, false, LOWREG>(
                        a, c, d, col, plane, gz0, n2, w, v, lds, nl, false);
                else
                    region_step<T, E, R, ZS, NW, MASKZ, DREG>(a, c, d, col, plane, gz0, n2, w, v,
                                                              lds, slots, pfac, false, tau);
                const T ck = (T)fp.cp[k + 2];
#pragma unroll
                for (int z = 0; z < E; ++z) g[z] += ck * v[z];
            }
        }

        // per axis: d_a gamma on the box, its projections, the node's term
        // (pacc[nl.par] is zero here: each step clears the next step's buffer)
#pragma unroll 1
        for (int ax = 0; ax < 3; ++ax) {
            __syncthreads();
            if (c.active) store_pencil<T, E, ZS>(c.mine, g);
            __syncthreads();
            T dg[E];
#pragma unroll
            for (int z = 0; z < E; ++z) dg[z] = (T)0;
            if (ax == 2) {
#pragma unroll
                for (int p = 1; p <= R; ++p) {
                    const T cf = (T)fp.grad[2][p];
#pragma unroll
                    for (int z = 0; z < E; ++z) {
                        T s = (T)0;
                        if (z + p < E) s += g[z + p];
                        if (z - p >= 0) s -= g[z - p];
                        dg[z] += cf * s;
                    }
                }
            } else {
#pragma unroll
                for (int p = 1; p <= R; ++p) {
                    const T cf = (T)(ax == 0 ? fp.grad[0][p] : fp.grad[1][p]);
                    const int up = ax == 0 ? ((c.active && px + p < c.dx) ? tid + p : npen)
                                           : ((c.active && py + p < c.dy) ? tid + p * c.dx : npen);
                    const int dn = ax == 0 ? ((c.active && px - p >= 0) ? tid - p : npen)
                                           : ((c.active && py - p >= 0) ? tid - p * c.dx : npen);
                    axpy_pencil<T, E, ZS>(dg, cf, lds + up * ZS);
                    axpy_pencil<T, E, ZS>(dg, -cf, lds + dn * ZS);
                }
            }
            __syncthreads();
            if (c.active) store_pencil<T, E, ZS>(c.mine, dg);
            __syncthreads();
            if constexpr (!COLNL) {
                // wave-per-atom path: raw projections of d_a gamma, then the lane
                // holding the node's support row (if any) adds the node's term
                if (c.nat)
                    projector_dots<T, ZS, NW, false>(a, slots, pfac, dots, nullptr, lds, c.nat,
                                                     c.dx, c.dy, c.dz, tau);
                __syncthreads();
                const int lane = tid & 63, wave = tid >> 6;
                for (int j = wave; j < c.nat; j += NW) {
                    const Slot sl = slots[j];
                    for (int e = lane; e < sl.count; e += 64) {
                        const int pk = a.sup_pack[sl.start + e];
                        if (sl.ox + (pk & 1023) != it.ctr[0] ||
                            sl.oy + ((pk >> 10) & 1023) != it.ctr[1] ||
                            sl.oz + ((pk >> 20) & 1023) != cz0)
                            continue;
                        const T *chq = a.chi + (int64_t)(sl.start + e) * NP;
                        const double *cj = a.cJ + (int64_t)sl.atom * NP;
                        double f = 0.0;
#pragma unroll
                        for (int l = 0; l < NP; ++l)
                            f += cj[l] * (double)chq[l] * (double)dots[j][l];
                        atomicAdd(&fp.force[3 * sl.atom + ax], -4.0 * a.h3 * f);
                    }
                }
                continue;
            } else {
            if (c.nat) col_dots<T, false>(a, nl, c.mine);
            __syncthreads();
            if (is_ctr) {
                const T *pa = nl.pacc + (int64_t)nl.par * nl.maxat * NP;
                for (int e = 0; e < nl.ncol; ++e) {
                    const ColEntry ce = nl.cols[e];
                    if (cz0 < ce.zlo || cz0 >= ce.zlo + ce.n) continue;
                    const int atom = slots[ce.slot].atom;
                    const T *chq = a.chi + (int64_t)(ce.row0 + (cz0 - ce.zlo)) * NP;
                    const double *cj = a.cJ + (int64_t)atom * NP;
                    double f = 0.0;
#pragma unroll
                    for (int l = 0; l < NP; ++l)
                        f += cj[l] * (double)chq[l] * (double)pa[ce.slot * NP + l];
                    atomicAdd(&fp.force[3 * atom + ax], -4.0 * a.h3 * f);
                }
            }
            __syncthreads();
            for (int i = tid; i < c.nat * NP; i += BLOCK) nl.pacc[(int64_t)nl.par * nl.maxat * NP + i] = (T)0;
            }
        }
        __syncthreads();
    }
    }
}

template <typename T, int E, int R, bool M>
static hipError_t launch_one(const void *args, const ForceParams &fp, int grid, hipStream_t s) {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    if constexpr (!force_supported<T, E>()) {
        return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((cc_force_kernel<T, E, R, M>), dim3(grid), dim3(BLOCK), 0, s,
                           *static_cast<const RegionArgs<T> *>(args), fp);
        return hipGetLastError();
    }
}

template <typename T, int E, int R, bool M>
static int occ_one() {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cc_force_kernel<T, E, R, M>, BLOCK, 0) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <typename T, int E>
static hipError_t by_r(int R, bool M, const void *args, const ForceParams *fp, int grid,
                       hipStream_t s, int *occ) {
#define SQ_CASE(RR)                                                                 \
    case RR:                                                                        \
        if (occ) {                                                                  \
            *occ = M ? occ_one<T, E, RR, true>() : occ_one<T, E, RR, false>();      \
            return hipSuccess;                                                      \
        }                                                                           \
        return M ? launch_one<T, E, RR, true>(args, *fp, grid, s)                   \
                 : launch_one<T, E, RR, false>(args, *fp, grid, s);
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
static hipError_t by_e(int E, int R, bool M, const void *args, const ForceParams *fp, int grid,
                       hipStream_t s, int *occ) {
    switch (E) {
        case 9: return by_r<T, 9>(R, M, args, fp, grid, s, occ);
        case 13: return by_r<T, 13>(R, M, args, fp, grid, s, occ);
        case 17: return by_r<T, 17>(R, M, args, fp, grid, s, occ);
        case 21: return by_r<T, 21>(R, M, args, fp, grid, s, occ);
        case 27: return by_r<T, 27>(R, M, args, fp, grid, s, occ);
        case 32:
            if constexpr (sizeof(T) == 4) return by_r<T, 32>(R, M, args, fp, grid, s, occ);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

bool cc_force_supported(int prec, int E) {
    auto pick = [](auto tag, int e) {
        using T = decltype(tag);
        switch (e) {
            case 9: return force_supported<T, 9>();
            case 13: return force_supported<T, 13>();
            case 17: return force_supported<T, 17>();
            case 21: return force_supported<T, 21>();
            case 27: return force_supported<T, 27>();
            case 32: return sizeof(T) == 4 && force_supported<T, 32>();
            default: return false;
        }
    };
    return prec == SQ_FP64 ? pick(double{}, E) : pick(float{}, E);
}

hipError_t launch_cc_force(int prec, int E, int R, bool maskz, const void *args,
                           const ForceParams &fp, int grid, hipStream_t s) {
    if (prec == SQ_FP64) return by_e<double>(E, R, maskz, args, &fp, grid, s, nullptr);
    return by_e<float>(E, R, maskz, args, &fp, grid, s, nullptr);
}

int cc_force_blocks_per_cu(int prec, int E, int R, bool maskz) {
    int occ = 1;
    if (prec == SQ_FP64) by_e<double>(E, R, maskz, nullptr, nullptr, 0, nullptr, &occ);
    else by_e<float>(E, R, maskz, nullptr, nullptr, 0, nullptr, &occ);
    return occ;
}

}  // namespace sqk
