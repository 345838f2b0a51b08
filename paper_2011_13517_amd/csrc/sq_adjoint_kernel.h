// Adjoint (reverse mode) of the region recurrence (gfx950).
//
// For node q with output y_q = sum_k a_k mu_k^q, a_k = 2 (g_rho c'_k + g_u d'_k)
// (the cotangents of rho^q and u^q; c'_0 = c_0/2), differentiating
// Eq. (Chebyshev) in reverse gives
//   vt_K = a_K e_q,   vt_k = a_k e_q + 2 Hs vt_{k+1} - vt_{k+2}   (k >= 1),
//   dy/dV(x)  = (1/tau) [vt_1(x) v_0(x) + 2 sum_{k=1}^{K-1} vt_{k+1}(x) v_k(x)],
//   dy/dR_J   = (h^3/tau) sum_k alpha_k sum_lm c_Jl
//               [(vt_{k+1}.dchi_Jlm)(chi_Jlm.v_k) + (vt_{k+1}.chi_Jlm)(dchi_Jlm.v_k)],
// alpha_0 = 1, alpha_k = 2, at fixed lambda_f, omega, tau.
//
// The reverse sweep needs v_k for k = K-1 .. 0.  The recurrence is run
// forward once, writing (v_c, v_{c+1}) to HBM every `ckpt_every` steps; the
// sweep then rebuilds v_{k-1} = 2 Hs v_k - v_{k+1} in registers alongside
// vt, and re-anchors on the stored exact pair at every checkpoint, so the
// rounding drift of the rebuilt vectors spans at most ckpt_every steps and
// the memory per in-flight region is 2 ceil(K / ckpt_every) boxes.  The
// dV contribution of a region is accumulated in VGPRs (one pencil per
// thread) and added to the grid with FP64 atomics; dR per atom of the box is
// accumulated in LDS (FP64) and added once per region.
#pragma once

#include "sq_region.h"

namespace sqk {

// projections of one vector (no recurrence step): publish, then dot products
template <typename T, int E, int R, int ZS, int NW, bool GRAD>
__device__ __forceinline__ void dots_only(const RegionArgs<T> &a, const StepCtx<T, E, R> &c,
                                          const T (&vec)[E], T *lds, const Slot *slots,
                                          T (*pfac)[NP], T (*dots)[NP], T (*ddots)[3 * NP],
                                          double tau) {
    if (c.active) store_pencil<T, E, ZS>(c.mine, vec);
    __syncthreads();
    if (c.nat)
        projector_dots<T, ZS, NW, GRAD>(a, slots, pfac, dots, ddots, lds, c.nat, c.dx, c.dy, c.dz,
                                        tau);
    __syncthreads();
}

template <typename T, int E, int R, bool MASKZ, bool GRAD>
__global__ void __launch_bounds__(((E * E + 63) / 64) * 64)
cheb_adjoint_kernel(const AdjointArgs<T> aa) {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    constexpr int ZS = pencil_stride<T, E>();
    constexpr int NW = BLOCK / 64;
    constexpr int EXTRA = GRAD ? (8 * NP * (int)sizeof(T) + 24) : 0;
    constexpr int MAXAT = max_atoms_in_region<T, E, EXTRA>();
    constexpr int AT = MAXAT > 0 ? MAXAT : 1;
    constexpr int GA = GRAD ? AT : 1;
    constexpr bool DREG = sizeof(T) == 4 ? E <= 21 : E <= 13;
    constexpr int EE = E * E;
    const RegionArgs<T> &a = aa.g;

    __shared__ __align__(16) T lds[region_lds_elems<T, E>()];
    __shared__ Slot slots[AT];
    __shared__ T pfac[AT][NP];
    __shared__ T dA[GA][NP], gA[GA][3 * NP], dB[GA][NP], gB[GA][3 * NP];
    __shared__ double dRacc[GA][3];
    __shared__ int s_item, s_nat;

    const int tid = threadIdx.x;
    const double tau = a.scal->tau;
    const int K = a.K, C = aa.ckpt_every;
    StepCtx<T, E, R> c;
#pragma unroll
    for (int p = 1; p <= R; ++p) {
        c.cx[p] = (T)(-a.w[p] * a.ih2[0] / tau);
        c.cy[p] = (T)(-a.w[p] * a.ih2[1] / tau);
        c.cz[p] = (T)(-a.w[p] * a.ih2[2] / tau);
    }
    T *ck = aa.ckpt + (int64_t)blockIdx.x * aa.ckpt_stride;

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
        const bool is_ctr = c.active && px == it.ctr[0] && py == it.ctr[1];
        const int cz0 = it.ctr[2];
#pragma unroll
        for (int p = 1; p <= R; ++p) {
            c.nb[4 * (p - 1) + 0] = (c.active && px + p < c.dx) ? tid + p : npen;
            c.nb[4 * (p - 1) + 1] = (c.active && px - p >= 0) ? tid - p : npen;
            c.nb[4 * (p - 1) + 2] = (c.active && py + p < c.dy) ? tid + p * c.dx : npen;
            c.nb[4 * (p - 1) + 3] = (c.active && py - p >= 0) ? tid - p * c.dx : npen;
        }
        c.mine = lds + tid * ZS;
        __syncthreads();
        c.nat = min(s_nat, MAXAT);
        if (tid == 0 && s_nat > MAXAT) atomicOr(a.status, 1);
        if constexpr (GRAD) {
            for (int j = tid; j < c.nat; j += BLOCK) dRacc[j][0] = dRacc[j][1] = dRacc[j][2] = 0.0;
        }
        // cotangent coefficients of this node
        const double gr = aa.g_rho ? aa.g_rho[it.out] : 0.0;
        const double gu = aa.g_u ? aa.g_u[it.out] : 0.0;
        auto coef = [&](int k) { return (T)(2.0 * (gr * aa.coef_c[k] + gu * aa.coef_d[k])); };

        auto ck_store = [&](int cidx, int which, const T(&vec)[E]) {
            if (!c.active) return;
#pragma unroll
            for (int z = 0; z < E; ++z) ck[((int64_t)(cidx * 2 + which) * E + z) * EE + tid] = vec[z];
        };
        auto ck_load = [&](int cidx, int which, T(&vec)[E]) {
            if (!c.active) return;
#pragma unroll
            for (int z = 0; z < E; ++z) vec[z] = ck[((int64_t)(cidx * 2 + which) * E + z) * EE + tid];
        };

        // ---- forward: v_0 .. v_K, checkpoints (v_cC, v_cC+1) for cC+1 <= K-1 ----
        T v[E], w[E];
#pragma unroll
        for (int z = 0; z < E; ++z) {
            v[z] = (is_ctr && z == cz0) ? (T)1 : (T)0;
            w[z] = (T)0;
        }
        for (int k = 0; k < K; k += 2) {
            region_step<T, E, R, ZS, NW, MASKZ, DREG>(a, c, d, col, plane, gz0, n2, v, w, lds, slots,
                                                      pfac, k == 0, tau);
            if (k % C == 0 && k + 1 <= K - 1) {
                ck_store(k / C, 0, v);
                ck_store(k / C, 1, w);
            }
            if (k + 1 < K) {
                region_step<T, E, R, ZS, NW, MASKZ, DREG>(a, c, d, col, plane, gz0, n2, w, v, lds,
                                                          slots, pfac, false, tau);
                if ((k + 1) % C == 0 && k + 2 <= K - 1) {
                    ck_store((k + 1) / C, 0, w);
                    ck_store((k + 1) / C, 1, v);
                }
            }
        }
        // (v_{K-1}, v_K) into (v, w)
        if ((K - 1) % 2) {
#pragma unroll
            for (int z = 0; z < E; ++z) {
                const T t = v[z];
                v[z] = w[z];
                w[z] = t;
            }
        }

        // ---- reverse sweep ----
        T t1[E], t2[E], G[E];
        {
            const T aK = coef(K);
#pragma unroll
            for (int z = 0; z < E; ++z) {
                t1[z] = (is_ctr && z == cz0) ? aK : (T)0;
                t2[z] = (T)0;
                G[z] = (T)0;
            }
        }
        // One reverse step: on entry cur = v_k, nxt = v_{k+1}, ta = vt_{k+1},
        // tb = vt_{k+2}; on exit nxt = v_{k-1} and tb = vt_k (k >= 1).
        auto rstep = [&](int k, T(&cur)[E], T(&nxt)[E], T(&ta)[E], T(&tb)[E]) {
            const bool anchor = k >= 1 && (k - 1) % C == 0;
            if (anchor) {
                ck_load((k - 1) / C, 1, cur);
                ck_load((k - 1) / C, 0, nxt);
            }
            const T alpha = k == 0 ? (T)1 : (T)2;
#pragma unroll
            for (int z = 0; z < E; ++z) G[z] += alpha * ta[z] * cur[z];
            if (k >= 1) {
                region_step<T, E, R, ZS, NW, MASKZ, DREG, GRAD>(a, c, d, col, plane, gz0, n2, ta, tb,
                                                                lds, slots, pfac, false, tau, dA, gA);
                if (is_ctr) {
                    const T ak = coef(k);
#pragma unroll
                    for (int z = 0; z < E; ++z) tb[z] += (z == cz0) ? ak : (T)0;
                }
                if (anchor) {
                    if constexpr (GRAD)
                        dots_only<T, E, R, ZS, NW, GRAD>(a, c, cur, lds, slots, pfac, dB, gB, tau);
                } else {
                    region_step<T, E, R, ZS, NW, MASKZ, DREG, GRAD>(a, c, d, col, plane, gz0, n2, cur,
                                                                    nxt, lds, slots, pfac, false,
                                                                    tau, dB, gB);
                }
            } else {
                if constexpr (GRAD) {
                    dots_only<T, E, R, ZS, NW, GRAD>(a, c, ta, lds, slots, pfac, dA, gA, tau);
                    dots_only<T, E, R, ZS, NW, GRAD>(a, c, cur, lds, slots, pfac, dB, gB, tau);
                }
            }
            if constexpr (GRAD) {
                const double f = (double)alpha * a.h3 / tau;
                for (int j = tid; j < c.nat; j += BLOCK) {
                    const double *cj = a.cJ + (int64_t)slots[j].atom * NP;
#pragma unroll
                    for (int x = 0; x < 3; ++x) {
                        double s = 0.0;
#pragma unroll
                        for (int l = 0; l < NP; ++l)
                            s += cj[l] * ((double)gA[j][3 * l + x] * (double)dB[j][l] +
                                          (double)dA[j][l] * (double)gB[j][3 * l + x]);
                        dRacc[j][x] += f * s;
                    }
                }
            }
        };
        for (int k = K - 1; k >= 0; k -= 2) {
            rstep(k, v, w, t1, t2);
            if (k - 1 >= 0) rstep(k - 1, w, v, t2, t1);
        }

        // ---- scatter: dV (FP64 atomics), dR per atom of the box ----
        if (aa.dV && c.active) {
            const double itau = 1.0 / tau;
#pragma unroll
            for (int z = 0; z < E; ++z) {
                if (z < c.dz) {
                    int gz = gz0 + z;
                    gz = gz >= n2 ? gz - n2 : gz;
                    unsafeAtomicAdd(aa.dV + col + plane * gz, (double)G[z] * itau);
                }
            }
        }
        __syncthreads();
        if constexpr (GRAD) {
            if (aa.dR)
                for (int j = tid; j < c.nat; j += BLOCK)
                    for (int x = 0; x < 3; ++x)
                        unsafeAtomicAdd(aa.dR + (int64_t)slots[j].atom * 3 + x, dRacc[j][x]);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------- //
// launch helpers for one FD radius R (instantiated in sq_adjoint_r<R>.hip)
// ------------------------------------------------------------------------- //
template <typename T, int E, int R, bool M, bool G>
static hipError_t adj_launch_one(const void *args, int grid, hipStream_t s) {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    hipLaunchKernelGGL((cheb_adjoint_kernel<T, E, R, M, G>), dim3(grid), dim3(BLOCK), 0, s,
                       *static_cast<const AdjointArgs<T> *>(args));
    return hipGetLastError();
}

template <typename T, int E, int R, bool M, bool G>
static int adj_occ_one() {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cheb_adjoint_kernel<T, E, R, M, G>, BLOCK,
                                                     0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <typename T, int E, int R>
static hipError_t adj_by_mg(bool M, bool G, const void *args, int grid, hipStream_t s, int *occ) {
    if (occ) {
        *occ = M ? (G ? adj_occ_one<T, E, R, true, true>() : adj_occ_one<T, E, R, true, false>())
                 : (G ? adj_occ_one<T, E, R, false, true>() : adj_occ_one<T, E, R, false, false>());
        return hipSuccess;
    }
    if (M) return G ? adj_launch_one<T, E, R, true, true>(args, grid, s)
                    : adj_launch_one<T, E, R, true, false>(args, grid, s);
    return G ? adj_launch_one<T, E, R, false, true>(args, grid, s)
             : adj_launch_one<T, E, R, false, false>(args, grid, s);
}

template <typename T, int R>
static hipError_t adj_by_e(int E, bool M, bool G, const void *args, int grid, hipStream_t s,
                           int *occ) {
    switch (E) {
        case 9: return adj_by_mg<T, 9, R>(M, G, args, grid, s, occ);
        case 13: return adj_by_mg<T, 13, R>(M, G, args, grid, s, occ);
        case 17: return adj_by_mg<T, 17, R>(M, G, args, grid, s, occ);
        case 21: return adj_by_mg<T, 21, R>(M, G, args, grid, s, occ);
        case 27:
            if constexpr (sizeof(T) == 4) return adj_by_mg<T, 27, R>(M, G, args, grid, s, occ);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <int R>
hipError_t adjoint_dispatch_r(int prec, int E, bool M, bool G, const void *args, int grid,
                              hipStream_t s, int *occ) {
    if (prec == SQ_FP64) return adj_by_e<double, R>(E, M, G, args, grid, s, occ);
    return adj_by_e<float, R>(E, M, G, args, grid, s, occ);
}

}  // namespace sqk
