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

// checkpoint slot I/O: layout [pair][which][z][pencil] so a wave's stores coalesce
template <typename T, int E>
__device__ __forceinline__ void ck_store(T *ck, bool active, int tid, int cidx, int which,
                                         const T (&vec)[E]) {
    if (!active) return;
#pragma unroll
    for (int z = 0; z < E; ++z) sgpr_ptr(ck + ((int64_t)(cidx * 2 + which) * E + z) * (E * E))[(uint32_t)tid] = vec[z];
}
template <typename T, int E>
__device__ __forceinline__ void ck_load(const T *ck, bool active, int tid, int cidx, int which,
                                        T (&vec)[E]) {
    if (!active) return;
#pragma unroll
    for (int z = 0; z < E; ++z) vec[z] = sgpr_ptr(ck + ((int64_t)(cidx * 2 + which) * E + z) * (E * E))[(uint32_t)tid];
}

// LDS tables of the atoms of the current box used by the reverse sweep
template <typename T, int AT, int GA>
struct AdjShared {
    Slot slots[AT];
    T pfac[AT][NP];
    T dA[GA][NP], gA[GA][3 * NP], dB[GA][NP], gB[GA][3 * NP];
    double dRacc[GA][3];
};

// per-region scalars of the reverse sweep
struct AdjNode {
    int64_t col, plane;
    int gz0, n2, cz0, C;
    bool is_ctr;
    double gr, gu;
};

// One reverse step: on entry cur = v_k, nxt = v_{k+1}, ta = vt_{k+1},
// tb = vt_{k+2}; on exit nxt = v_{k-1} and tb = vt_k (k >= 1).  G += alpha vt_{k+1} v_k,
// and (GRAD) dR_J += alpha h^3/tau sum_lm c [(vt.dchi)(chi.v) + (vt.chi)(dchi.v)].
template <typename T, int E, int R, int ZS, int NW, int BLOCK, bool MASKZ, bool DREG, bool GRAD,
          int AT, int GA>
__device__ __forceinline__ void adjoint_rstep(const AdjointArgs<T> &aa, const StepCtx<T, E, R> &c,
                                              const AdjNode &nd, const T (&d)[DREG ? E : 1],
                                              T *lds, AdjShared<T, AT, GA> &sh, const T *ck,
                                              int k, T (&cur)[E], T (&nxt)[E], T (&ta)[E],
                                              T (&tb)[E], T (&G)[E], double tau) {
    const RegionArgs<T> &a = aa.g;
    const int tid = threadIdx.x;
    const bool anchor = k >= 1 && (k - 1) % nd.C == 0;
    if (anchor) {
        ck_load<T, E>(ck, c.active, tid, (k - 1) / nd.C, 1, cur);
        ck_load<T, E>(ck, c.active, tid, (k - 1) / nd.C, 0, nxt);
    }
    const T alpha = k == 0 ? (T)1 : (T)2;
#pragma unroll
    for (int z = 0; z < E; ++z) G[z] += alpha * ta[z] * cur[z];
    if (k >= 1) {
        region_step<T, E, R, ZS, NW, MASKZ, DREG, GRAD>(a, c, d, nd.col, nd.plane, nd.gz0, nd.n2,
                                                        ta, tb, lds, sh.slots, sh.pfac, false, tau,
                                                        sh.dA, sh.gA);
        if (nd.is_ctr) {
            const T ak = (T)(2.0 * (nd.gr * aa.coef_c[k] + nd.gu * aa.coef_d[k]));
#pragma unroll
            for (int z = 0; z < E; ++z) tb[z] += (z == nd.cz0) ? ak : (T)0;
        }
        if (anchor) {
            if constexpr (GRAD)
                dots_only<T, E, R, ZS, NW, GRAD>(a, c, cur, lds, sh.slots, sh.pfac, sh.dB, sh.gB,
                                                 tau);
        } else {
            region_step<T, E, R, ZS, NW, MASKZ, DREG, GRAD>(a, c, d, nd.col, nd.plane, nd.gz0,
                                                            nd.n2, cur, nxt, lds, sh.slots,
                                                            sh.pfac, false, tau, sh.dB, sh.gB);
        }
    } else {
        if constexpr (GRAD) {
            dots_only<T, E, R, ZS, NW, GRAD>(a, c, ta, lds, sh.slots, sh.pfac, sh.dA, sh.gA, tau);
            dots_only<T, E, R, ZS, NW, GRAD>(a, c, cur, lds, sh.slots, sh.pfac, sh.dB, sh.gB, tau);
        }
    }
    if constexpr (GRAD) {
        const double f = (double)alpha * a.h3 / tau;
        for (int j = tid; j < c.nat; j += BLOCK) {
            const double *cj = a.cJ + (int64_t)sh.slots[j].atom * NP;
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < NP; ++l)
                    s += cj[l] * ((double)sh.gA[j][3 * l + x] * (double)sh.dB[j][l] +
                                  (double)sh.dA[j][l] * (double)sh.gB[j][3 * l + x]);
                sh.dRacc[j][x] += f * s;
            }
        }
    }
}

// Reverse step with the column projector path: the vt and v recurrences keep
// their own projection buffers (nlA, nlB); the dR term reads the raw
// projections each step left behind.
template <typename T, int E, int R, int ZS, int BLOCK, bool MASKZ, bool DREG, bool GRAD>
__device__ __forceinline__ void adjoint_rstep_col(const AdjointArgs<T> &aa,
                                                  const StepCtx<T, E, R> &c, const AdjNode &nd,
                                                  const T (&d)[DREG ? E : 1], T *lds,
                                                  ColNL<T> &nlA, ColNL<T> &nlB, const Slot *slots,
                                                  double (*dRacc)[3], const T *ck, int k,
                                                  T (&cur)[E], T (&nxt)[E], T (&ta)[E],
                                                  T (&tb)[E], T (&G)[E], double tau) {
    const RegionArgs<T> &a = aa.g;
    const int tid = threadIdx.x;
    const bool anchor = k >= 1 && (k - 1) % nd.C == 0;
    if (anchor) {
        ck_load<T, E>(ck, c.active, tid, (k - 1) / nd.C, 1, cur);
        ck_load<T, E>(ck, c.active, tid, (k - 1) / nd.C, 0, nxt);
    }
    const T alpha = k == 0 ? (T)1 : (T)2;
#pragma unroll
    for (int z = 0; z < E; ++z) G[z] += alpha * ta[z] * cur[z];
    if (k >= 1) {
        region_step_col<T, E, R, ZS, BLOCK, MASKZ, DREG, GRAD, true>(a, c, d, nd.col, nd.plane, nd.gz0,
                                                               nd.n2, ta, tb, lds, nlA, false);
        if (nd.is_ctr) {
            const T ak = (T)(2.0 * (nd.gr * aa.coef_c[k] + nd.gu * aa.coef_d[k]));
#pragma unroll
            for (int z = 0; z < E; ++z) tb[z] += (z == nd.cz0) ? ak : (T)0;
        }
        if (anchor) {
            if constexpr (GRAD) col_dots_only<T, E, R, ZS, BLOCK, GRAD>(a, c, cur, nlB);
        } else {
            region_step_col<T, E, R, ZS, BLOCK, MASKZ, DREG, GRAD, true>(a, c, d, nd.col, nd.plane,
                                                                   nd.gz0, nd.n2, cur, nxt, lds,
                                                                   nlB, false);
        }
    } else {
        if constexpr (GRAD) {
            col_dots_only<T, E, R, ZS, BLOCK, GRAD>(a, c, ta, nlA);
            col_dots_only<T, E, R, ZS, BLOCK, GRAD>(a, c, cur, nlB);
        }
    }
    if constexpr (GRAD) {
        const double f = (double)alpha * a.h3 / tau;
        const T *dA = nlA.pacc + (int64_t)(nlA.par ^ 1) * nlA.maxat * NP;
        const T *gA = nlA.gacc + (int64_t)(nlA.par ^ 1) * nlA.maxat * 3 * NP;
        const T *dB = nlB.pacc + (int64_t)(nlB.par ^ 1) * nlB.maxat * NP;
        const T *gB = nlB.gacc + (int64_t)(nlB.par ^ 1) * nlB.maxat * 3 * NP;
        for (int j = tid; j < c.nat; j += BLOCK) {
            const double *cj = a.cJ + (int64_t)slots[j].atom * NP;
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < NP; ++l)
                    s += cj[l] * ((double)gA[(j * NP + l) * 3 + x] * (double)dB[j * NP + l] +
                                  (double)dA[j * NP + l] * (double)gB[(j * NP + l) * 3 + x]);
                dRacc[j][x] += f * s;
            }
        }
    }
}

// G += alpha vt_{k+1} v_k with v_k read from its stored slot.  All loads are
// issued before the FMAs (one memory wait; left alone, the allocator issues
// load, wait, FMA per z).
template <typename T, int E, typename Ctx>
__device__ __forceinline__ void sa_gupdate(const Ctx &c, const T *ck, int k, T alpha,
                                           const T (&ta)[E], T (&G)[E]) {
    constexpr int EE = E * E;
    if (!c.active) return;
    const uint32_t t = threadIdx.x;
    T vk[E];
#pragma unroll
    for (int z = 0; z < E; ++z) vk[z] = sgpr_ptr(ck + ((int64_t)k * E + z) * EE)[t];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int z = 0; z < E; ++z) G[z] += alpha * ta[z] * vk[z];
}

// Reverse step when the forward pass stored every v_k (checkpoint stride 1):
// G += alpha vt_{k+1} v_k and tb <- vt_k.  v_k is read from its HBM slot where
// it is used (the G update) instead of being held as a register pencil, so only
// vt_{k+1}, vt_{k+2} and G stay resident; the projections of v_k needed for dR
// were stored by the forward sweep next to the vectors.
template <typename T, int E, int R, int ZS, int BLOCK, bool MASKZ, bool DREG, bool GRAD>
__device__ __forceinline__ void adjoint_rstep_sa(const AdjointArgs<T> &aa,
                                                 const StepCtx<T, E, R> &c, const AdjNode &nd,
                                                 const T (&d)[DREG ? E : 1], T *lds, ColNL<T> &nlA,
                                                 const Slot *slots, double (*dRacc)[3],
                                                 const T *ck, int k, T (&ta)[E], T (&tb)[E],
                                                 T (&G)[E], double tau) {
    const RegionArgs<T> &a = aa.g;
    constexpr int EE = E * E;
    const T alpha = k == 0 ? (T)1 : (T)2;
    sa_gupdate<T, E>(c, ck, k, alpha, ta, G);
    if (k >= 1) {
        region_step_col<T, E, R, ZS, BLOCK, MASKZ, DREG, GRAD, true>(
            a, c, d, nd.col, nd.plane, nd.gz0, nd.n2, ta, tb, lds, nlA, false);
        if (nd.is_ctr) {
            const T ak = (T)(2.0 * (nd.gr * aa.coef_c[k] + nd.gu * aa.coef_d[k]));
#pragma unroll
            for (int z = 0; z < E; ++z) tb[z] += (z == nd.cz0) ? ak : (T)0;
        }
    } else {
        if constexpr (GRAD) col_dots_only<T, E, R, ZS, BLOCK, GRAD>(a, c, ta, nlA);
    }
    if constexpr (GRAD) {
        const double f = (double)alpha * a.h3 / tau;
        const T *dA = nlA.pacc + (int64_t)(nlA.par ^ 1) * nlA.maxat * NP;
        const T *gA = nlA.gacc + (int64_t)(nlA.par ^ 1) * nlA.maxat * 3 * NP;
        const T *pk = ck + (int64_t)a.K * E * EE + (int64_t)k * MAX_REGION_ATOMS * 4 * NP;
        for (int j = threadIdx.x; j < c.nat; j += BLOCK) {
            // all loads of the atom first (one memory wait), then the sums
            const double *cjp = a.cJ + (int64_t)slots[j].atom * NP;
            const T *pj = pk + j * 4 * NP;
            double cj[NP];
            T pv[4 * NP];
#pragma unroll
            for (int l = 0; l < NP; ++l) cj[l] = cjp[l];
#pragma unroll
            for (int q = 0; q < 4 * NP; ++q) pv[q] = pj[q];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < NP; ++l)
                    s += cj[l] * ((double)gA[(j * NP + l) * 3 + x] * (double)pv[l] +
                                  (double)dA[j * NP + l] * (double)pv[NP + l * 3 + x]);
                dRacc[j][x] += f * s;
            }
        }
    }
}

// copy the projections of the vector the last step projected (parity buffer
// par ^ 1 of nl) into the store-all slot, row k
template <typename T, int BLOCK, bool WITHG = true>
__device__ __forceinline__ void store_projections(const ColNL<T> &nl, int nat, T *ck, int K,
                                                  int E3, int k) {
    T *pk = ck + (int64_t)K * E3 + (int64_t)k * MAX_REGION_ATOMS * 4 * NP;
    const T *pa = nl.pacc + (int64_t)(nl.par ^ 1) * nl.maxat * NP;
    if constexpr (WITHG) {
        const T *ga = nl.gacc + (int64_t)(nl.par ^ 1) * nl.maxat * 3 * NP;
        for (int i = threadIdx.x; i < nat * 4 * NP; i += BLOCK) {
            const int j = i / (4 * NP), q = i - j * 4 * NP;
            pk[i] = q < NP ? pa[j * NP + q] : ga[j * 3 * NP + (q - NP)];
        }
    } else {
        for (int i = threadIdx.x; i < nat * NP; i += BLOCK) {
            const int j = i / NP, q = i - j * NP;
            pk[j * 4 * NP + q] = pa[i];
        }
    }
}

// dR in W mode (store-all adjoint).  With p_k = chi . v_k (stored by the
// forward sweep) and q_k = chi . vt_{k+1} (the reverse step's projections),
// the dR sum over k of alpha_k [(vt_{k+1} . dchi)(chi . v_k) +
// (vt_{k+1} . chi)(dchi . v_k)] equals dchi . W with
// W(y) = sum_k alpha_k (p_k vt_{k+1}(y) + q_k v_k(y)) on the support rows.  W is
// accumulated per row of the thread's column pieces (in the slot,
// [row][thread][l], the thread's rows numbered densely over its pieces) inside
// the reverse steps, and contracted with
// dchi once per region, so no dchi projections are formed per step.
// contraction of W with dchi/dR into the per-atom accumulators of the box
template <typename T, int E, int BLOCK>
__device__ __forceinline__ void w_contract(const RegionArgs<T> &a, const ColNL<T> &nl,
                                           const Slot *slots, const T *wb, double (*cdR)[3],
                                           double scale) {
    constexpr int NB = 2;
    const uint32_t t = threadIdx.x;
    int ebase = 0;
    for (int cc = 0; cc < nl.ncol; ++cc) {
        const ColEntry e = nl.cols[cc];
        double cj[NP];
#pragma unroll
        for (int l = 0; l < NP; ++l) cj[l] = a.cJ[(int64_t)slots[e.slot].atom * NP + l];
        const WVec<T> *wc = reinterpret_cast<const WVec<T> *>(wb) + ((int64_t)ebase * BLOCK + t);
        ebase += e.n;
        double sx[3] = {0.0, 0.0, 0.0};
        for (int i0 = 0; i0 < e.n; i0 += NB) {
            T dc[NB][3 * NP];
            WVec<T> wv[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int i = min(i0 + b, e.n - 1);
                const T *dcp = a.dchi + (int64_t)(e.row0 + i) * 3 * NP;
#pragma unroll
                for (int q = 0; q < 3 * NP; ++q) dc[b][q] = dcp[q];
                wv[b] = wc[(int64_t)i * BLOCK];
                if (i0 + b >= e.n) wv[b] = WVec<T>{{0, 0, 0, 0}};
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int l = 0; l < NP; ++l)
#pragma unroll
                    for (int x = 0; x < 3; ++x)
                        sx[x] += cj[l] * (double)dc[b][l * 3 + x] * (double)wv[b].v[l];
        }
#pragma unroll
        for (int x = 0; x < 3; ++x) atomicAdd(&cdR[e.slot][x], sx[x] * scale);
    }
}

// Reverse step of the store-all adjoint with dR in W mode.  Reverse step k
// (own pencil vt_{k+1} after its first barrier, the projection buffer of step
// k+1 still holding q_{k+1}) adds alpha_k p_k vt_{k+1} + alpha_{k+1} q_{k+1} v_{k+1};
// the last term alpha_0 q_0 v_0 is added after the k = 0 projections.
template <typename T, int E, int R, int ZS, int BLOCK, bool MASKZ, bool DREG>
__device__ __forceinline__ void adjoint_rstep_saw(const AdjointArgs<T> &aa,
                                                  const StepCtx<T, E, R> &c, const AdjNode &nd,
                                                  const T (&d)[DREG ? E : 1], T *lds,
                                                  ColNL<T> &nlA, const T *ck, T *wb, int k,
                                                  T (&ta)[E], T (&tb)[E], T (&G)[E]) {
    const RegionArgs<T> &a = aa.g;
    const T alpha = k == 0 ? (T)1 : (T)2;
    sa_gupdate<T, E>(c, ck, k, alpha, ta, G);
    WArgs<T> w{ck, wb, k, alpha, k + 1 <= a.K - 1 ? k + 1 : -1, (T)2, nlA.par ^ 1};
    if (k >= 1) {
        region_step_col<T, E, R, ZS, BLOCK, MASKZ, DREG, false, true, true>(
            a, c, d, nd.col, nd.plane, nd.gz0, nd.n2, ta, tb, lds, nlA, false, nullptr, &w);
        if (nd.is_ctr) {
            const T ak = (T)(2.0 * (nd.gr * aa.coef_c[k] + nd.gu * aa.coef_d[k]));
#pragma unroll
            for (int z = 0; z < E; ++z) tb[z] += (z == nd.cz0) ? ak : (T)0;
        }
    } else {
        col_dots_only<T, E, R, ZS, BLOCK, false, true>(a, c, ta, nlA, &w);
        // alpha_0 q_0 v_0 (q_0 now in buffer par ^ 1; own pencil unused: ap = 0)
        WArgs<T> w0{ck, wb, 0, (T)0, 0, (T)1, nlA.par ^ 1};
        if (nlA.ncol) w_update<T, E, BLOCK>(a, nlA, w0, c.mine);
    }
}

template <typename T, int E, int R, bool MASKZ, bool GRAD, bool STOREALL>
__global__ void __launch_bounds__(((E * E + 63) / 64) * 64)
cheb_adjoint_kernel(const AdjointArgs<T> aa) {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    constexpr int ZS = pencil_stride<T, E>();
    constexpr int NW = BLOCK / 64;
    constexpr int COLBYTES = BLOCK * MAXC * (int)sizeof(ColEntry);
    // column path: two projection states (vt and v), each [2][AT][NP] (+ [2][AT][3NP]
    // with dR, except in the store-all W mode), and the dR accumulators
    constexpr int CEXTRA = !GRAD ? 4 * NP * (int)sizeof(T)
                                 : (STOREALL ? 4 * NP * (int)sizeof(T) + 24
                                             : 16 * NP * (int)sizeof(T) + 24);
    constexpr bool COLNL = max_atoms_in_region<T, E, CEXTRA, COLBYTES>() >= 32;
    constexpr bool WM = COLNL && STOREALL && GRAD;
    constexpr int EXTRA = GRAD ? (8 * NP * (int)sizeof(T) + 24) : 0;
    constexpr int MAXAT = COLNL ? max_atoms_in_region<T, E, CEXTRA, COLBYTES>()
                                : max_atoms_in_region<T, E, EXTRA>();
    constexpr int AT = MAXAT > 0 ? MAXAT : 1;
    constexpr int GA = (GRAD && !COLNL) ? AT : 1;
    constexpr int CA = COLNL ? AT : 1;
    constexpr int CG = (COLNL && GRAD && !WM) ? AT : 1;
    constexpr bool DREG = sizeof(T) == 4 ? E <= 21 : E <= 13;
    constexpr int EE = E * E;
    const RegionArgs<T> &a = aa.g;

    __shared__ __align__(16) T lds[region_lds_elems<T, E>()];
    __shared__ AdjShared<T, AT, GA> sh;
    __shared__ T cpA[2][CA][NP], cpB[2][CA][NP];
    __shared__ T cgA[2][CG][3 * NP], cgB[2][CG][3 * NP];
    __shared__ double cdR[COLNL && GRAD ? AT : 1][3];
    __shared__ ColEntry colbuf[COLNL ? BLOCK * MAXC : 1];
    __shared__ T ncoef[4 * R];
    __shared__ int s_item, s_nat;
    Slot *slots = sh.slots;
    T(*pfac)[NP] = sh.pfac;

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
    if (tid < 4 * R) {
        const int p = (tid >> 2) + 1;
        ncoef[tid] = (T)(-a.w[p] * a.ih2[(tid & 3) < 2 ? 0 : 1] / tau);
    }
    c.ncoef = ncoef;

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
        c.px = px;
        c.py = py;
        c.npen = npen;
        __syncthreads();
        c.nat = min(s_nat, MAXAT);
        if (tid == 0 && s_nat > MAXAT) atomicOr(a.status, 1);
        if constexpr (GRAD) {
            for (int j = tid; j < c.nat; j += BLOCK)
                sh.dRacc[j][0] = sh.dRacc[j][1] = sh.dRacc[j][2] = 0.0;
        }
        AdjNode nd;
        nd.col = col;
        nd.plane = plane;
        nd.gz0 = gz0;
        nd.n2 = n2;
        nd.cz0 = cz0;
        nd.C = C;
        nd.is_ctr = is_ctr;
        nd.gr = aa.g_rho ? aa.g_rho[it.out] : 0.0;
        nd.gu = aa.g_u ? aa.g_u[it.out] : 0.0;

        ColNL<T> nlA{}, nlB{};
        if constexpr (COLNL) {
            for (int j = tid; j < c.nat; j += BLOCK) {
                const double f = 2.0 * a.h3 / tau;
                const double *cj = a.cJ + (int64_t)slots[j].atom * NP;
#pragma unroll
                for (int l = 0; l < NP; ++l) {
                    pfac[j][l] = (T)(f * cj[l]);
                    cpA[0][j][l] = cpA[1][j][l] = cpB[0][j][l] = cpB[1][j][l] = (T)0;
                }
                if constexpr (GRAD) {
                    if constexpr (!WM) {
                        for (int q = 0; q < 3 * NP; ++q)
                            cgA[0][j][q] = cgA[1][j][q] = cgB[0][j][q] = cgB[1][j][q] = (T)0;
                    }
                    cdR[j][0] = cdR[j][1] = cdR[j][2] = 0.0;
                }
            }
            int ncol = build_columns<T>(a, slots, c.nat, c.active, px, py, c.dz, colbuf + tid * MAXC);
            if (ncol > MAXC) {
                atomicOr(a.status, 2);
                ncol = MAXC;
            }
            nlA.cols = nlB.cols = colbuf + tid * MAXC;
            nlA.ncol = nlB.ncol = ncol;
            nlA.scale = nlB.scale = &pfac[0][0];
            nlA.maxat = nlB.maxat = CA;
            nlA.pacc = &cpA[0][0][0];
            nlB.pacc = &cpB[0][0][0];
            nlA.gacc = (GRAD && !WM) ? &cgA[0][0][0] : nullptr;
            nlB.gacc = (GRAD && !WM) ? &cgB[0][0][0] : nullptr;
            __syncthreads();
        }

        T v[E], G[E];
        T *wb = ck + storeall_w_offset(K, E);
        if constexpr (COLNL && STOREALL) {
            // ---- forward storing v_0 .. v_{K-1}; reverse reads them back ----
            T w[E];
#pragma unroll
            for (int z = 0; z < E; ++z) {
                v[z] = (is_ctr && z == cz0) ? (T)1 : (T)0;
                w[z] = (T)0;
            }
            // slot layout [k][z][pencil]: a wave's stores coalesce
            // (v_K itself is never needed by the reverse sweep).  With GRAD the
            // step's projections of v_k (chi and dchi/dR) go to the slot too.
            // A step that advances v_k also stores v_k (its input) inside the
            // step; the last vector v_{K-1} is stored after the loop.
            constexpr int E3 = E * E * E;
            // In W mode (dR) only the value projections chi . v_k are kept.
            // The forward sweep holds two pencils only, so it keeps the
            // diagonal in registers even where the reverse sweep cannot.
            constexpr bool FG = GRAD && !WM;
            T dF[E];
#pragma unroll
            for (int z = 0; z < E; ++z) {
                if constexpr (DREG) {
                    dF[z] = d[z];
                } else {
                    int gz = gz0 + z;
                    gz = gz >= n2 ? gz - n2 : gz;
                    dF[z] = (c.active && z < c.dz) ? a.D[col + plane * gz] : (T)0;
                }
            }
            for (int k = 0; k + 1 <= K - 1; k += 2) {
                region_step_col<T, E, R, ZS, BLOCK, MASKZ, true, FG, true>(
                    a, c, dF, col, plane, gz0, n2, v, w, lds, nlB, k == 0, ck + (int64_t)k * E3);
                if constexpr (GRAD) store_projections<T, BLOCK, FG>(nlB, c.nat, ck, K, E3, k);
                if (k + 2 <= K - 1) {
                    region_step_col<T, E, R, ZS, BLOCK, MASKZ, true, FG, true>(
                        a, c, dF, col, plane, gz0, n2, w, v, lds, nlB, false,
                        ck + (int64_t)(k + 1) * E3);
                    if constexpr (GRAD) store_projections<T, BLOCK, FG>(nlB, c.nat, ck, K, E3, k + 1);
                }
            }
            if ((K - 1) % 2 == 0) ck_store<T, E>(ck, c.active, tid, 0, K - 1, v);
            else ck_store<T, E>(ck, c.active, tid, 0, K - 1, w);
            if constexpr (GRAD) {
                // projections of v_{K-1}, the last stored vector
                if ((K - 1) % 2 == 0) col_dots_only<T, E, R, ZS, BLOCK, FG>(a, c, v, nlB);
                else col_dots_only<T, E, R, ZS, BLOCK, FG>(a, c, w, nlB);
                store_projections<T, BLOCK, FG>(nlB, c.nat, ck, K, E3, K - 1);
            }
            if constexpr (WM) {
                // zero the W rows of this thread's column pieces (numbered
                // densely over its pieces: row ebase + i of piece cc)
                int ebase = 0;
                for (int cc = 0; cc < nlA.ncol; ++cc) {
                    const ColEntry e = nlA.cols[cc];
                    for (int i = 0; i < e.n; ++i)
                        reinterpret_cast<WVec<T> *>(wb)[(int64_t)(ebase + i) * BLOCK + tid] =
                            WVec<T>{{0, 0, 0, 0}};
                    ebase += e.n;
                }
            }
            T t1[E], t2[E];
            const T aK = (T)(2.0 * (nd.gr * aa.coef_c[K] + nd.gu * aa.coef_d[K]));
#pragma unroll
            for (int z = 0; z < E; ++z) {
                t1[z] = (is_ctr && z == cz0) ? aK : (T)0;
                t2[z] = (T)0;
                G[z] = (T)0;
            }
            if constexpr (WM) {
                for (int k = K - 1; k >= 0; k -= 2) {
                    adjoint_rstep_saw<T, E, R, ZS, BLOCK, MASKZ, DREG>(
                        aa, c, nd, d, lds, nlA, ck, wb, k, t1, t2, G);
                    if (k - 1 >= 0)
                        adjoint_rstep_saw<T, E, R, ZS, BLOCK, MASKZ, DREG>(
                            aa, c, nd, d, lds, nlA, ck, wb, k - 1, t2, t1, G);
                }
                w_contract<T, E, BLOCK>(a, nlA, slots, wb, cdR, a.h3 / tau);
            } else {
                for (int k = K - 1; k >= 0; k -= 2) {
                    adjoint_rstep_sa<T, E, R, ZS, BLOCK, MASKZ, DREG, GRAD>(
                        aa, c, nd, d, lds, nlA, slots, cdR, ck, k, t1, t2, G, tau);
                    if (k - 1 >= 0)
                        adjoint_rstep_sa<T, E, R, ZS, BLOCK, MASKZ, DREG, GRAD>(
                            aa, c, nd, d, lds, nlA, slots, cdR, ck, k - 1, t2, t1, G, tau);
                }
            }
        } else {
            // ---- forward: v_0 .. v_K, checkpoints (v_cC, v_cC+1) for cC+1 <= K-1 ----
            T w[E];
    #pragma unroll
            for (int z = 0; z < E; ++z) {
                v[z] = (is_ctr && z == cz0) ? (T)1 : (T)0;
                w[z] = (T)0;
            }
            for (int k = 0; k < K; k += 2) {
                if constexpr (COLNL)
                    region_step_col<T, E, R, ZS, BLOCK, MASKZ, DREG, false, true>(a, c, d, col, plane, gz0, n2,
                                                                            v, w, lds, nlB, k == 0);
                else
                    region_step<T, E, R, ZS, NW, MASKZ, DREG>(a, c, d, col, plane, gz0, n2, v, w, lds,
                                                              slots, pfac, k == 0, tau);
                if (k % C == 0 && k + 1 <= K - 1) {
                    ck_store<T, E>(ck, c.active, tid, k / C, 0, v);
                    ck_store<T, E>(ck, c.active, tid, k / C, 1, w);
                }
                if (k + 1 < K) {
                    if constexpr (COLNL)
                        region_step_col<T, E, R, ZS, BLOCK, MASKZ, DREG, false, true>(a, c, d, col, plane, gz0,
                                                                                n2, w, v, lds, nlB, false);
                    else
                        region_step<T, E, R, ZS, NW, MASKZ, DREG>(a, c, d, col, plane, gz0, n2, w, v,
                                                                  lds, slots, pfac, false, tau);
                    if ((k + 1) % C == 0 && k + 2 <= K - 1) {
                        ck_store<T, E>(ck, c.active, tid, (k + 1) / C, 0, w);
                        ck_store<T, E>(ck, c.active, tid, (k + 1) / C, 1, v);
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
            T t1[E], t2[E];
            {
                const T aK = (T)(2.0 * (nd.gr * aa.coef_c[K] + nd.gu * aa.coef_d[K]));
    #pragma unroll
                for (int z = 0; z < E; ++z) {
                    t1[z] = (is_ctr && z == cz0) ? aK : (T)0;
                    t2[z] = (T)0;
                    G[z] = (T)0;
                }
            }
            if constexpr (COLNL) {
                for (int k = K - 1; k >= 0; k -= 2) {
                    adjoint_rstep_col<T, E, R, ZS, BLOCK, MASKZ, DREG, GRAD>(
                        aa, c, nd, d, lds, nlA, nlB, slots, cdR, ck, k, v, w, t1, t2, G, tau);
                    if (k - 1 >= 0)
                        adjoint_rstep_col<T, E, R, ZS, BLOCK, MASKZ, DREG, GRAD>(
                            aa, c, nd, d, lds, nlA, nlB, slots, cdR, ck, k - 1, w, v, t2, t1, G, tau);
                }
            } else {
                for (int k = K - 1; k >= 0; k -= 2) {
                    adjoint_rstep<T, E, R, ZS, NW, BLOCK, MASKZ, DREG, GRAD, AT, GA>(
                        aa, c, nd, d, lds, sh, ck, k, v, w, t1, t2, G, tau);
                    if (k - 1 >= 0)
                        adjoint_rstep<T, E, R, ZS, NW, BLOCK, MASKZ, DREG, GRAD, AT, GA>(
                            aa, c, nd, d, lds, sh, ck, k - 1, w, v, t2, t1, G, tau);
                }
            }


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
                        unsafeAtomicAdd(aa.dR + (int64_t)slots[j].atom * 3 + x,
                                        COLNL ? cdR[j][x] : sh.dRacc[j][x]);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------- //
// launch helpers for one FD radius R (instantiated in sq_adjoint_r<R>.hip)
// ------------------------------------------------------------------------- //
// z masking is always on in the adjoint (one select per point and step) so the
// instantiations cover (gradient) x (store-all or rebuild) only.
template <typename T, int E, int R, bool G, bool SA>
static hipError_t adj_launch_one(const void *args, int grid, hipStream_t s) {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    hipLaunchKernelGGL((cheb_adjoint_kernel<T, E, R, true, G, SA>), dim3(grid), dim3(BLOCK), 0, s,
                       *static_cast<const AdjointArgs<T> *>(args));
    return hipGetLastError();
}

template <typename T, int E, int R, bool G, bool SA>
static int adj_occ_one() {
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cheb_adjoint_kernel<T, E, R, true, G, SA>,
                                                     BLOCK, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <typename T, int E, int R>
static hipError_t adj_by_mg(bool SA, bool G, const void *args, int grid, hipStream_t s, int *occ) {
    if (occ) {
        *occ = SA ? (G ? adj_occ_one<T, E, R, true, true>() : adj_occ_one<T, E, R, false, true>())
                  : (G ? adj_occ_one<T, E, R, true, false>() : adj_occ_one<T, E, R, false, false>());
        return hipSuccess;
    }
    if (SA) return G ? adj_launch_one<T, E, R, true, true>(args, grid, s)
                     : adj_launch_one<T, E, R, false, true>(args, grid, s);
    return G ? adj_launch_one<T, E, R, true, false>(args, grid, s)
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
hipError_t adjoint_dispatch_r(int prec, int E, bool SA, bool G, const void *args, int grid,
                              hipStream_t s, int *occ) {
    if (prec == SQ_FP64) return adj_by_e<double, R>(E, SA, G, args, grid, s, occ);
    return adj_by_e<float, R>(E, SA, G, args, grid, s, occ);
}

}  // namespace sqk
