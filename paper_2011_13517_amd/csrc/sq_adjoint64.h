// FP64 adjoint of the region recurrence for the largest boxes (gfx950).
//
// Same mathematics as the adjoint in sq_adjoint_kernel.h: for node q with
// y_q = sum_k a_k mu_k^q, a_k = 2 (g_rho c'_k + g_u d'_k),
//   vt_K = a_K e_q,   vt_k = a_k e_q + 2 Hs vt_{k+1} - vt_{k+2}   (k >= 1),
//   dy/dV(x) = (1/tau) sum_{k=0}^{K-1} alpha_k vt_{k+1}(x) v_k(x),
//   dy/dR_J  = (h^3/tau) sum_k alpha_k sum_lm c_Jl
//              [(vt_{k+1}.dchi_Jlm)(chi_Jlm.v_k) + (vt_{k+1}.chi_Jlm)(dchi_Jlm.v_k)],
// alpha_0 = 1, alpha_k = 2 (the reverse of Eq. (Chebyshev) at fixed lambda_f,
// omega, tau).  The gradient sums cancel by three to four decades, so every
// vector and the dV sum are FP64 here: FP32 rounding of any one of v_k, vt_k or
// the dV accumulator alone leaves 1e-5..1e-4 relative error at K ~ 80.
//
// Layout for FP64 boxes whose pencil array fills the LDS (edge 27: 157 KB of
// 160 KB), leaving room only for the per-atom projections:
//  * Thread t owns the z-pencil (t mod dx, t / dx) of the two live vectors in
//    VGPRs; the LDS holds the box once (x/y neighbours) plus one zero pencil.
//  * Projector block one wave per atom (the atom's support rows spread over
//    the lanes, wave reductions, LDS atomics into the box for the rank-4
//    term); the atom list of the box lives in the workgroup's HBM slot.
//  * Forward sweep: v_0 .. v_{K-1} and their projections (chi . v_k, and
//    dchi . v_k for dR) go to the slot.  Reverse sweep: vt_{k+1} goes to the
//    slot, and the dR term of step k is formed at once from its own
//    projections and the stored ones, in FP64 registers of thread j for atom j.
//  * A final pass of each thread over its own pencil streams vt_{k+1}(z) and
//    v_k(z) back from the slot and accumulates dV(z) in FP64 registers (the
//    sweeps' two pencils leave no room for a third FP64 pencil).
//  * dV is added to the grid with FP64 atomics, dR once per atom per region.
#pragma once

#include "sq_region.h"

namespace sqk {

constexpr int A64_EDGE = 27;
constexpr int A64_PROJ = 4 * NP;   // chi . v (NP), then dchi . v ([l][x], 3 NP)
constexpr int A64_SLOT_ATOMS = (MAX_REGION_ATOMS * (int)sizeof(Slot) + 7) / 8;   // doubles

// slot of one workgroup (doubles): v_k rows, vt_{k+1} rows ([k][z][pencil],
// E^3 each), forward projections [k][atom][A64_PROJ], the atom list
constexpr int64_t a64_slot_elems(int K, int E) {
    return round_np(2 * (int64_t)K * E * E * E + (int64_t)K * MAX_REGION_ATOMS * A64_PROJ +
                    A64_SLOT_ATOMS);
}

// prev[z] = D[z] cur[z] - prev[z], D read from L2 CH planes at a time (loads
// of a batch first, then its FMAs); z is clamped into the box so the loads
// need no branch (planes past dz are zeroed by the z mask).
template <int E, int CH>
__device__ __forceinline__ void a64_diag(const double *D, int64_t col, int64_t plane, int gz0,
                                         int n2, int dz, const double (&cur)[E],
                                         double (&prev)[E]) {
    int salt = 0;
    asm volatile("" : "+s"(salt));
    const uint32_t cl = (uint32_t)col;
    const int zmax = dz - 1 + salt;
#pragma unroll
    for (int z0 = 0; z0 < E; z0 += CH) {
        double dv[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (z0 + i < E) {
                int gz = gz0 + min(z0 + i, zmax);
                gz = gz >= n2 ? gz - n2 : gz;
                dv[i] = sgpr_ptr(D + plane * gz)[cl];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < CH; ++i)
            if (z0 + i < E) prev[z0 + i] = dv[i] * cur[z0 + i] - prev[z0 + i];
    }
}

// a pencil to a slot row [z][pencil] (E^2 apart; a wave's stores coalesce)
template <int E>
__device__ __forceinline__ void a64_store_row(double *row, bool active, const double (&v)[E]) {
    if (!active) return;
#pragma unroll
    for (int z = 0; z < E; ++z) sgpr_ptr(row + (int64_t)z * E * E)[threadIdx.x] = v[z];
}

struct A64Geo {
    int64_t col, plane;
    int gz0, n2;
};

// One step in place, prev <- scale (2 Hs cur) - prev (scale = 1/2 and prev = 0
// on the first step give v_1 = Hs v_0).  The raw projections of cur (chi . cur,
// and dchi . cur with GRAD) are left in dots / ddots.
template <int E, int R, int ZS, int NW, bool GRAD>
__device__ __forceinline__ void a64_step(const RegionArgs<double> &a,
                                         const StepCtx<double, E, R> &c, const A64Geo &g,
                                         double (&cur)[E], double (&prev)[E], double *lds,
                                         const Slot *slots, double (*pfac)[NP],
                                         double (*dots)[NP], double (*ddots)[3 * NP], bool first,
                                         double tau) {
    if (c.active) store_pencil<double, E, ZS>(c.mine, cur);
    __syncthreads();
    if (c.nat)
        projector_dots<double, ZS, NW, GRAD>(a, slots, pfac, dots, ddots, lds, c.nat, c.dx, c.dy,
                                             c.dz, tau);
    a64_diag<E, 9>(a.D, g.col, g.plane, g.gz0, g.n2, c.dz, cur, prev);
#pragma unroll
    for (int p = 1; p <= R; ++p) {
#pragma unroll
        for (int z = 0; z < E; ++z) {
            double s = 0.0;
            if (z + p < E) s += cur[z + p];
            if (z - p >= 0) s += cur[z - p];
            prev[z] = fma(c.cz[p], s, prev[z]);
        }
    }
    // neighbour offsets recomputed per step from an opaque zero, so the
    // compiler keeps none of the 4R of them live across the step loop
    int salt = 0;
    asm volatile("" : "+v"(salt));
    const int tid = threadIdx.x + salt;
    const int px = c.px + salt, py = c.py + salt;
#pragma unroll
    for (int p = 1; p <= R; ++p) {
        const int n0 = (c.active && px + p < c.dx) ? tid + p : c.npen;
        axpy_pencil<double, E, ZS>(prev, c.cx[p], lds + n0 * ZS);
        const int n1 = (c.active && px - p >= 0) ? tid - p : c.npen;
        axpy_pencil<double, E, ZS>(prev, c.cx[p], lds + n1 * ZS);
        const int n2_ = (c.active && py + p < c.dy) ? tid + p * c.dx : c.npen;
        axpy_pencil<double, E, ZS>(prev, c.cy[p], lds + n2_ * ZS);
        const int n3 = (c.active && py - p >= 0) ? tid - p * c.dx : c.npen;
        axpy_pencil<double, E, ZS>(prev, c.cy[p], lds + n3 * ZS);
    }
    __syncthreads();
    if (c.nat) {
        if (c.active) store_pencil<double, E, ZS>(c.mine, prev);
        __syncthreads();
        projector_update<double, ZS, NW>(a, slots, pfac, lds, c.nat, c.dx, c.dy, c.dz);
        __syncthreads();
        if (c.active) load_pencil<double, E, ZS>(c.mine, prev);
    }
    if (first) {
#pragma unroll
        for (int z = 0; z < E; ++z) prev[z] *= 0.5;
    }
#pragma unroll
    for (int z = 0; z < E; ++z) prev[z] = (z < c.dz) ? prev[z] : 0.0;
}

// projections of one vector without a step
template <int E, int R, int ZS, int NW, bool GRAD>
__device__ __forceinline__ void a64_dots(const RegionArgs<double> &a,
                                         const StepCtx<double, E, R> &c, const double (&vec)[E],
                                         double *lds, const Slot *slots, double (*pfac)[NP],
                                         double (*dots)[NP], double (*ddots)[3 * NP],
                                         double tau) {
    if (c.active) store_pencil<double, E, ZS>(c.mine, vec);
    __syncthreads();
    if (c.nat)
        projector_dots<double, ZS, NW, GRAD>(a, slots, pfac, dots, ddots, lds, c.nat, c.dx, c.dy,
                                             c.dz, tau);
    __syncthreads();
}

template <int E, int R, bool GRAD>
__global__ void __launch_bounds__(((E * E + 63) / 64) * 64)
cheb_adjoint64_kernel(const AdjointArgs<double> aa) {
    using T = double;
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    constexpr int NW = BLOCK / 64;
    constexpr int ZS = pencil_stride<T, E>();
    constexpr int EE = E * E;
    constexpr int64_t E3 = (int64_t)E * E * E;
    constexpr int BOXB = region_lds_elems<T, E>() * (int)sizeof(T);
    constexpr int PER = NP * 8 + (GRAD ? A64_PROJ * 8 : 0);   // pfac (+ dots, ddots)
    constexpr int AT0 = (LDS_BYTES - BOXB - 64) / PER;
    constexpr int AT = AT0 > MAX_REGION_ATOMS ? MAX_REGION_ATOMS : AT0;
    static_assert(AT >= 32, "the box leaves too little LDS for the atom projections");
    const RegionArgs<T> &a = aa.g;

    __shared__ __align__(16) T lds[region_lds_elems<T, E>()];
    __shared__ T pfac[AT][NP];
    __shared__ T dots[GRAD ? AT : 1][NP];
    __shared__ T ddots[GRAD ? AT : 1][3 * NP];
    __shared__ int s_item, s_nat;

    const int tid = threadIdx.x;
    const double tau = a.scal->tau;
    const int K = a.K;
    StepCtx<T, E, R> c;
#pragma unroll
    for (int p = 1; p <= R; ++p) {
        c.cx[p] = -a.w[p] * a.ih2[0] / tau;
        c.cy[p] = -a.w[p] * a.ih2[1] / tau;
        c.cz[p] = -a.w[p] * a.ih2[2] / tau;
    }
    T *slot = aa.ckpt + (int64_t)blockIdx.x * aa.ckpt_stride;
    T *Vrow = slot;                          // v_k       at Vrow + k E^3
    T *Trow = slot + (int64_t)K * E3;        // vt_{k+1}  at Trow + k E^3
    T *Prow = slot + 2 * (int64_t)K * E3;    // projections of v_k, [k][atom][A64_PROJ]
    Slot *slots = reinterpret_cast<Slot *>(Prow + (int64_t)K * MAX_REGION_ATOMS * A64_PROJ);
    T(*dp)[NP] = GRAD ? dots : nullptr;
    T(*ddp)[3 * NP] = GRAD ? ddots : nullptr;
    const double hs = a.h3 / tau;

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
        for (int i = tid; i < (npen + 1) * ZS; i += BLOCK) lds[i] = 0.0;
        if (a.n_atoms) gather_atoms<T, AT, BLOCK>(a, it, slots, &s_nat);
        int gx = it.lo[0] + px, gy = it.lo[1] + py;
        if (a.periodic) {
            gx = wrap(gx, a.N[0]);
            gy = wrap(gy, a.N[1]);
        }
        A64Geo g;
        g.col = (int64_t)gx + (int64_t)a.N[0] * gy;
        g.plane = (int64_t)a.N[0] * a.N[1];
        g.gz0 = a.periodic ? wrap(it.lo[2], a.N[2]) : it.lo[2];
        g.n2 = a.periodic ? a.N[2] : (1 << 30);
        const bool is_ctr = c.active && px == it.ctr[0] && py == it.ctr[1];
        const int cz0 = it.ctr[2];
        c.mine = lds + tid * ZS;
        c.px = px;
        c.py = py;
        c.npen = npen;
        __syncthreads();
        c.nat = min(s_nat, AT);
        if (tid == 0 && s_nat > AT) atomicOr(a.status, 1);
        const double gr = aa.g_rho ? aa.g_rho[it.out] : 0.0;
        const double gu = aa.g_u ? aa.g_u[it.out] : 0.0;

        // ---- forward sweep: v_0 .. v_{K-1} (and projections) to the slot ----
        T v[E], w[E];
#pragma unroll
        for (int z = 0; z < E; ++z) {
            v[z] = (is_ctr && z == cz0) ? 1.0 : 0.0;
            w[z] = 0.0;
        }
        // projections of v_k (dots / ddots) into the slot, row k
        auto store_proj = [&](int k) {
            T *pk = Prow + (int64_t)k * MAX_REGION_ATOMS * A64_PROJ;
            for (int i = tid; i < c.nat * A64_PROJ; i += BLOCK) {
                const int j = i / A64_PROJ, q = i - j * A64_PROJ;
                pk[i] = q < NP ? dots[j][q] : ddots[j][q - NP];
            }
        };
        for (int k = 0; k + 1 <= K - 1; k += 2) {
            a64_store_row<E>(Vrow + k * E3, c.active, v);
            a64_step<E, R, ZS, NW, GRAD>(a, c, g, v, w, lds, slots, pfac, dp, ddp, k == 0, tau);
            if constexpr (GRAD) store_proj(k);
            if (k + 2 <= K - 1) {
                a64_store_row<E>(Vrow + (k + 1) * E3, c.active, w);
                a64_step<E, R, ZS, NW, GRAD>(a, c, g, w, v, lds, slots, pfac, dp, ddp, false, tau);
                if constexpr (GRAD) store_proj(k + 1);
            }
        }
        // v_{K-1} (in v when K-1 is even): stored, and projected for dR
        if ((K - 1) % 2 == 0) {
            a64_store_row<E>(Vrow + (K - 1) * E3, c.active, v);
            if constexpr (GRAD) a64_dots<E, R, ZS, NW, GRAD>(a, c, v, lds, slots, pfac, dp, ddp, tau);
        } else {
            a64_store_row<E>(Vrow + (K - 1) * E3, c.active, w);
            if constexpr (GRAD) a64_dots<E, R, ZS, NW, GRAD>(a, c, w, lds, slots, pfac, dp, ddp, tau);
        }
        if constexpr (GRAD) store_proj(K - 1);

        // ---- reverse sweep: vt_{k+1} to the slot, dR per step ----
        {
            const T aK = 2.0 * (gr * aa.coef_c[K] + gu * aa.coef_d[K]);
#pragma unroll
            for (int z = 0; z < E; ++z) {
                v[z] = (is_ctr && z == cz0) ? aK : 0.0;   // vt_K
                w[z] = 0.0;                                // vt_{K+1}
            }
        }
        double dRr[3] = {0.0, 0.0, 0.0};   // thread j: atom j of the box
        auto rstep = [&](int k, T (&ta)[E], T (&tb)[E]) {
            a64_store_row<E>(Trow + k * E3, c.active, ta);
            if (k >= 1) {
                a64_step<E, R, ZS, NW, GRAD>(a, c, g, ta, tb, lds, slots, pfac, dp, ddp, false, tau);
                if (is_ctr) {
                    const T ak = 2.0 * (gr * aa.coef_c[k] + gu * aa.coef_d[k]);
#pragma unroll
                    for (int z = 0; z < E; ++z) tb[z] += (z == cz0) ? ak : 0.0;
                }
            } else if constexpr (GRAD) {
                a64_dots<E, R, ZS, NW, GRAD>(a, c, ta, lds, slots, pfac, dp, ddp, tau);
            }
            if constexpr (GRAD) {
                if (tid < c.nat) {
                    const T *pj = Prow + ((int64_t)k * MAX_REGION_ATOMS + tid) * A64_PROJ;
                    const double *cjp = a.cJ + (int64_t)slots[tid].atom * NP;
                    const double f = (k == 0 ? 1.0 : 2.0) * hs;
#pragma unroll
                    for (int x = 0; x < 3; ++x) {
                        double s = 0.0;
#pragma unroll
                        for (int l = 0; l < NP; ++l)
                            s += cjp[l] * (ddots[tid][l * 3 + x] * pj[l] +
                                           dots[tid][l] * pj[NP + l * 3 + x]);
                        dRr[x] += f * s;
                    }
                }
            }
        };
        for (int k = K - 1; k >= 0; k -= 2) {
            rstep(k, v, w);
            if (k - 1 >= 0) rstep(k - 1, w, v);
        }

        // ---- dV: G(z) = sum_k alpha_k vt_{k+1}(z) v_k(z), own pencil, FP64 ----
        if (aa.dV && c.active) {
            T G[E];
#pragma unroll
            for (int z = 0; z < E; ++z) G[z] = 0.0;
            constexpr int ZB = 9;   // planes per pass (loads in flight vs registers)
#pragma unroll
            for (int z0 = 0; z0 < E; z0 += ZB) {
                for (int k = 0; k < K; ++k) {
                    const T al = k == 0 ? 1.0 : 2.0;
                    T tv[ZB], vv[ZB];
#pragma unroll
                    for (int i = 0; i < ZB; ++i) {
                        if (z0 + i < E) {
                            tv[i] = sgpr_ptr(Trow + k * E3 + (int64_t)(z0 + i) * EE)[(uint32_t)tid];
                            vv[i] = sgpr_ptr(Vrow + k * E3 + (int64_t)(z0 + i) * EE)[(uint32_t)tid];
                        }
                    }
#pragma unroll
                    for (int i = 0; i < ZB; ++i)
                        if (z0 + i < E) G[z0 + i] = fma(al * tv[i], vv[i], G[z0 + i]);
                }
            }
            const double itau = 1.0 / tau;
#pragma unroll
            for (int z = 0; z < E; ++z) {
                if (z < c.dz) {
                    int gz = g.gz0 + z;
                    gz = gz >= g.n2 ? gz - g.n2 : gz;
                    unsafeAtomicAdd(aa.dV + g.col + g.plane * gz, G[z] * itau);
                }
            }
        }
        if constexpr (GRAD) {
            if (aa.dR && tid < c.nat)
                for (int x = 0; x < 3; ++x)
                    unsafeAtomicAdd(aa.dR + (int64_t)slots[tid].atom * 3 + x, dRr[x]);
        }
        __syncthreads();
    }
}

// launch / occupancy of the FP64 edge-27 adjoint for one radius
template <int R, bool G>
static hipError_t a64_launch_one(const void *args, int grid, hipStream_t s, int *occ) {
    constexpr int E = A64_EDGE;
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    if (occ) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cheb_adjoint64_kernel<E, R, G>, BLOCK,
                                                         0) != hipSuccess)
            n = 1;
        *occ = n > 0 ? n : 1;
        return hipSuccess;
    }
    hipLaunchKernelGGL((cheb_adjoint64_kernel<E, R, G>), dim3(grid), dim3(BLOCK), 0, s,
                       *static_cast<const AdjointArgs<double> *>(args));
    return hipGetLastError();
}

}  // namespace sqk
