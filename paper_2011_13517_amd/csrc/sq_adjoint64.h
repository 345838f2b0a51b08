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
// 160 KB):
//  * Thread t owns the z-pencil (t mod dx, t / dx) of the two live vectors in
//    VGPRs; the LDS holds the box once (x/y neighbours) plus one zero pencil,
//    and the per-atom projections.
//  * Projector block on the column path of the other region kernels (each
//    thread projects its own pencil's pieces of the atom supports and adds the
//    rank-4 term to its own pencil); the atom list and the column entries of the
//    box live in the workgroup's HBM slot instead of the LDS.
//  * Forward sweep: v_0 .. v_{K-1} go to the slot, and the projections
//    p_k = chi . v_k that the recurrence forms anyway.  Reverse sweep: vt_{k+1}
//    goes to the slot, and q_k = chi . vt_{k+1}.  No dchi projections are
//    formed per step.
//  * A final pass of each thread over its own pencil streams vt_{k+1}(z) and
//    v_k(z) back from the slot and accumulates, in FP64 registers,
//      dV(z) = (1/tau) sum_k alpha_k vt_{k+1}(z) v_k(z)
//    and, on the support rows of its column pieces, the row accumulators
//      W_l(y) = sum_k alpha_k (p_k,l vt_{k+1}(y) + q_k,l v_k(y)),
//    whose contraction with dchi gives dR (by linearity the dR sum above is
//    (h^3/tau) sum_l c_l sum_y dchi_l(y) W_l(y)); dchi is read once per row.
//  * dV is added to the grid with FP64 atomics; dR is reduced per atom in LDS
//    and added once per atom per region.
#pragma once

#include "sq_region.h"

namespace sqk {

// a block-uniform FP64 value pinned in scalar registers (the stencil weights:
// 3(R+1) doubles that would otherwise hold 6(R+1) VGPRs for the whole kernel)
__device__ __forceinline__ double uniform_f64(double x) {
    const long long b = __double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(b & 0xffffffffLL));
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | lo);
}

constexpr int A64_EDGE = 27;
constexpr int A64_ATOMS = 48;      // atoms per box (the LDS left beside the FP64 box)

// slot of one workgroup (doubles): v_k rows and vt_{k+1} rows ([k][z][pencil],
// E^3 each), projections p_k and q_k ([k][atom][NP] each), then the atom list
// (Slot) and the column entries ([thread][MAXC] ColEntry) of the box
constexpr int64_t a64_proj_elems(int K) { return (int64_t)K * A64_ATOMS * NP; }
constexpr int64_t a64_tables_elems(int E) {
    return ((int64_t)A64_ATOMS * sizeof(Slot) +
            (int64_t)((E * E + 63) / 64 * 64) * MAXC * sizeof(ColEntry) + 7) / 8;
}
constexpr int64_t a64_slot_elems(int K, int E) {
    return round_np(2 * (int64_t)K * E * E * E + 2 * a64_proj_elems(K) + a64_tables_elems(E));
}

// projections of the last step (parity buffer par ^ 1 of nl) to a slot row
template <int BLOCK>
__device__ __forceinline__ void a64_store_proj(const ColNL<double> &nl, int nat, double *row) {
    const double *pa = nl.pacc + (int64_t)(nl.par ^ 1) * nl.maxat * NP;
    for (int i = threadIdx.x; i < nat * NP; i += BLOCK) row[i] = pa[i];
}

// One recurrence step with one pencil in registers:
//   acc <- scale (2 Hs acc) - prev  (+ inj at plane inj_z of the owning thread),
// scale = 1/2 on the first step.  On entry acc holds cur; cur is published to
// the LDS box, and the register part (D cur - prev and the z neighbours) re-reads
// cur from the thread's own LDS pencil in batches of ZB planes while acc is
// overwritten batch by batch; prev (the vector two steps back) streams from its
// slot row (PREV false: zero; a compile-time choice, so the batch of loads has
// no branches between them).  The result is written to out_row.  The
// projections chi . cur are left in parity buffer nl.par ^ 1.
template <int E, int R, int ZS, int BLOCK, bool PREV>
__device__ __forceinline__ void a64_step(const RegionArgs<double> &a,
                                         const StepCtx<double, E, R> &c, int64_t col,
                                         int64_t plane, int gz0, int n2, double (&acc)[E],
                                         double *lds, ColNL<double> &nl, bool first,
                                         const double *prev_row, double *out_row, int inj_z,
                                         double inj) {
    constexpr int EE = E * E;
    constexpr int ZB = 9;
    if (c.active) store_pencil<double, E, ZS>(c.mine, acc);
    __syncthreads();
    if (c.nat) col_dots<double, false>(a, nl, c.mine);
    if (c.active) {
        int salt = 0;
        asm volatile("" : "+s"(salt));
        const uint32_t cl = (uint32_t)col;
        const int zmax = c.dz - 1 + salt;
        const uint32_t t = threadIdx.x;
#pragma unroll
        for (int z0 = 0; z0 < E; z0 += ZB) {
            double cw[ZB + 2 * R], dv[ZB], pv[ZB];
#pragma unroll
            for (int i = 0; i < ZB + 2 * R; ++i) {
                const int z = z0 - R + i;
                cw[i] = (z >= 0 && z < E) ? c.mine[z] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < ZB; ++i) {
                if (z0 + i < E) {
                    int gz = gz0 + min(z0 + i, zmax);
                    gz = gz >= n2 ? gz - n2 : gz;
                    dv[i] = sgpr_ptr(a.D + plane * gz)[cl];
                    pv[i] = PREV ? sgpr_ptr(prev_row + (int64_t)(z0 + i) * EE)[t] : 0.0;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < ZB; ++i) {
                if (z0 + i < E) {
                    double r = dv[i] * cw[i + R] - pv[i];
#pragma unroll
                    for (int p = 1; p <= R; ++p) r = fma(c.cz[p], cw[i + R + p] + cw[i + R - p], r);
                    acc[z0 + i] = r;
                }
            }
        }
        // x/y neighbours from the LDS box (offsets recomputed from an opaque zero
        // so that none of the 4R stays live across the step loop)
        int s2 = 0;
        asm volatile("" : "+v"(s2));
        const int tid = threadIdx.x + s2;
        const int px = c.px + s2, py = c.py + s2;
#pragma unroll
        for (int p = 1; p <= R; ++p) {
            const int n0 = (px + p < c.dx) ? tid + p : c.npen;
            axpy_pencil<double, E, ZS>(acc, c.cx[p], lds + n0 * ZS);
            const int n1 = (px - p >= 0) ? tid - p : c.npen;
            axpy_pencil<double, E, ZS>(acc, c.cx[p], lds + n1 * ZS);
            const int n2_ = (py + p < c.dy) ? tid + p * c.dx : c.npen;
            axpy_pencil<double, E, ZS>(acc, c.cy[p], lds + n2_ * ZS);
            const int n3 = (py - p >= 0) ? tid - p * c.dx : c.npen;
            axpy_pencil<double, E, ZS>(acc, c.cy[p], lds + n3 * ZS);
        }
    }
    __syncthreads();
    if (first) {
#pragma unroll
        for (int z = 0; z < E; ++z) acc[z] *= 0.5;
    }
#pragma unroll
    for (int z = 0; z < E; ++z) acc[z] = (z < c.dz) ? acc[z] : 0.0;
    if (c.nat) {
        if (c.active) store_pencil<double, E, ZS>(c.mine, acc);
        if (nl.ncol) col_update<double>(a, nl, c.mine, first ? 0.5 : 1.0);
        if (c.active) load_pencil<double, E, ZS>(c.mine, acc);
        col_zero_next<double, BLOCK, false>(nl, c.nat);
    }
    nl.par ^= 1;
    if (inj_z >= 0) {
#pragma unroll
        for (int z = 0; z < E; ++z) acc[z] += (z == inj_z) ? inj : 0.0;
    }
    if (c.active && out_row) {
#pragma unroll
        for (int z = 0; z < E; ++z) sgpr_ptr(out_row + (int64_t)z * EE)[threadIdx.x] = acc[z];
    }
}

template <int E, int R>
__global__ void __launch_bounds__(((E * E + 63) / 64) * 64)
cheb_adjoint64_kernel(const AdjointArgs<double> aa) {
    using T = double;
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    constexpr int ZS = pencil_stride<T, E>();
    constexpr int EE = E * E;
    constexpr int64_t E3 = (int64_t)E * E * E;
    constexpr int AT = A64_ATOMS;
    const RegionArgs<T> &a = aa.g;

    __shared__ __align__(16) T lds[region_lds_elems<T, E>()];
    __shared__ T pfac[AT][NP];         // 2 h^3 c_Jl / tau
    __shared__ T pacc[2][AT][NP];      // raw projections by step parity
    __shared__ double cdR[AT][3];      // dR of the box
    __shared__ int s_item, s_nat;

    const int tid = threadIdx.x;
    const double tau = a.scal->tau;
    const int K = a.K;
    StepCtx<T, E, R> c;
#pragma unroll
    for (int p = 1; p <= R; ++p) {
        c.cx[p] = uniform_f64(-a.w[p] * a.ih2[0] / tau);
        c.cy[p] = uniform_f64(-a.w[p] * a.ih2[1] / tau);
        c.cz[p] = uniform_f64(-a.w[p] * a.ih2[2] / tau);
    }
    T *slot = aa.ckpt + (int64_t)blockIdx.x * aa.ckpt_stride;
    T *Vrow = slot;                          // v_k       at Vrow + k E^3
    T *Trow = slot + (int64_t)K * E3;        // vt_{k+1}  at Trow + k E^3
    T *Prow = slot + 2 * (int64_t)K * E3;    // p_k = chi . v_k        [k][atom][NP]
    T *Qrow = Prow + a64_proj_elems(K);      // q_k = chi . vt_{k+1}   [k][atom][NP]
    Slot *slots = reinterpret_cast<Slot *>(Qrow + a64_proj_elems(K));
    ColEntry *colbuf = reinterpret_cast<ColEntry *>(slots + AT);

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
        const int64_t col = (int64_t)gx + (int64_t)a.N[0] * gy;
        const int64_t plane = (int64_t)a.N[0] * a.N[1];
        const int gz0 = a.periodic ? wrap(it.lo[2], a.N[2]) : it.lo[2];
        const int n2 = a.periodic ? a.N[2] : (1 << 30);
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
        for (int j = tid; j < c.nat; j += BLOCK) {
            const double f = 2.0 * a.h3 / tau;
            const double *cj = a.cJ + (int64_t)slots[j].atom * NP;
#pragma unroll
            for (int l = 0; l < NP; ++l) {
                pfac[j][l] = f * cj[l];
                pacc[0][j][l] = pacc[1][j][l] = 0.0;
            }
            cdR[j][0] = cdR[j][1] = cdR[j][2] = 0.0;
        }
        ColEntry *mycols = colbuf + tid * MAXC;
        int ncol = build_columns<T>(a, slots, c.nat, c.active, px, py, c.dz, mycols);
        if (ncol > MAXC) {
            atomicOr(a.status, 2);
            ncol = MAXC;
        }
        ColNL<T> nl{};
        nl.cols = mycols;
        nl.ncol = ncol;
        nl.pacc = &pacc[0][0][0];
        nl.scale = &pfac[0][0];
        nl.maxat = AT;
        __syncthreads();

        // ---- forward sweep: v_0 .. v_{K-1} and p_k = chi . v_k to the slot ----
        T acc[E];
#pragma unroll
        for (int z = 0; z < E; ++z) acc[z] = (is_ctr && z == cz0) ? 1.0 : 0.0;
        if (c.active)
            for (int z = 0; z < E; ++z) sgpr_ptr(Vrow + (int64_t)z * EE)[tid] = acc[z];
        for (int k = 0; k + 1 <= K - 1; ++k) {
            if (k == 0)
                a64_step<E, R, ZS, BLOCK, false>(a, c, col, plane, gz0, n2, acc, lds, nl, true,
                                                 nullptr, Vrow + E3, -1, 0.0);
            else
                a64_step<E, R, ZS, BLOCK, true>(a, c, col, plane, gz0, n2, acc, lds, nl, false,
                                                Vrow + (k - 1) * E3, Vrow + (k + 1) * E3, -1, 0.0);
            a64_store_proj<BLOCK>(nl, c.nat, Prow + (int64_t)k * AT * NP);
        }
        // acc = v_{K-1}: its projections without a step
        col_dots_only<T, E, R, ZS, BLOCK, false>(a, c, acc, nl);
        a64_store_proj<BLOCK>(nl, c.nat, Prow + (int64_t)(K - 1) * AT * NP);

        // ---- reverse sweep: vt_{k+1} and q_k = chi . vt_{k+1} to the slot ----
        const T aK = 2.0 * (gr * aa.coef_c[K] + gu * aa.coef_d[K]);
#pragma unroll
        for (int z = 0; z < E; ++z) acc[z] = (is_ctr && z == cz0) ? aK : 0.0;   // vt_K
        if (c.active)
            for (int z = 0; z < E; ++z) sgpr_ptr(Trow + (K - 1) * E3 + (int64_t)z * EE)[tid] = acc[z];
        for (int k = K - 1; k >= 1; --k) {
            // vt_k = a_k e_q + 2 Hs vt_{k+1} - vt_{k+2}   (vt_{K+1} = 0)
            const T ak = 2.0 * (gr * aa.coef_c[k] + gu * aa.coef_d[k]);
            if (k == K - 1)
                a64_step<E, R, ZS, BLOCK, false>(a, c, col, plane, gz0, n2, acc, lds, nl, false,
                                                 nullptr, Trow + (k - 1) * E3, is_ctr ? cz0 : -1,
                                                 ak);
            else
                a64_step<E, R, ZS, BLOCK, true>(a, c, col, plane, gz0, n2, acc, lds, nl, false,
                                                Trow + (k + 1) * E3, Trow + (k - 1) * E3,
                                                is_ctr ? cz0 : -1, ak);
            a64_store_proj<BLOCK>(nl, c.nat, Qrow + (int64_t)k * AT * NP);
        }
        // acc = vt_1: its projections q_0 without a step
        col_dots_only<T, E, R, ZS, BLOCK, false>(a, c, acc, nl);
        a64_store_proj<BLOCK>(nl, c.nat, Qrow);
        __syncthreads();   // the slot's projection rows are read by other threads below

        // ---- dV: G(z) = sum_k alpha_k vt_{k+1}(z) v_k(z), own pencil, FP64 ----
        if (aa.dV && c.active) {
            T G[E];
#pragma unroll
            for (int z = 0; z < E; ++z) G[z] = 0.0;
            constexpr int ZB = 9;   // planes per pass (loads in flight vs registers)
            const uint32_t t = (uint32_t)tid;
#pragma unroll
            for (int z0 = 0; z0 < E; z0 += ZB) {
                // two steps per iteration: 4 ZB loads in flight
                for (int k = 0; k < K; k += 2) {
                    const bool two = k + 1 < K;
                    const int k1 = two ? k + 1 : k;
                    const T a0 = k == 0 ? 1.0 : 2.0, a1 = two ? 2.0 : 0.0;
                    T tv[2][ZB], vv[2][ZB];
#pragma unroll
                    for (int i = 0; i < ZB; ++i) {
                        if (z0 + i < E) {
                            tv[0][i] = sgpr_ptr(Trow + k * E3 + (int64_t)(z0 + i) * EE)[t];
                            vv[0][i] = sgpr_ptr(Vrow + k * E3 + (int64_t)(z0 + i) * EE)[t];
                            tv[1][i] = sgpr_ptr(Trow + k1 * E3 + (int64_t)(z0 + i) * EE)[t];
                            vv[1][i] = sgpr_ptr(Vrow + k1 * E3 + (int64_t)(z0 + i) * EE)[t];
                        }
                    }
#pragma unroll
                    for (int i = 0; i < ZB; ++i) {
                        if (z0 + i < E) {
                            G[z0 + i] = fma(a0 * tv[0][i], vv[0][i], G[z0 + i]);
                            G[z0 + i] = fma(a1 * tv[1][i], vv[1][i], G[z0 + i]);
                        }
                    }
                }
            }
            const double itau = 1.0 / tau;
#pragma unroll
            for (int z = 0; z < E; ++z) {
                if (z < c.dz) {
                    int gz = gz0 + z;
                    gz = gz >= n2 ? gz - n2 : gz;
                    unsafeAtomicAdd(aa.dV + col + plane * gz, G[z] * itau);
                }
            }
        }

        // ---- dR: row accumulators W on this pencil's support rows ----
        if (aa.dR) {
            constexpr int RB = 4;   // rows per pass
            for (int cc = 0; cc < nl.ncol; ++cc) {
                const ColEntry e = mycols[cc];
                const double *cj = a.cJ + (int64_t)slots[e.slot].atom * NP;
                double sx[3] = {0.0, 0.0, 0.0};
                for (int i0 = 0; i0 < e.n; i0 += RB) {
                    double W[RB][NP];
#pragma unroll
                    for (int r = 0; r < RB; ++r)
#pragma unroll
                        for (int l = 0; l < NP; ++l) W[r][l] = 0.0;
                    for (int k = 0; k < K; k += 2) {
                        // two steps per iteration (the second weighted 0 past K - 1)
                        const bool two = k + 1 < K;
                        const int k1 = two ? k + 1 : k;
                        const T al[2] = {k == 0 ? 1.0 : 2.0, two ? 2.0 : 0.0};
                        double p[2][NP], q[2][NP], tv[2][RB], vv[2][RB];
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int kk = h ? k1 : k;
                            const double *pk = Prow + ((int64_t)kk * AT + e.slot) * NP;
                            const double *qk = Qrow + ((int64_t)kk * AT + e.slot) * NP;
#pragma unroll
                            for (int l = 0; l < NP; ++l) {
                                p[h][l] = pk[l];
                                q[h][l] = qk[l];
                            }
                            // z differs between lanes here (each lane's own piece),
                            // so the row address is a per-lane one
#pragma unroll
                            for (int r = 0; r < RB; ++r) {
                                const int64_t o =
                                    kk * E3 + (int64_t)(e.zlo + min(i0 + r, e.n - 1)) * EE + tid;
                                tv[h][r] = Trow[o];
                                vv[h][r] = Vrow[o];
                            }
                        }
#pragma unroll
                        for (int h = 0; h < 2; ++h)
#pragma unroll
                            for (int r = 0; r < RB; ++r)
#pragma unroll
                                for (int l = 0; l < NP; ++l)
                                    W[r][l] += al[h] * (p[h][l] * tv[h][r] + q[h][l] * vv[h][r]);
                    }
#pragma unroll
                    for (int r = 0; r < RB; ++r) {
                        if (i0 + r < e.n) {
                            const double *dc = a.dchi + (int64_t)(e.row0 + i0 + r) * 3 * NP;
#pragma unroll
                            for (int l = 0; l < NP; ++l)
#pragma unroll
                                for (int x = 0; x < 3; ++x) sx[x] += cj[l] * dc[l * 3 + x] * W[r][l];
                        }
                    }
                }
                const double hs = a.h3 / tau;
#pragma unroll
                for (int x = 0; x < 3; ++x) atomicAdd(&cdR[e.slot][x], sx[x] * hs);
            }
            __syncthreads();
            for (int j = tid; j < c.nat; j += BLOCK)
                for (int x = 0; x < 3; ++x)
                    unsafeAtomicAdd(aa.dR + (int64_t)slots[j].atom * 3 + x, cdR[j][x]);
        }
        __syncthreads();
    }
}

// launch / occupancy of the FP64 edge-27 adjoint for one radius
template <int R>
static hipError_t a64_launch_one(const void *args, int grid, hipStream_t s, int *occ) {
    constexpr int E = A64_EDGE;
    constexpr int BLOCK = ((E * E + 63) / 64) * 64;
    if (occ) {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cheb_adjoint64_kernel<E, R>, BLOCK,
                                                         0) != hipSuccess)
            n = 1;
        *occ = n > 0 ? n : 1;
        return hipSuccess;
    }
    hipLaunchKernelGGL((cheb_adjoint64_kernel<E, R>), dim3(grid), dim3(BLOCK), 0, s,
                       *static_cast<const AdjointArgs<double> *>(args));
    return hipGetLastError();
}

}  // namespace sqk
