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
//    and the per-atom projections.  The box keeps planes 0 .. E-2 of every
//    pencil at an even stride (16-byte reads and writes of plane pairs) and
//    plane E-1 of all pencils in a block of its own.
//  * Projector block atom-major: at region start the box's support rows are
//    listed atom by atom in chunks of 64 (row, LDS offset) entries; in every
//    step each wave walks its share of the chunks, forming chi . v with wave
//    reductions and adding the rank-4 term with LDS atomics.  The atom list,
//    the row list and the column entries of the box (used by the final pass)
//    live in the workgroup's HBM slot instead of the LDS.
//  * Forward sweep: v_0 .. v_{K-1} go to the slot, and the projections
//    p_k = chi . v_k that the recurrence forms anyway.  Reverse sweep: vt_{k+1}
//    goes to the slot, and q_k = chi . vt_{k+1}.  No dchi projections are
//    formed per step.  Both live vectors of a sweep stay in registers (the one
//    being advanced is updated in place; the other is published to the LDS box
//    and read back after the step), so a step reads nothing back from the slot.
//  * Slot rows and the diagonal are addressed as one block-uniform base plus a
//    32-bit lane offset (one scalar pair per stream instead of one per plane);
//    this bounds the V grid to A64_MAX_GRID points.
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

#include <type_traits>
#include <utility>

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
constexpr int A64_DB = 9;          // planes of the diagonal per load batch
#ifndef A64_FZB
#define A64_FZB 3                  // planes per batch of the final dV / dR pass
#endif
#ifndef A64_XY_SPLIT
#define A64_XY_SPLIT 3             // x/y pipeline units per pencil
#endif
#ifndef A64_MFMA_DOTS
#define A64_MFMA_DOTS 0            // projections with FP64 matrix instructions (1) or VALU (0)
#endif
#ifndef A64_NCB
#define A64_NCB 2                  // chunks per load batch of the atom-major block
#endif
// V grids up to this many points keep every byte offset of the diagonal in 32 bits
// (slot rows: K up to 512 keeps 2 K E^3 doubles below 2^32 bytes)
constexpr int64_t A64_MAX_GRID = (int64_t)1 << 29;

// Slot rows and the diagonal are read and written with raw buffer
// instructions: a resource in scalar registers, a 32-bit lane offset (one
// VGPR per stream, whatever the plane) and a scalar plane offset.  The
// resource's extent is the stream's byte size; in-range offsets are what the
// kernel forms, and the hardware returns zero for (and drops) anything past it.
typedef unsigned int a64_u2 __attribute__((ext_vector_type(2)));
constexpr int A64_RSRC_WORD3 = 0x00020000;   // raw 32-bit data format (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t a64_rsrc(const void *base, int64_t bytes) {
    const uint32_t n = bytes >= (int64_t)0xffffffffLL ? 0xffffffffu : (uint32_t)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)n,
                                             A64_RSRC_WORD3);
}
// Cache policy of the streams: the slot rows are written once per step and
// read once in the final passes, so they go non-temporal (their 157 KB per
// step and workgroup would otherwise evict the diagonal and the projector
// table, which every step reads again, from the L2).
constexpr int A64_CACHED = 0;
#ifndef A64_STREAM_POLICY
#define A64_STREAM_POLICY 2        // nt
#endif
#ifndef A64_REREAD_POLICY
#define A64_REREAD_POLICY 2        // nt
#endif
constexpr int A64_STREAM = A64_STREAM_POLICY;
constexpr int A64_REREAD = A64_REREAD_POLICY;   // the final passes' reads of the rows

// byte offsets: voff per lane, soff block-uniform
template <int POL = A64_CACHED>
__device__ __forceinline__ double a64_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const a64_u2 v =
        __builtin_amdgcn_raw_buffer_load_b64(r, voff, __builtin_amdgcn_readfirstlane(soff), POL);
    return __builtin_bit_cast(double, v);
}
template <int POL = A64_STREAM>
__device__ __forceinline__ void a64_st(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                       double x) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(a64_u2, x), r, voff,
                                          __builtin_amdgcn_readfirstlane(soff), POL);
}

constexpr int64_t a64_proj_elems(int K) { return (int64_t)K * A64_ATOMS * NP; }
// per-workgroup tables behind the rows: atom slots, column entries, the
// atom-major list of the box's support rows (int2, at most one entry per
// column-entry row plus a chunk of padding per atom) and its per-atom counts
constexpr int64_t a64_list_cap_elems(int E) {
    return (int64_t)((E * E + 63) / 64 * 64) * MAXC * E + (int64_t)A64_ATOMS * 64;
}
constexpr int64_t a64_tables_elems(int E) {
    return ((int64_t)A64_ATOMS * sizeof(Slot) +
            (int64_t)((E * E + 63) / 64 * 64) * MAXC * sizeof(ColEntry) +
            a64_list_cap_elems(E) * 8 + (int64_t)A64_ATOMS * 4 + 7) / 8;
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

// x/y neighbours: acc += sum over the 4R neighbouring pencils of their
// weight times the pencil, read from the LDS box in NS units of a pencil
// (A64Units: runs of an even number of planes) through a two-deep pipeline: the reads of the next unit are in flight while
// the FMAs of the current one run (left to itself the compiler issues the
// reads one at a time, each waiting for the previous).  Every unit is its own
// compile-time instance, so both buffers stay in registers.  A neighbour
// outside the box is the zero pencil npen.
struct A64Lane {
    int tid, px, py;
};

// LDS box of this kernel: planes 0 .. E-2 of pencil n at n (E - 1), an even
// stride, so every pencil starts 16-byte aligned and pairs of planes move as
// 16-byte reads and writes; plane E - 1 of every pencil after them, at
// a64_xb + n.  The same size as pencils of E planes; with odd E-plane pencils
// half of them start 8 bytes off and the reads go as 8-byte pairs, which an
// LDS read probe of this pattern measured at 112 B/clk/CU against 157.
template <int E>
constexpr int a64_xb() {
    static_assert(E % 2 == 1, "an even stride E - 1");
    return (E * E + 1) * (E - 1);
}
template <int E>
__device__ __forceinline__ int a64_off(int n, int z) {
    return z < E - 1 ? n * (E - 1) + z : a64_xb<E>() + n;
}
// planes Z0 .. Z0 + H - 1 (those below E) of pencil n to q[0 .. H-1]
template <int E, int Z0, int H, typename Q>
__device__ __forceinline__ void a64_box_get(Q &q, const double *lds, int n) {
    constexpr int PS = E - 1;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const int z = Z0 + i;
        if (z >= E) continue;
        const bool pair = (z % 2 == 0) && z + 1 < PS && i + 1 < H;
        const bool second = (z % 2 == 1) && i > 0 && z < PS;
        if (pair) {
            const double2 d = *reinterpret_cast<const double2 *>(lds + n * PS + z);
            q[i] = d.x;
            q[i + 1] = d.y;
        } else if (!second) {
            q[i] = z < PS ? lds[n * PS + z] : lds[a64_xb<E>() + n];
        }
    }
}
// all E planes of v to pencil n
template <int E>
__device__ __forceinline__ void a64_box_put(double *lds, int n, const double (&v)[E]) {
    constexpr int PS = E - 1;
#pragma unroll
    for (int z = 0; z < PS; z += 2) {
        double2 d;
        d.x = v[z];
        d.y = v[z + 1];
        *reinterpret_cast<double2 *>(lds + n * PS + z) = d;
    }
    lds[a64_xb<E>() + n] = v[E - 1];
}

// units of a pencil: NS runs of planes of an even length (the last one shorter:
// 10, 10, 7 at E = 27), so that every unit starts on a 16-byte plane pair and
// reads only pairs (and plane E-1 from its own block).  Thirds of 9 planes put
// an 8-byte read at an odd plane into two units in three, and 8-byte reads at
// the even pencil stride meet in pairs on the LDS banks.
template <int E, int NS>
struct A64Units {
    static constexpr int H = ((E + NS - 1) / NS + 1) / 2 * 2;   // planes per unit
    static constexpr int z0(int k) { return k * H; }
    static constexpr int hz(int k) { return k + 1 < NS ? H : E - k * H; }
    using Buf = double[H];   // one unit of a neighbour pencil
};

template <int E, int R, int ZS, int NS, int U>
__device__ __forceinline__ void a64_xy_load(typename A64Units<E, NS>::Buf &q,
                                            const StepCtx<double, E, R> &c, const A64Lane &l,
                                            const double *lds) {
    constexpr int HZ = A64Units<E, NS>::hz(U % NS);
    constexpr int j = U / NS, p = j / 4 + 1, dir = j % 4, z0 = A64Units<E, NS>::z0(U % NS);
    int n;
    if constexpr (dir == 0) n = (l.px + p < c.dx) ? l.tid + p : c.npen;
    else if constexpr (dir == 1) n = (l.px - p >= 0) ? l.tid - p : c.npen;
    else if constexpr (dir == 2) n = (l.py + p < c.dy) ? l.tid + p * c.dx : c.npen;
    else n = (l.py - p >= 0) ? l.tid - p * c.dx : c.npen;
    a64_box_get<E, z0, HZ>(q, lds, n);
}

template <int E, int R, int ZS, int NS, int U>
__device__ __forceinline__ void a64_xy_unit(double (&acc)[E], typename A64Units<E, NS>::Buf &qa,
                                            typename A64Units<E, NS>::Buf &qb,
                                            const StepCtx<double, E, R> &c, const A64Lane &l,
                                            const double *lds) {
    constexpr int HZ = A64Units<E, NS>::hz(U % NS);
    constexpr int HM = A64Units<E, NS>::H;
    constexpr int NU = 4 * R * NS;
    if constexpr (U + 1 < NU) {
        if constexpr ((U + 1) & 1) a64_xy_load<E, R, ZS, NS, U + 1>(qb, c, l, lds);
        else a64_xy_load<E, R, ZS, NS, U + 1>(qa, c, l, lds);
    }
    __builtin_amdgcn_sched_barrier(0);
    constexpr int j = U / NS, p = j / 4 + 1, z0 = A64Units<E, NS>::z0(U % NS);
    const double w = (j % 4 < 2) ? c.cx[p] : c.cy[p];
    const double(&q)[HM] = (U & 1) ? qb : qa;
#pragma unroll
    for (int i = 0; i < HZ; ++i)
        if (z0 + i < E) acc[z0 + i] = fma(w, q[i], acc[z0 + i]);
    __builtin_amdgcn_sched_barrier(0);
}

template <int E, int R, int ZS, int NS, int... U>
__device__ __forceinline__ void a64_xy_run(double (&acc)[E], const StepCtx<double, E, R> &c,
                                           const A64Lane &l, const double *lds,
                                           std::integer_sequence<int, U...>) {
    double qa[A64Units<E, NS>::H], qb[A64Units<E, NS>::H];
    a64_xy_load<E, R, ZS, NS, 0>(qa, c, l, lds);
    (a64_xy_unit<E, R, ZS, NS, U>(acc, qa, qb, c, l, lds), ...);
}

template <int E, int R, int ZS>
__device__ __forceinline__ void a64_xy(double (&acc)[E], const StepCtx<double, E, R> &c,
                                       const double *lds) {
    constexpr int NS = A64_XY_SPLIT;
    // lane offsets recomputed from an opaque zero so that none of the 4R
    // neighbour addresses stays live across the step loop
    int s2 = 0;
    asm volatile("" : "+v"(s2));
    const A64Lane l{(int)threadIdx.x + s2, c.px + s2, c.py + s2};
    static_assert(NS > 0, "x/y units of the box");
    a64_xy_run<E, R, ZS, NS>(acc, c, l, lds, std::make_integer_sequence<int, 4 * R * NS>{});
}

// the wave's largest column-entry count (the final pass runs every lane to it)
__device__ __forceinline__ int a64_wave_max(int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m));
    return __builtin_amdgcn_readfirstlane(v);
}

// ---- atom-major projector block ----
// The support rows of the box are listed atom by atom, in support-table order
// (x-fastest columns, z contiguous, so consecutive entries are mostly
// consecutive rows of chi): entry (row, off | slot << 16), off the element
// offset of the point in the LDS box.  Every atom's run is padded to whole
// chunks of 64 entries; a padding entry points at the zero pencil and has bit
// 31 set.  The chunks of the box are split into one contiguous range per
// wave, so a wave reads 64 consecutive entries per chunk (coalesced chi rows,
// the same number of rows in every lane) where the column path has each lane
// read its own pencil's rows, with run lengths that differ between lanes.
constexpr int A64_CHUNK = 64;
constexpr int A64_PAD = (int)0x80000000;
template <int E>
constexpr int64_t a64_list_cap() {
    static_assert(A64_CHUNK == 64, "one chunk per wave");
    return a64_list_cap_elems(E);
}

// sum over the 64 lanes of the wave, the same in every lane: rotations
// within each row of 16 lanes (DPP), then the four row sums
__device__ __forceinline__ double a64_wave_sum(double x) {
    x += dpp_f<0x128>(x);   // row_ror:8
    x += dpp_f<0x124>(x);   // row_ror:4
    x += dpp_f<0x122>(x);   // row_ror:2
    x += dpp_f<0x121>(x);   // row_ror:1
    auto lane_val = [&](int l) {
        const long long b = __double_as_longlong(x);
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)(b & 0xffffffffLL), l);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), l);
        return __longlong_as_double(((long long)hi << 32) | lo);
    };
    return (lane_val(0) + lane_val(16)) + (lane_val(32) + lane_val(48));
}

// in-box run of column (cx, cy) of atom slot sl: first row, box pencil and
// first plane, length
__device__ __forceinline__ int a64_run(const RegionArgs<double> &a, const Slot &sl, int cx,
                                       int cy, int dx, int dz, int &row, int &pen, int &zfirst) {
    const int64_t ci = 2 * ((int64_t)sl.col + (int64_t)cy * sl.bx + cx);
    const int r0 = a.colidx[ci], zc = a.colidx[ci + 1];
    const int z0 = sl.oz + (zc & 0xffff);
    const int zlo = max(z0, 0), zhi = min(z0 + (zc >> 16), dz);
    row = r0 + (zlo - z0);
    pen = (sl.oy + cy) * dx + (sl.ox + cx);
    zfirst = zlo;
    return max(zhi - zlo, 0);
}

// Builds the list for the nat atoms of the box into list (capacity
// a64_list_cap entries) with per-atom row counts in acnt; returns the number
// of chunks (block-uniform).  Atoms whose chunks would pass the capacity are
// left out and status bit 2 is raised (the same condition as more than MAXC
// supports crossing one pencil).
template <int E, int ZS, int BLOCK>
__device__ int a64_build_list(const RegionArgs<double> &a, const Slot *slots, int nat, int dx,
                              int dy, int dz, int zero_off, int2 *list, int *acnt) {
    constexpr int NW = BLOCK / 64;
    constexpr int64_t CAP = a64_list_cap<E>();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    auto cols = [&](const Slot &sl, int &cx0, int &cy0, int &wx) {
        cx0 = max(0, -sl.ox);
        cy0 = max(0, -sl.oy);
        wx = max(min(sl.bx, dx - sl.ox) - cx0, 0);
        const int wy = max(min(sl.by, dy - sl.oy) - cy0, 0);
        return wx * wy;
    };
    // pass 1: in-box rows per atom
    for (int j = wave; j < nat; j += NW) {
        const Slot sl = slots[j];
        int cx0, cy0, wx;
        const int ncols = cols(sl, cx0, cy0, wx);
        int cnt = 0;
        for (int q0 = 0; q0 < ncols; q0 += 64) {
            const int q = q0 + lane;
            int n = 0, row, pen, zf;
            if (q < ncols) n = a64_run(a, sl, cx0 + q % wx, cy0 + q / wx, dx, dz, row, pen, zf);
            cnt += wave_sum(n);
        }
        if (lane == 0) acnt[j] = cnt;
    }
    __syncthreads();
    // chunk offsets: atoms in slot order, each padded to whole chunks
    int nch = 0, fit = 0;
    for (int j = 0; j < nat; ++j) {
        nch += (acnt[j] + A64_CHUNK - 1) / A64_CHUNK;
        if ((int64_t)nch * A64_CHUNK <= CAP) fit = nch;
    }
    if (fit < nch && threadIdx.x == 0) atomicOr(a.status, 2);
    // pass 2: the entries
    for (int j = wave; j < nat; j += NW) {
        int base = 0;
        for (int i = 0; i < j; ++i) base += (acnt[i] + A64_CHUNK - 1) / A64_CHUNK;
        const int cnt = acnt[j], nj = (cnt + A64_CHUNK - 1) / A64_CHUNK;
        if (base + nj > fit) continue;
        int2 *out = list + (int64_t)base * A64_CHUNK;
        const Slot sl = slots[j];
        int cx0, cy0, wx;
        const int ncols = cols(sl, cx0, cy0, wx);
        int pos = 0;
        for (int q0 = 0; q0 < ncols; q0 += 64) {
            const int q = q0 + lane;
            int n = 0, row = 0, pen = 0, zf = 0;
            if (q < ncols) n = a64_run(a, sl, cx0 + q % wx, cy0 + q / wx, dx, dz, row, pen, zf);
            int inc = n;   // inclusive scan over the lanes
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(inc, o, 64);
                if (lane >= o) inc += t;
            }
            for (int i = 0; i < n; ++i)
                out[pos + inc - n + i] = make_int2(row + i, a64_off<E>(pen, zf + i) | (j << 16));
            pos += __shfl(inc, 63, 64);
        }
        for (int e = cnt + lane; e < nj * A64_CHUNK; e += 64)
            out[e] = make_int2(sl.start, zero_off | (j << 16) | A64_PAD);
    }
    return fit;
}

struct A64List {
    const int2 *ent;
    int g0, g1;   // this wave's chunks
};

// p_J += chi_J . v over the wave's chunks (v in the LDS box), summed per atom
// in registers and added to pacc (the current parity) once per atom and wave
template <int NCB>
__device__ __forceinline__ void a64_am_dots(const RegionArgs<double> &a, const A64List &L,
                                            const double *lds, double *pacc) {
    const int lane = threadIdx.x & 63;
    double s[NP] = {0.0, 0.0, 0.0, 0.0};
    int cj = -1;
    auto flush = [&]() {
        double t[NP];
#pragma unroll
        for (int l = 0; l < NP; ++l) t[l] = a64_wave_sum(s[l]);
        if (lane == 0) {
#pragma unroll
            for (int l = 0; l < NP; ++l) atomicAdd(&pacc[cj * NP + l], t[l]);
        }
    };
    for (int g = L.g0; g < L.g1; g += NCB) {
        int2 en[NCB];
#pragma unroll
        for (int b = 0; b < NCB; ++b)
            en[b] = g + b < L.g1 ? L.ent[(int64_t)(g + b) * A64_CHUNK + lane] : make_int2(0, 0);
        double ch[NCB][NP], v[NCB];
#pragma unroll
        for (int b = 0; b < NCB; ++b) {
            if (g + b < L.g1) {
                const double *chp = a.chi + (int64_t)en[b].x * NP;
#pragma unroll
                for (int l = 0; l < NP; ++l) ch[b][l] = chp[l];
                v[b] = lds[en[b].y & 0xffff];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < NCB; ++b) {
            if (g + b < L.g1) {
                const int j = __builtin_amdgcn_readfirstlane((en[b].y >> 16) & 0x7fff);
                if (j != cj) {
                    if (cj >= 0) flush();
                    cj = j;
#pragma unroll
                    for (int l = 0; l < NP; ++l) s[l] = 0.0;
                }
#pragma unroll
                for (int l = 0; l < NP; ++l) s[l] = fma(ch[b][l], v[b], s[l]);
            }
        }
    }
    if (cj >= 0) flush();
}

// Projections with FP64 matrix instructions (v_mfma_f64_4x4x4f64: four
// independent 4x4x4 blocks per wave; lane 16k + 4b + i holds A[b][i][k] and
// B[b][k][i], lane 16i + 4b + j holds D[b][i][j]).  Per chunk, four
// instructions take 16 rows each: in block b, A[i][k] = chi_i of row
// 16t + 4b + k and B[k][0] = v of that row (the other three columns of B are
// zero), so D[i][0] of the four blocks accumulates the atom's projections.
// A compile-time alternative to the VALU routine above (A64_MFMA_DOTS), kept
// for the measured comparison: one useful column in four, and four entry,
// chi and LDS loads per lane and chunk instead of one.
template <int NCB>
__device__ __forceinline__ void a64_am_dots_mfma(const RegionArgs<double> &a, const A64List &L,
                                                 const double *lds, double *pacc) {
    const int lane = threadIdx.x & 63;
    double acc = 0.0;
    int cj = -1;
    auto flush = [&]() {
        // D[i][0] of block b is in lane 16 i + 4 b
        auto at = [&](int l) {
            const long long bb = __double_as_longlong(acc);
            const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)(bb & 0xffffffffLL), l);
            const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(bb >> 32), l);
            return __longlong_as_double(((long long)hi << 32) | lo);
        };
        double t[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i)
            t[i] = (at(16 * i) + at(16 * i + 4)) + (at(16 * i + 8) + at(16 * i + 12));
        if (lane == 0) {
#pragma unroll
            for (int l = 0; l < NP; ++l) atomicAdd(&pacc[cj * NP + l], t[l]);
        }
    };
    for (int g = L.g0; g < L.g1; g += NCB) {
        int2 en[NCB][4];
        double av[NCB][4], bv[NCB][4];
#pragma unroll
        for (int b = 0; b < NCB; ++b)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                en[b][t] = g + b < L.g1
                               ? L.ent[(int64_t)(g + b) * A64_CHUNK + 16 * t +
                                       4 * ((lane >> 2) & 3) + (lane >> 4)]
                               : make_int2(0, 0);
#pragma unroll
        for (int b = 0; b < NCB; ++b)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                av[b][t] = a.chi[(int64_t)en[b][t].x * NP + (lane & 3)];
                const double v = lds[en[b][t].y & 0xffff];
                bv[b][t] = (lane & 3) == 0 ? v : 0.0;
            }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < NCB; ++b) {
            if (g + b < L.g1) {
                const int j = __builtin_amdgcn_readfirstlane((en[b][0].y >> 16) & 0x7fff);
                if (j != cj) {
                    if (cj >= 0) flush();
                    cj = j;
                    acc = 0.0;
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc = __builtin_amdgcn_mfma_f64_4x4x4f64(av[b][t], bv[b][t], acc, 0, 0, 0);
            }
        }
    }
    if (cj >= 0) flush();
}

template <int NCB>
__device__ __forceinline__ void a64_dots(const RegionArgs<double> &a, const A64List &L,
                                         const double *lds, double *pacc) {
    if constexpr (A64_MFMA_DOTS) a64_am_dots_mfma<NCB>(a, L, lds, pacc);
    else a64_am_dots<NCB>(a, L, lds, pacc);
}

// v(x) += sum_l chi_Jl(x) f_Jl, f_Jl = half * scale_Jl * p_Jl, over the wave's
// chunks, with LDS atomics (supports of several atoms overlap)
template <int NCB>
__device__ __forceinline__ void a64_am_update(const RegionArgs<double> &a, const A64List &L,
                                              double *lds, const double *pacc,
                                              const double *scale, double half) {
    const int lane = threadIdx.x & 63;
    double f[NP] = {0.0, 0.0, 0.0, 0.0};
    int cj = -1;
    for (int g = L.g0; g < L.g1; g += NCB) {
        int2 en[NCB];
#pragma unroll
        for (int b = 0; b < NCB; ++b)
            en[b] = g + b < L.g1 ? L.ent[(int64_t)(g + b) * A64_CHUNK + lane] : make_int2(0, 0);
        double ch[NCB][NP];
#pragma unroll
        for (int b = 0; b < NCB; ++b) {
            if (g + b < L.g1) {
                const double *chp = a.chi + (int64_t)en[b].x * NP;
#pragma unroll
                for (int l = 0; l < NP; ++l) ch[b][l] = chp[l];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int b = 0; b < NCB; ++b) {
            if (g + b < L.g1) {
                const int j = __builtin_amdgcn_readfirstlane((en[b].y >> 16) & 0x7fff);
                if (j != cj) {
                    cj = j;
#pragma unroll
                    for (int l = 0; l < NP; ++l) f[l] = scale[j * NP + l] * pacc[j * NP + l] * half;
                }
                const double u = ch[b][0] * f[0] + ch[b][1] * f[1] + ch[b][2] * f[2] + ch[b][3] * f[3];
                if (en[b].y >= 0) atomicAdd(&lds[en[b].y & 0xffff], u);
            }
        }
    }
}

// One recurrence step with the two live vectors in registers:
//   v_{k+1} = scale (2 Hs v_k - v_{k-1})  (+ inj at plane inj_z of the owning
// thread), scale = 1/2 on the first step.  The rank-4 projector term of each
// new vector is deferred into the next step: on entry cur holds v_k without
// it (pend = the halving factor it takes, 0 when there is none) and nw holds
// v_{k-1}.  cur is published to the LDS box; with atoms in the box the waves
// add the deferred term to the box with LDS atomics (chunks of the row list,
// projections of the previous step in parity buffer nl.par ^ 1) and the
// thread reads its completed pencil back.  The completed v_k goes to slot row
// in_row (element offset; svo is the lane's byte offset in a row, dvo its
// byte offset in a plane of D) from the diagonal term's reads of the own
// pencil, batch by batch: loads and stores share one memory counter, so
// stores issued before the step's loads would have to drain before those
// loads could be used.  The z neighbours come from the registers of cur
// (its last use in the step); the projections chi . v_k go to parity buffer
// nl.par; the x/y neighbours and the diagonal come from the box, D in batches
// of A64_DB planes, the first before the x/y part (whose LDS work hides it)
// and each next one before the diagonal term of the current batch.  The new
// vector is formed in place in nw and, after the last barrier, moved to cur,
// and nw re-reads v_k from the own pencil.  Three barriers per step with
// atoms in the box (the term added at the end of its own step would take two
// more barriers and a store and read-back of the own pencil).
template <int E, int R, int ZS, int BLOCK>
__device__ __forceinline__ void a64_step_d(const RegionArgs<double> &a,
                                           const StepCtx<double, E, R> &c,
                                           __amdgpu_buffer_rsrc_t Dr, uint32_t dvo,
                                           uint32_t plane, int gz0, int n2, double (&cur)[E],
                                           double (&nw)[E], double *lds, ColNL<double> &nl,
                                           bool first, __amdgpu_buffer_rsrc_t Sr, uint32_t svo,
                                           uint32_t in_row, int inj_z, double inj,
                                           const A64List &L, double pend) {
    constexpr int EE = E * E;
    constexpr int DB = A64_DB;
    constexpr int NDB = (E + DB - 1) / DB;
    if (c.active) a64_box_put<E>(lds, threadIdx.x, cur);
    __syncthreads();
    if (c.nat && pend != 0.0) {
        a64_am_update<A64_NCB>(a, L, lds, nl.pacc + (int64_t)(nl.par ^ 1) * nl.maxat * NP,
                               nl.scale, pend);
        __syncthreads();
        if (c.active) a64_box_get<E, 0, E>(cur, lds, threadIdx.x);
    }
    if (c.active) {
        // z neighbours from the registers of cur (its last use in the step):
        // nw <- sum_p cz_p (cur[z + p] + cur[z - p]) - nw
#pragma unroll
        for (int z = 0; z < E; ++z) {
            double r = -nw[z];
#pragma unroll
            for (int p = 1; p <= R; ++p) {
                if (z + p < E && z - p >= 0)
                    r = fma(c.cz[p], cur[z + p] + cur[z - p], r);
                else if (z + p < E)
                    r = fma(c.cz[p], cur[z + p], r);
                else if (z - p >= 0)
                    r = fma(c.cz[p], cur[z - p], r);
            }
            nw[z] = r;
        }
    }
    if (c.nat) a64_dots<A64_NCB>(a, L, lds, nl.pacc + (int64_t)nl.par * nl.maxat * NP);
    if (c.active) {
        int salt = 0;
        asm volatile("" : "+s"(salt));
        const int zmax = c.dz - 1 + salt;
        double d[NDB][DB];
        auto load_d = [&](int b) {
#pragma unroll
            for (int i = 0; i < DB; ++i) {
                const int z = b * DB + i;
                if (z < E) {
                    int gz = gz0 + min(z, zmax);
                    gz = gz >= n2 ? gz - n2 : gz;
                    d[b][i] = a64_ld(Dr, dvo, plane * (uint32_t)gz * 8u);
                }
            }
        };
        load_d(0);
        __builtin_amdgcn_sched_barrier(0);
        a64_xy<E, R, ZS>(nw, c, lds);
        __builtin_amdgcn_sched_barrier(0);
        int s3 = 0;
        asm volatile("" : "+v"(s3));
        const int own = (int)threadIdx.x + s3;
#pragma unroll
        for (int b = 0; b < NDB; ++b) {
            if (b + 1 < NDB) load_d(b + 1);
#pragma unroll
            for (int i = 0; i < DB; ++i) {
                const int z = b * DB + i;
                if (z < E) {
                    // the completed v_k to its slot row, from the own-pencil value the
                    // diagonal term reads anyway: issued here, after the batch's loads,
                    // the stores stay in flight while the next batch is waited for
                    const double vz = lds[a64_off<E>(own, z)];
                    nw[z] = fma(d[b][i], vz, nw[z]);
                    a64_st(Sr, svo, (in_row + (uint32_t)(z * EE)) * 8u, vz);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int z = 0; z < E; ++z) cur[z] = nw[z];
    if (c.active) a64_box_get<E, 0, E>(nw, lds, threadIdx.x);
    if (first) {
#pragma unroll
        for (int z = 0; z < E; ++z) cur[z] *= 0.5;
    }
    {
        int salt = 0;
        asm volatile("" : "+s"(salt));
        const int dz = c.dz + salt;
        if (dz < E) {
#pragma unroll
            for (int z = 0; z < E; ++z) cur[z] = (z < dz) ? cur[z] : 0.0;
        }
    }
    if (c.nat) col_zero_next<double, BLOCK, false>(nl, c.nat);
    nl.par ^= 1;
    if (inj_z >= 0) {
        int iz = inj_z;
        asm volatile("" : "+v"(iz));
#pragma unroll
        for (int z = 0; z < E; ++z) cur[z] += (z == iz) ? inj : 0.0;
    }
}

// the last vector of a sweep: its deferred rank-4 term, its slot row and its
// projections chi . v (to parity buffer nl.par, then flipped), without a step
template <int E, int R, int ZS, int BLOCK>
__device__ __forceinline__ void a64_finish_d(const RegionArgs<double> &a,
                                             const StepCtx<double, E, R> &c, double (&cur)[E],
                                             ColNL<double> &nl, const A64List &L, double *lds,
                                             __amdgpu_buffer_rsrc_t Sr, uint32_t svo,
                                             uint32_t in_row, double pend) {
    constexpr int EE = E * E;
    if (c.active) a64_box_put<E>(lds, threadIdx.x, cur);
    __syncthreads();
    if (c.nat && pend != 0.0) {
        a64_am_update<A64_NCB>(a, L, lds, nl.pacc + (int64_t)(nl.par ^ 1) * nl.maxat * NP,
                               nl.scale, pend);
        __syncthreads();
        if (c.active) a64_box_get<E, 0, E>(cur, lds, threadIdx.x);
    }
    if (c.active) {
#pragma unroll
        for (int z = 0; z < E; ++z) a64_st(Sr, svo, (in_row + (uint32_t)(z * EE)) * 8u, cur[z]);
    }
    if (c.nat) a64_dots<A64_NCB>(a, L, lds, nl.pacc + (int64_t)nl.par * nl.maxat * NP);
    __syncthreads();
    col_zero_next<double, BLOCK, false>(nl, c.nat);
    nl.par ^= 1;
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
    // slot rows at element offsets: v_k at k E^3, vt_{k+1} at (K + k) E^3
    const __amdgpu_buffer_rsrc_t Sr = a64_rsrc(slot, 2 * (int64_t)K * E3 * 8);
    const __amdgpu_buffer_rsrc_t Dr =
        a64_rsrc(a.D, (int64_t)a.N[0] * a.N[1] * a.N[2] * 8);
    const uint32_t VO = 0, TO = (uint32_t)(K * E3);
    const uint32_t svo = (uint32_t)tid * 8u;
    T *Prow = slot + 2 * (int64_t)K * E3;    // p_k = chi . v_k        [k][atom][NP]
    T *Qrow = Prow + a64_proj_elems(K);      // q_k = chi . vt_{k+1}   [k][atom][NP]
    Slot *slots = reinterpret_cast<Slot *>(Qrow + a64_proj_elems(K));
    ColEntry *colbuf = reinterpret_cast<ColEntry *>(slots + AT);
    int2 *alist = reinterpret_cast<int2 *>(colbuf + BLOCK * MAXC);
    int *acnt = reinterpret_cast<int *>(alist + a64_list_cap<E>());
    static_assert(region_lds_elems<T, E>() == a64_xb<E>() + E * E + 1, "the box layout");
    static_assert(region_lds_elems<T, E>() < 65536, "box offsets fit 16 bits");

    for (;;) {
        if (tid == 0) {
            s_item = atomicAdd(a.counter, 1);
            s_nat = 0;
        }
        __syncthreads();
        // block-uniform: the item and everything derived from it stay in
        // scalar registers
        const int itn = __builtin_amdgcn_readfirstlane(s_item);
        if (itn >= a.n_items) break;
        const Item it = a.items[itn];
        c.dx = it.dim[0];
        c.dy = it.dim[1];
        c.dz = it.dim[2];
        const int npen = c.dx * c.dy;
        c.active = tid < npen;
        const int px = c.active ? tid % c.dx : 0, py = c.active ? tid / c.dx : 0;
        for (int i = tid; i < region_lds_elems<T, E>(); i += BLOCK) lds[i] = 0.0;
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
        c.mine = nullptr;   // the box is addressed through a64_off (split planes)
        c.px = px;
        c.py = py;
        c.npen = npen;
        __syncthreads();
        c.nat = min(__builtin_amdgcn_readfirstlane(s_nat), AT);
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
        const int ncw = a64_wave_max(ncol);   // passes of the final pass's column loop
        nl.pacc = &pacc[0][0][0];
        nl.scale = &pfac[0][0];
        nl.maxat = AT;
        A64List L{alist, 0, 0};
        if (c.nat) {
            const int nch = a64_build_list<E, ZS, BLOCK>(a, slots, c.nat, c.dx, c.dy, c.dz,
                                                        a64_off<E>(npen, 0), alist, acnt);
            const int w = tid >> 6;
            L.g0 = w * nch / (BLOCK / 64);
            L.g1 = (w + 1) * nch / (BLOCK / 64);
        }
        __syncthreads();

        // ---- forward sweep: v_0 .. v_{K-1} and p_k = chi . v_k to the slot ----
        // X = cur, Y = prev; each step leaves the next pair in place
        const uint32_t dvo = (uint32_t)col * 8u, pl = (uint32_t)plane;
        T X[E], Y[E];
#pragma unroll
        for (int z = 0; z < E; ++z) {
            X[z] = (is_ctr && z == cz0) ? 1.0 : 0.0;
            Y[z] = 0.0;
        }
        // step k stores v_k; the rank-4 term of v_{k+1} (halved after the
        // first step) is added at the start of step k + 1
        for (int k = 0; k + 1 <= K - 1; ++k) {
            const double pend = k == 0 ? 0.0 : (k == 1 ? 0.5 : 1.0);
            a64_step_d<E, R, ZS, BLOCK>(a, c, Dr, dvo, pl, gz0, n2, X, Y, lds, nl, k == 0,
                                        Sr, svo, VO + (uint32_t)(k * E3), -1, 0.0, L, pend);
            a64_store_proj<BLOCK>(nl, c.nat, Prow + (int64_t)k * AT * NP);
        }
        a64_finish_d<E, R, ZS, BLOCK>(a, c, X, nl, L, lds, Sr, svo,
                                      VO + (uint32_t)((K - 1) * E3),
                                      K == 1 ? 0.0 : (K == 2 ? 0.5 : 1.0));
        a64_store_proj<BLOCK>(nl, c.nat, Prow + (int64_t)(K - 1) * AT * NP);

        // ---- reverse sweep: vt_{k+1} and q_k = chi . vt_{k+1} to the slot ----
        // vt_k = a_k e_q + 2 Hs vt_{k+1} - vt_{k+2}  (vt_{K+1} = 0)
        const T aK = 2.0 * (gr * aa.coef_c[K] + gu * aa.coef_d[K]);
#pragma unroll
        for (int z = 0; z < E; ++z) {
            X[z] = (is_ctr && z == cz0) ? aK : 0.0;   // vt_K
            Y[z] = 0.0;
        }
        const int iz = is_ctr ? cz0 : -1;
        // step k stores vt_{k+1}
        for (int k = K - 1; k >= 1; --k) {
            const T ak = 2.0 * (gr * aa.coef_c[k] + gu * aa.coef_d[k]);
            a64_step_d<E, R, ZS, BLOCK>(a, c, Dr, dvo, pl, gz0, n2, X, Y, lds, nl, false,
                                        Sr, svo, TO + (uint32_t)(k * E3), iz, ak, L,
                                        k == K - 1 ? 0.0 : 1.0);
            a64_store_proj<BLOCK>(nl, c.nat, Qrow + (int64_t)k * AT * NP);
        }
        a64_finish_d<E, R, ZS, BLOCK>(a, c, X, nl, L, lds, Sr, svo, TO, K >= 2 ? 1.0 : 0.0);
        a64_store_proj<BLOCK>(nl, c.nat, Qrow);
        __syncthreads();   // the slot's projection rows are read by other threads below

        // ---- final pass: dV and dR from the stored rows ----
        // Every lane streams its own pencil's rows plane by plane (one plane of
        // all lanes is one contiguous slot row, so the loads coalesce) in
        // batches of A64_FZB planes over all k, and accumulates
        //   G(z)   = sum_k alpha_k vt_{k+1}(z) v_k(z)                    (dV)
        //   W_l(z) = sum_k alpha_k (p_k,l vt_{k+1}(z) + q_k,l v_k(z))   (dR)
        // for the planes of the batch and (W) up to two of its column entries
        // at a time; a batch's W rows that lie in an entry's support piece are
        // contracted with dchi at once.  p_k and q_k of the box's atoms are read
        // from the idle LDS box when they fit it, else from the slot.
        const bool want_dV = aa.dV != nullptr, want_dR = aa.dR != nullptr;
        if (want_dV || want_dR) {
            const int pq = K * c.nat * NP;
            const bool staged = want_dR && 2 * (int64_t)pq <= (int64_t)region_lds_elems<T, E>();
            if (staged) {
                for (int i = tid; i < pq; i += BLOCK) {
                    const int k = i / (c.nat * NP), rest = i - k * (c.nat * NP);
                    lds[i] = Prow[(int64_t)k * AT * NP + rest];
                    lds[pq + i] = Qrow[(int64_t)k * AT * NP + rest];
                }
            }
            __syncthreads();
            const double itau = 1.0 / tau, hs = a.h3 / tau;
            auto final_pass = [&](auto staged_tag) {
                constexpr bool ST = decltype(staged_tag)::value;
                constexpr int ZB = A64_FZB, WC = 2;
                const int pstride = ST ? c.nat : AT;
                const int npass = want_dR ? max(1, (ncw + WC - 1) / WC) : 1;
                for (int pass = 0; pass < npass; ++pass) {
                    const bool do_g = want_dV && pass == 0;
                    ColEntry en[WC];
                    bool has[WC];
#pragma unroll
                    for (int w = 0; w < WC; ++w) {
                        const int ci = pass * WC + w;
                        has[w] = want_dR && ci < nl.ncol;
                        en[w] = has[w] ? mycols[ci] : ColEntry{0, 0, 0, 0};
                    }
                    double sx[WC][3];
#pragma unroll
                    for (int w = 0; w < WC; ++w) sx[w][0] = sx[w][1] = sx[w][2] = 0.0;
                    for (int z0 = 0; z0 < E; z0 += ZB) {
                        bool ov[WC], wov[WC];
                        bool any_w = false;
#pragma unroll
                        for (int w = 0; w < WC; ++w) {
                            ov[w] = has[w] && en[w].zlo < z0 + ZB && en[w].zlo + en[w].n > z0;
                            wov[w] = __any(ov[w]) != 0;   // wave-uniform
                            any_w = any_w || wov[w];
                        }
                        if (!do_g && !any_w) continue;
                        double G[ZB], W[WC][ZB][NP];
#pragma unroll
                        for (int i = 0; i < ZB; ++i) G[i] = 0.0;
#pragma unroll
                        for (int w = 0; w < WC; ++w)
#pragma unroll
                            for (int i = 0; i < ZB; ++i)
#pragma unroll
                                for (int l = 0; l < NP; ++l) W[w][i][l] = 0.0;
                        for (int k = 0; k < K; k += 2) {
                            // two steps per iteration (the second weighted 0 past K - 1)
                            const bool two = k + 1 < K;
                            const int k1 = two ? k + 1 : k;
                            const T al[2] = {k == 0 ? 1.0 : 2.0, two ? 2.0 : 0.0};
                            double tv[2][ZB], vv[2][ZB];
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                const int kk = h ? k1 : k;
#pragma unroll
                                for (int i = 0; i < ZB; ++i) {
                                    const uint32_t o = (uint32_t)(kk * E3 + min(z0 + i, E - 1) * EE);
                                    tv[h][i] = a64_ld<A64_REREAD>(Sr, svo, (TO + o) * 8u);
                                    vv[h][i] = a64_ld<A64_REREAD>(Sr, svo, (VO + o) * 8u);
                                }
                            }
                            if (do_g) {
#pragma unroll
                                for (int i = 0; i < ZB; ++i) {
                                    G[i] = fma(al[0] * tv[0][i], vv[0][i], G[i]);
                                    G[i] = fma(al[1] * tv[1][i], vv[1][i], G[i]);
                                }
                            }
#pragma unroll
                            for (int w = 0; w < WC; ++w) {
                                if (!wov[w]) continue;
                                double pk[2][NP], qk[2][NP];
#pragma unroll
                                for (int h = 0; h < 2; ++h) {
                                    const int64_t o =
                                        ((int64_t)(h ? k1 : k) * pstride + en[w].slot) * NP;
#pragma unroll
                                    for (int l = 0; l < NP; ++l) {
                                        if constexpr (ST) {
                                            pk[h][l] = lds[o + l];
                                            qk[h][l] = lds[pq + o + l];
                                        } else {
                                            pk[h][l] = Prow[o + l];
                                            qk[h][l] = Qrow[o + l];
                                        }
                                    }
                                }
#pragma unroll
                                for (int h = 0; h < 2; ++h)
#pragma unroll
                                    for (int i = 0; i < ZB; ++i)
#pragma unroll
                                        for (int l = 0; l < NP; ++l)
                                            W[w][i][l] += al[h] * (pk[h][l] * tv[h][i] +
                                                                   qk[h][l] * vv[h][i]);
                            }
                        }
                        if (do_g && c.active) {
#pragma unroll
                            for (int i = 0; i < ZB; ++i) {
                                const int z = z0 + i;
                                if (z < E && z < c.dz) {
                                    int gz = gz0 + z;
                                    gz = gz >= n2 ? gz - n2 : gz;
                                    unsafeAtomicAdd(aa.dV + col + plane * gz, G[i] * itau);
                                }
                            }
                        }
                        // rows of this batch inside an entry's support piece
#pragma unroll
                        for (int w = 0; w < WC; ++w) {
                            if (!ov[w]) continue;
                            const double *cj = a.cJ + (int64_t)slots[en[w].slot].atom * NP;
#pragma unroll
                            for (int i = 0; i < ZB; ++i) {
                                const int z = z0 + i;
                                if (z >= en[w].zlo && z < en[w].zlo + en[w].n) {
                                    const double *dc =
                                        a.dchi + (int64_t)(en[w].row0 + z - en[w].zlo) * 3 * NP;
#pragma unroll
                                    for (int l = 0; l < NP; ++l)
#pragma unroll
                                        for (int x = 0; x < 3; ++x)
                                            sx[w][x] += cj[l] * dc[l * 3 + x] * W[w][i][l];
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int w = 0; w < WC; ++w)
                        if (has[w])
#pragma unroll
                            for (int x = 0; x < 3; ++x) atomicAdd(&cdR[en[w].slot][x], sx[w][x] * hs);
                }
            };
            if (staged) final_pass(std::true_type{});
            else final_pass(std::false_type{});
            if (want_dR) {
                __syncthreads();
                for (int j = tid; j < c.nat; j += BLOCK)
                    for (int x = 0; x < 3; ++x)
                        unsafeAtomicAdd(aa.dR + (int64_t)slots[j].atom * 3 + x, cdR[j][x]);
            }
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
