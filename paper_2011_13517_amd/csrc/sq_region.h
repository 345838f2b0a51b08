// Device helpers shared by the forward and adjoint region kernels: LDS pencil
// I/O, the atom list of a box, the projector block and one in-place step of
// the Chebyshev recurrence  prev <- 2 Hs cur - prev  on a region box.
#pragma once

#include "sq_internal.h"

namespace sqk {

struct Slot {              // an atom touching the current box
    int32_t start, count;  // rows in the support tables
    int32_t ox, oy, oz;    // atom box origin relative to the region box
    int32_t atom;
    int32_t bx, by;        // atom box extent in x and y
    int32_t col;           // first entry of the atom's column index
};

// Column path of the projector block: every thread handles the pieces of
// atom supports that cross its own z-pencil.  An entry names the atom slot,
// the first support row of the piece and its z range in the box.
struct ColEntry {
    int32_t slot, row0, zlo, n;
};

// atoms per region that fit the LDS left over by the box and FIXED bytes of
// other tables (EXTRA bytes of per-atom state beyond the slot and its four
// scaled projections)
template <typename T, int E, int EXTRA = 0, int FIXED = 0>
constexpr int max_atoms_in_region() {
    constexpr int used = region_lds_elems<T, E>() * (int)sizeof(T) + 512 + FIXED;
    constexpr int per = (int)sizeof(Slot) + NP * (int)sizeof(T) + EXTRA;
    constexpr int n = (LDS_BYTES - used) / per;
    return n > MAX_REGION_ATOMS ? MAX_REGION_ATOMS : (n < 0 ? 0 : n);
}

// A block-uniform pointer pinned in scalar registers.  Per-z loads of a
// pencil then address as (SGPR base) + (32-bit thread offset); without the pin
// the compiler folds the thread offset into E hoisted 64-bit VGPR addresses
// and spills them in the large-region kernels.
// The result is a global (address space 1) pointer so that the accesses
// stay global loads and stores rather than flat ones.
template <typename T>
using global_ptr = __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ global_ptr<T> sgpr_ptr(T *p) {
    const uint64_t u = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return reinterpret_cast<global_ptr<T>>(((uint64_t)hi << 32) | lo);
}

template <typename T, int E, int ZS>
__device__ __forceinline__ void store_pencil(T *dst, const T (&v)[E]) {
    if constexpr (sizeof(T) == 4 && ZS % 4 == 0) {
#pragma unroll
        for (int i = 0; i < (E + 3) / 4; ++i) {
            float4 q;
            q.x = v[4 * i];
            q.y = (4 * i + 1 < E) ? v[4 * i + 1] : 0.f;
            q.z = (4 * i + 2 < E) ? v[4 * i + 2] : 0.f;
            q.w = (4 * i + 3 < E) ? v[4 * i + 3] : 0.f;
            reinterpret_cast<float4 *>(dst)[i] = q;
        }
    } else if constexpr (sizeof(T) == 8 && ZS % 2 == 0) {
#pragma unroll
        for (int i = 0; i < (E + 1) / 2; ++i) {
            double2 q;
            q.x = v[2 * i];
            q.y = (2 * i + 1 < E) ? v[2 * i + 1] : 0.0;
            reinterpret_cast<double2 *>(dst)[i] = q;
        }
    } else {
#pragma unroll
        for (int z = 0; z < E; ++z) dst[z] = v[z];
    }
}

template <typename T, int E, int ZS>
__device__ __forceinline__ void load_pencil(const T *src, T (&v)[E]) {
    if constexpr (sizeof(T) == 4 && ZS % 4 == 0) {
#pragma unroll
        for (int i = 0; i < (E + 3) / 4; ++i) {
            const float4 q = reinterpret_cast<const float4 *>(src)[i];
            v[4 * i] = q.x;
            if (4 * i + 1 < E) v[4 * i + 1] = q.y;
            if (4 * i + 2 < E) v[4 * i + 2] = q.z;
            if (4 * i + 3 < E) v[4 * i + 3] = q.w;
        }
    } else if constexpr (sizeof(T) == 8 && ZS % 2 == 0) {
#pragma unroll
        for (int i = 0; i < (E + 1) / 2; ++i) {
            const double2 q = reinterpret_cast<const double2 *>(src)[i];
            v[2 * i] = q.x;
            if (2 * i + 1 < E) v[2 * i + 1] = q.y;
        }
    } else {
#pragma unroll
        for (int z = 0; z < E; ++z) v[z] = src[z];
    }
}

// acc[z] += c * pencil[z] for a neighbouring pencil in LDS
template <typename T, int E, int ZS>
__device__ __forceinline__ void axpy_pencil(T (&acc)[E], T c, const T *src) {
    if constexpr (sizeof(T) == 4 && ZS % 4 == 0) {
#pragma unroll
        for (int i = 0; i < (E + 3) / 4; ++i) {
            const float4 q = reinterpret_cast<const float4 *>(src)[i];
            acc[4 * i] = fmaf(c, q.x, acc[4 * i]);
            if (4 * i + 1 < E) acc[4 * i + 1] = fmaf(c, q.y, acc[4 * i + 1]);
            if (4 * i + 2 < E) acc[4 * i + 2] = fmaf(c, q.z, acc[4 * i + 2]);
            if (4 * i + 3 < E) acc[4 * i + 3] = fmaf(c, q.w, acc[4 * i + 3]);
        }
    } else if constexpr (sizeof(T) == 8 && ZS % 2 == 0) {
#pragma unroll
        for (int i = 0; i < (E + 1) / 2; ++i) {
            const double2 q = reinterpret_cast<const double2 *>(src)[i];
            acc[2 * i] = fma(c, q.x, acc[2 * i]);
            if (2 * i + 1 < E) acc[2 * i + 1] = fma(c, q.y, acc[2 * i + 1]);
        }
    } else {
#pragma unroll
        for (int z = 0; z < E; ++z) acc[z] = fma(c, src[z], acc[z]);
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ int wrap(int x, int n) {
    x %= n;
    return x < 0 ? x + n : x;
}

// Build the list of atoms whose support box meets the region box (LDS).
template <typename T, int MAXAT, int BLOCK>
__device__ void gather_atoms(const RegionArgs<T> &a, const Item &it, Slot *slots, int *s_nat) {
    for (int j = threadIdx.x; j < a.n_atoms; j += BLOCK) {
        const AtomDev at = a.atoms[j];
        int off[3];
        bool hit = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int o = at.lo[d] - it.lo[d];
            if (a.periodic) {
                o = wrap(o, a.N[d]);
                if (o >= it.dim[d]) o -= a.N[d];
            }
            off[d] = o;
            hit = hit && (o < it.dim[d]) && (o + at.dim[d] > 0);
        }
        if (hit) {
            const int slot = atomicAdd(s_nat, 1);
            if (slot < MAXAT) {
                slots[slot].start = at.start;
                slots[slot].count = at.count;
                slots[slot].ox = off[0];
                slots[slot].oy = off[1];
                slots[slot].oz = off[2];
                slots[slot].atom = j;
                slots[slot].bx = at.dim[0];
                slots[slot].by = at.dim[1];
                slots[slot].col = at.col_start;
            }
        }
    }
}

// Per-region context shared by the steps of one box.
template <typename T, int E, int R>
struct StepCtx {
    T cx[R + 1], cy[R + 1], cz[R + 1];
    int nb[4 * R];
    int dx, dy, dz;
    int nat;
    bool active;
    T *mine;
    int px, py, npen;      // pencil of this thread, pencils in the box
    const T *ncoef;        // LDS [4R]: x+, x-, y+, y- weights per distance (low-register path)
};

// Raw projections of the LDS vector onto the projectors of every atom of the
// box (one wave per atom): p_Jlm = chi_Jlm . v and, when GRAD, the
// position derivatives dp_Jlm,x = (d chi_Jlm / d R_J,x) . v.  The forward
// scaling 2 h^3 c_Jl / tau goes to pfac; the raw values to dots / ddots.
template <typename T, int ZS, int NW, bool GRAD>
__device__ __forceinline__ void projector_dots(const RegionArgs<T> &a, const Slot *slots,
                                               T (*pfac)[NP], T (*dots)[NP],
                                               T (*ddots)[3 * NP], const T *lds, int nat,
                                               int dx, int dy, int dz, double tau) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = wave; j < nat; j += NW) {
        const Slot sl = slots[j];
        T s[NP] = {0, 0, 0, 0};
        T g[GRAD ? 3 * NP : 1];
        if constexpr (GRAD) {
#pragma unroll
            for (int i = 0; i < 3 * NP; ++i) g[i] = 0;
        }
        for (int e = lane; e < sl.count; e += 64) {
            const int pk = a.sup_pack[sl.start + e];
            const int lx = sl.ox + (pk & 1023), ly = sl.oy + ((pk >> 10) & 1023),
                      lz = sl.oz + ((pk >> 20) & 1023);
            if (lx >= 0 && lx < dx && ly >= 0 && ly < dy && lz >= 0 && lz < dz) {
                const T val = lds[(ly * dx + lx) * ZS + lz];
                const T *ch = a.chi + (int64_t)(sl.start + e) * NP;
#pragma unroll
                for (int l = 0; l < NP; ++l) s[l] += ch[l] * val;
                if constexpr (GRAD) {
                    const T *dc = a.dchi + (int64_t)(sl.start + e) * 3 * NP;
#pragma unroll
                    for (int i = 0; i < 3 * NP; ++i) g[i] += dc[i] * val;
                }
            }
        }
#pragma unroll
        for (int l = 0; l < NP; ++l) s[l] = wave_sum(s[l]);
        if constexpr (GRAD) {
#pragma unroll
            for (int i = 0; i < 3 * NP; ++i) g[i] = wave_sum(g[i]);
        }
        if (lane == 0) {
            const double f = 2.0 * a.h3 / tau;
            const double *c = a.cJ + (int64_t)sl.atom * NP;
#pragma unroll
            for (int l = 0; l < NP; ++l) {
                pfac[j][l] = (T)(f * c[l]) * s[l];
                if (dots) dots[j][l] = s[l];
            }
            if constexpr (GRAD) {
#pragma unroll
                for (int i = 0; i < 3 * NP; ++i) ddots[j][i] = g[i];
            }
        }
    }
}

// rank-4 update of the LDS copy: v(x) += sum_lm chi_Jlm(x) pfac_Jlm
template <typename T, int ZS, int NW>
__device__ __forceinline__ void projector_update(const RegionArgs<T> &a, const Slot *slots,
                                                 const T (*pfac)[NP], T *lds, int nat, int dx,
                                                 int dy, int dz) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = wave; j < nat; j += NW) {
        const Slot sl = slots[j];
        const T f0 = pfac[j][0], f1 = pfac[j][1], f2 = pfac[j][2], f3 = pfac[j][3];
        for (int e = lane; e < sl.count; e += 64) {
            const int pk = a.sup_pack[sl.start + e];
            const int lx = sl.ox + (pk & 1023), ly = sl.oy + ((pk >> 10) & 1023),
                      lz = sl.oz + ((pk >> 20) & 1023);
            if (lx >= 0 && lx < dx && ly >= 0 && ly < dy && lz >= 0 && lz < dz) {
                const T *ch = a.chi + (int64_t)(sl.start + e) * NP;
                const T u = ch[0] * f0 + ch[1] * f1 + ch[2] * f2 + ch[3] * f3;
                atomicAdd(&lds[(ly * dx + lx) * ZS + lz], u);
            }
        }
    }
}

// prev <- D cur - prev.  Without DREG the diagonal is re-read from L2 every
// step: z is clamped into the box so the loads need no branch (entries past dz
// are zeroed by the z mask, and boxes without one have dz = E), and an opaque
// zero keeps the E uniform plane addresses from being hoisted out of the step
// loop into spilled registers.
template <typename T, int E, int R, bool DREG>
__device__ __forceinline__ void diag_part(const RegionArgs<T> &a, const StepCtx<T, E, R> &c,
                                          const T (&d)[DREG ? E : 1], int64_t col,
                                          int64_t plane, int gz0, int n2, const T (&cur)[E],
                                          T (&prev)[E]) {
    if constexpr (DREG) {
#pragma unroll
        for (int z = 0; z < E; ++z) prev[z] = d[z] * cur[z] - prev[z];
    } else {
        int salt = 0;
        asm volatile("" : "+s"(salt));
        const uint32_t cl = (uint32_t)col;
        const int zmax = c.dz - 1 + salt;
        // all loads of a batch first, then its FMAs: one memory wait per batch
        // (left alone, the allocator issues load, wait, FMA per z); FP64 pencils
        // go in batches of 9 so the loads do not need 2E registers at once
        constexpr int CH = sizeof(T) == 8 ? 9 : E;
#pragma unroll
        for (int z0 = 0; z0 < E; z0 += CH) {
            T dv[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                if (z0 + i < E) {
                    int gz = gz0 + min(z0 + i, zmax);
                    gz = gz >= n2 ? gz - n2 : gz;
                    dv[i] = sgpr_ptr(a.D + plane * gz)[cl];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int i = 0; i < CH; ++i)
                if (z0 + i < E) prev[z0 + i] = dv[i] * cur[z0 + i] - prev[z0 + i];
        }
    }
}

// One recurrence step in place: prev <- scale * (2 Hs cur) - prev.
// (scale = 1/2 with prev = 0 gives v_1 = Hs v_0.)
template <typename T, int E, int R, int ZS, int NW, bool MASKZ, bool DREG, bool GRAD = false>
__device__ __forceinline__ void region_step(const RegionArgs<T> &a, const StepCtx<T, E, R> &c,
                                            const T (&d)[DREG ? E : 1], int64_t col,
                                            int64_t plane, int gz0, int n2, T (&cur)[E],
                                            T (&prev)[E], T *lds, const Slot *slots,
                                            T (*pfac)[NP], bool first, double tau,
                                            T (*dots)[NP] = nullptr,
                                            T (*ddots)[3 * NP] = nullptr) {
    if (c.active) store_pencil<T, E, ZS>(c.mine, cur);
    __syncthreads();
    if (c.nat)
        projector_dots<T, ZS, NW, GRAD>(a, slots, pfac, dots, ddots, lds, c.nat, c.dx, c.dy,
                                        c.dz, tau);

    // local part: D cur - prev, z neighbours from registers, x/y from LDS
    diag_part<T, E, R, DREG>(a, c, d, col, plane, gz0, n2, cur, prev);
#pragma unroll
    for (int p = 1; p <= R; ++p) {
#pragma unroll
        for (int z = 0; z < E; ++z) {
            T s = (T)0;
            if (z + p < E) s += cur[z + p];
            if (z - p >= 0) s += cur[z - p];
            prev[z] += c.cz[p] * s;
        }
    }
#pragma unroll
    for (int p = 1; p <= R; ++p) {
        axpy_pencil<T, E, ZS>(prev, c.cx[p], lds + c.nb[4 * (p - 1) + 0] * ZS);
        axpy_pencil<T, E, ZS>(prev, c.cx[p], lds + c.nb[4 * (p - 1) + 1] * ZS);
        axpy_pencil<T, E, ZS>(prev, c.cy[p], lds + c.nb[4 * (p - 1) + 2] * ZS);
        axpy_pencil<T, E, ZS>(prev, c.cy[p], lds + c.nb[4 * (p - 1) + 3] * ZS);
    }
    __syncthreads();

    if (c.nat) {
        if (c.active) store_pencil<T, E, ZS>(c.mine, prev);
        __syncthreads();
        projector_update<T, ZS, NW>(a, slots, pfac, lds, c.nat, c.dx, c.dy, c.dz);
        __syncthreads();
        if (c.active) load_pencil<T, E, ZS>(c.mine, prev);
    }
    if (first) {
#pragma unroll
        for (int z = 0; z < E; ++z) prev[z] *= (T)0.5;
    }
    if constexpr (MASKZ) {
#pragma unroll
        for (int z = 0; z < E; ++z) prev[z] = (z < c.dz) ? prev[z] : (T)0;
    }
}

// --------------------------------------------------------------------------
// Column path of the projector block.
// --------------------------------------------------------------------------
template <typename T>
struct ColNL {
    const ColEntry *cols;  // this thread's entries (LDS)
    int ncol;
    T *pacc;               // [2][maxat][NP] raw projections chi . v, by step parity
    T *gacc;               // [2][maxat][3 NP] raw d chi / d R . v (gradient), or null
    const T *scale;        // [maxat][NP] 2 h^3 c_Jl / tau
    int maxat;
    int par;               // parity buffer of the current step (zero on entry)
};

// entries of the atom supports crossing pencil (px, py) of the box
template <typename T>
__device__ __forceinline__ int build_columns(const RegionArgs<T> &a, const Slot *slots, int nat,
                                             bool active, int px, int py, int dz, ColEntry *mine) {
    int n = 0;
    if (!active) return 0;
    for (int j = 0; j < nat; ++j) {
        const Slot sl = slots[j];
        const int cx = px - sl.ox, cy = py - sl.oy;
        if (cx < 0 || cy < 0 || cx >= sl.bx || cy >= sl.by) continue;
        const int64_t ci = 2 * ((int64_t)sl.col + (int64_t)cy * sl.bx + cx);
        const int row = a.colidx[ci], zc = a.colidx[ci + 1];
        const int cnt = zc >> 16;
        if (cnt == 0) continue;
        const int z0 = sl.oz + (zc & 0xffff);
        const int zlo = max(z0, 0), zhi = min(z0 + cnt, dz);
        if (zlo >= zhi) continue;
        if (n < MAXC) mine[n] = ColEntry{j, row + (zlo - z0), zlo, zhi - zlo};
        ++n;
    }
    return n;
}

// raw projections of this thread's pencil (in LDS) onto the crossing supports,
// reduced over the box with LDS atomics into the current parity buffer
// Lanes l and l ^ m (m = 1, 2) that add into the same atom slot merge their
// values first (DPP quad permutes, no LDS): the lane with bit m clear keeps
// the sum, the other drops out.  Neighbouring pencils usually cross the same
// atoms in the same order, so this cuts the same-address conflicts of the LDS
// atomics that follow by up to four.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL>((int)(b & 0xffffffffLL));
    const int hi = dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T, int NV, int CTRL, int M>
__device__ __forceinline__ void merge_level(T (&v)[NV], int &slot) {
    const int lane = (int)(threadIdx.x & 63);
    const int so = dpp_i<CTRL>(slot);
    T vo[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) vo[i] = dpp_f<CTRL>(v[i]);
    if (so == slot && slot >= 0) {
        if (lane & M) {
            slot = -1;
#pragma unroll
            for (int i = 0; i < NV; ++i) v[i] = (T)0;
        } else {
#pragma unroll
            for (int i = 0; i < NV; ++i) v[i] += vo[i];
        }
    }
}
template <typename T, int NV>
__device__ __forceinline__ void merge_equal_slots(T (&v)[NV], int &slot) {
    merge_level<T, NV, 0xB1, 1>(v, slot);   // quad_perm(1,0,3,2): partner lane ^ 1
    merge_level<T, NV, 0x4E, 2>(v, slot);   // quad_perm(2,3,0,1): partner lane ^ 2
}

// The support rows of a column piece are read in batches of NB (loads of the
// batch first, then its FMAs), so one L2 round trip serves NB rows.
#ifndef SQ_NB64
#define SQ_NB64 2
#endif
constexpr int NB64 = SQ_NB64;   // FP64 batch
template <typename T, bool GRAD, int NBX = 0>
__device__ __forceinline__ void col_dots(const RegionArgs<T> &a, const ColNL<T> &nl,
                                         const T *pencil) {
    // FP64 batches stay small: the two FP64 pencils already hold 4E VGPRs
    // (NBX > 0: a caller with registers to spare sets the batch)
    constexpr int NB = NBX > 0 ? NBX : sizeof(T) == 8 ? (GRAD ? 1 : NB64) : (GRAD ? 2 : 4);
    // every lane runs the wave's largest column count (the DPP merge needs its
    // partner lanes active); lanes past their own count contribute nothing
    int ncw = nl.ncol;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) ncw = max(ncw, __shfl_xor(ncw, m));
    for (int c = 0; c < ncw; ++c) {
        const bool has = c < nl.ncol;
        const ColEntry e = has ? nl.cols[c] : ColEntry{-1, 0, 0, 0};
        T s[NP] = {0, 0, 0, 0};
        T g[GRAD ? 3 * NP : 1];
        if constexpr (GRAD) {
#pragma unroll
            for (int i = 0; i < 3 * NP; ++i) g[i] = 0;
        }
        for (int i0 = 0; i0 < e.n; i0 += NB) {
            T ch[NB][NP], dc[GRAD ? NB : 1][GRAD ? 3 * NP : 1], v[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int i = min(i0 + b, e.n - 1);   // a short batch re-reads its last row
                const T *chp = a.chi + (int64_t)(e.row0 + i) * NP;
#pragma unroll
                for (int l = 0; l < NP; ++l) ch[b][l] = chp[l];
                if constexpr (GRAD) {
                    const T *dcp = a.dchi + (int64_t)(e.row0 + i) * 3 * NP;
#pragma unroll
                    for (int q = 0; q < 3 * NP; ++q) dc[b][q] = dcp[q];
                }
                v[b] = i0 + b < e.n ? pencil[e.zlo + i] : (T)0;
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
#pragma unroll
                for (int l = 0; l < NP; ++l) s[l] += ch[b][l] * v[b];
                if constexpr (GRAD) {
#pragma unroll
                    for (int q = 0; q < 3 * NP; ++q) g[q] += dc[b][q] * v[b];
                }
            }
        }
        int slot = e.slot;
        if constexpr (GRAD) {
            T sg[NP + 3 * NP];
#pragma unroll
            for (int l = 0; l < NP; ++l) sg[l] = s[l];
#pragma unroll
            for (int q = 0; q < 3 * NP; ++q) sg[NP + q] = g[q];
            merge_equal_slots<T, 4 * NP>(sg, slot);
#pragma unroll
            for (int l = 0; l < NP; ++l) s[l] = sg[l];
#pragma unroll
            for (int q = 0; q < 3 * NP; ++q) g[q] = sg[NP + q];
        } else {
            merge_equal_slots<T, NP>(s, slot);
        }
        if (slot >= 0) {
            T *pa = nl.pacc + ((int64_t)nl.par * nl.maxat + slot) * NP;
#pragma unroll
            for (int l = 0; l < NP; ++l) atomicAdd(&pa[l], s[l]);
            if constexpr (GRAD) {
                T *ga = nl.gacc + ((int64_t)nl.par * nl.maxat + slot) * 3 * NP;
#pragma unroll
                for (int q = 0; q < 3 * NP; ++q) atomicAdd(&ga[q], g[q]);
            }
        }
    }
}

// rank-4 update of this thread's own pencil in LDS (no other thread writes it)
template <typename T, int NBX = 0>
__device__ __forceinline__ void col_update(const RegionArgs<T> &a, const ColNL<T> &nl, T *pencil,
                                           T half) {
    constexpr int NB = NBX > 0 ? NBX : sizeof(T) == 8 ? NB64 : 4;
    for (int c = 0; c < nl.ncol; ++c) {
        const ColEntry e = nl.cols[c];
        const T *pa = nl.pacc + ((int64_t)nl.par * nl.maxat + e.slot) * NP;
        const T *sc = nl.scale + (int64_t)e.slot * NP;
        T f[NP];
#pragma unroll
        for (int l = 0; l < NP; ++l) f[l] = sc[l] * pa[l] * half;
        for (int i0 = 0; i0 < e.n; i0 += NB) {
            T ch[NB][NP];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int i = min(i0 + b, e.n - 1);
                const T *chp = a.chi + (int64_t)(e.row0 + i) * NP;
#pragma unroll
                for (int l = 0; l < NP; ++l) ch[b][l] = chp[l];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int b = 0; b < NB; ++b)
                if (i0 + b < e.n)
                    pencil[e.zlo + i0 + b] +=
                        ch[b][0] * f[0] + ch[b][1] * f[1] + ch[b][2] * f[2] + ch[b][3] * f[3];
        }
    }
}

template <typename T, int BLOCK, bool GRAD>
__device__ __forceinline__ void col_zero_next(const ColNL<T> &nl, int nat) {
    T *pa = nl.pacc + (int64_t)(nl.par ^ 1) * nl.maxat * NP;
    for (int i = threadIdx.x; i < nat * NP; i += BLOCK) pa[i] = (T)0;
    if constexpr (GRAD) {
        T *ga = nl.gacc + (int64_t)(nl.par ^ 1) * nl.maxat * 3 * NP;
        for (int i = threadIdx.x; i < nat * 3 * NP; i += BLOCK) ga[i] = (T)0;
    }
}

// local part of prev <- 2 Hs cur - prev (no projector term): D cur - prev,
// z neighbours from registers, x / y neighbours from the LDS copy of cur
template <typename T, int E, int R, int ZS, bool DREG>
__device__ __forceinline__ void local_part(const RegionArgs<T> &a, const StepCtx<T, E, R> &c,
                                           const T (&d)[DREG ? E : 1], int64_t col,
                                           int64_t plane, int gz0, int n2, const T (&cur)[E],
                                           T (&prev)[E], const T *lds) {
    diag_part<T, E, R, DREG>(a, c, d, col, plane, gz0, n2, cur, prev);
#pragma unroll
    for (int p = 1; p <= R; ++p) {
#pragma unroll
        for (int z = 0; z < E; ++z) {
            T s = (T)0;
            if (z + p < E) s += cur[z + p];
            if (z - p >= 0) s += cur[z - p];
            prev[z] += c.cz[p] * s;
        }
    }
#pragma unroll
    for (int p = 1; p <= R; ++p) {
        axpy_pencil<T, E, ZS>(prev, c.cx[p], lds + c.nb[4 * (p - 1) + 0] * ZS);
        axpy_pencil<T, E, ZS>(prev, c.cx[p], lds + c.nb[4 * (p - 1) + 1] * ZS);
        axpy_pencil<T, E, ZS>(prev, c.cy[p], lds + c.nb[4 * (p - 1) + 2] * ZS);
        axpy_pencil<T, E, ZS>(prev, c.cy[p], lds + c.nb[4 * (p - 1) + 3] * ZS);
    }
}

// Same as local_part with a runtime loop over the 4R neighbour pencils, for
// kernels that keep more pencils resident (the adjoint): one neighbour pencil
// is in flight at a time instead of all 4R.
// With st non-null, cur is also stored to st ([z][pencil], E^2 apart) right
// after its last register use: the stores then overlap the LDS half of the
// step instead of delaying the next step's loads (which share the vector
// memory counter with them).
template <typename T, int E, int R, int ZS, bool DREG>
__device__ __forceinline__ void local_part_lowreg(const RegionArgs<T> &a,
                                                  const StepCtx<T, E, R> &c,
                                                  const T (&d)[DREG ? E : 1], int64_t col,
                                                  int64_t plane, int gz0, int n2,
                                                  const T (&cur)[E], T (&prev)[E],
                                                  const T *lds, T *st) {
    diag_part<T, E, R, DREG>(a, c, d, col, plane, gz0, n2, cur, prev);
#pragma unroll
    for (int p = 1; p <= R; ++p) {
#pragma unroll
        for (int z = 0; z < E; ++z) {
            T s = (T)0;
            if (z + p < E) s += cur[z + p];
            if (z - p >= 0) s += cur[z - p];
            prev[z] += c.cz[p] * s;
        }
    }
    if (st && c.active) {
#pragma unroll
        for (int z = 0; z < E; ++z) sgpr_ptr(st + (int64_t)z * E * E)[threadIdx.x] = cur[z];
    }
    // neighbour offsets are recomputed per step from an opaque zero so the
    // compiler does not keep 4R of them live across the step loop
    int salt = 0;
    asm volatile("" : "+v"(salt));
    const int tid = threadIdx.x + salt;
    const int px = c.px + salt, py = c.py + salt;
#pragma unroll
    for (int p = 1; p <= R; ++p) {
        const int n0 = (c.active && px + p < c.dx) ? tid + p : c.npen;
        axpy_pencil<T, E, ZS>(prev, c.cx[p], lds + n0 * ZS);
        const int n1 = (c.active && px - p >= 0) ? tid - p : c.npen;
        axpy_pencil<T, E, ZS>(prev, c.cx[p], lds + n1 * ZS);
        const int n2_ = (c.active && py + p < c.dy) ? tid + p * c.dx : c.npen;
        axpy_pencil<T, E, ZS>(prev, c.cy[p], lds + n2_ * ZS);
        const int n3 = (c.active && py - p >= 0) ? tid - p * c.dx : c.npen;
        axpy_pencil<T, E, ZS>(prev, c.cy[p], lds + n3 * ZS);
    }
}

// One step with the column projector path (two barriers per step):
//   A: cur complete in LDS -> projections of cur (own pencil, LDS atomics) and
//      the local stencil;  B: all reads of cur done -> publish the local part,
//      add the projector term to the own pencil, reload it.
// cur is written to LDS at the start even when the previous step left the
// same values there: a conditional store costs more registers than it saves.
// A per-row update the store-all adjoint runs inside a step, right after the
// projections of cur (the own pencil in LDS holds cur; the projection buffer
// of the previous step is still intact there).
// NP-vector of W (one support row, all projectors), moved as one aligned unit
template <typename T>
struct alignas(4 * sizeof(T)) WVec {
    T v[4];
    __device__ T &operator[](int i) { return v[i]; }
};
static_assert(NP == 4, "WVec holds NP values");

template <typename T>
struct WArgs {
    const T *ck;     // the region's stored vectors
    T *wb;           // accumulator rows
    int kp;          // p-term: projections chi . v_kp of the forward sweep ...
    T ap;            //   ... weight, times the own pencil
    int kq;          // q-term (kq >= 0): projection buffer parq of nl ...
    T aq;            //   ... weight, times v_kq
    int parq;
};

template <typename T, int E, int BLOCK>
__device__ __forceinline__ void w_update(const RegionArgs<T> &a, const ColNL<T> &nl,
                                         const WArgs<T> &w, const T *mine);

// First half of a step (up to the second barrier): publish cur, project it,
// local part of prev.  (st: see local_part_lowreg; LOWREG steps only.)
template <typename T, int E, int R, int ZS, bool DREG, bool GRAD, bool LOWREG, int BLOCK = 64,
          bool WH = false>
__device__ __forceinline__ void step_col_a(const RegionArgs<T> &a, const StepCtx<T, E, R> &c,
                                           const T (&d)[DREG ? E : 1], int64_t col,
                                           int64_t plane, int gz0, int n2, T (&cur)[E],
                                           T (&prev)[E], T *lds, ColNL<T> &nl,
                                           T *st = nullptr, const WArgs<T> *w = nullptr) {
    if (c.active) store_pencil<T, E, ZS>(c.mine, cur);
    __syncthreads();
    // all lanes of the block (c.nat is uniform): the merge exchanges between lanes
    if (c.nat) col_dots<T, GRAD>(a, nl, c.mine);
    if constexpr (WH) {
        if (nl.ncol) w_update<T, E, BLOCK>(a, nl, *w, c.mine);
    }
    if constexpr (LOWREG)
        local_part_lowreg<T, E, R, ZS, DREG>(a, c, d, col, plane, gz0, n2, cur, prev, lds, st);
    else
        local_part<T, E, R, ZS, DREG>(a, c, d, col, plane, gz0, n2, cur, prev, lds);
}

template <typename T, int E, int R, int ZS, int BLOCK, bool MASKZ, bool DREG, bool GRAD,
          bool LOWREG = false, bool WH = false>
__device__ __forceinline__ void region_step_col(const RegionArgs<T> &a, const StepCtx<T, E, R> &c,
                                                const T (&d)[DREG ? E : 1], int64_t col,
                                                int64_t plane, int gz0, int n2, T (&cur)[E],
                                                T (&prev)[E], T *lds, ColNL<T> &nl, bool first,
                                                T *st = nullptr, const WArgs<T> *w = nullptr) {
    step_col_a<T, E, R, ZS, DREG, GRAD, LOWREG, BLOCK, WH>(a, c, d, col, plane, gz0, n2, cur,
                                                           prev, lds, nl, st, w);
    __syncthreads();
    if (first) {
#pragma unroll
        for (int z = 0; z < E; ++z) prev[z] *= (T)0.5;
    }
    if constexpr (MASKZ) {
#pragma unroll
        for (int z = 0; z < E; ++z) prev[z] = (z < c.dz) ? prev[z] : (T)0;
    }
    if (c.nat) {
        if (c.active) store_pencil<T, E, ZS>(c.mine, prev);
        if (nl.ncol) col_update<T>(a, nl, c.mine, first ? (T)0.5 : (T)1);
        if (c.active) load_pencil<T, E, ZS>(c.mine, prev);
        col_zero_next<T, BLOCK, GRAD>(nl, c.nat);
    }
    nl.par ^= 1;
}

// projections of one vector without a recurrence step (column path)
template <typename T, int E, int R, int ZS, int BLOCK, bool GRAD, bool WH = false>
__device__ __forceinline__ void col_dots_only(const RegionArgs<T> &a, const StepCtx<T, E, R> &c,
                                              const T (&vec)[E], ColNL<T> &nl,
                                              const WArgs<T> *w = nullptr) {
    if (c.active) store_pencil<T, E, ZS>(c.mine, vec);
    __syncthreads();
    // all lanes of the block (c.nat is uniform): the merge exchanges between lanes
    if (c.nat) col_dots<T, GRAD>(a, nl, c.mine);
    if constexpr (WH) {
        if (nl.ncol) w_update<T, E, BLOCK>(a, nl, *w, c.mine);
    }
    __syncthreads();
    col_zero_next<T, BLOCK, GRAD>(nl, c.nat);
    nl.par ^= 1;
}

// W(y) += ap p_kp vt(y) + aq q v_kq(y) on the rows of this thread's column
// pieces; rows are handled in batches (loads first, then the FMAs).
template <typename T, int E, int BLOCK>
__device__ __forceinline__ void w_update(const RegionArgs<T> &a, const ColNL<T> &nl,
                                         const WArgs<T> &w, const T *mine) {
    constexpr int EE = E * E;
    constexpr int NB = 4;
    const uint32_t t = threadIdx.x;
    const T *pk = w.ck + (int64_t)a.K * E * EE + (int64_t)w.kp * MAX_REGION_ATOMS * 4 * NP;
    const bool hq = w.kq >= 0;
    const T *vk = w.ck + (int64_t)(hq ? w.kq : 0) * E * EE + t;
    int ebase = 0;   // this thread's rows are numbered densely over its pieces
    for (int cc = 0; cc < nl.ncol; ++cc) {
        const ColEntry e = nl.cols[cc];
        T q[NP], p[NP];
#pragma unroll
        for (int l = 0; l < NP; ++l) {
            p[l] = w.ap * pk[e.slot * 4 * NP + l];
            q[l] = hq ? w.aq * nl.pacc[((int64_t)w.parq * nl.maxat + e.slot) * NP + l] : (T)0;
        }
        // row i of this piece: one NP-vector per thread, wc[i * BLOCK]
        WVec<T> *wc = reinterpret_cast<WVec<T> *>(w.wb) + ((int64_t)ebase * BLOCK + t);
        ebase += e.n;
        for (int i0 = 0; i0 < e.n; i0 += NB) {
            T tv[NB], vv[NB];
            WVec<T> wv[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int i = min(i0 + b, e.n - 1);
                tv[b] = mine[e.zlo + i];
                vv[b] = hq ? vk[(int64_t)(e.zlo + i) * EE] : (T)0;
                wv[b] = wc[(int64_t)i * BLOCK];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (i0 + b < e.n) {
                    WVec<T> r = wv[b];
#pragma unroll
                    for (int l = 0; l < NP; ++l) r[l] += p[l] * tv[b] + q[l] * vv[b];
                    wc[(int64_t)(i0 + b) * BLOCK] = r;
                }
            }
        }
    }
}

template <typename T, int E>
__device__ __forceinline__ double pick(const T (&v)[E], int z0) {
    T m = 0;
#pragma unroll
    for (int z = 0; z < E; ++z) m = (z == z0) ? v[z] : m;
    return (double)m;
}

}  // namespace sqk
