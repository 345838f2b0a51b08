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
};

// atoms per region that fit the LDS left over by the box (EXTRA bytes of
// per-atom state beyond the slot and its four scaled projections)
template <typename T, int E, int EXTRA = 0>
constexpr int max_atoms_in_region() {
    constexpr int used = region_lds_elems<T, E>() * (int)sizeof(T) + 512;
    constexpr int per = (int)sizeof(Slot) + NP * (int)sizeof(T) + EXTRA;
    constexpr int n = (LDS_BYTES - used) / per;
    return n > 128 ? 128 : n;
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
    if constexpr (DREG) {
#pragma unroll
        for (int z = 0; z < E; ++z) prev[z] = d[z] * cur[z] - prev[z];
    } else {
        // D read back from L2 each step (its VGPRs are needed for the FP64 pencils)
#pragma unroll
        for (int z = 0; z < E; ++z) {
            int gz = gz0 + z;
            gz = gz >= n2 ? gz - n2 : gz;
            const T dz = (c.active && z < c.dz) ? a.D[col + plane * gz] : (T)0;
            prev[z] = dz * cur[z] - prev[z];
        }
    }
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

template <typename T, int E>
__device__ __forceinline__ double pick(const T (&v)[E], int z0) {
    T m = 0;
#pragma unroll
    for (int z = 0; z < E; ++z) m = (z == z0) ? v[z] : m;
    return (double)m;
}

}  // namespace sqk
