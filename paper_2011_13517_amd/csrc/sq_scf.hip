// SCF outer loop around the density path (Section 3's flowchart), periodic
// cells: the electron density from rho^q, the electrostatic potential of Eq.
// (Poisson) by conjugate gradients on the FD Laplacian, the LDA
// exchange-correlation potential, and mixing of the effective potential.
//
// Every vector here lives on the V grid in FP64.  Reductions are deterministic
// (fixed per-block partials, summed in a fixed order by one wave), and the
// scalars of the iteration stay on the device, so only the convergence tests
// of the host loop synchronise.
#include <cfloat>

#include "sq_scf.h"

namespace sqk {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ double blk_sum(double x, double *sh) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = x;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < TPB / 64; ++i) t += sh[i];
    return t;
}

// partial[block] = sum over the block's grid-stride share of x . y
__global__ void dot_partial_kernel(const double *x, const double *y, int64_t n, double *partial) {
    __shared__ double sh[TPB / 64];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB)
        acc += x[i] * y[i];
    const double t = blk_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// one wave: lane l sums partial[l], partial[l + 64], ... in order, then a fixed
// butterfly (the same order on every run)
__global__ void sum_finish_kernel(const double *partial, int nb, double *out) {
    const int l = threadIdx.x;
    double t = 0.0;
    for (int i = l; i < nb; i += 64) t += partial[i];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o, 64);
    if (l == 0 && blockIdx.x == 0) *out = t;
}

// the node of Omega at V-grid point i, or -1 on the padding
__device__ __forceinline__ int64_t omega_index(const ScfGrid &g, int64_t i) {
    const int x = (int)(i % g.N[0]) - g.pad[0];
    const int y = (int)((i / g.N[0]) % g.N[1]) - g.pad[1];
    const int z = (int)(i / ((int64_t)g.N[0] * g.N[1])) - g.pad[2];
    if (x < 0 || y < 0 || z < 0 || x >= g.n[0] || y >= g.n[1] || z >= g.n[2]) return -1;
    return x + (int64_t)g.n[0] * (y + (int64_t)g.n[1] * z);
}

// n = rho^q / (h1 h2 h3) and the Poisson source n + b at the nodes of Omega
__global__ void source_kernel(ScfGrid g, const double *rho_q, const double *b, double inv_h3,
                              double *nx, double *src) {
    const int64_t nv = (int64_t)g.N[0] * g.N[1] * g.N[2];
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < nv;
         i += (int64_t)gridDim.x * TPB) {
        const int64_t q = omega_index(g, i);
        const double d = q >= 0 ? rho_q[q] * inv_h3 : 0.0;
        nx[i] = d;
        src[i] = q >= 0 ? d + b[i] : 0.0;
    }
}

// x <- scale * (x - s[0] / n)   (zero mean, then the 4 pi of Eq. (Poisson))
__global__ void center_scale_kernel(double *x, int64_t n, const double *s, double scale) {
    const double m = *s / (double)n;
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * TPB)
        x[i] = scale * (x[i] - m);
}

// y = -Lap_h x: -sum_a (w_0 x + sum_p w_p (x_{+p} + x_{-p})) / h_a^2, wrapped on
// periodic grids; on embedded grids at the nodes of Omega only (the padding,
// at least r deep, holds the Dirichlet values) and 0 on the padding
__global__ void neg_lap_kernel(ScfGrid g, const double *x, double *y) {
    const int64_t nv = (int64_t)g.N[0] * g.N[1] * g.N[2];
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < nv;
         i += (int64_t)gridDim.x * TPB) {
        const int ix = (int)(i % g.N[0]);
        const int iy = (int)((i / g.N[0]) % g.N[1]);
        const int iz = (int)(i / ((int64_t)g.N[0] * g.N[1]));
        if (!g.periodic && omega_index(g, i) < 0) {
            y[i] = 0.0;
            continue;
        }
        const int64_t sy = g.N[0], sz = (int64_t)g.N[0] * g.N[1];
        const double xc = x[i];
        double ax = g.w[0] * xc, ay = g.w[0] * xc, az = g.w[0] * xc;
        for (int p = 1; p <= g.r; ++p) {
            int a = ix + p, b = ix - p;
            a = a >= g.N[0] ? a - g.N[0] : a;
            b = b < 0 ? b + g.N[0] : b;
            ax += g.w[p] * (x[i - ix + a] + x[i - ix + b]);
            a = iy + p;
            b = iy - p;
            a = a >= g.N[1] ? a - g.N[1] : a;
            b = b < 0 ? b + g.N[1] : b;
            ay += g.w[p] * (x[i + (a - iy) * sy] + x[i + (b - iy) * sy]);
            a = iz + p;
            b = iz - p;
            a = a >= g.N[2] ? a - g.N[2] : a;
            b = b < 0 ? b + g.N[2] : b;
            az += g.w[p] * (x[i + (a - iz) * sz] + x[i + (b - iz) * sz]);
        }
        y[i] = -(ax * g.ih2[0] + ay * g.ih2[1] + az * g.ih2[2]);
    }
}

// r <- src - r (r holds A phi on entry), p <- r
__global__ void cg_init_kernel(const double *src, double *r, double *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * TPB) {
        const double v = src[i] - r[i];
        r[i] = v;
        p[i] = v;
    }
}

// alpha = rr / pAp;  phi += alpha p;  r -= alpha Ap
__global__ void cg_update_kernel(const double *sc, double *phi, double *r, const double *p,
                                 const double *Ap, int64_t n) {
    const double rr = sc[SC_RR], pap = sc[SC_PAP];
    const double alpha = pap != 0.0 ? rr / pap : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * TPB) {
        phi[i] += alpha * p[i];
        r[i] -= alpha * Ap[i];
    }
}

// beta = rr_new / rr;  p = r + beta p;  then rr <- rr_new (one thread, after the
// grid has read rr: done by cg_shift_kernel)
__global__ void cg_direction_kernel(const double *sc, const double *r, double *p, int64_t n) {
    const double rr = sc[SC_RR], rn = sc[SC_RRN];
    const double beta = rr != 0.0 ? rn / rr : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * TPB)
        p[i] = r[i] + beta * p[i];
}

__global__ void zero_kernel(double *x) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *x = 0.0;
}

__global__ void cg_shift_kernel(double *sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sc[SC_RR] = sc[SC_RRN];
}

// LDA: Slater exchange and the Perdew-Wang (1992) correlation, unpolarised
__device__ __forceinline__ double vxc_pw92(double n) {
    if (!(n > 0.0)) return 0.0;
    const double A = 0.031091, a1 = 0.21370, b1 = 7.5957, b2 = 3.5876, b3 = 1.6382,
                 b4 = 0.49294;
    const double ex = -0.75 * cbrt(3.0 * n / M_PI);
    const double rs = cbrt(3.0 / (4.0 * M_PI * n));
    const double sr = sqrt(rs);
    const double q0 = -2.0 * A * (1.0 + a1 * rs);
    const double q1 = 2.0 * A * (b1 * sr + b2 * rs + b3 * rs * sr + b4 * rs * rs);
    const double dq1 = A * (b1 / sr + 2.0 * b2 + 3.0 * b3 * sr + 4.0 * b4 * rs);
    const double lg = log1p(1.0 / q1);
    const double ec = q0 * lg;
    const double dec = -2.0 * A * a1 * lg - q0 * dq1 / (q1 * q1 + q1);
    return 4.0 / 3.0 * ex + ec - rs / 3.0 * dec;
}

// V_out = phi + v_xc(n) at the nodes of Omega (V_in on the padding);  F = V_out - V_in
__global__ void vout_kernel(ScfGrid g, const double *phi, const double *nx, const double *vin,
                            double *vout, double *F) {
    const int64_t n = (int64_t)g.N[0] * g.N[1] * g.N[2];
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * TPB) {
        const double vo = omega_index(g, i) >= 0 ? phi[i] + vxc_pw92(nx[i]) : vin[i];
        vout[i] = vo;
        F[i] = vo - vin[i];
    }
}

// F . (F - F') and |F - F'|^2 partials, in one pass
__global__ void anderson_partial_kernel(const double *F, const double *Fp, int64_t n,
                                        double *part_a, double *part_b) {
    __shared__ double sh[TPB / 64];
    double a = 0.0, b = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * TPB) {
        const double d = F[i] - Fp[i];
        a += F[i] * d;
        b += d * d;
    }
    a = blk_sum(a, sh);
    __syncthreads();
    b = blk_sum(b, sh);
    if (threadIdx.x == 0) {
        part_a[blockIdx.x] = a;
        part_b[blockIdx.x] = b;
    }
}

// mixing: linear (first step) V <- V + beta F, or Anderson with the previous pair:
// g = F.(F - F') / |F - F'|^2, V <- (V - g (V - V')) + beta (F - g (F - F'));
// V' <- V, F' <- F for the next step
__global__ void mix_kernel(double *V, double *Vp, const double *F, double *Fp, int64_t n,
                           double beta, int anderson, const double *sc) {
    double g = 0.0;
    if (anderson) {
        const double num = sc[SC_FDF], den = sc[SC_DFDF];
        g = den > 0.0 ? num / den : 0.0;
    }
    for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * TPB) {
        const double v = V[i], f = F[i];
        double vn;
        if (anderson)
            vn = (v - g * (v - Vp[i])) + beta * (f - g * (f - Fp[i]));
        else
            vn = v + beta * f;
        Vp[i] = v;
        Fp[i] = f;
        V[i] = vn;
    }
}

}  // namespace

hipError_t scf_dot(const double *x, const double *y, int64_t n, double *partial, int nb,
                   double *out, hipStream_t st) {
    hipLaunchKernelGGL(dot_partial_kernel, dim3(nb), dim3(TPB), 0, st, x, y, n, partial);
    hipLaunchKernelGGL(sum_finish_kernel, dim3(1), dim3(64), 0, st, partial, nb, out);
    return hipGetLastError();
}

hipError_t scf_source(const ScfGrid &g, const double *rho_q, const double *b, double inv_h3,
                      double *nx, double *src, const double *ones, double *partial, int nb,
                      double *sc, hipStream_t st) {
    const int64_t n = (int64_t)g.N[0] * g.N[1] * g.N[2];
    hipLaunchKernelGGL(source_kernel, dim3(nb), dim3(TPB), 0, st, g, rho_q, b, inv_h3, nx, src);
    if (g.periodic) {   // the neutral cell: remove the mean
        hipError_t e = scf_dot(src, ones, n, partial, nb, sc + SC_MEAN, st);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, st, sc + SC_MEAN);
    }
    hipLaunchKernelGGL(center_scale_kernel, dim3(nb), dim3(TPB), 0, st, src, n,
                       (const double *)(sc + SC_MEAN), 4.0 * M_PI);
    return hipGetLastError();
}

hipError_t scf_cg_start(const ScfGrid &g, const double *src, double *phi, double *r, double *p,
                        double *partial, int nb, double *sc, hipStream_t st) {
    const int64_t n = (int64_t)g.N[0] * g.N[1] * g.N[2];
    hipLaunchKernelGGL(neg_lap_kernel, dim3(nb), dim3(TPB), 0, st, g, phi, r);
    hipLaunchKernelGGL(cg_init_kernel, dim3(nb), dim3(TPB), 0, st, src, r, p, n);
    hipError_t e = scf_dot(r, r, n, partial, nb, sc + SC_RR, st);
    if (e != hipSuccess) return e;
    return scf_dot(src, src, n, partial, nb, sc + SC_BB, st);
}

hipError_t scf_cg_iter(const ScfGrid &g, double *phi, double *r, double *p, double *Ap,
                       double *partial, int nb, double *sc, hipStream_t st) {
    const int64_t n = (int64_t)g.N[0] * g.N[1] * g.N[2];
    hipLaunchKernelGGL(neg_lap_kernel, dim3(nb), dim3(TPB), 0, st, g, p, Ap);
    hipError_t e = scf_dot(p, Ap, n, partial, nb, sc + SC_PAP, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cg_update_kernel, dim3(nb), dim3(TPB), 0, st, (const double *)sc, phi, r,
                       (const double *)p, (const double *)Ap, n);
    e = scf_dot(r, r, n, partial, nb, sc + SC_RRN, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cg_direction_kernel, dim3(nb), dim3(TPB), 0, st, (const double *)sc,
                       (const double *)r, p, n);
    hipLaunchKernelGGL(cg_shift_kernel, dim3(1), dim3(64), 0, st, sc);
    return hipGetLastError();
}

hipError_t scf_center(double *x, int64_t n, const double *ones, double *partial, int nb,
                      double *sc, hipStream_t st) {
    hipError_t e = scf_dot(x, ones, n, partial, nb, sc + SC_MEAN, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(center_scale_kernel, dim3(nb), dim3(TPB), 0, st, x, n,
                       (const double *)(sc + SC_MEAN), 1.0);
    return hipGetLastError();
}

hipError_t scf_vout(const ScfGrid &g, const double *phi, const double *nx, const double *vin,
                    double *vout, double *F, double *partial, int nb, double *sc,
                    hipStream_t st) {
    const int64_t n = (int64_t)g.N[0] * g.N[1] * g.N[2];
    hipLaunchKernelGGL(vout_kernel, dim3(nb), dim3(TPB), 0, st, g, phi, nx, vin, vout, F);
    return scf_dot(F, F, n, partial, nb, sc + SC_FF, st);
}

hipError_t scf_mix(double *V, double *Vp, const double *F, double *Fp, int64_t n, double beta,
                   int anderson, double *partial, int nb, double *sc, hipStream_t st) {
    if (anderson) {
        hipLaunchKernelGGL(anderson_partial_kernel, dim3(nb), dim3(TPB), 0, st, F,
                           (const double *)Fp, n, partial, partial + nb);
        hipLaunchKernelGGL(sum_finish_kernel, dim3(1), dim3(64), 0, st, (const double *)partial,
                           nb, sc + SC_FDF);
        hipLaunchKernelGGL(sum_finish_kernel, dim3(1), dim3(64), 0, st,
                           (const double *)(partial + nb), nb, sc + SC_DFDF);
    }
    hipLaunchKernelGGL(mix_kernel, dim3(nb), dim3(TPB), 0, st, V, Vp, F, Fp, n, beta, anderson,
                       (const double *)sc);
    return hipGetLastError();
}

}  // namespace sqk
