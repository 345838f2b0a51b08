// Spectral Gauss quadrature (LSSGQ) of Section 2.2 after the Lanczos sweep:
// Gauss nodes and weights of every node's Jacobi matrix, the Fermi level of
// Eq. (Ne) by bisection over the rules, and the pointwise fields
// rho^q, u^q, s^q of Eqs. (rhoq), (uq), (sq) with their domain totals.
//
// Nodes are the eigenvalues of the node's Jacobi matrix (mapped back from the
// scaled spectrum, lambda = tau theta + omega) and the weights the squared
// first components of its normalised eigenvectors (Golub and Welsch, 1969).
// The eigensolve is the implicit QL iteration with shifts (Bowdler, Martin,
// Reinsch and Wilkinson, 1968) carrying only the first row of the eigenvector
// matrix: one thread per node, its three length-K arrays in LDS, interleaved
// across the threads of the block so that the lanes of a wave hit distinct
// banks whatever index each of them is at.
#include <cfloat>

#include "sq_kernels.h"

namespace sqk {

namespace {

// LDS column j of thread t of a block of nt threads
struct Col {
    double *p;
    int nt;
    __device__ double &operator[](int j) const { return p[j * nt]; }
};

// Implicit QL on the symmetric tridiagonal (d[0..n), e[0..n-1)), e[n-1] = 0.
// On return d holds the eigenvalues and z the first row of the eigenvector
// matrix (z starts as e_0).  Returns false when an eigenvalue did not settle
// in 60 sweeps.
__device__ bool ql_first_row(const Col &d, const Col &e, const Col &z, int n) {
    bool ok = true;
    for (int l = 0; l < n; ++l) {
        for (int sweep = 0;; ++sweep) {
            // first negligible coupling at or after l
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = fabs(d[m]) + fabs(d[m + 1]);
                if (fabs(e[m]) <= DBL_EPSILON * dd) break;
            }
            if (m == l) break;
            if (sweep == 60) {
                ok = false;
                break;
            }
            // shift: eigenvalue of the leading 2x2 block nearer to d[l]
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool split = false;
            for (int i = m - 1; i >= l; --i) {
                double f = s * e[i];
                const double b = c * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {   // the bulge vanished: the block splits here
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    split = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                // the rotation acting on columns i, i+1 of the eigenvector matrix
                f = z[i + 1];
                z[i + 1] = s * z[i] + c * f;
                z[i] = c * z[i] - s * f;
            }
            if (split) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return ok;
}

// In place per node: lam[K] holds a_1..a_K and wgt[K] b_1..b_K on entry (the
// rule ends at the first zero b); on exit lam holds the nodes in ascending
// order (the last node repeated past the rule's end) and wgt the weights (0
// past the end).  Dynamic LDS: 3 K doubles per thread.
__global__ void gauss_eig_kernel(double *lam, double *wgt, int64_t n, int K, const Scalars *s,
                                 int32_t *status) {
    HIP_DYNAMIC_SHARED(double, sh)
    const int nt = blockDim.x, t = threadIdx.x;
    const int64_t q = (int64_t)blockIdx.x * nt + t;
    if (q >= n) return;
    const Col d{sh + t, nt}, e{sh + (int64_t)K * nt + t, nt}, z{sh + 2 * (int64_t)K * nt + t, nt};
    double *L = lam + q * K, *W = wgt + q * K;
    int m = K;
    for (int j = 0; j < K; ++j) {
        d[j] = L[j];
        const double b = W[j];
        e[j] = b;
        z[j] = j == 0 ? 1.0 : 0.0;
        if (b == 0.0 && m == K) m = j + 1;
    }
    e[m - 1] = 0.0;
    if (!ql_first_row(d, e, z, m)) atomicOr(status, 4);
    // ascending order (selection sort; m <= K is small)
    for (int i = 0; i < m - 1; ++i) {
        int k = i;
        for (int j = i + 1; j < m; ++j)
            if (d[j] < d[k]) k = j;
        if (k != i) {
            const double td = d[i], tz = z[i];
            d[i] = d[k];
            z[i] = z[k];
            d[k] = td;
            z[k] = tz;
        }
    }
    const double tau = s->tau, om = s->omega;
    for (int j = 0; j < K; ++j) {
        const int jj = j < m ? j : m - 1;
        L[j] = tau * d[jj] + om;
        W[j] = j < m ? z[j] * z[j] : 0.0;
    }
}

__device__ __forceinline__ double gsum(double x, double *sh) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = x;
    __syncthreads();
    double t = 0.0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) t += sh[i];
    return t;
}

__device__ __forceinline__ double occ(double lam, double lf, double kT) {
    return 0.5 * (1.0 - tanh((lam - lf) / (2.0 * kT)));
}

__global__ void gauss_fermi_init_kernel(Scalars *s, double Ne, double tol, int max_iter,
                                        const double *lf_in) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    s->lo = s->lmin;
    s->hi = s->lmax;
    s->ne_target = Ne;
    s->tol = tol;
    s->iters = 0;
    s->max_iter = max_iter;
    s->done = 0;
    s->status = SQ_OK;   // a new solve: no status from an earlier one survives
    if (max_iter == 0) {
        s->lambda_f = *lf_in;
        s->done = 1;
    }
}

// One evaluation of N_e = 2 sum_q sum_k w g(lambda) at lo (phase 0), hi
// (phase 1) or the midpoint (phase 2).  The last block to finish sums the
// block partials in block order and moves the bracket: lo = mid when
// N_e(mid) < target, else hi = mid; stop at |N_e - target| < tol, at a 4-ulp
// bracket or after max_iter midpoints, with lambda_f = the last midpoint.
__global__ void gauss_eval_kernel(Scalars *s, const double *lam, const double *wgt, int64_t nk,
                                  double kT, int phase, double *partial, int *ticket) {
    __shared__ double sh[16];
    __shared__ int last;
    if (s->done) return;
    const double x = phase == 0 ? s->lo : (phase == 1 ? s->hi : s->lo + 0.5 * (s->hi - s->lo));
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nk;
         i += (int64_t)gridDim.x * blockDim.x)
        acc += wgt[i] * occ(lam[i], x, kT);
    const double t = gsum(acc, sh);
    if (threadIdx.x == 0) {
        __hip_atomic_store(&partial[blockIdx.x], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int old =
            __hip_atomic_fetch_add(ticket, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (old == (int)gridDim.x - 1);
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    double S = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b)
        S += __hip_atomic_load(&partial[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double ne = 2.0 * S;
    *ticket = 0;
    if (phase == 0) {
        s->ne_lo = ne;
    } else if (phase == 1) {
        s->ne_hi = ne;
        if (s->ne_lo > s->ne_target || ne < s->ne_target) {
            s->status = SQ_ERR_NOT_CONVERGED;
            s->lambda_f = __builtin_nan("");
            s->done = 1;
        }
    } else {
        s->iters += 1;
        s->ne_mid = ne;
        s->lambda_f = x;
        if (fabs(ne - s->ne_target) < s->tol) {
            s->done = 1;
            return;
        }
        if (ne < s->ne_target) s->lo = x; else s->hi = x;
        // a 4-ulp bracket or max_iter midpoints without |N_e - target| < tol:
        // lambda_f keeps the last midpoint, flagged as not converged
        const double big = fmax(fabs(s->lo), fabs(s->hi));
        if (s->hi - s->lo < 4.0 * DBL_EPSILON * big || s->iters >= s->max_iter) {
            s->done = 1;
            s->status = SQ_ERR_NOT_CONVERGED;
        }
    }
}

// rho^q = 2 sum_k w g, u^q = 2 sum_k w lambda g, s^q = -2 sum_k w sfn (units
// of k_B) with sfn = g log g + (1 - g) log(1 - g) written as
// -(t e^-t / (1 + e^-t) + log(1 + e^-t)), t = |lambda - lambda_f| / kT;
// per-block partial sums of the three for the totals.
__global__ void gauss_fields_kernel(const double *lam, const double *wgt, int64_t n, int K,
                                    double kT, const Scalars *s, double *rho, double *u,
                                    double *sq, double *partial) {
    __shared__ double sh[16];
    const double lf = s->lambda_f;
    double pr = 0.0, pu = 0.0, ps = 0.0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        double r = 0.0, e = 0.0, h = 0.0;
        for (int k = 0; k < K; ++k) {
            const double x = lam[q * K + k], w = wgt[q * K + k];
            const double g = occ(x, lf, kT);
            const double t = fabs(x - lf) / kT, ex = exp(-t);
            r += w * g;
            e += w * x * g;
            h += w * -(t * ex / (1.0 + ex) + log1p(ex));
        }
        r *= 2.0;
        e *= 2.0;
        h *= -2.0;
        if (rho) rho[q] = r;
        if (u) u[q] = e;
        if (sq) sq[q] = h;
        pr += r;
        pu += e;
        ps += h;
    }
    pr = gsum(pr, sh);
    pu = gsum(pu, sh);
    ps = gsum(ps, sh);
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x + 0] = pr;
        partial[3 * blockIdx.x + 1] = pu;
        partial[3 * blockIdx.x + 2] = ps;
    }
}

__global__ void gauss_totals_kernel(const double *partial, int nb, double kT, const Scalars *s,
                                    double *totals, double *lf_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = 0; i < nb; ++i) {
        a += partial[3 * i + 0];
        b += partial[3 * i + 1];
        c += partial[3 * i + 2];
    }
    if (totals) {
        totals[0] = a;
        totals[1] = b;
        totals[2] = c;
        totals[3] = b - kT * c;
        totals[4] = s->omega;
        totals[5] = s->tau;
        totals[6] = (double)s->iters;
        totals[7] = (double)s->status;
    }
    if (lf_out) *lf_out = s->lambda_f;
}

}  // namespace

int gauss_eig_threads(int K) {
    int nt = 64;
    while (nt > 1 && (int64_t)nt * 3 * K * (int64_t)sizeof(double) > LDS_BYTES) nt >>= 1;
    return nt;
}

hipError_t k_gauss_eig(double *lam, double *wgt, int64_t n, int K, const Scalars *s,
                       int32_t *status, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const int nt = gauss_eig_threads(K);
    const size_t lds = (size_t)nt * 3 * K * sizeof(double);
    // more than 64 KiB of dynamic LDS needs the kernel attribute raised, once per
    // device (a host call: it is kept out of every later, possibly captured, call)
    static bool raised[64] = {};
    if (lds > 65536) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if (dev >= 64 || !raised[dev]) {
            e = hipFuncSetAttribute((const void *)gauss_eig_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, LDS_BYTES);
            if (e != hipSuccess) return e;
            if (dev < 64) raised[dev] = true;
        }
    }
    const int64_t grid = (n + nt - 1) / nt;
    hipLaunchKernelGGL(gauss_eig_kernel, dim3((unsigned)grid), dim3(nt), lds, st, lam, wgt, n, K, s,
                       status);
    return hipGetLastError();
}

hipError_t k_gauss_fermi(const FermiWork &f, Scalars *s, const double *lam, const double *wgt,
                         int64_t nk, double kT, double Ne, double tol, int max_iter,
                         const double *lf_in, hipStream_t st) {
    hipLaunchKernelGGL(gauss_fermi_init_kernel, dim3(1), dim3(64), 0, st, s, Ne, tol, max_iter,
                       lf_in);
    if (max_iter > 0) {
        const int G = f.n_partial;
        for (int ph = 0; ph < 2; ++ph)
            hipLaunchKernelGGL(gauss_eval_kernel, dim3(G), dim3(256), 0, st, s, lam, wgt, nk, kT,
                               ph, f.partial, f.ticket);
        for (int it = 0; it < max_iter; ++it)
            hipLaunchKernelGGL(gauss_eval_kernel, dim3(G), dim3(256), 0, st, s, lam, wgt, nk, kT,
                               2, f.partial, f.ticket);
    }
    return hipGetLastError();
}

hipError_t k_gauss_fields(const double *lam, const double *wgt, int64_t n, int K, double kT,
                          const Scalars *s, double *rho, double *u, double *sq, double *partial,
                          int n_partial, double *totals, double *lf_out, hipStream_t st) {
    const int64_t want = (n + 255) / 256;
    const int nb = (int)(want < 1 ? 1 : (want > n_partial ? n_partial : want));
    hipLaunchKernelGGL(gauss_fields_kernel, dim3(nb), dim3(256), 0, st, lam, wgt, n, K, kT, s, rho,
                       u, sq, partial);
    hipLaunchKernelGGL(gauss_totals_kernel, dim3(1), dim3(64), 0, st, partial, nb, kT, s, totals,
                       lf_out);
    return hipGetLastError();
}

}  // namespace sqk
