// FP64 device work around the recurrence (gfx950): spectral bounds, scaled
// diagonal, moment sums, Chebyshev coefficients, Fermi-level bisection and the
// pointwise contraction.  Every reduction is deterministic (fixed per-block
// partials summed in block order), and nothing here synchronises the host, so
// the whole sequence is graph-capturable.
#include <cfloat>

#include "sq_kernels.h"

namespace sqk {

// ------------------------------------------------------------------------- //
// small helpers
// ------------------------------------------------------------------------- //
__device__ __forceinline__ double block_sum(double x, double *sh) {
    // blockDim.x is a multiple of 64 and at most 1024
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = x;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int i = 0; i < nw; ++i) t += sh[i];
        sh[0] = t;
    }
    __syncthreads();
    t = sh[0];
    __syncthreads();
    return t;
}

// sum of partial[0..n) in index order, computed redundantly by every block
__device__ __forceinline__ double ordered_sum(const double *partial, int n, double *sh) {
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < n; ++i) t += partial[i];
        sh[0] = t;
    }
    __syncthreads();
    t = sh[0];
    __syncthreads();
    return t;
}

// splitmix64 (Steele, Lea & Flood 2014) as a counter-based generator:
// value i of stream `seed` mixes seed + (i + 1) * golden-gamma.
__device__ __forceinline__ double splitmix_uniform(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

// cos(k t_j), t_j = pi (j + 1/2) / N, with the angle reduced exactly in integers:
// k t_j = pi k (2j + 1) / (2N) = (pi / 2N) * (k (2j + 1) mod 4N)
__device__ __forceinline__ double cos_ktj(int64_t k, int64_t j, int64_t N) {
    const int64_t m = (k * (2 * j + 1)) % (4 * N);
    return cos(M_PI * (double)m / (double)(2 * N));
}

// Fermi-Dirac in scaled variables, (1 - tanh((x - lf) / (2 th))) / 2
__device__ __forceinline__ double fermi(double x, double lf, double th) {
    return 0.5 * (1.0 - tanh((x - lf) / (2.0 * th)));
}

// ------------------------------------------------------------------------- //
// scalars, diagonal, utility fills
// ------------------------------------------------------------------------- //
__global__ void set_bounds_kernel(Scalars *s, double lmin, double lmax) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        s->lmin = lmin;
        s->lmax = lmax;
        s->omega = 0.5 * (lmax + lmin);
        s->tau = 0.5 * (lmax - lmin);
        s->status = 0;
    }
}

__global__ void fill_i32_kernel(int32_t *p, int32_t v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void fill_f64_kernel(double *p, double v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// D = 2 (V + kin - omega) / tau, the diagonal of 2 Hs without the nonlocal part
__global__ void build_diag_kernel(const double *V, int64_t n, double kin, const Scalars *s,
                                  double *D64, float *D32) {
    const double om = s->omega, tau = s->tau;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double x = 2.0 * (V[i] + kin - om) / tau;
        if (D64) D64[i] = x;
        if (D32) D32[i] = (float)x;
    }
}

// ------------------------------------------------------------------------- //
// whole-domain Hamiltonian (FP64) for the Lanczos spectral bounds
// ------------------------------------------------------------------------- //
__global__ void full_apply_local_kernel(FullOp op, const double *q, double *y) {
    const int64_t n = (int64_t)op.N[0] * op.N[1] * op.N[2];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % op.N[0]);
        const int yy = (int)((i / op.N[0]) % op.N[1]);
        const int z = (int)(i / ((int64_t)op.N[0] * op.N[1]));
        const int pos[3] = {x, yy, z};
        const int64_t st[3] = {1, op.N[0], (int64_t)op.N[0] * op.N[1]};
        double s = (op.kin + op.V[i]) * q[i];
        for (int a = 0; a < 3; ++a) {
            for (int p = 1; p <= op.r; ++p) {
                const double off = -0.5 * op.w[p] * op.ih2[a];
                int t = pos[a] + p;
                if (op.periodic) {
                    if (t >= op.N[a]) t -= op.N[a];
                    s += off * q[i + (t - pos[a]) * st[a]];
                } else if (t < op.N[a]) {
                    s += off * q[i + p * st[a]];
                }
                t = pos[a] - p;
                if (op.periodic) {
                    if (t < 0) t += op.N[a];
                    s += off * q[i + (t - pos[a]) * st[a]];
                } else if (t >= 0) {
                    s += off * q[i - p * st[a]];
                }
            }
        }
        y[i] = s;
    }
}

// cp[J][l] = h^3 c_Jl (chi_Jl . q); one block per atom
__global__ void full_proj_dot_kernel(FullOp op, const double *q, double *cp) {
    __shared__ double sh[16];
    const int J = blockIdx.x;
    const int64_t s0 = op.sup_off[J], s1 = op.sup_off[J + 1];
    double acc[NP] = {0, 0, 0, 0};
    for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
        const double v = q[op.sup_idx[s]];
#pragma unroll
        for (int l = 0; l < NP; ++l) acc[l] += op.chi[s * NP + l] * v;
    }
#pragma unroll
    for (int l = 0; l < NP; ++l) {
        const double t = block_sum(acc[l], sh);
        if (threadIdx.x == 0) cp[J * NP + l] = op.h3 * op.cJ[J * NP + l] * t;
    }
}

// y[x] += sum over (atom, support row) at x of sum_l chi cp  (point-major table)
__global__ void full_proj_scatter_kernel(FullOp op, const double *cp, double *y) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < op.n_upts;
         u += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int64_t e = op.pt_off[u]; e < op.pt_off[u + 1]; ++e) {
            const int64_t row = op.pt_row[e];
            const int J = op.pt_atom[e];
#pragma unroll
            for (int l = 0; l < NP; ++l) s += op.chi[row * NP + l] * cp[J * NP + l];
        }
        y[op.pt_idx[u]] += s;
    }
}

__global__ void lz_init_kernel(double *q, double *qp, int64_t n, uint64_t seed, double *partial) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = splitmix_uniform(seed, (uint64_t)i);
        q[i] = v;
        qp[i] = 0.0;
        acc += v * v;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void lz_scale_kernel(double *q, int64_t n, const double *partial, int np) {
    __shared__ double sh[16];
    const double nrm = sqrt(ordered_sum(partial, np, sh));
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        q[i] /= nrm;
}

__global__ void lz_dot_kernel(const double *a, const double *b, int64_t n, double *partial) {
    __shared__ double sh[16];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        acc += a[i] * b[i];
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// alpha_j = q.y;  y -= alpha_j q + beta_{j-1} qp;  partial2 = |y|^2
__global__ void lz_update_kernel(double *y, const double *q, const double *qp, int64_t n,
                                 const double *partial, int np, double *alpha, double *beta,
                                 int j, double *partial2) {
    __shared__ double sh[16];
    const double al = ordered_sum(partial, np, sh);
    const double be = j > 0 ? beta[j - 1] : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) alpha[j] = al;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double v = y[i] - al * q[i] - be * qp[i];
        y[i] = v;
        acc += v * v;
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial2[blockIdx.x] = t;
}

// beta_j = |y|;  qp = q;  q = y / beta_j
__global__ void lz_next_kernel(double *q, double *qp, const double *y, int64_t n,
                               const double *partial2, int np, double *beta, int j) {
    __shared__ double sh[16];
    double be = sqrt(ordered_sum(partial2, np, sh));
    if (blockIdx.x == 0 && threadIdx.x == 0) beta[j] = be;
    const double inv = be > 0.0 ? 1.0 / be : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        qp[i] = q[i];
        q[i] = y[i] * inv;
    }
}

// number of eigenvalues of the tridiagonal (alpha, beta) below x (Sturm count)
__device__ int sturm_count(const double *al, const double *be, int m, double x) {
    int c = 0;
    double d = 1.0;
    for (int i = 0; i < m; ++i) {
        const double b2 = i ? be[i - 1] * be[i - 1] : 0.0;
        d = al[i] - x - (i ? b2 / d : 0.0);
        if (d == 0.0) d = -DBL_MIN;
        if (d < 0.0) ++c;
    }
    return c;
}

// extreme eigenvalues of the Lanczos matrix by Sturm bisection, then the
// widened bounds and the scaling of Section 2.2
__global__ void lz_finish_kernel(const double *al, const double *be, int m, double margin,
                                 Scalars *s) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double glo = 1e300, ghi = -1e300;
    for (int i = 0; i < m; ++i) {
        const double r = (i ? fabs(be[i - 1]) : 0.0) + (i + 1 < m ? fabs(be[i]) : 0.0);
        glo = fmin(glo, al[i] - r);
        ghi = fmax(ghi, al[i] + r);
    }
    double lo = glo, hi = ghi;
    for (int it = 0; it < 200; ++it) {          // smallest: count(x) >= 1
        const double mid = 0.5 * (lo + hi);
        if (sturm_count(al, be, m, mid) >= 1) hi = mid; else lo = mid;
    }
    const double emin = hi;
    lo = glo;
    hi = ghi;
    for (int it = 0; it < 200; ++it) {          // largest: count(x) >= m
        const double mid = 0.5 * (lo + hi);
        if (sturm_count(al, be, m, mid) >= m) hi = mid; else lo = mid;
    }
    const double emax = lo;
    const double wdt = emax - emin;
    s->lmin = emin - margin * wdt;
    s->lmax = emax + margin * wdt;
    s->omega = 0.5 * (s->lmax + s->lmin);
    s->tau = 0.5 * (s->lmax - s->lmin);
    s->status = 0;
}

// ------------------------------------------------------------------------- //
// moments: M_k = sum_q mu_k^q, deterministic two-pass
// ------------------------------------------------------------------------- //
__global__ void moment_partial_kernel(const double *mu, int64_t n, int K, double *partial) {
    const int64_t q0 = n * blockIdx.x / gridDim.x, q1 = n * (blockIdx.x + 1) / gridDim.x;
    for (int k = threadIdx.x; k <= K; k += blockDim.x) {
        double s = 0.0;
        for (int64_t q = q0; q < q1; ++q) s += mu[q * (K + 1) + k];
        partial[(int64_t)blockIdx.x * (K + 1) + k] = s;
    }
}

__global__ void moment_final_kernel(const double *partial, int np, int K, double *M,
                                    double *M_user) {
    for (int k = threadIdx.x; k <= K; k += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < np; ++b) s += partial[(int64_t)b * (K + 1) + k];
        M[k] = s;
        if (M_user) M_user[k] = s;
    }
}

// ------------------------------------------------------------------------- //
// Fermi level (Eq. (Ne)) and coefficients (Eq. (ChebyshevWeights))
// ------------------------------------------------------------------------- //
// Chebyshev-Gauss with N_q points: c_k = (2/N_q) sum_j f(x_j) cos(k t_j).
// Then sum'_k c_k M_k = (2/N_q) sum_j f(x_j) P_j with the lambda_f-independent
// P_j = M_0/2 + sum_{k>=1} M_k cos(k t_j), so each bisection step costs O(N_q).
__global__ void fermi_init_kernel(Scalars *s, double kT, int K, double Ne, double tol,
                                  int max_iter, const double *lf_in, int nq_cap_log2) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double th = kT / s->tau;
    double need = fmax(4.0 * (K + 1), fmax(1024.0, 8.0 / th));
    int l2 = 10;
    while ((double)(1LL << l2) < need && l2 < nq_cap_log2) ++l2;
    s->nq_log2 = l2;
    s->status = SQ_OK;   // a new solve: no status from an earlier one survives
    if ((double)(1LL << l2) < need) s->status = SQ_ERR_ARG;
    s->lo = s->lmin;
    s->hi = s->lmax;
    s->ne_target = Ne;
    s->tol = tol;
    s->iters = 0;
    s->max_iter = max_iter;
    s->done = 0;
    if (max_iter == 0) {
        s->lambda_f = *lf_in;
        s->done = 1;
    }
}

__global__ void cheb_prep_kernel(const double *M, int K, const Scalars *s, double *P) {
    const int64_t N = 1LL << s->nq_log2;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N;
         j += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.5 * M[0];
        for (int k = 1; k <= K; ++k) acc += M[k] * cos_ktj(k, j, N);
        P[j] = acc;
    }
}

// One evaluation of N_e at lo (phase 0), hi (phase 1) or mid (phase 2); the
// last block to finish sums the partials in block order and updates the bracket.
__global__ void fermi_eval_kernel(Scalars *s, const double *P, double kT, int phase,
                                  double *partial, int *ticket) {
    __shared__ double sh[16];
    __shared__ int last;
    if (s->done) return;
    const double lam = phase == 0 ? s->lo : (phase == 1 ? s->hi : s->lo + 0.5 * (s->hi - s->lo));
    const double lf = (lam - s->omega) / s->tau, th = kT / s->tau;
    const int64_t N = 1LL << s->nq_log2;
    double acc = 0.0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double x = cos(M_PI * ((double)j + 0.5) / (double)N);
        acc += fermi(x, lf, th) * P[j];
    }
    const double t = block_sum(acc, sh);
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
    const double ne = 2.0 * (2.0 / (double)N) * S;
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
        if (fabs(ne - s->ne_target) < s->tol) {
            s->lambda_f = lam;
            s->done = 1;
            return;
        }
        if (ne < s->ne_target) s->lo = lam; else s->hi = lam;
        // a 4-ulp bracket or max_iter midpoints without |N_e - target| < tol:
        // the estimate is returned, flagged as not converged
        const double big = fmax(fabs(s->lo), fabs(s->hi));
        if (s->hi - s->lo < 4.0 * DBL_EPSILON * big) {
            s->lambda_f = s->lo + 0.5 * (s->hi - s->lo);
            s->done = 1;
            s->status = SQ_ERR_NOT_CONVERGED;
        } else if (s->iters >= s->max_iter) {
            s->lambda_f = lam;
            s->done = 1;
            s->status = SQ_ERR_NOT_CONVERGED;
        }
    }
}

// primed coefficients at lambda_f (c'_0 = c_0/2): c (density), d (band
// energy), and their lambda_f derivatives; one block per k
__global__ void coeff_kernel(const Scalars *s, double kT, int K, double *cp, double *dp,
                             double *dcp, double *dup) {
    __shared__ double sh[16];
    const int k = blockIdx.x;
    const double tau = s->tau, om = s->omega;
    const double lf = (s->lambda_f - om) / tau, th = kT / tau;
    const int64_t N = 1LL << s->nq_log2;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int64_t j = threadIdx.x; j < N; j += blockDim.x) {
        const double x = cos(M_PI * ((double)j + 0.5) / (double)N);
        const double ck = cos_ktj(k, j, N);
        const double z = (x - lf) / (2.0 * th);
        const double g = 0.5 * (1.0 - tanh(z));
        const double ch = cosh(z);
        const double dg = 1.0 / (4.0 * ch * ch * th * tau);   // dg/dlambda_f
        const double e = tau * x + om;
        a0 += g * ck;
        a1 += e * g * ck;
        a2 += dg * ck;
        a3 += e * dg * ck;
    }
    const double sc = (2.0 / (double)N) * (k == 0 ? 0.5 : 1.0);
    a0 = block_sum(a0, sh);
    a1 = block_sum(a1, sh);
    a2 = block_sum(a2, sh);
    a3 = block_sum(a3, sh);
    if (threadIdx.x == 0) {
        cp[k] = a0 * sc;
        dp[k] = a1 * sc;
        dcp[k] = a2 * sc;
        dup[k] = a3 * sc;
    }
}

__global__ void totals_kernel(const double *M, int K, const double *cp, const double *dp,
                              const double *dcp, const double *dup, const Scalars *s,
                              double *totals, double *lf_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0, b = 0, c = 0, d = 0;
    for (int k = 0; k <= K; ++k) {
        a += cp[k] * M[k];
        b += dp[k] * M[k];
        c += dcp[k] * M[k];
        d += dup[k] * M[k];
    }
    if (totals) {
        totals[0] = 2.0 * a;
        totals[1] = 2.0 * b;
        totals[2] = 2.0 * c;
        totals[3] = 2.0 * d;
        totals[4] = s->omega;
        totals[5] = s->tau;
        totals[6] = (double)s->iters;
        totals[7] = (double)s->status;
    }
    if (lf_out) *lf_out = s->lambda_f;
}

// Entropy, Eq. (sq): coefficients of g log g + (1 - g) log(1 - g) at the
// solved Fermi level, primed and negated, so that contracting the moments
// with them (2 sum'_k e_k mu_k) gives s^q = -2 int s dmu_q (units of k_B).
// With t = |x - lf| / th the integrand is -(t e^-t / (1 + e^-t) + log(1 + e^-t)).
__global__ void entropy_coeff_kernel(const Scalars *s, double kT, int K, double *ep) {
    __shared__ double sh[16];
    const int k = blockIdx.x;
    const double tau = s->tau, om = s->omega;
    const double lf = (s->lambda_f - om) / tau, th = kT / tau;
    const int64_t N = 1LL << s->nq_log2;
    double a = 0.0;
    for (int64_t j = threadIdx.x; j < N; j += blockDim.x) {
        const double x = cos(M_PI * ((double)j + 0.5) / (double)N);
        const double t = fabs(x - lf) / th, e = exp(-t);
        a += (t * e / (1.0 + e) + log1p(e)) * cos_ktj(k, j, N);   // minus the integrand
    }
    a = block_sum(a, sh);
    if (threadIdx.x == 0) ep[k] = a * (2.0 / (double)N) * (k == 0 ? 0.5 : 1.0);
}

// S = sum_q s^q = 2 sum'_k e_k M_k and the band free energy U - kT S
__global__ void entropy_totals_kernel(const double *M, int K, const double *ep, const double *dp,
                                      double kT, double *totals) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double S = 0.0, U = 0.0;
    for (int k = 0; k <= K; ++k) {
        S += ep[k] * M[k];
        U += dp[k] * M[k];
    }
    totals[0] = 2.0 * S;
    totals[1] = 2.0 * U - kT * 2.0 * S;
}

// rho^q = 2 sum'_k c_k mu_k^q, u^q = 2 sum'_k d_k mu_k^q  (one wave per node)
__global__ void contract_kernel(const double *mu, int64_t n, int K, const double *cp,
                                const double *dp, double *rho, double *u) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t q = wave; q < n; q += nwaves) {
        double a = 0.0, b = 0.0;
        for (int k = lane; k <= K; k += 64) {
            const double m = mu[q * (K + 1) + k];
            a += cp[k] * m;
            b += dp[k] * m;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            a += __shfl_xor(a, o, 64);
            b += __shfl_xor(b, o, 64);
        }
        if (lane == 0) {
            if (rho) rho[q] = 2.0 * a;
            if (u) u[q] = 2.0 * b;
        }
    }
}

// ------------------------------------------------------------------------- //
// host-side launch wrappers
// ------------------------------------------------------------------------- //
static int grid_for(int64_t n, int block, int cap = 2048) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t k_set_bounds(Scalars *s, double lmin, double lmax, hipStream_t st) {
    hipLaunchKernelGGL(set_bounds_kernel, dim3(1), dim3(64), 0, st, s, lmin, lmax);
    return hipGetLastError();
}

hipError_t k_fill_i32(int32_t *p, int32_t v, int n, hipStream_t st) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t k_fill_f64(double *p, double v, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t k_build_diag(const double *V, int64_t n, double kin, const Scalars *s, double *D64,
                        float *D32, hipStream_t st) {
    hipLaunchKernelGGL(build_diag_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, V, n, kin, s,
                       D64, D32);
    return hipGetLastError();
}

hipError_t k_lanczos_bounds(const FullOp &op, LanczosWork &w, int m, uint64_t seed,
                            double margin, Scalars *s, hipStream_t st) {
    const int64_t n = (int64_t)op.N[0] * op.N[1] * op.N[2];
    const int B = 256, G = w.n_partial;
    hipLaunchKernelGGL(lz_init_kernel, dim3(G), dim3(B), 0, st, w.q, w.qp, n, seed, w.partial);
    hipLaunchKernelGGL(lz_scale_kernel, dim3(G), dim3(B), 0, st, w.q, n, w.partial, G);
    for (int j = 0; j < m; ++j) {
        hipLaunchKernelGGL(full_apply_local_kernel, dim3(grid_for(n, B)), dim3(B), 0, st, op, w.q,
                           w.y);
        if (op.n_atoms > 0) {
            hipLaunchKernelGGL(full_proj_dot_kernel, dim3(op.n_atoms), dim3(256), 0, st, op, w.q,
                               w.cp);
            hipLaunchKernelGGL(full_proj_scatter_kernel, dim3(grid_for(op.n_upts, B)), dim3(B), 0,
                               st, op, w.cp, w.y);
        }
        hipLaunchKernelGGL(lz_dot_kernel, dim3(G), dim3(B), 0, st, w.q, w.y, n, w.partial);
        hipLaunchKernelGGL(lz_update_kernel, dim3(G), dim3(B), 0, st, w.y, w.q, w.qp, n,
                           w.partial, G, w.alpha, w.beta, j, w.partial2);
        if (j + 1 < m)
            hipLaunchKernelGGL(lz_next_kernel, dim3(G), dim3(B), 0, st, w.q, w.qp, w.y, n,
                               w.partial2, G, w.beta, j);
    }
    hipLaunchKernelGGL(lz_finish_kernel, dim3(1), dim3(64), 0, st, w.alpha, w.beta, m, margin, s);
    return hipGetLastError();
}

hipError_t k_moment_sum(const double *mu, int64_t n, int K, double *partial, int np, double *M,
                        double *M_user, hipStream_t st) {
    hipLaunchKernelGGL(moment_partial_kernel, dim3(np), dim3(256), 0, st, mu, n, K, partial);
    hipLaunchKernelGGL(moment_final_kernel, dim3(1), dim3(256), 0, st, partial, np, K, M, M_user);
    return hipGetLastError();
}

hipError_t k_fermi(const FermiWork &f, Scalars *s, const double *M, int K, double kT, double Ne,
                   double tol, int max_iter, const double *lf_in, hipStream_t st) {
    hipLaunchKernelGGL(fermi_init_kernel, dim3(1), dim3(64), 0, st, s, kT, K, Ne, tol, max_iter,
                       lf_in, f.nq_cap_log2);
    if (max_iter > 0) {
        hipLaunchKernelGGL(cheb_prep_kernel, dim3(1024), dim3(256), 0, st, M, K, s, f.P);
        const int G = f.n_partial;
        for (int ph = 0; ph < 2; ++ph)
            hipLaunchKernelGGL(fermi_eval_kernel, dim3(G), dim3(256), 0, st, s, f.P, kT, ph,
                               f.partial, f.ticket);
        for (int it = 0; it < max_iter; ++it)
            hipLaunchKernelGGL(fermi_eval_kernel, dim3(G), dim3(256), 0, st, s, f.P, kT, 2,
                               f.partial, f.ticket);
    }
    hipLaunchKernelGGL(coeff_kernel, dim3(K + 1), dim3(256), 0, st, s, kT, K, f.cp, f.dp, f.dcp,
                       f.dup);
    return hipGetLastError();
}

hipError_t k_totals(const FermiWork &f, const double *M, int K, const Scalars *s, double *totals,
                    double *lf_out, hipStream_t st) {
    hipLaunchKernelGGL(totals_kernel, dim3(1), dim3(64), 0, st, M, K, f.cp, f.dp, f.dcp, f.dup, s,
                       totals, lf_out);
    return hipGetLastError();
}

hipError_t k_entropy(const FermiWork &f, const double *M, int K, double kT, const Scalars *s,
                     double *totals, hipStream_t st) {
    hipLaunchKernelGGL(entropy_coeff_kernel, dim3(K + 1), dim3(256), 0, st, s, kT, K, f.ep);
    if (totals)
        hipLaunchKernelGGL(entropy_totals_kernel, dim3(1), dim3(64), 0, st, M, K, f.ep, f.dp, kT,
                           totals);
    return hipGetLastError();
}

hipError_t k_contract(const double *mu, int64_t n, int K, const double *cp, const double *dp,
                      double *rho, double *u, hipStream_t st) {
    hipLaunchKernelGGL(contract_kernel, dim3(grid_for(n * 64, 256, 8192)), dim3(256), 0, st, mu,
                       n, K, cp, dp, rho, u);
    return hipGetLastError();
}

}  // namespace sqk
