/*
 * sq_oracle.c -- plain, slow, FP64 CPU oracle of the spectral-quadrature (SQ)
 * density hot path (Ghosh & Bhattacharya, "Spectral quadrature for the first
 * principles study of crystal defects: application to magnesium").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file: only the test-suite, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header or table with the HIP library.
 *
 * Every routine follows the paper's statement of the method in the paper's
 * order; where the paper is silent the reading used is stated at the routine.
 *
 *  - finite-difference Laplacian weights: Section 3 "Discretization" (the
 *    paper defers the weights to its references; the standard central
 *    second-derivative weights of radius r are used);
 *  - Kohn-Sham Hamiltonian H = -1/2 Lap + V + V_nl: Section 2.1, the equation
 *    after the fixed point equation and the action of the nonlocal operator;
 *    the nonlocal integral becomes a grid sum with weight h1*h2*h3;
 *  - node Hamiltonian H^q: Section 3 "Hamiltonian at each grid point": the
 *    restriction of H to the region of influence around node q, i.e. the
 *    principal submatrix of H on that box (zero outside it);
 *  - scaled Hamiltonian (H - omega)/tau: Section 2.2, Clenshaw-Curtis part;
 *  - Chebyshev recurrence v_0 = e_q, v_1 = Hs v_0, v_{k+1} = 2 Hs v_k - v_{k-1}:
 *    Eq. (Chebyshev), read as v_k = T_k(Hs) e_q;
 *  - coefficients c_k = (2/pi) int g T_k / sqrt(1-x^2): Eq. (ChebyshevWeights);
 *  - pointwise density / band energy: Eqs. (rhoq), (uq) with the Chebyshev
 *    expansion f = c_0/2 + sum_{k>=1} c_k T_k;
 *  - Fermi level from the electron count: Eq. (Ne) (bisection here);
 *  - adjoint of the recurrence: reverse-mode differentiation of Eq. (Chebyshev).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC sq_oracle.c -o _liboracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t n[3];          /* Omega grid */
    double h[3];           /* spacing (bohr) */
    int32_t r;             /* FD radius (order / 2) */
    int32_t bc;            /* 0 periodic, 1 Dirichlet (clip), 2 embedded (V on Omega') */
    int32_t pad[3];        /* embedded: Omega' = Omega padded by pad nodes per side */
    int32_t n_atoms;
    int32_t n_proj;
    const int64_t *sup_off;   /* [n_atoms+1] */
    const int64_t *sup_idx;   /* [nnz] linear index in V's grid */
    const double *chi;        /* [nnz][n_proj] */
    const double *dchi;       /* [nnz][n_proj][3], may be NULL */
    const double *c;          /* [n_atoms][n_proj] */
} orc_problem;

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the node loops from here on (timing on one core or all) */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* FD weights: central second derivative, radius r (2r-th order accurate).     */
/* w_p = 2 (-1)^{p+1} (r!)^2 / (p^2 (r-p)! (r+p)!),  w_0 = -2 sum_{p>=1} w_p.   */
/* ------------------------------------------------------------------------- */
void orc_fd_weights(int r, double *w) {
    double s = 0.0;
    for (int p = 1; p <= r; ++p) {
        double ratio = 1.0;   /* (r!)^2 / ((r-p)! (r+p)!) = prod_{j=1}^{p} (r-p+j)/(r+j) */
        for (int j = 1; j <= p; ++j) ratio *= (double)(r - p + j) / (double)(r + j);
        double wp = 2.0 * ratio / ((double)p * (double)p);
        if ((p + 1) % 2) wp = -wp;
        w[p] = wp;
        s += wp;
    }
    w[0] = -2.0 * s;
}

/* ------------------------------------------------------------------------- */
/* geometry of the grid that V lives on                                        */
/* ------------------------------------------------------------------------- */
static void vgrid(const orc_problem *P, int64_t N[3]) {
    for (int a = 0; a < 3; ++a) N[a] = (int64_t)P->n[a] + 2 * (int64_t)P->pad[a];
}

/* Region of influence of node `node` (linear index in Omega) with half-widths m:
 * box origin lo (in V-grid coordinates, unwrapped), extent dim, centre position. */
static int node_box(const orc_problem *P, int64_t node, const int32_t m[3],
                    int64_t lo[3], int32_t dim[3], int32_t ctr[3]) {
    int64_t q[3];
    q[0] = node % P->n[0];
    q[1] = (node / P->n[0]) % P->n[1];
    q[2] = node / ((int64_t)P->n[0] * P->n[1]);
    for (int a = 0; a < 3; ++a) {
        if (m[a] < 0) return -1;
        if (P->bc == 0) {                        /* periodic: full box, wrapped */
            if (2 * m[a] + 1 + P->r > P->n[a]) return -1;
            lo[a] = q[a] - m[a];
            dim[a] = 2 * m[a] + 1;
            ctr[a] = m[a];
        } else if (P->bc == 1) {                 /* Dirichlet: clipped at the boundary */
            int64_t l = q[a] - m[a], u = q[a] + m[a];
            if (l < 0) l = 0;
            if (u > P->n[a] - 1) u = P->n[a] - 1;
            lo[a] = l;
            dim[a] = (int32_t)(u - l + 1);
            ctr[a] = (int32_t)(q[a] - l);
        } else {                                 /* embedded: V given on Omega' */
            if (m[a] > P->pad[a]) return -1;
            lo[a] = q[a] + P->pad[a] - m[a];
            dim[a] = 2 * m[a] + 1;
            ctr[a] = m[a];
        }
    }
    return 0;
}

/* map V-grid coordinate along axis a into box coordinate; -1 when outside */
static int64_t to_box(const orc_problem *P, const int64_t N[3], int a, int64_t g,
                      const int64_t lo[3], const int32_t dim[3]) {
    int64_t t = g - lo[a];
    if (P->bc == 0) {
        t %= N[a];
        if (t < 0) t += N[a];
    }
    return (t >= 0 && t < dim[a]) ? t : -1;
}

/* The node operator: everything the matrix-free product with H^q needs. */
typedef struct {
    int32_t dim[3];
    int64_t npts;
    int64_t ctr;          /* box index of node q */
    int64_t *gidx;        /* [npts] V-grid linear index of each box point */
    double *diag;         /* [npts] -1/2 sum_a w_0/h_a^2 + V(x) */
    /* nonlocal: for every atom touching the box, the support points inside it */
    int32_t n_at;
    int32_t *at;          /* [n_at] atom id */
    int64_t *at_off;      /* [n_at+1] */
    int64_t *bi;          /* box index of the support point */
    int64_t *si;          /* row in the projector table */
} node_op;

static void free_op(node_op *o) {
    free(o->gidx); free(o->diag); free(o->at); free(o->at_off); free(o->bi); free(o->si);
}

static int build_op(const orc_problem *P, const double *V, const double *w,
                    int64_t node, const int32_t m[3], node_op *o) {
    int64_t lo[3], N[3];
    int32_t ctr[3];
    memset(o, 0, sizeof(*o));
    if (node_box(P, node, m, lo, o->dim, ctr)) return -1;
    vgrid(P, N);
    o->npts = (int64_t)o->dim[0] * o->dim[1] * o->dim[2];
    o->ctr = ctr[0] + (int64_t)o->dim[0] * (ctr[1] + (int64_t)o->dim[1] * ctr[2]);
    o->gidx = (int64_t *)malloc(sizeof(int64_t) * o->npts);
    o->diag = (double *)malloc(sizeof(double) * o->npts);
    double kin = 0.0;
    for (int a = 0; a < 3; ++a) kin += -0.5 * w[0] / (P->h[a] * P->h[a]);
    for (int64_t k = 0; k < o->dim[2]; ++k)
        for (int64_t j = 0; j < o->dim[1]; ++j)
            for (int64_t i = 0; i < o->dim[0]; ++i) {
                int64_t g[3] = {lo[0] + i, lo[1] + j, lo[2] + k};
                for (int a = 0; a < 3; ++a) {
                    if (P->bc == 0) { g[a] %= N[a]; if (g[a] < 0) g[a] += N[a]; }
                }
                int64_t b = i + o->dim[0] * (j + o->dim[1] * k);
                int64_t gl = g[0] + N[0] * (g[1] + N[1] * g[2]);
                o->gidx[b] = gl;
                o->diag[b] = kin + V[gl];
            }
    /* support points of every atom that fall inside the box */
    o->at = (int32_t *)malloc(sizeof(int32_t) * (P->n_atoms + 1));
    o->at_off = (int64_t *)malloc(sizeof(int64_t) * (P->n_atoms + 2));
    int64_t cap = 1024, cnt = 0;
    o->bi = (int64_t *)malloc(sizeof(int64_t) * cap);
    o->si = (int64_t *)malloc(sizeof(int64_t) * cap);
    o->at_off[0] = 0;
    for (int32_t J = 0; J < P->n_atoms; ++J) {
        int64_t start = cnt;
        for (int64_t s = P->sup_off[J]; s < P->sup_off[J + 1]; ++s) {
            int64_t gl = P->sup_idx[s];
            int64_t gx = gl % N[0], gy = (gl / N[0]) % N[1], gz = gl / (N[0] * N[1]);
            int64_t bx = to_box(P, N, 0, gx, lo, o->dim);
            int64_t by = to_box(P, N, 1, gy, lo, o->dim);
            int64_t bz = to_box(P, N, 2, gz, lo, o->dim);
            if (bx < 0 || by < 0 || bz < 0) continue;
            if (cnt == cap) {
                cap *= 2;
                o->bi = (int64_t *)realloc(o->bi, sizeof(int64_t) * cap);
                o->si = (int64_t *)realloc(o->si, sizeof(int64_t) * cap);
            }
            o->bi[cnt] = bx + o->dim[0] * (by + o->dim[1] * bz);
            o->si[cnt] = s;
            ++cnt;
        }
        if (cnt > start) {
            o->at[o->n_at] = J;
            o->at_off[++o->n_at] = cnt;
        }
    }
    return 0;
}

/* out = (H^q - omega I) v / tau, matrix free (Section 3: the product with the
 * node Hamiltonian is applied without storing the matrix). */
static void apply_scaled(const orc_problem *P, const double *w, const node_op *o,
                         double omega, double tau, const double *v, double *out) {
    const int32_t d0 = o->dim[0], d1 = o->dim[1], d2 = o->dim[2];
    const int64_t st[3] = {1, d0, (int64_t)d0 * d1};
    const int32_t dims[3] = {d0, d1, d2};
    for (int32_t k = 0; k < d2; ++k)
        for (int32_t j = 0; j < d1; ++j)
            for (int32_t i = 0; i < d0; ++i) {
                const int64_t b = i + (int64_t)d0 * (j + (int64_t)d1 * k);
                const int32_t pos[3] = {i, j, k};
                double s = (o->diag[b] - omega) * v[b];
                for (int a = 0; a < 3; ++a) {
                    const double ih2 = 1.0 / (P->h[a] * P->h[a]);
                    for (int p = 1; p <= P->r; ++p) {
                        const double off = -0.5 * w[p] * ih2;
                        if (pos[a] + p < dims[a]) s += off * v[b + p * st[a]];
                        if (pos[a] - p >= 0) s += off * v[b - p * st[a]];
                    }
                }
                out[b] = s / tau;
            }
    /* nonlocal: (V_nl v)(x) = h^3 sum_J sum_lm c_Jl chi_Jlm(x) sum_x' chi_Jlm(x') v(x') */
    const double h3 = P->h[0] * P->h[1] * P->h[2];
    const int np = P->n_proj;
    for (int32_t t = 0; t < o->n_at; ++t) {
        const int32_t J = o->at[t];
        for (int l = 0; l < np; ++l) {
            double proj = 0.0;
            for (int64_t e = o->at_off[t]; e < o->at_off[t + 1]; ++e)
                proj += P->chi[o->si[e] * np + l] * v[o->bi[e]];
            proj *= h3 * P->c[(int64_t)J * np + l] / tau;
            for (int64_t e = o->at_off[t]; e < o->at_off[t + 1]; ++e)
                out[o->bi[e]] += P->chi[o->si[e] * np + l] * proj;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Chebyshev moments mu_k^q = e_q^T T_k(Hs_q) e_q via the three-term recurrence */
/* ------------------------------------------------------------------------- */
static int moments_one(const orc_problem *P, const double *V, const double *w,
                       int64_t node, const int32_t m[3], double omega, double tau,
                       int K, double *mu) {
    node_op o;
    if (build_op(P, V, w, node, m, &o)) return -1;
    double *vm = (double *)calloc(o.npts, sizeof(double));   /* v_{k-1} */
    double *vk = (double *)calloc(o.npts, sizeof(double));   /* v_k */
    double *vn = (double *)calloc(o.npts, sizeof(double));   /* v_{k+1} */
    vk[o.ctr] = 1.0;                                          /* v_0 = e_q */
    mu[0] = vk[o.ctr];
    if (K >= 1) {
        apply_scaled(P, w, &o, omega, tau, vk, vn);           /* v_1 = Hs v_0 */
        mu[1] = vn[o.ctr];
        double *t = vm; vm = vk; vk = vn; vn = t;
    }
    for (int k = 1; k < K; ++k) {                             /* v_{k+1} = 2 Hs v_k - v_{k-1} */
        apply_scaled(P, w, &o, omega, tau, vk, vn);
        for (int64_t b = 0; b < o.npts; ++b) vn[b] = 2.0 * vn[b] - vm[b];
        mu[k + 1] = vn[o.ctr];
        double *t = vm; vm = vk; vk = vn; vn = t;
    }
    free(vm); free(vk); free(vn);
    free_op(&o);
    return 0;
}

/* mu[n_nodes][K+1]; node_m may be NULL (then m_default for all nodes). */
int orc_moments(const orc_problem *P, const double *V, double lmin, double lmax,
                const int64_t *nodes, const int32_t *node_m, const int32_t *m_default,
                int64_t n_nodes, int K, double *mu) {
    double w[16];
    if (P->r < 1 || P->r > 15 || K < 0 || !(lmax > lmin)) return -1;
    orc_fd_weights(P->r, w);
    const double omega = 0.5 * (lmax + lmin), tau = 0.5 * (lmax - lmin);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t q = 0; q < n_nodes; ++q) {
        const int32_t *m = node_m ? node_m + 3 * q : m_default;
        err |= moments_one(P, V, w, nodes[q], m, omega, tau, K, mu + q * (K + 1)) ? 1 : 0;
    }
    return err ? -1 : 0;
}

/* Apply the scaled node operator once (used by the dense-matrix checks). */
int orc_apply_node(const orc_problem *P, const double *V, int64_t node, const int32_t m[3],
                   double lmin, double lmax, const double *v, double *out,
                   int32_t *dim_out, int64_t *ctr_out) {
    double w[16];
    node_op o;
    orc_fd_weights(P->r, w);
    if (build_op(P, V, w, node, m, &o)) return -1;
    for (int a = 0; a < 3; ++a) dim_out[a] = o.dim[a];
    *ctr_out = o.ctr;
    if (v && out) apply_scaled(P, w, &o, 0.5 * (lmax + lmin), 0.5 * (lmax - lmin), v, out);
    free_op(&o);
    return 0;
}

/* box geometry of a node: origin (V-grid coordinates) / extent / centre */
int orc_node_box(const orc_problem *P, int64_t node, const int32_t m[3],
                 int64_t lo[3], int32_t dim[3], int32_t ctr[3]) {
    return node_box(P, node, m, lo, dim, ctr);
}

/* ------------------------------------------------------------------------- */
/* Chebyshev coefficients, Eq. (ChebyshevWeights):                             */
/*   c_k = (2/pi) int_{-1}^{1} f(x) T_k(x) / sqrt(1 - x^2) dx                   */
/* evaluated with the N-point Chebyshev-Gauss rule, x_j = cos t_j,              */
/* t_j = pi (j + 1/2) / N:  c_k = (2/N) sum_j f(x_j) cos(k t_j),                */
/* doubling N from max(4(K+1), 1024) until the change is below 1e-15.           */
/*   kind 0: f = g  (Fermi-Dirac in scaled variables, Eq. (FermiDirac))         */
/*   kind 1: f = (tau x + omega) g         (band energy integrand, Eq. (uq))    */
/*   kind 2: f = d g / d lambda_f          (unscaled lambda_f, per Ha)          */
/*   kind 3: f = (tau x + omega) d g / d lambda_f                               */
/*   kind 4: f = g log g + (1 - g) log(1 - g)  (entropy integrand, Eq. (sq))     */
/* g(x) = 1 / (1 + exp((x - lf)/th)) = (1 - tanh((x - lf) / (2 th))) / 2.        */
/* For kind 4, with t = |x - lf| / th (the integrand is even in x - lf):          */
/*   g log g + (1 - g) log(1 - g) = -(t e^-t / (1 + e^-t) + log(1 + e^-t)).      */
/* ------------------------------------------------------------------------- */
static double integrand(int kind, double x, double lf, double th, double tau, double omega) {
    const double z = (x - lf) / (2.0 * th);
    if (kind == 4) {
        const double t = fabs(x - lf) / th, e = exp(-t);
        return -(t * e / (1.0 + e) + log1p(e));
    }
    if (kind == 0) return 0.5 * (1.0 - tanh(z));
    if (kind == 1) return (tau * x + omega) * 0.5 * (1.0 - tanh(z));
    const double ch = cosh(z);
    const double gg = 1.0 / (4.0 * ch * ch);              /* g (1 - g) */
    const double dg = gg / (th * tau);                    /* dg/dlambda_f, lambda_f unscaled */
    if (kind == 2) return dg;
    return (tau * x + omega) * dg;
}

/* The sum over j is split into a fixed number of blocks (independent of the
 * thread count) so the result does not depend on how many threads run it. */
#define CC_BLOCKS 64
static void cc_rule(int kind, double lf, double th, double tau, double omega, int K,
                    int64_t N, double *out) {
    double *part = (double *)calloc((size_t)CC_BLOCKS * (K + 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int blk = 0; blk < CC_BLOCKS; ++blk) {
        double *p = part + (size_t)blk * (K + 1);
        const int64_t j0 = N * blk / CC_BLOCKS, j1 = N * (blk + 1) / CC_BLOCKS;
        for (int64_t j = j0; j < j1; ++j) {
            const double t = M_PI * ((double)j + 0.5) / (double)N;
            const double f = integrand(kind, cos(t), lf, th, tau, omega);
            for (int k = 0; k <= K; ++k) p[k] += f * cos((double)k * t);
        }
    }
    for (int k = 0; k <= K; ++k) {
        double s = 0.0;
        for (int blk = 0; blk < CC_BLOCKS; ++blk) s += part[(size_t)blk * (K + 1) + k];
        out[k] = s * (2.0 / (double)N);
    }
    free(part);
}

/* lf_hat, th_hat: scaled Fermi level and temperature (Section 2.2). */
int64_t orc_cheb_coeffs(int kind, double lf_hat, double th_hat, double tau, double omega,
                        int K, double *out) {
    int64_t N = 4 * (int64_t)(K + 1);
    if (N < 1024) N = 1024;
    double *a = (double *)malloc(sizeof(double) * (K + 1));
    double *b = (double *)malloc(sizeof(double) * (K + 1));
    cc_rule(kind, lf_hat, th_hat, tau, omega, K, N, a);
    for (;;) {
        const int64_t N2 = 2 * N;
        cc_rule(kind, lf_hat, th_hat, tau, omega, K, N2, b);
        double d = 0.0, sc = 1.0;
        for (int k = 0; k <= K; ++k) {
            double e = fabs(b[k] - a[k]);
            if (e > d) d = e;
        }
        if (kind == 1 || kind == 3) sc = fabs(tau) + fabs(omega);   /* size of (tau x + omega) */
        if (kind == 2 || kind == 3) sc /= tau;                      /* d/dlambda_f carries 1/tau */
        N = N2;
        memcpy(a, b, sizeof(double) * (K + 1));
        if (d <= 1e-15 * sc || N >= ((int64_t)1 << 24)) break;
    }
    memcpy(out, a, sizeof(double) * (K + 1));
    free(a); free(b);
    return N;
}

/* ------------------------------------------------------------------------- */
/* pointwise fields, Eqs. (rhoq), (uq), with f ~ c_0/2 + sum_{k>=1} c_k T_k:     */
/*   rho^q = 2 (c_0 mu_0 / 2 + sum_k c_k mu_k),   u^q likewise with d_k          */
/* ------------------------------------------------------------------------- */
void orc_contract(const double *mu, int64_t n_nodes, int K, const double *c, const double *d,
                  double *rho, double *u) {
    for (int64_t q = 0; q < n_nodes; ++q) {
        const double *m = mu + q * (K + 1);
        double sr = 0.5 * c[0] * m[0], su = 0.5 * d[0] * m[0];
        for (int k = 1; k <= K; ++k) { sr += c[k] * m[k]; su += d[k] * m[k]; }
        rho[q] = 2.0 * sr;
        u[q] = 2.0 * su;
    }
}

/* N_e(lambda_f) = sum_q rho^q = 2 (c_0 M_0 / 2 + sum_k c_k M_k), M_k = sum_q mu_k^q */
double orc_electron_count(const double *M, int K, double lambda_f, double kT,
                          double lmin, double lmax) {
    const double omega = 0.5 * (lmax + lmin), tau = 0.5 * (lmax - lmin);
    double *c = (double *)malloc(sizeof(double) * (K + 1));
    orc_cheb_coeffs(0, (lambda_f - omega) / tau, kT / tau, tau, omega, K, c);
    double s = 0.5 * c[0] * M[0];
    for (int k = 1; k <= K; ++k) s += c[k] * M[k];
    free(c);
    return 2.0 * s;
}

/* Fermi level, Eq. (Ne): bisection on [lmin, lmax] for N_e(lambda_f) = target.
 * mid = lo + (hi - lo)/2; N_e(mid) < target -> lo = mid, else hi = mid;
 * stop when |N_e(mid) - target| < tol or hi - lo < 4 eps max(|lo|, |hi|).
 * Returns 0, 1 when it stops (4-ulp bracket, max_iter midpoints) without
 * |N_e - target| < tol, or -4 when the bracket does not hold the target. */
int orc_fermi_level(const double *M, int K, double kT, double lmin, double lmax,
                    double target, double tol, int max_iter, double *lambda_f, int *iters) {
    double lo = lmin, hi = lmax;
    const double nlo = orc_electron_count(M, K, lo, kT, lmin, lmax);
    const double nhi = orc_electron_count(M, K, hi, kT, lmin, lmax);
    *iters = 0;
    if (nlo > target || nhi < target) { *lambda_f = NAN; return -4; }
    double mid = lo + 0.5 * (hi - lo);
    int converged = 0;
    for (int it = 0; it < max_iter; ++it) {
        mid = lo + 0.5 * (hi - lo);
        const double ne = orc_electron_count(M, K, mid, kT, lmin, lmax);
        *iters = it + 1;
        if (fabs(ne - target) < tol) { converged = 1; break; }
        if (ne < target) lo = mid; else hi = mid;
        const double big = fabs(lo) > fabs(hi) ? fabs(lo) : fabs(hi);
        if (hi - lo < 4.0 * 2.220446049250313e-16 * big) { mid = lo + 0.5 * (hi - lo); break; }
    }
    *lambda_f = mid;
    /* 1: stopped (4-ulp bracket or max_iter midpoints) without |N_e - target| < tol */
    return converged ? 0 : 1;
}

/* ------------------------------------------------------------------------- */
/* Adjoint of the recurrence.  For a node with output y = sum_k a_k mu_k:        */
/*   vt_K = a_K e_q,  vt_k = a_k e_q + 2 Hs vt_{k+1} - vt_{k+2}  (k >= 1),        */
/*   dy/dHs = vt_1 v_0^T + 2 sum_{k=1}^{K-1} vt_{k+1} v_k^T,                     */
/*   dy/dV_j = (1/tau) [vt_1[j] v_0[j] + 2 sum_{k=1}^{K-1} vt_{k+1}[j] v_k[j]],  */
/*   dy/dR_J = (h^3/tau) sum_lm c_Jl sum_k alpha_k                              */
/*             [(vt_{k+1}.dchi)(chi.v_k) + (vt_{k+1}.chi)(dchi.v_k)],            */
/*   alpha_0 = 1, alpha_k = 2 (k >= 1).  Partial derivatives at fixed            */
/*   lambda_f, omega, tau.  dV and dR are accumulated (+=).                      */
/* ------------------------------------------------------------------------- */
static int adjoint_one(const orc_problem *P, const double *V, const double *w, int64_t node,
                       const int32_t m[3], double omega, double tau, int K, const double *a,
                       double *gV, double *dR) {
    node_op o;
    if (build_op(P, V, w, node, m, &o)) return -1;
    const int64_t n = o.npts;
    double *vs = (double *)calloc((size_t)(K + 1) * n, sizeof(double));  /* all v_k */
    double *tmp = (double *)calloc(n, sizeof(double));
    vs[o.ctr] = 1.0;
    if (K >= 1) apply_scaled(P, w, &o, omega, tau, vs, vs + n);
    for (int k = 1; k < K; ++k) {
        apply_scaled(P, w, &o, omega, tau, vs + k * n, vs + (k + 1) * n);
        for (int64_t b = 0; b < n; ++b) vs[(k + 1) * n + b] = 2.0 * vs[(k + 1) * n + b] - vs[(k - 1) * n + b];
    }
    double *t1 = (double *)calloc(n, sizeof(double));   /* vt_{k+1} */
    double *t2 = (double *)calloc(n, sizeof(double));   /* vt_{k+2} */
    double *G = (double *)calloc(n, sizeof(double));
    const double h3 = P->h[0] * P->h[1] * P->h[2];
    const int np = P->n_proj;
    if (K >= 1) t1[o.ctr] = a[K];                       /* vt_K */
    for (int k = K - 1; k >= 0; --k) {
        const double alpha = (k == 0) ? 1.0 : 2.0;
        const double *vk = vs + (int64_t)k * n;
        for (int64_t b = 0; b < n; ++b) G[b] += alpha * t1[b] * vk[b];
        if (dR && P->dchi) {
            for (int32_t t = 0; t < o.n_at; ++t) {
                const int32_t J = o.at[t];
                for (int l = 0; l < np; ++l) {
                    double A = 0.0, B = 0.0, dA[3] = {0, 0, 0}, dB[3] = {0, 0, 0};
                    for (int64_t e = o.at_off[t]; e < o.at_off[t + 1]; ++e) {
                        const double ch = P->chi[o.si[e] * np + l];
                        const double vt = t1[o.bi[e]], vv = vk[o.bi[e]];
                        A += ch * vt;
                        B += ch * vv;
                        for (int x = 0; x < 3; ++x) {
                            const double dc = P->dchi[(o.si[e] * np + l) * 3 + x];
                            dA[x] += dc * vt;
                            dB[x] += dc * vv;
                        }
                    }
                    const double f = alpha * h3 * P->c[(int64_t)J * np + l] / tau;
                    for (int x = 0; x < 3; ++x) {
                        const double g = f * (dA[x] * B + A * dB[x]);
#pragma omp atomic
                        dR[(int64_t)J * 3 + x] += g;
                    }
                }
            }
        }
        if (k >= 1) {                                  /* vt_k from vt_{k+1}, vt_{k+2} */
            apply_scaled(P, w, &o, omega, tau, t1, tmp);
            for (int64_t b = 0; b < n; ++b) tmp[b] = 2.0 * tmp[b] - t2[b];
            tmp[o.ctr] += a[k];
            double *s = t2; t2 = t1; t1 = tmp; tmp = s;
        }
    }
    for (int64_t b = 0; b < n; ++b) {
        const double g = G[b] / tau;
#pragma omp atomic
        gV[o.gidx[b]] += g;
    }
    free(vs); free(tmp); free(t1); free(t2); free(G);
    free_op(&o);
    return 0;
}

/* a: [n_nodes][K+1] cotangent coefficients; gV: V-grid sized, accumulated;
 * dR: [n_atoms][3] accumulated or NULL. */
int orc_adjoint(const orc_problem *P, const double *V, double lmin, double lmax,
                const int64_t *nodes, const int32_t *node_m, const int32_t *m_default,
                int64_t n_nodes, int K, const double *a, double *gV, double *dR) {
    double w[16];
    if (P->r < 1 || P->r > 15 || K < 1 || !(lmax > lmin)) return -1;
    orc_fd_weights(P->r, w);
    const double omega = 0.5 * (lmax + lmin), tau = 0.5 * (lmax - lmin);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t q = 0; q < n_nodes; ++q) {
        const int32_t *m = node_m ? node_m + 3 * q : m_default;
        err |= adjoint_one(P, V, w, nodes[q], m, omega, tau, K, a + q * (K + 1), gV, dR) ? 1 : 0;
    }
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------- */
/* Whole-domain Hamiltonian (unscaled), for spectral bounds.  Periodic wraps;    */
/* Dirichlet and embedded are zero outside the V grid.                          */
/* ------------------------------------------------------------------------- */
void orc_apply_full(const orc_problem *P, const double *V, const double *v, double *out) {
    double w[16];
    int64_t N[3];
    orc_fd_weights(P->r, w);
    vgrid(P, N);
    double kin = 0.0;
    for (int a = 0; a < 3; ++a) kin += -0.5 * w[0] / (P->h[a] * P->h[a]);
    const int64_t st[3] = {1, N[0], N[0] * N[1]};
#pragma omp parallel for
    for (int64_t k = 0; k < N[2]; ++k)
        for (int64_t j = 0; j < N[1]; ++j)
            for (int64_t i = 0; i < N[0]; ++i) {
                const int64_t b = i + N[0] * (j + N[1] * k);
                const int64_t pos[3] = {i, j, k};
                double s = (kin + V[b]) * v[b];
                for (int a = 0; a < 3; ++a) {
                    const double off0 = -0.5 / (P->h[a] * P->h[a]);
                    for (int p = 1; p <= P->r; ++p) {
                        const double off = off0 * w[p];
                        for (int sg = -1; sg <= 1; sg += 2) {
                            int64_t t = pos[a] + sg * p;
                            if (P->bc == 0) { t %= N[a]; if (t < 0) t += N[a]; }
                            else if (t < 0 || t >= N[a]) continue;
                            s += off * v[b + (t - pos[a]) * st[a]];
                        }
                    }
                }
                out[b] = s;
            }
    const double h3 = P->h[0] * P->h[1] * P->h[2];
    const int np = P->n_proj;
    for (int32_t J = 0; J < P->n_atoms; ++J)
        for (int l = 0; l < np; ++l) {
            double proj = 0.0;
            for (int64_t s = P->sup_off[J]; s < P->sup_off[J + 1]; ++s)
                proj += P->chi[s * np + l] * v[P->sup_idx[s]];
            proj *= h3 * P->c[(int64_t)J * np + l];
            for (int64_t s = P->sup_off[J]; s < P->sup_off[J + 1]; ++s)
                out[P->sup_idx[s]] += P->chi[s * np + l] * proj;
        }
}

/* splitmix64 (Steele, Lea & Flood 2014), used as a counter-based generator:
 * value i of stream `seed` is mix(seed + (i + 1) * 0x9E3779B97F4A7C15). */
static uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64(uint64_t seed, uint64_t i) { return splitmix64_at(seed, i); }

double orc_splitmix_uniform(uint64_t seed, uint64_t i) {   /* in [-1, 1) */
    return (double)(splitmix64_at(seed, i) >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

/* Plain Lanczos (no reorthogonalisation) on the whole-domain H from the
 * splitmix start vector; returns the tridiagonal alpha[0..m-1], beta[0..m-2]. */
int orc_lanczos(const orc_problem *P, const double *V, int m, uint64_t seed,
                double *alpha, double *beta) {
    int64_t N[3];
    vgrid(P, N);
    const int64_t n = N[0] * N[1] * N[2];
    double *q0 = (double *)calloc(n, sizeof(double));
    double *q1 = (double *)malloc(sizeof(double) * n);
    double *wv = (double *)malloc(sizeof(double) * n);
    double nrm = 0.0;
    for (int64_t i = 0; i < n; ++i) { q1[i] = orc_splitmix_uniform(seed, (uint64_t)i); nrm += q1[i] * q1[i]; }
    nrm = sqrt(nrm);
    for (int64_t i = 0; i < n; ++i) q1[i] /= nrm;
    double b = 0.0;
    for (int j = 0; j < m; ++j) {
        orc_apply_full(P, V, q1, wv);
        double a = 0.0;
        for (int64_t i = 0; i < n; ++i) a += q1[i] * wv[i];
        alpha[j] = a;
        if (j == m - 1) break;
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) { wv[i] -= a * q1[i] + b * q0[i]; s += wv[i] * wv[i]; }
        b = sqrt(s);
        beta[j] = b;
        if (b == 0.0) { for (int t = j + 1; t < m; ++t) { alpha[t] = a; beta[t - 1] = 0.0; } break; }
        for (int64_t i = 0; i < n; ++i) { q0[i] = q1[i]; q1[i] = wv[i] / b; }
    }
    free(q0); free(q1); free(wv);
    return 0;
}

/* Gershgorin interval of the whole-domain H (rows of the stencil, V and V_nl). */
void orc_gershgorin(const orc_problem *P, const double *V, double *lo, double *hi) {
    double w[16];
    int64_t N[3];
    orc_fd_weights(P->r, w);
    vgrid(P, N);
    const int64_t n = N[0] * N[1] * N[2];
    double kin = 0.0, off = 0.0;
    for (int a = 0; a < 3; ++a) {
        kin += -0.5 * w[0] / (P->h[a] * P->h[a]);
        for (int p = 1; p <= P->r; ++p) off += 2.0 * fabs(0.5 * w[p] / (P->h[a] * P->h[a]));
    }
    double *dg = (double *)calloc(n, sizeof(double));
    double *rs = (double *)calloc(n, sizeof(double));
    const double h3 = P->h[0] * P->h[1] * P->h[2];
    const int np = P->n_proj;
    for (int32_t J = 0; J < P->n_atoms; ++J) {
        for (int64_t s = P->sup_off[J]; s < P->sup_off[J + 1]; ++s)
            for (int64_t t = P->sup_off[J]; t < P->sup_off[J + 1]; ++t) {
                double e = 0.0;
                for (int l = 0; l < np; ++l) e += P->c[(int64_t)J * np + l] * P->chi[s * np + l] * P->chi[t * np + l];
                e *= h3;
                if (P->sup_idx[s] == P->sup_idx[t]) dg[P->sup_idx[s]] += e;
                else rs[P->sup_idx[s]] += fabs(e);
            }
    }
    double l = INFINITY, u = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        const double d = kin + V[i] + dg[i], r = off + rs[i];
        if (d - r < l) l = d - r;
        if (d + r > u) u = d + r;
    }
    *lo = l; *hi = u;
    free(dg); free(rs);
}
