/*
 * sq.h -- C ABI of the MI355X (gfx950) spectral-quadrature density library.
 *
 * Method: linear-scaling spectral quadrature (Ghosh & Bhattacharya, "Spectral
 * quadrature for the first principles study of crystal defects: application
 * to magnesium").  For every finite-difference node q the Kohn-Sham
 * Hamiltonian restricted to the node's region of influence (Section 3,
 * "Hamiltonian at each grid point"), scaled to [-1, 1] (Section 2.2), drives
 * the Chebyshev recurrence of Eq. (Chebyshev); the diagonal entries
 * mu_k^q = e_q^T T_k(Hs_q) e_q ("moments") are contracted with the
 * Clenshaw-Curtis coefficients of Eq. (ChebyshevWeights) into the pointwise
 * electron density and band energy of Eqs. (rhoq), (uq); the Fermi level is
 * fixed by the electron count of Eq. (Ne).
 *
 * Conventions for every entry point
 *  - Every function returns an sq_status (0 = success, < 0 = error) and never
 *    throws; sq_last_error() returns a thread-local message for the last error.
 *  - Array arguments named "device" are HIP device pointers owned by the
 *    caller; arguments named "host" are host pointers read during the call.
 *  - Grids are flattened with x fastest: idx = i + n0*(j + n1*k).
 *  - sq_density, sq_fermi_level and sq_density_backward only enqueue work on
 *    the given stream (a hipStream_t; NULL = the default stream): they never
 *    synchronise the host and never allocate, so a sequence of them can be
 *    captured into a HIP graph and replayed.  Argument errors detectable on the
 *    host are reported at the call; conditions found on the device (Fermi level
 *    not bracketed, region atom list overflow) are written to the `totals`
 *    status word and to sq_device_status().
 *  - A context is not thread-safe; use one context per stream.
 */
#ifndef SQ_H
#define SQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SQ_OK = 0,
    SQ_ERR_ARG = -1,            /* invalid argument or unsupported shape */
    SQ_ERR_HIP = -2,            /* a HIP runtime call failed */
    SQ_ERR_OOM = -3,            /* device allocation failed (sq_setup only) */
    SQ_ERR_NOT_CONVERGED = -4,  /* Fermi level not bracketed / not converged */
    SQ_ERR_SPECTRUM = -5,       /* spectral bounds invalid (lambda_max <= lambda_min) */
    SQ_ERR_STATE = -6           /* call out of order (e.g. backward before forward) */
} sq_status;

typedef enum {
    SQ_BC_PERIODIC = 0,   /* wrap; needs 2*rcut_a + 1 + r <= n_a (no self-overlap)        */
    SQ_BC_DIRICHLET = 1,  /* region clipped at the domain boundary, zero outside          */
    SQ_BC_EMBEDDED = 2    /* V given on Omega' = Omega padded by rcut_a nodes per side;   */
                          /* regions never clipped (Section 3, embedded domain Omega')    */
} sq_bc;

typedef enum {
    SQ_FP64 = 0,          /* recurrence in FP64 */
    SQ_FP32_ACC64 = 1     /* recurrence and stencil in FP32, moments and all else FP64 */
} sq_precision;

/* Problem parameters, following the paper's statement of the problem:
 * grid n_a and spacing h_a (Section 3, Discretization), FD order n_o (the
 * Laplacian's central-difference order, radius r = n_o/2), truncation of the
 * node Hamiltonian to a box of 2*rcut_a + 1 nodes per axis (Section 3, region
 * of influence), quadrature order K (Section 2.2) and smearing k_B*theta
 * (Eq. (FermiDirac)). */
typedef struct {
    int32_t n[3];        /* Omega grid, nodes per axis (>= 1)                      */
    double h[3];         /* spacing in bohr (> 0)                                   */
    int32_t fd_order;    /* even, 2..12 (radius r = fd_order/2)                     */
    int32_t bc;          /* sq_bc                                                   */
    int32_t rcut[3];     /* default region half-width in nodes per axis (>= 0)      */
    int32_t order;       /* Chebyshev degree K, 1..512                              */
    double kT;           /* smearing in Ha (> 0)                                    */
    int32_t precision;   /* sq_precision                                            */
    int32_t ckpt_every;  /* adjoint: 1 = keep every v_k of the in-flight regions     */
                         /* (no rebuild); C > 1 = checkpoint pairs every C steps and  */
                         /* rebuild v_k backwards; 0 = 1 if that pool fits in 8 GiB,  */
                         /* else 10                                                    */
    int32_t adjoint_precision;  /* sq_precision of sq_density_backward (default 0 =  */
                         /* SQ_FP64: the gradient sums cancel strongly, so FP32      */
                         /* vectors lose ~1e-4 relative at K ~ 80); both support     */
                         /* region edges <= 27 (FP64 at edge 27: V grids of at most  */
                         /* 2^29 points)                                             */
    int32_t tune;        /* launch plan when regions fall in several edge buckets   */
                         /* (9, 13, 17, 21, 27, 32): 0 = sq_setup times, on a sample */
                         /* of the regions, one launch at the largest bucket against */
                         /* one launch per bucket, each launch at 1, 1/2 and 1/4 of  */
                         /* its occupancy limit of resident workgroups per CU, and   */
                         /* keeps the fastest (cached per geometry in the process);  */
                         /* 1 = one launch per bucket at the occupancy limit;        */
                         /* 2 = one launch of one workgroup per region (the plain,   */
                         /* unbatched path, kept as the baseline of the batching)    */
} sq_params;

/* Nonlocal Kleinman-Bylander projectors (Section 2.1, the nonlocal operator
 * V_nl(x, x') = sum_J sum_lm c_Jl chi_Jlm(x) chi_Jlm(x'); its action is the
 * grid sum (V_nl f)(x) = h1 h2 h3 sum_J sum_lm c_Jl chi_Jlm(x) sum_x' chi_Jlm(x') f(x')).
 * Host arrays, copied by sq_setup.  Supports are lists of grid points. */
typedef struct {
    int32_t n_atoms;        /* >= 0                                                  */
    int32_t n_proj;         /* projectors per atom, 1..4 (e.g. s, px, py, pz)         */
    const int64_t *sup_off; /* [n_atoms+1] CSR offsets                                */
    const int64_t *sup_idx; /* [nnz] linear index in V's grid (Omega, or Omega')      */
    const double *chi;      /* [nnz][n_proj]    chi_Jlm at the support point          */
    const double *dchi;     /* [nnz][n_proj][3] d chi_Jlm / d R_J, or NULL (no dR)    */
    const double *c;        /* [n_atoms][n_proj] c_Jl (repeated over m)               */
} sq_projectors;

typedef struct sq_ctx sq_ctx;

/* Geometry and sizes of a context (filled by sq_get_info). */
typedef struct {
    int64_t n_nodes;
    int32_t order;          /* K: moments per node are K+1                             */
    int32_t vgrid[3];       /* grid V lives on (Omega, or Omega' for SQ_BC_EMBEDDED)   */
    int32_t n_atoms;
    int32_t max_region[3];  /* largest region box                                      */
    int64_t region_points;  /* sum over nodes of the region size |R_q|                 */
    int64_t workspace_bytes;/* device memory held by the context                       */
    int32_t n_launches;     /* persistent region launches per pass (the launch plan)   */
    int32_t forward_blocks; /* resident forward workgroups summed over those launches  */
    int64_t n_force_nodes;  /* nodes inside some projector support (sq_nonlocal_force) */
    int64_t force_region_points; /* sum of their region sizes                          */
} sq_info;

/* Builds a context: validates parameters, builds the region work list and
 * uploads projector tables.  The only call that allocates device memory and
 * synchronises.
 *   params      host, required.
 *   proj        host, NULL for a local-only Hamiltonian.
 *   nodes       host [n_nodes] linear node indices in Omega, or NULL = every
 *               node of Omega in linear order (then n_nodes must be n0*n1*n2).
 *   node_rcut   host [n_nodes][3] per-node half-widths, or NULL = params->rcut.
 *   out         receives the context (NULL on failure).
 * Errors: SQ_ERR_ARG (bad shapes, region larger than supported, periodic box
 * overlapping itself), SQ_ERR_OOM, SQ_ERR_HIP. */
sq_status sq_setup(const sq_params *params, const sq_projectors *proj, const int64_t *nodes,
                   const int32_t *node_rcut, int64_t n_nodes, sq_ctx **out);

/* Releases the context and its device memory (waits for its work). */
sq_status sq_destroy(sq_ctx *ctx);

const char *sq_last_error(void);

sq_status sq_get_info(const sq_ctx *ctx, sq_info *info);

/* Forward pass: Section 2.2 scaling, Eq. (Chebyshev) recurrence on every node
 * region, moments mu_k^q and their sum M_k = sum_q mu_k^q (the per-process
 * sum before the global reduction of Eq. (Ne)).
 *   V            device, FP64, the local potential on V's grid (read only).
 *   lambda_min,
 *   lambda_max   spectral bounds of the whole-domain H used for the scaling
 *                omega = (max+min)/2, tau = (max-min)/2; pass NaN, NaN to
 *                estimate them on the device (FP64 Lanczos on the whole-domain
 *                H, widened by 1% of the width on each side).
 *   moments      device [n_nodes][K+1] FP64 output, or NULL (kept internally);
 *                a caller buffer must stay valid until the next sq_density on
 *                this context, because sq_fermi_level contracts it.
 *   moment_sum   device [K+1] FP64 output, or NULL.
 *   stream       hipStream_t.
 * The context keeps the scaled diagonal and the bounds for sq_fermi_level and
 * sq_density_backward. */
sq_status sq_density(sq_ctx *ctx, const double *V, double lambda_min, double lambda_max,
                     double *moments, double *moment_sum, void *stream);

/* Fermi level and pointwise fields, Eqs. (Ne), (rhoq), (uq).
 * Bisection on [lambda_min, lambda_max] for N_e(lambda_f) = Ne_target with
 * N_e = 2 (c_0 M_0/2 + sum_k c_k M_k); mid = lo + (hi-lo)/2, lo = mid when
 * N_e(mid) < target, stop when |N_e(mid) - target| < tol_Ne or the bracket
 * is below 4 eps.  max_iter == 0 skips the solve and uses *lambda_f as given.
 *   lambda_f  device scalar FP64: output (input when max_iter == 0).
 *   rho, u    device [n_nodes] FP64 outputs (electrons per node and band
 *             energy per node), or NULL.
 *   totals    device [8] FP64 output: {N_e, U, dN_e/dlambda_f, dU/dlambda_f,
 *             omega, tau, iterations, status} with status 0 or SQ_ERR_*.
 * Device status (totals[7] and sq_device_status): SQ_ERR_NOT_CONVERGED when
 * [lambda_min, lambda_max] does not bracket the target (lambda_f = NaN), or
 * when the bisection stops at max_iter midpoints or at a 4-eps bracket
 * without |N_e - target| < tol_Ne (lambda_f = the last estimate); every new
 * solve starts from SQ_OK.
 * Requires a preceding sq_density on the same context. */
sq_status sq_fermi_level(sq_ctx *ctx, double Ne_target, double tol_Ne, int32_t max_iter,
                         double *lambda_f, double *rho, double *u, double *totals,
                         void *stream);

/* Electronic entropy, Eq. (sq), and the band part of the free energy, from the
 * moments of the last sq_density at the Fermi level of the last
 * sq_fermi_level:
 *   s^q = -2 int s(lambda) dmu_q,  s = g log g + (1 - g) log(1 - g),
 * evaluated like rho^q with the Chebyshev coefficients of s (Eq.
 * (ChebyshevWeights)); s^q is in units of k_B and is >= 0 up to the
 * quadrature error.  The paper's free-energy expression writes the entropy
 * term as -2 theta s^q with s^q already carrying -2 k_B; this library takes
 * the band free energy as sum_q (u^q - kT s^q).
 *   s       device [n_nodes] FP64 output, or NULL.
 *   totals  device [2] FP64 output {S = sum_q s^q, U - kT S}, or NULL.
 * Requires sq_density and sq_fermi_level on the same context before it. */
sq_status sq_entropy(sq_ctx *ctx, double *s, double *totals, void *stream);

/* Adjoint (reverse mode) of the forward pass at fixed lambda_f, omega, tau:
 * for y = sum_q (g_rho[q] rho^q + g_u[q] u^q) accumulates
 *   dV[x] += dy/dV(x)          (V's grid, FP64)
 *   dR[J] += dy/dR_J           ([n_atoms][3] FP64, gradient through chi(x - R_J);
 *                                the nonlocal force is its negative)
 * by the reverse Chebyshev recurrence; v_k comes back from stored vectors
 * (ckpt_every = 1) or is rebuilt backwards from checkpoints (ckpt_every > 1).
 *   g_rho, g_u  device [n_nodes] FP64 cotangents (either may be NULL = 0).
 *   dV          device, accumulated (+=), or NULL.
 *   dR          device, accumulated (+=), or NULL; needs dchi at setup.
 * Requires sq_density and sq_fermi_level on the same context before it. */
sq_status sq_density_backward(sq_ctx *ctx, const double *g_rho, const double *g_u, double *dV,
                              double *dR, void *stream);

/* Spectral Gauss quadrature (LSSGQ), Section 2.2: K-point Gauss rule of the
 * local spectral measure of every node from K steps of Eq. (Lanczos) on the
 * node Hamiltonian (K = params.order), started at e_q without
 * reorthogonalisation.  The rule's nodes are the eigenvalues of the node's
 * K x K Jacobi matrix (lambda = tau theta + omega) and its weights the squared
 * first components of the normalised eigenvectors (the paper's text swaps the
 * two symbols; this is the Golub-Welsch reading).  A Krylov space that closes
 * before K steps (b_{k+1} <= 1e-14) gives the shorter exact rule: the last
 * node is repeated and its extra weights are 0.  The Lanczos vectors run in
 * params.precision; a_k, b_k and the eigensolve are FP64.
 *   V            device, FP64, the local potential on V's grid (read only).
 *   lambda_min,
 *   lambda_max   scaling bounds as in sq_density (NaN, NaN: device estimate).
 *   nodes,
 *   weights      device [n_nodes][K] FP64 outputs, both given or both NULL
 *                (kept internally); they hold the rules that
 *                sq_gauss_fermi_level reads, so caller buffers must stay valid
 *                until then.  Nodes of a row ascend.
 * The first call with NULL outputs allocates 2 n_nodes K doubles, and every
 * context's first call a small partial-sum buffer; later calls allocate
 * nothing.  Invalidates the state of sq_density / sq_fermi_level (both share
 * the scaling), so sq_entropy and sq_density_backward need a new sq_density.
 * Eigensolve failures (none expected) show in sq_device_status as
 * SQ_ERR_NOT_CONVERGED. */
sq_status sq_gauss_density(sq_ctx *ctx, const double *V, double lambda_min, double lambda_max,
                           double *nodes, double *weights, void *stream);

/* Fermi level and pointwise fields from the Gauss rules of the last
 * sq_gauss_density, Eqs. (Ne), (rhoq), (uq), (sq):
 *   N_e = 2 sum_q sum_k w_k g(lambda_k),   rho^q = 2 sum_k w_k g(lambda_k),
 *   u^q = 2 sum_k w_k lambda_k g(lambda_k),
 *   s^q = -2 sum_k w_k (g log g + (1 - g) log(1 - g))  (units of k_B),
 * g = 1 / (1 + exp((lambda - lambda_f) / kT)).  Bisection as in
 * sq_fermi_level, except that lambda_f is the last midpoint evaluated on
 * every stop.  max_iter == 0 uses *lambda_f as given.
 *   lambda_f       device scalar FP64: output (input when max_iter == 0).
 *   rho, u, s      device [n_nodes] FP64 outputs, or NULL.
 *   totals         device [8] FP64 output: {N_e, U, S, U - kT S, omega, tau,
 *                  iterations, status}, or NULL.
 * Device status as in sq_fermi_level (not bracketed, or stopped without
 * |N_e - target| < tol_Ne: SQ_ERR_NOT_CONVERGED).
 * Requires a preceding sq_gauss_density on the same context. */
sq_status sq_gauss_fermi_level(sq_ctx *ctx, double Ne_target, double tol_Ne, int32_t max_iter,
                               double *lambda_f, double *rho, double *u, double *s,
                               double *totals, void *stream);

/* Nonlocal atomic force by the spectral Clenshaw-Curtis quadrature, Eq.
 * (NLforceSQ) in the discrete form of Section 3:
 *   f_J,nl = -4 sum_q e_q^T V_J^q grad_h (sum'_k c_k v_k^q),
 * with v_k^q the Chebyshev vectors of the node's region (Eq. (Chebyshev)), c_k
 * the Fermi-function coefficients at the Fermi level of the last
 * sq_fermi_level (c_0 halved), grad_h the radius-r central first-derivative
 * stencil, w_p = (-1)^{p+1} (r!)^2 / (p (r-p)! (r+p)!), on the region box with
 * zero outside it, and e_q^T V_J^q f = h1 h2 h3 sum_lm c_Jl chi_Jlm(q)
 * (chi_Jlm . f) over the box.  Only nodes inside some projector support
 * contribute; sq_setup lists them.  The recurrence runs in params.precision;
 * the contraction and the accumulation are FP64.
 *   f_nl  device [n_atoms][3] FP64 output (overwritten).
 * Errors: SQ_ERR_STATE without sq_density and sq_fermi_level before it,
 * SQ_ERR_ARG without projectors. */
sq_status sq_nonlocal_force(sq_ctx *ctx, double *f_nl, void *stream);

/* SCF outer loop (Section 3's flowchart) on a periodic cell or an embedded
 * region, every node of Omega a quadrature node (sq_setup with nodes == NULL):
 *   V_in -> sq_density, sq_fermi_level (rho^q, lambda_f) -> n = rho^q / (h1 h2 h3)
 *   -> phi of Eq. (Poisson), -Lap_h phi = 4 pi (n + b) with the FD Laplacian at
 *      the nodes of Omega, by conjugate gradients: periodic cells remove the
 *      source's mean and return phi of zero mean (warm-started from the last
 *      phi); embedded regions hold phi = phi_bc on the padding of Omega' (the
 *      paper's Dirichlet values from the surrounding crystal; the padding,
 *      rcut, must be at least the FD radius deep) and start from phi_bc
 *   -> V_out = phi + v_xc(n) (LDA: Slater exchange and the Perdew-Wang 1992
 *      correlation, unpolarised) at the nodes of Omega; embedded regions keep
 *      V_in on the padding -> F = V_out - V_in
 *   -> stop when RMS(F) over the nodes of Omega < tol, else mix: V_in + beta F
 *      on the first step, then
 *      Anderson with the previous pair, g = F.(F - F') / |F - F'|^2,
 *      V_in <- (V_in - g (V_in - V')) + beta (F - g (F - F')).
 * CG (the operator is symmetric positive definite: on zero-mean functions for
 * periodic cells) stands in for the paper's GMRES.  The loop synchronises the stream at
 * every CG check and SCF test; the first call allocates 11 V-grid vectors of
 * workspace. */
typedef struct {
    double beta;            /* mixing parameter (> 0)                                   */
    double tol;             /* stop when the RMS of V_out - V_in is below tol (Ha)      */
    double fermi_tol;       /* |N_e(lambda_f) - Ne| tolerance of every Fermi solve      */
    double poisson_rtol;    /* CG stop: |residual| / |source| below this                */
    int32_t max_iter;       /* SCF iterations (>= 1)                                    */
    int32_t anderson;       /* 1: Anderson after the first step; 0: linear throughout   */
    int32_t poisson_max_iter; /* CG steps per solve (>= 1)                              */
    int32_t pad_;
} sq_scf_params;

typedef struct {
    int32_t iterations;         /* SCF iterations run                                   */
    int32_t converged;          /* 1 when RMS(V_out - V_in) < tol                       */
    int32_t poisson_iterations; /* CG steps over all solves                             */
    int32_t poisson_converged;  /* 1 when every solve reached poisson_rtol              */
    double residual;            /* RMS(V_out - V_in) of the last iteration              */
    double poisson_relres;      /* largest final relative CG residual                   */
} sq_scf_info;

/*   b         device [n_V] FP64 pseudocharge density of the nuclei on V's grid (a
 *             periodic cell: sum b h^3 = -Ne for neutrality; its mean is removed
 *             with n's).
 *   phi_bc    device [n_V] FP64: embedded regions, the electrostatic potential
 *             whose padding values are the Dirichlet data; NULL for periodic cells.
 *   Ne        electron count of every Fermi solve.
 *   lambda_min,
 *   lambda_max  scaling bounds held for the whole loop (NaN, NaN: re-estimated on
 *             the device at every iteration).
 *   V         device [n_V] FP64: the starting V_in on entry; on return the last
 *             V_in (the converged effective potential when info->converged).
 *   rho       device [n_nodes] FP64 output: rho^q of the last iteration, or NULL.
 *   lambda_f  device scalar FP64 output, or NULL.
 *   info      host output.
 * Errors: SQ_ERR_ARG for a Dirichlet-clipped context, a node list, an embedded
 * context without phi_bc or with padding shallower than the FD radius, or bad params;
 * SQ_ERR_NOT_CONVERGED from a Fermi solve; loop non-convergence is reported in
 * info, not as an error. */
sq_status sq_scf(sq_ctx *ctx, const double *b, const double *phi_bc, double Ne,
                 double lambda_min, double lambda_max, const sq_scf_params *params, double *V,
                 double *rho, double *lambda_f, sq_scf_info *info, void *stream);

/* The Fermi-level solve of sq_fermi_level, without a context and without any
 * allocation: for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Given
 * the moment sums M_k of a density pass (sq_density's moment_sum) and the
 * scaling bounds that pass used, it bisects N_e(lambda_f) = 2 (c_0 M_0/2 +
 * sum_k c_k M_k) = Ne_target exactly as sq_fermi_level does (same kernels, same
 * rule, same Chebyshev-Gauss rule for the coefficients) and gives the same
 * lambda_f and totals.  Its scratch (bracket, partial sums, the rule's sums) is
 * one static array of 8.6 MB per GPU, kept until the process ends.
 *   M            device [K+1] FP64 moment sums (read only).
 *   K            Chebyshev degree, 1..512.
 *   lambda_min,
 *   lambda_max   the bounds the moments were scaled with (finite, max > min).
 *   kT           smearing in Ha (> 0); kT / tau must leave the coefficient rule
 *                at most 2^20 points (8 / (kT / tau) <= 2^20), else SQ_ERR_ARG.
 *   Ne_target, tol_Ne, max_iter   as in sq_fermi_level (max_iter 0: *lambda_f
 *                is an input and no bisection runs).
 *   lambda_f     device scalar FP64, output (input when max_iter == 0).
 *   coef         device [4][K+1] FP64 output {c', d', dc'/dlambda_f,
 *                dd'/dlambda_f} (c'_0 = c_0/2), or NULL.
 *   totals       device [8] FP64 output as in sq_fermi_level, or NULL.
 * Every call on a GPU uses that GPU's one scratch array: calls that overlap on
 * one GPU (two streams, two threads) race and must be serialised by the
 * caller.  Host-detectable argument errors return at the call; the device
 * status goes to totals[7]. */
sq_status sq_fermi_level_noalloc(const double *M, int32_t K, double lambda_min, double lambda_max,
                                 double kT, double Ne_target, double tol_Ne, int32_t max_iter,
                                 double *lambda_f, double *coef, double *totals, void *stream);

/* Synchronises the context's last stream and returns the device-side status
 * word (SQ_OK, SQ_ERR_NOT_CONVERGED, SQ_ERR_ARG on region atom-list overflow). */
sq_status sq_device_status(sq_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SQ_H */
