// Declarations of the FP64 support kernels (sq_kernels.hip) used by the API.
#pragma once

#include "sq_internal.h"

namespace sqk {

// Whole-domain Hamiltonian operands (device pointers).
struct FullOp {
    int32_t N[3];
    int32_t periodic;
    int32_t r;
    double w[MAX_R + 1];
    double ih2[3];
    double kin;                 // -1/2 sum_a w_0 / h_a^2
    double h3;
    const double *V;
    int32_t n_atoms;
    const int64_t *sup_off;     // [n_atoms+1]
    const int64_t *sup_idx;     // [nnz]
    const double *chi;          // [nnz][NP]
    const double *cJ;           // [n_atoms][NP]
    // point-major view of the supports: unique points and their (row, atom)
    int64_t n_upts;
    const int64_t *pt_idx;      // [n_upts] V-grid index
    const int64_t *pt_off;      // [n_upts+1]
    const int64_t *pt_row;      // [nnz] support row
    const int32_t *pt_atom;     // [nnz] atom
};

struct LanczosWork {
    double *q, *qp, *y;         // V-grid vectors
    double *alpha, *beta;       // [max steps]
    double *partial, *partial2; // [n_partial]
    double *cp;                 // [n_atoms][NP]
    int n_partial;
};

struct FermiWork {
    double *P;                  // [2^nq_cap_log2]
    double *partial;            // [n_partial]
    int *ticket;
    double *cp, *dp, *dcp, *dup;  // [K+1] primed coefficients
    double *ep;                 // [K+1] primed entropy coefficients, negated
    int n_partial;
    int nq_cap_log2;
};

hipError_t k_set_bounds(Scalars *s, double lmin, double lmax, hipStream_t st);
hipError_t k_fill_i32(int32_t *p, int32_t v, int n, hipStream_t st);
hipError_t k_fill_f64(double *p, double v, int64_t n, hipStream_t st);
hipError_t k_build_diag(const double *V, int64_t n, double kin, const Scalars *s, double *D64,
                        float *D32, hipStream_t st);
hipError_t k_lanczos_bounds(const FullOp &op, LanczosWork &w, int m, uint64_t seed, double margin,
                            Scalars *s, hipStream_t st);
hipError_t k_moment_sum(const double *mu, int64_t n, int K, double *partial, int np, double *M,
                        double *M_user, hipStream_t st);
hipError_t k_fermi(const FermiWork &f, Scalars *s, const double *M, int K, double kT, double Ne,
                   double tol, int max_iter, const double *lf_in, hipStream_t st);
hipError_t k_totals(const FermiWork &f, const double *M, int K, const Scalars *s, double *totals,
                    double *lf_out, hipStream_t st);
hipError_t k_entropy(const FermiWork &f, const double *M, int K, double kT, const Scalars *s,
                     double *totals, hipStream_t st);
hipError_t k_contract(const double *mu, int64_t n, int K, const double *cp, const double *dp,
                      double *rho, double *u, hipStream_t st);

// Gauss quadrature (LSSGQ): per-node eigensolve of the Jacobi matrices held in
// (lam, wgt) in place, the Fermi-level bisection over the rules, and the
// pointwise fields with their totals {N_e, U, S, U - kT S, omega, tau, iters,
// status}.
hipError_t k_gauss_eig(double *lam, double *wgt, int64_t n, int K, const Scalars *s,
                       int32_t *status, hipStream_t st);
hipError_t k_gauss_fermi(const FermiWork &f, Scalars *s, const double *lam, const double *wgt,
                         int64_t nk, double kT, double Ne, double tol, int max_iter,
                         const double *lf_in, hipStream_t st);
hipError_t k_gauss_fields(const double *lam, const double *wgt, int64_t n, int K, double kT,
                          const Scalars *s, double *rho, double *u, double *sq, double *partial,
                          int n_partial, double *totals, double *lf_out, hipStream_t st);

}  // namespace sqk
