// SCF outer loop: device pieces (sq_scf.hip) used by the API's host loop.
#pragma once

#include "sq_internal.h"

namespace sqk {

// V grid (Omega, or Omega' = Omega padded by pad[a] for embedded problems) and
// the FD Laplacian weights (w[0..r], Section 3)
struct ScfGrid {
    int32_t N[3];
    int32_t n[3];       // Omega
    int32_t pad[3];     // 0 for periodic grids
    int32_t r;
    int32_t periodic;
    int32_t pad_;
    double w[MAX_R + 1];
    double ih2[3];
};

// device scalars of the loop
enum {
    SC_MEAN = 0,   // sum used for a mean
    SC_RR,         // r . r of the current CG step
    SC_RRN,        // r . r after the update
    SC_PAP,        // p . A p
    SC_BB,         // |source|^2
    SC_FF,         // |F|^2 of the SCF residual
    SC_FDF,        // F . (F - F')
    SC_DFDF,       // |F - F'|^2
    SC_COUNT
};

hipError_t scf_dot(const double *x, const double *y, int64_t n, double *partial, int nb,
                   double *out, hipStream_t st);
// nx = rho^q / h^3 at the nodes of Omega (0 on the padding); src = 4 pi (nx + b),
// made zero-mean on periodic grids, 0 on the padding
hipError_t scf_source(const ScfGrid &g, const double *rho_q, const double *b, double inv_h3,
                      double *nx, double *src, const double *ones, double *partial, int nb,
                      double *sc, hipStream_t st);
// r = src - A phi, p = r, rr, |src|^2 (A = -Lap_h)
hipError_t scf_cg_start(const ScfGrid &g, const double *src, double *phi, double *r, double *p,
                        double *partial, int nb, double *sc, hipStream_t st);
hipError_t scf_cg_iter(const ScfGrid &g, double *phi, double *r, double *p, double *Ap,
                       double *partial, int nb, double *sc, hipStream_t st);
hipError_t scf_center(double *x, int64_t n, const double *ones, double *partial, int nb,
                      double *sc, hipStream_t st);
// V_out = phi + v_xc(nx) at the nodes of Omega (V_in on the padding),
// F = V_out - V_in, |F|^2
hipError_t scf_vout(const ScfGrid &g, const double *phi, const double *nx, const double *vin,
                    double *vout, double *F, double *partial, int nb, double *sc,
                    hipStream_t st);
hipError_t scf_mix(double *V, double *Vp, const double *F, double *Fp, int64_t n, double beta,
                   int anderson, double *partial, int nb, double *sc, hipStream_t st);

}  // namespace sqk
