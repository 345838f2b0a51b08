// sq_fermi_level_noalloc: the Fermi-level solve of sq_fermi_level on
// caller-given moment sums, with its scratch in a static device array instead
// of a context's workspace, so that it allocates nothing (and needs no
// sq_setup).  It runs the same kernels as sq_fermi_level.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "sq_kernels.h"

namespace {

using namespace sqk;

constexpr int NA_MAX_K = 512;        // largest Chebyshev degree
constexpr int NA_NQ_LOG2 = 20;       // largest Chebyshev-Gauss rule: 2^20 points
constexpr int NA_PARTIAL = 512;      // blocks of the bisection's reductions
constexpr int NA_MAX_DEVICES = 64;

// layout of the scratch array (8.6 MB)
struct NoAllocScratch {
    Scalars s;                       // bracket, scaling and status of the solve
    int32_t ticket;                  // last-block ticket of the reductions (zeroed per call)
    int32_t pad_[63];
    double partial[NA_PARTIAL];
    double cp[NA_MAX_K + 1], dp[NA_MAX_K + 1], dcp[NA_MAX_K + 1], dup[NA_MAX_K + 1];
    double ep[NA_MAX_K + 1];
    double P[(size_t)1 << NA_NQ_LOG2];   // lambda_f-independent sums of the rule
};

// Every GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` is only a stand-in for the symbol: the device address
// comes from hipGetSymbolAddress, per device, and only that address is used.
static __device__ __align__(256) unsigned char scratch[sizeof(NoAllocScratch)];

std::mutex g_mu;
void *g_scratch_ptr[NA_MAX_DEVICES] = {};

sq_status fail(sq_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return set_error(st, buf);
}

// device address of this device's scratch, resolved once per device with that
// device current
sq_status scratch_for_current_device(NoAllocScratch **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SQ_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= NA_MAX_DEVICES) return fail(SQ_ERR_ARG, "device %d not supported", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SQ_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<NoAllocScratch *>(g_scratch_ptr[dev]);
    return SQ_OK;
}

}  // namespace

extern "C" sq_status sq_fermi_level_noalloc(const double *M, int32_t K, double lambda_min,
                                            double lambda_max, double kT, double Ne_target,
                                            double tol_Ne, int32_t max_iter, double *lambda_f,
                                            double *coef, double *totals, void *stream) {
    if (!M || !lambda_f) return fail(SQ_ERR_ARG, "M and lambda_f must not be NULL");
    if (K < 1 || K > NA_MAX_K) return fail(SQ_ERR_ARG, "K = %d not in [1, %d]", K, NA_MAX_K);
    if (!(kT > 0.0)) return fail(SQ_ERR_ARG, "kT must be > 0");
    if (!(lambda_max > lambda_min && std::isfinite(lambda_min) && std::isfinite(lambda_max)))
        return fail(SQ_ERR_SPECTRUM, "need finite lambda_max > lambda_min");
    if (max_iter < 0 || max_iter > 100000) return fail(SQ_ERR_ARG, "max_iter out of range");
    if (max_iter > 0 && !(tol_Ne >= 0.0)) return fail(SQ_ERR_ARG, "tol_Ne must be >= 0");
    // Chebyshev-Gauss points of the coefficient rule: the power of two >=
    // max(4 (K+1), 1024, 8 / theta), theta = kT / tau (as sq_fermi_level)
    const double theta = kT / (0.5 * (lambda_max - lambda_min));
    const double need = std::fmax(4.0 * (K + 1), std::fmax(1024.0, 8.0 / theta));
    if (need > (double)(1LL << NA_NQ_LOG2))
        return fail(SQ_ERR_ARG, "kT / tau = %.3e needs %.0f quadrature points; the "
                    "no-allocation solve holds at most 2^%d", theta, need, NA_NQ_LOG2);
    NoAllocScratch *sc = nullptr;
    const sq_status ss = scratch_for_current_device(&sc);
    if (ss != SQ_OK) return ss;
    hipStream_t st = static_cast<hipStream_t>(stream);
    FermiWork f{};
    f.P = sc->P;
    f.partial = sc->partial;
    f.ticket = &sc->ticket;
    const int64_t K1 = K + 1;
    f.cp = coef ? coef : sc->cp;
    f.dp = coef ? coef + K1 : sc->dp;
    f.dcp = coef ? coef + 2 * K1 : sc->dcp;
    f.dup = coef ? coef + 3 * K1 : sc->dup;
    f.ep = sc->ep;
    f.n_partial = NA_PARTIAL;
    f.nq_cap_log2 = NA_NQ_LOG2;
    hipError_t e;
    // the ticket must start at zero; a fill kernel (not a memset) keeps the call
    // safe to capture into a graph
    if ((e = k_fill_i32(&sc->ticket, 0, 1, st)) != hipSuccess ||
        (e = k_set_bounds(&sc->s, lambda_min, lambda_max, st)) != hipSuccess ||
        (e = k_fermi(f, &sc->s, M, K, kT, Ne_target, tol_Ne, max_iter, lambda_f, st)) !=
            hipSuccess ||
        (e = k_totals(f, M, K, &sc->s, totals, lambda_f, st)) != hipSuccess)
        return fail(SQ_ERR_HIP, "launch failed: %s", hipGetErrorString(e));
    return SQ_OK;
}
