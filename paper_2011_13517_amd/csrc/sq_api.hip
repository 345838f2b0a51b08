// C ABI of libsq: context setup (work list, projector tables, workspaces) and
// the host side of sq_density / sq_fermi_level / sq_density_backward.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "sq_force.h"
#include "sq_scf.h"
#include "sq_kernels.h"

using namespace sqk;

namespace {

thread_local std::string g_err;

sq_status fail(sq_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(SQ_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));          \
    } while (0)

constexpr int LANCZOS_STEPS = 100;
constexpr double LANCZOS_MARGIN = 0.01;
constexpr uint64_t LANCZOS_SEED = 0x5EEDULL;
constexpr int NQ_CAP_LOG2 = 22;
#ifndef SQ_N_PARTIAL
#define SQ_N_PARTIAL 512   // blocks of the deterministic grid reductions
#endif
constexpr int N_PARTIAL = SQ_N_PARTIAL;

// central second-derivative weights of radius r (the paper's FD Laplacian,
// Section 3): w_p = 2 (-1)^{p+1} (r!)^2 / (p^2 (r-p)! (r+p)!), w_0 = -2 sum w_p
void fd_weights(int r, double *w) {
    double s = 0.0;
    for (int p = 1; p <= r; ++p) {
        double f = 1.0;
        for (int j = 1; j <= p; ++j) f *= double(r - p + j) / double(r + j);
        w[p] = ((p % 2) ? 2.0 : -2.0) * f / double(p * p);
        s += w[p];
    }
    w[0] = -2.0 * s;
}

// central first-derivative weights of radius r (the FD gradient of Section 3):
// w_p = (-1)^{p+1} (r!)^2 / (p (r-p)! (r+p)!), applied as sum_p w_p (f_{+p} - f_{-p}) / h
void fd_first_weights(int r, double *w) {
    w[0] = 0.0;
    for (int p = 1; p <= r; ++p) {
        double f = 1.0;
        for (int j = 1; j <= p; ++j) f *= double(r - p + j) / double(r + j);
        w[p] = ((p % 2) ? 1.0 : -1.0) * f / double(p);
    }
}

}  // namespace

// error reporting for entry points defined in other sources of the library
namespace sqk {
sq_status set_error(sq_status st, const char *msg) {
    g_err = msg;
    return st;
}
}  // namespace sqk

// A launch group: a contiguous range of the sorted work list run by one
// persistent kernel instantiated for edge bucket E.
struct Group {
    int E = 0;
    bool maskz = false;
    int begin = 0, count = 0;
    int grid_fwd = 1, grid_adj = 1;
    int grid_gauss = 0;   // set on the first Gauss sweep
    int bpc = 0;          // resident forward workgroups per CU (0: the occupancy limit)
};
enum { PLAN_MERGED = 0, PLAN_SPLIT = 1, PLAN_PER_REGION = 2 };

static int item_bucket(const Item &it) {
    return edge_bucket(std::max(it.dim[0], std::max(it.dim[1], it.dim[2])));
}

// groups of a sorted work list: one group at the largest bucket (merged), one
// group per edge bucket (split), or one launch of one workgroup per region (the
// plain, unbatched path)
static std::vector<Group> make_groups(const std::vector<Item> &items, int plan) {
    std::vector<Group> g;
    const int n = (int)items.size();
    if (plan == PLAN_PER_REGION) {
        for (int i = 0; i < n; ++i) {
            Group gr;
            gr.begin = i;
            gr.count = 1;
            gr.E = item_bucket(items[i]);
            gr.maskz = items[i].dim[2] != gr.E;
            g.push_back(gr);
        }
        return g;
    }
    for (int i = 0; i < n;) {
        Group gr;
        gr.begin = i;
        gr.E = item_bucket(items[i]);
        int j = i;
        while (j < n && (plan == PLAN_MERGED || item_bucket(items[j]) == gr.E)) {
            gr.E = std::max(gr.E, item_bucket(items[j]));
            ++j;
        }
        gr.count = j - i;
        for (int q = i; q < j; ++q)
            if (items[q].dim[2] != gr.E) gr.maskz = true;
        g.push_back(gr);
        i = j;
    }
    return g;
}

// plans measured by the tuner, per geometry (process-wide): the plan and the
// resident forward workgroups per CU of each edge bucket
struct TuneChoice {
    int plan = 1;
    std::map<int, int> bpc;
};
static std::mutex g_tune_mu;
static std::map<std::string, TuneChoice> g_tune_cache;

// persistent grid of a group: its resident workgroups per CU (the occupancy
// limit, or the tuner's smaller choice) times the CUs, at most one per region
static void set_forward_grid(int prec, int r, int ncu, Group &g) {
    const int occ = forward_blocks_per_cu(prec, g.E, r, g.maskz);
    const int b = g.bpc > 0 ? std::min(g.bpc, occ) : occ;
    g.grid_fwd = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)b * ncu, g.count));
}

struct sq_ctx {
    sq_params p{};
    int r = 1;
    double w[MAX_R + 1] = {};
    double ih2[3] = {}, kin = 0, h3 = 0;
    int N[3] = {};
    int64_t nv = 0;
    int periodic = 0;
    int64_t n_nodes = 0;
    int K = 0;
    int prec = 0;
    int aprec = 0;   // precision of the adjoint
    int E = 0;                    // largest edge bucket of the work list
    std::vector<Group> groups;    // launch plan: one persistent launch per group
    int plan = 0;                 // PLAN_MERGED, PLAN_SPLIT or PLAN_PER_REGION
    std::map<int, int> tuned_bpc; // tuner: resident forward workgroups per CU, by edge bucket
    int max_region[3] = {};
    int64_t region_points = 0;
    int64_t bytes = 0;
    // device
    std::vector<void *> allocs;
    Item *d_items = nullptr;
    int n_items = 0;
    int32_t *d_counter = nullptr;
    int32_t *d_status = nullptr;
    Scalars *d_scal = nullptr;
    float *d_D32 = nullptr;
    double *d_D64 = nullptr;
    double *d_mu = nullptr;       // internal moments
    const double *mu_last = nullptr;
    double *d_M = nullptr;
    double *d_mpartial = nullptr;
    int n_mpart = 0;
    // projectors
    int n_atoms = 0, n_proj = 0;
    bool have_dchi = false;
    AtomDev *d_atoms = nullptr;
    int32_t *d_pack = nullptr;
    float *d_chi32 = nullptr, *d_dchi32 = nullptr;
    double *d_chi64 = nullptr, *d_dchi64 = nullptr;
    double *d_cJ = nullptr;
    double *d_chi_full = nullptr;   // caller's row order, whole-domain operator
    int32_t *d_colidx = nullptr;
    int64_t *d_sup_off = nullptr, *d_sup_idx = nullptr;
    int64_t n_upts = 0;
    int64_t *d_pt_idx = nullptr, *d_pt_off = nullptr, *d_pt_row = nullptr;
    int32_t *d_pt_atom = nullptr;
    LanczosWork lz{};
    FermiWork fw{};
    // adjoint
    bool adj_ok = false;
    bool adj_grid_ok = true;   // V grid within the FP64 edge-27 kernel's offset range
    bool storeall = false;
    int n_ckpt = 1;
    int64_t ckpt_stride = 0;
    void *d_ckpt = nullptr;
    bool have_density = false, have_fermi = false;
    // Gauss quadrature: rules of the last sq_gauss_density (caller's buffers
    // or the internal ones, allocated on first use) and field partials
    double *d_glam = nullptr, *d_gwgt = nullptr, *d_gpart = nullptr;
    double *glam_last = nullptr, *gwgt_last = nullptr;
    bool have_gauss = false;
    // nonlocal force: the regions of nodes inside some projector support
    Item *d_fitems = nullptr;
    std::vector<Group> fgroups;
    int64_t n_force_nodes = 0, force_region_points = 0;
    // SCF loop: every node of Omega in linear order; workspace on first use
    bool all_nodes = false;
    double *d_scf = nullptr, *d_scf_part = nullptr, *d_scf_sc = nullptr;
    double *d_scf_rho = nullptr, *d_scf_lf = nullptr;
    hipStream_t last_stream = nullptr;

    template <typename T>
    sq_status alloc(T **ptr, size_t n) {
        *ptr = nullptr;
        if (n == 0) n = 1;
        void *q = nullptr;
        const hipError_t e = hipMalloc(&q, n * sizeof(T));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(SQ_ERR_OOM, "hipMalloc of %zu bytes failed: %s", n * sizeof(T),
                        hipGetErrorString(e));
        }
        allocs.push_back(q);
        bytes += (int64_t)(n * sizeof(T));
        *ptr = static_cast<T *>(q);
        return SQ_OK;
    }
    template <typename T>
    sq_status upload(T **ptr, const T *src, size_t n) {
        sq_status st = alloc(ptr, n);
        if (st) return st;
        if (n) {
            const hipError_t e = hipMemcpy(*ptr, src, n * sizeof(T), hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(SQ_ERR_HIP, "hipMemcpy: %s", hipGetErrorString(e));
        }
        return SQ_OK;
    }
    ~sq_ctx() {
        for (void *q : allocs) (void)hipFree(q);
    }
};

namespace {

#define TRY(expr)                    \
    do {                             \
        sq_status s_ = (expr);       \
        if (s_ != SQ_OK) return s_;  \
    } while (0)

sq_status validate(const sq_params *p) {
    if (!p) return fail(SQ_ERR_ARG, "params is NULL");
    for (int a = 0; a < 3; ++a) {
        if (p->n[a] < 1) return fail(SQ_ERR_ARG, "n[%d] = %d must be >= 1", a, p->n[a]);
        if (!(p->h[a] > 0.0)) return fail(SQ_ERR_ARG, "h[%d] must be > 0", a);
        if (p->rcut[a] < 0) return fail(SQ_ERR_ARG, "rcut[%d] must be >= 0", a);
    }
    if (p->fd_order < 2 || p->fd_order > 2 * MAX_R || p->fd_order % 2)
        return fail(SQ_ERR_ARG, "fd_order %d must be even in [2, %d]", p->fd_order, 2 * MAX_R);
    if (p->bc < 0 || p->bc > 2) return fail(SQ_ERR_ARG, "bc %d unknown", p->bc);
    if (p->order < 1 || p->order > 512) return fail(SQ_ERR_ARG, "order %d not in [1, 512]", p->order);
    if (!(p->kT > 0.0)) return fail(SQ_ERR_ARG, "kT must be > 0");
    if (p->precision != SQ_FP64 && p->precision != SQ_FP32_ACC64)
        return fail(SQ_ERR_ARG, "precision %d unknown", p->precision);
    if (p->ckpt_every < 0) return fail(SQ_ERR_ARG, "ckpt_every must be >= 0");
    if (p->adjoint_precision != SQ_FP64 && p->adjoint_precision != SQ_FP32_ACC64)
        return fail(SQ_ERR_ARG, "adjoint_precision %d unknown", p->adjoint_precision);
    if (p->tune < 0 || p->tune > 2) return fail(SQ_ERR_ARG, "tune %d unknown", p->tune);
    return SQ_OK;
}

// unwrapped bounding box of a set of coordinates on a ring of n cells
void ring_bbox(std::vector<int> &c, int n, bool periodic, int *lo, int *dim) {
    if (!periodic) {
        const auto mm = std::minmax_element(c.begin(), c.end());
        *lo = *mm.first;
        *dim = *mm.second - *mm.first + 1;
        return;
    }
    std::vector<char> occ(n, 0);
    for (int x : c) occ[x] = 1;
    // the support starts right after the longest circular run of empty cells
    int best_len = -1, best_end = 0;
    for (int s = 0; s < n; ++s) {
        if (occ[s] || !occ[(s + n - 1) % n]) continue;   // not the start of an empty run
        int len = 0;
        while (len < n && !occ[(s + len) % n]) ++len;
        if (len > best_len) {
            best_len = len;
            best_end = (s + len) % n;
        }
    }
    if (best_len <= 0) {   // fills the ring
        *lo = 0;
        *dim = n;
        return;
    }
    *lo = best_end;
    int mx = 0;
    for (int x : c) mx = std::max(mx, ((x - best_end) % n + n) % n);
    *dim = mx + 1;
}

template <typename T>
void fill_region_args(const sq_ctx &c, RegionArgs<T> &a) {
    for (int x = 0; x < 3; ++x) {
        a.N[x] = c.N[x];
        a.ih2[x] = c.ih2[x];
    }
    a.periodic = c.periodic;
    a.scal = c.d_scal;
    for (int p = 0; p <= MAX_R; ++p) a.w[p] = c.w[p];
    a.h3 = c.h3;
    a.K = c.K;
    a.n_atoms = c.n_atoms;
    a.atoms = c.d_atoms;
    a.sup_pack = c.d_pack;
    a.colidx = c.d_colidx;
    a.cJ = c.d_cJ;
    a.status = c.d_status;
    if constexpr (sizeof(T) == 8) {
        a.D = c.d_D64;
        a.chi = c.d_chi64;
        a.dchi = c.d_dchi64;
    } else {
        a.D = c.d_D32;
        a.chi = c.d_chi32;
        a.dchi = c.d_dchi32;
    }
}

// forward recurrence of every group of a plan (one persistent launch each,
// its own work counter)
template <typename T>
sq_status run_forward_t(const sq_ctx &c, const std::vector<Group> &groups, const Item *items,
                        double *mu, hipStream_t st) {
    HIP_TRY(k_fill_i32(c.d_counter, 0, (int64_t)groups.size(), st));
    for (size_t g = 0; g < groups.size(); ++g) {
        RegionArgs<T> a{};
        fill_region_args(c, a);
        a.items = items + groups[g].begin;
        a.n_items = groups[g].count;
        a.counter = c.d_counter + g;
        a.moments = mu;
        HIP_TRY(launch_forward(c.prec, groups[g].E, c.r, groups[g].maskz, &a, groups[g].grid_fwd, st));
    }
    return SQ_OK;
}

sq_status run_forward(const sq_ctx &c, const std::vector<Group> &groups, const Item *items,
                      double *mu, hipStream_t st) {
    return c.prec == SQ_FP64 ? run_forward_t<double>(c, groups, items, mu, st)
                             : run_forward_t<float>(c, groups, items, mu, st);
}

// Launch-plan tuner.  On an evenly strided sample of at most 8192 regions
// (same bucket mix), with a zero potential (the cost does not depend on the
// values), it times for every launch group of the merged and of the split plan
// the persistent grid at the occupancy limit and at one half and one quarter
// of it (fewer resident workgroups per CU trade latency hiding for less
// contention on the LDS, L2 and the work counter), keeps each group's fastest
// grid, and then the plan whose groups sum to less.  The choice (plan and
// workgroups per CU of each edge bucket) is cached per geometry key, which
// includes the CU count and each bucket's occupancy limit, for the process.
sq_status tune_plan(sq_ctx &c, const std::vector<Item> &items, int ncu) {
    std::string key;
    {
        std::map<int, int64_t> hist;
        for (const Item &it : items) hist[item_bucket(it)] += 1;
        char buf[160];
        std::snprintf(buf, sizeof buf, "p%d r%d K%d a%d n%d bc%d cu%d", c.prec, c.r, c.K,
                      c.n_atoms, (int)items.size(), c.p.bc, ncu);
        key = buf;
        for (auto &kv : hist)
            key += " " + std::to_string(kv.first) + ":" + std::to_string(kv.second) + "/" +
                   std::to_string(forward_blocks_per_cu(c.prec, kv.first, c.r, true));
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto f = g_tune_cache.find(key);
        if (f != g_tune_cache.end()) {
            c.plan = f->second.plan;
            c.tuned_bpc = f->second.bpc;
            return SQ_OK;
        }
    }
    const int n = (int)items.size();
    const int stride = std::max(1, n / 8192);
    std::vector<Item> sample;
    for (int i = 0; i < n; i += stride) {
        Item it = items[i];
        it.out = (int32_t)sample.size();
        sample.push_back(it);
    }
    Item *d_sample = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&d_sample), sample.size() * sizeof(Item)) != hipSuccess)
        return fail(SQ_ERR_OOM, "tuner: hipMalloc failed");
    std::vector<Group> plans[2] = {make_groups(sample, PLAN_MERGED), make_groups(sample, PLAN_SPLIT)};
    Scalars s{};
    s.omega = 0.0;
    s.tau = 1.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    sq_status st = SQ_OK;
    if (hipMemcpy(d_sample, sample.data(), sample.size() * sizeof(Item), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(c.d_scal, &s, sizeof(s), hipMemcpyHostToDevice) != hipSuccess ||
        (c.d_D64 && hipMemset(c.d_D64, 0, c.nv * sizeof(double)) != hipSuccess) ||
        (c.d_D32 && hipMemset(c.d_D32, 0, c.nv * sizeof(float)) != hipSuccess) ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = fail(SQ_ERR_HIP, "tuner setup failed");
    }
    // one group at one grid: an untimed run (first grid only), then a timed one
    auto time_group = [&](const Group &g, bool warm, float *ms) -> sq_status {
        const std::vector<Group> one{g};
        sq_status t = SQ_OK;
        if (warm) t = run_forward(c, one, d_sample, c.d_mu, nullptr);
        if (t == SQ_OK && hipEventRecord(e0, nullptr) != hipSuccess) t = fail(SQ_ERR_HIP, "event");
        if (t == SQ_OK) t = run_forward(c, one, d_sample, c.d_mu, nullptr);
        if (t == SQ_OK && (hipEventRecord(e1, nullptr) != hipSuccess ||
                           hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(ms, e0, e1) != hipSuccess))
            t = fail(SQ_ERR_HIP, "tuner timing failed");
        return t;
    };
    float best = -1.0f;
    TuneChoice choice;
    for (int pl = 0; pl < 2 && st == SQ_OK; ++pl) {
        float total = 0.0f;
        std::map<int, int> bpc;
        for (Group &g : plans[pl]) {
            const int occ = forward_blocks_per_cu(c.prec, g.E, c.r, g.maskz);
            float gbest = -1.0f;
            int gb = occ;
            for (int b : {occ, occ / 2, occ / 4}) {
                if (st != SQ_OK || b < 1 || (b != occ && b == gb)) continue;
                if (b != occ && (int64_t)b * ncu >= g.count && (int64_t)gb * ncu >= g.count)
                    continue;   // both grids already cover every region of the group
                g.bpc = b;
                set_forward_grid(c.prec, c.r, ncu, g);
                float ms = 0.0f;
                st = time_group(g, b == occ, &ms);
                if (st == SQ_OK && (gbest < 0.0f || ms < gbest)) {
                    gbest = ms;
                    gb = b;
                }
            }
            total += gbest > 0.0f ? gbest : 0.0f;
            bpc[g.E] = gb;
        }
        if (st == SQ_OK && (best < 0.0f || total < best)) {
            best = total;
            choice.plan = pl == 0 ? PLAN_MERGED : PLAN_SPLIT;
            choice.bpc = bpc;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipDeviceSynchronize();
    (void)hipFree(d_sample);
    if (hipMemset(c.d_scal, 0, sizeof(Scalars)) != hipSuccess ||
        hipMemset(c.d_status, 0, sizeof(int32_t)) != hipSuccess)
        return fail(SQ_ERR_HIP, "tuner reset failed");
    if (st != SQ_OK) return st;
    c.plan = choice.plan;
    c.tuned_bpc = choice.bpc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = choice;
    return SQ_OK;
}

// spectral bounds (given, or both NaN: device Lanczos estimate) and the
// scaled diagonal of V
sq_status prepare_operator(sq_ctx &c, const double *V, double lambda_min, double lambda_max,
                           hipStream_t st) {
    const bool estimate = std::isnan(lambda_min) && std::isnan(lambda_max);
    if (!estimate && !(lambda_max > lambda_min && std::isfinite(lambda_min) &&
                       std::isfinite(lambda_max)))
        return fail(SQ_ERR_SPECTRUM, "need lambda_max > lambda_min (or both NaN)");
    if (estimate) {
        FullOp op{};
        for (int a = 0; a < 3; ++a) {
            op.N[a] = c.N[a];
            op.ih2[a] = c.ih2[a];
        }
        op.periodic = c.periodic;
        op.r = c.r;
        for (int p = 0; p <= MAX_R; ++p) op.w[p] = c.w[p];
        op.kin = c.kin;
        op.h3 = c.h3;
        op.V = V;
        op.n_atoms = c.n_atoms;
        op.sup_off = c.d_sup_off;
        op.sup_idx = c.d_sup_idx;
        op.chi = c.d_chi_full;
        op.cJ = c.d_cJ;
        op.n_upts = c.n_upts;
        op.pt_idx = c.d_pt_idx;
        op.pt_off = c.d_pt_off;
        op.pt_row = c.d_pt_row;
        op.pt_atom = c.d_pt_atom;
        HIP_TRY(k_lanczos_bounds(op, c.lz, LANCZOS_STEPS, LANCZOS_SEED, LANCZOS_MARGIN, c.d_scal, st));
    } else {
        HIP_TRY(k_set_bounds(c.d_scal, lambda_min, lambda_max, st));
    }
    HIP_TRY(k_build_diag(V, c.nv, c.kin, c.d_scal, c.d_D64, c.d_D32, st));
    return SQ_OK;
}

}  // namespace

extern "C" {

const char *sq_last_error(void) { return g_err.c_str(); }

sq_status sq_setup(const sq_params *params, const sq_projectors *proj, const int64_t *nodes,
                   const int32_t *node_rcut, int64_t n_nodes, sq_ctx **out) {
    if (!out) return fail(SQ_ERR_ARG, "out is NULL");
    *out = nullptr;
    TRY(validate(params));
    auto ctx = new (std::nothrow) sq_ctx;
    if (!ctx) return fail(SQ_ERR_OOM, "host allocation failed");
    sq_ctx &c = *ctx;
    auto bail = [&](sq_status st) {
        delete ctx;
        return st;
    };
    c.p = *params;
    if (c.p.ckpt_every == 0) c.p.ckpt_every = 10;
    c.r = c.p.fd_order / 2;
    fd_weights(c.r, c.w);
    c.kin = 0.0;
    for (int a = 0; a < 3; ++a) {
        c.ih2[a] = 1.0 / (c.p.h[a] * c.p.h[a]);
        c.kin += -0.5 * c.w[0] * c.ih2[a];
    }
    c.h3 = c.p.h[0] * c.p.h[1] * c.p.h[2];
    c.periodic = c.p.bc == SQ_BC_PERIODIC;
    int pad[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
        if (c.p.bc == SQ_BC_EMBEDDED) pad[a] = c.p.rcut[a];
        c.N[a] = c.p.n[a] + 2 * pad[a];
    }
    c.nv = (int64_t)c.N[0] * c.N[1] * c.N[2];
    c.K = c.p.order;
    c.prec = c.p.precision;
    c.aprec = c.p.adjoint_precision;
    const int64_t n_omega = (int64_t)c.p.n[0] * c.p.n[1] * c.p.n[2];
    if (!nodes) {
        if (n_nodes != n_omega)
            return bail(fail(SQ_ERR_ARG, "nodes == NULL needs n_nodes == %lld", (long long)n_omega));
    } else if (n_nodes < 1) {
        return bail(fail(SQ_ERR_ARG, "n_nodes must be >= 1"));
    }
    if (n_nodes > INT32_MAX) return bail(fail(SQ_ERR_ARG, "too many nodes"));
    c.n_nodes = n_nodes;
    c.all_nodes = nodes == nullptr && node_rcut == nullptr;

    // ---- work list -------------------------------------------------------
    std::vector<Item> items(n_nodes);
    int emax = 0;
    for (int64_t q = 0; q < n_nodes; ++q) {
        const int64_t g = nodes ? nodes[q] : q;
        if (g < 0 || g >= n_omega)
            return bail(fail(SQ_ERR_ARG, "node %lld out of range", (long long)g));
        const int pos[3] = {(int)(g % c.p.n[0]), (int)((g / c.p.n[0]) % c.p.n[1]),
                            (int)(g / ((int64_t)c.p.n[0] * c.p.n[1]))};
        Item &it = items[q];
        it.out = (int32_t)q;
        for (int a = 0; a < 3; ++a) {
            const int m = node_rcut ? node_rcut[3 * q + a] : c.p.rcut[a];
            if (m < 0) return bail(fail(SQ_ERR_ARG, "node_rcut must be >= 0"));
            if (c.p.bc == SQ_BC_PERIODIC) {
                if (2 * m + 1 + c.r > c.p.n[a])
                    return bail(fail(SQ_ERR_ARG,
                                     "periodic region of half-width %d overlaps itself on axis %d "
                                     "(needs 2*rcut+1+r <= n)", m, a));
                it.lo[a] = pos[a] - m;
                it.dim[a] = 2 * m + 1;
                it.ctr[a] = m;
            } else if (c.p.bc == SQ_BC_DIRICHLET) {
                const int l = std::max(pos[a] - m, 0), u = std::min(pos[a] + m, c.p.n[a] - 1);
                it.lo[a] = l;
                it.dim[a] = u - l + 1;
                it.ctr[a] = pos[a] - l;
            } else {
                if (m > pad[a])
                    return bail(fail(SQ_ERR_ARG, "embedded node half-width %d exceeds the padding "
                                     "%d", m, pad[a]));
                it.lo[a] = pos[a] + pad[a] - m;
                it.dim[a] = 2 * m + 1;
                it.ctr[a] = m;
            }
            emax = std::max(emax, it.dim[a]);
            c.max_region[a] = std::max(c.max_region[a], it.dim[a]);
        }
        c.region_points += (int64_t)it.dim[0] * it.dim[1] * it.dim[2];
    }
    if (emax > max_edge(c.prec))
        return bail(fail(SQ_ERR_ARG, "region edge %d exceeds the supported %d for this precision",
                         emax, max_edge(c.prec)));
    c.E = edge_bucket(emax);
    bool uniform = true;
    for (const Item &it : items) {
        if (it.dim[0] != items[0].dim[0] || it.dim[1] != items[0].dim[1] ||
            it.dim[2] != items[0].dim[2])
            uniform = false;
    }
    if (!uniform) {   // by edge bucket, then largest regions first (LPT order)
        std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) {
            const int ea = item_bucket(a), eb = item_bucket(b);
            if (ea != eb) return ea > eb;
            return (int64_t)a.dim[0] * a.dim[1] * a.dim[2] > (int64_t)b.dim[0] * b.dim[1] * b.dim[2];
        });
    }
    c.n_items = (int)n_nodes;

    // ---- projectors ------------------------------------------------------
    std::vector<AtomDev> atoms;
    std::vector<int32_t> rpack, colidx;     // region tables (see below)
    std::vector<double> rchi, rdchi;
    std::vector<double> chi64, cJ;
    std::vector<int64_t> sup_off, sup_idx;
    if (proj && proj->n_atoms > 0) {
        if (proj->n_proj < 1 || proj->n_proj > NP)
            return bail(fail(SQ_ERR_ARG, "n_proj %d not in [1, %d]", proj->n_proj, NP));
        if (!proj->sup_off || !proj->sup_idx || !proj->chi || !proj->c)
            return bail(fail(SQ_ERR_ARG, "projector tables incomplete"));
        c.n_atoms = proj->n_atoms;
        c.n_proj = proj->n_proj;
        c.have_dchi = proj->dchi != nullptr;
        const int np = proj->n_proj;
        const int64_t nnz = proj->sup_off[proj->n_atoms];
        if (proj->sup_off[0] != 0 || nnz < 0 || nnz > INT32_MAX)
            return bail(fail(SQ_ERR_ARG, "bad sup_off"));
        // the whole offset array is checked before any table is read: every
        // atom's rows must lie inside [0, nnz]
        for (int J = 0; J < proj->n_atoms; ++J)
            if (proj->sup_off[J + 1] < proj->sup_off[J] || proj->sup_off[J + 1] > nnz)
                return bail(fail(SQ_ERR_ARG, "sup_off not monotone within [0, %lld] at atom %d",
                                 (long long)nnz, J));
        atoms.resize(c.n_atoms);
        chi64.assign(nnz * NP, 0.0);
        cJ.assign((size_t)c.n_atoms * NP, 0.0);
        sup_off.assign(proj->sup_off, proj->sup_off + c.n_atoms + 1);
        sup_idx.assign(proj->sup_idx, proj->sup_idx + nnz);
        int bbmax[3] = {0, 0, 0};
        std::vector<int> cc[3];
        for (int J = 0; J < c.n_atoms; ++J) {
            const int64_t s0 = proj->sup_off[J], s1 = proj->sup_off[J + 1];
            if (s1 < s0) return bail(fail(SQ_ERR_ARG, "sup_off not monotone"));
            for (int l = 0; l < np; ++l) cJ[(size_t)J * NP + l] = proj->c[(int64_t)J * np + l];
            AtomDev &at = atoms[J];
            at.start = (int32_t)rpack.size();
            at.count = 0;
            at.col_start = (int32_t)(colidx.size() / 2);
            if (s1 == s0) {
                for (int a = 0; a < 3; ++a) { at.lo[a] = 0; at.dim[a] = 0; }
                continue;
            }
            for (int a = 0; a < 3; ++a) cc[a].clear();
            for (int64_t s = s0; s < s1; ++s) {
                const int64_t g = proj->sup_idx[s];
                if (g < 0 || g >= c.nv)
                    return bail(fail(SQ_ERR_ARG, "support index %lld out of range", (long long)g));
                cc[0].push_back((int)(g % c.N[0]));
                cc[1].push_back((int)((g / c.N[0]) % c.N[1]));
                cc[2].push_back((int)(g / ((int64_t)c.N[0] * c.N[1])));
            }
            for (int a = 0; a < 3; ++a) {
                ring_bbox(cc[a], c.N[a], c.periodic != 0, &at.lo[a], &at.dim[a]);
                if (at.dim[a] > 1023)
                    return bail(fail(SQ_ERR_ARG, "projector support too wide (%d nodes)", at.dim[a]));
                bbmax[a] = std::max(bbmax[a], at.dim[a]);
            }
            // whole-domain tables keep the caller's row order
            for (int64_t s = s0; s < s1; ++s)
                for (int l = 0; l < np; ++l) chi64[s * NP + l] = proj->chi[s * np + l];
            // region tables: the support on its box, column-major (x, y) with z
            // contiguous; a column's rows span its z range (gaps padded with
            // zero rows) so a pencil's piece of the support is one run of rows.
            const int bd[3] = {at.dim[0], at.dim[1], at.dim[2]};
            const int64_t bvol = (int64_t)bd[0] * bd[1] * bd[2];
            if (bvol > (1LL << 26)) return bail(fail(SQ_ERR_ARG, "projector support box too large"));
            std::vector<int64_t> where(bvol, -1);   // box cell -> first caller row there
            std::vector<int> zmin(bd[0] * bd[1], INT32_MAX), zmax(bd[0] * bd[1], -1);
            std::vector<int64_t> cell(s1 - s0);
            for (int64_t s = s0; s < s1; ++s) {
                int o[3];
                for (int a = 0; a < 3; ++a) {
                    int x = cc[a][s - s0] - at.lo[a];
                    if (c.periodic) x = ((x % c.N[a]) + c.N[a]) % c.N[a];
                    o[a] = x;
                }
                const int col = o[1] * bd[0] + o[0];
                zmin[col] = std::min(zmin[col], o[2]);
                zmax[col] = std::max(zmax[col], o[2]);
                const int64_t ci = (int64_t)col * bd[2] + o[2];
                cell[s - s0] = ci;
                if (where[ci] < 0) where[ci] = s;
            }
            at.start = (int32_t)(rpack.size());
            at.col_start = (int32_t)(colidx.size() / 2);
            for (int col = 0; col < bd[0] * bd[1]; ++col) {
                if (zmax[col] < 0) {
                    colidx.push_back(0);
                    colidx.push_back(0);
                    continue;
                }
                const int n = zmax[col] - zmin[col] + 1;
                colidx.push_back((int32_t)rpack.size());
                colidx.push_back(zmin[col] | (n << 16));
                for (int z = zmin[col]; z <= zmax[col]; ++z) {
                    rpack.push_back((col % bd[0]) | ((col / bd[0]) << 10) | (z << 20));
                    for (int q = 0; q < NP; ++q) rchi.push_back(0.0);
                    for (int q = 0; q < 3 * NP; ++q) rdchi.push_back(0.0);
                }
            }
            // scatter the caller's rows (rows at the same cell add up, which
            // leaves both the projections and the rank-4 term unchanged)
            for (int64_t s = s0; s < s1; ++s) {
                const int64_t ci = cell[s - s0];
                const int col = (int)(ci / bd[2]), z = (int)(ci % bd[2]);
                const int64_t row = colidx[2 * ((int64_t)at.col_start + col)] + (z - zmin[col]);
                for (int l = 0; l < np; ++l) {
                    rchi[row * NP + l] += proj->chi[s * np + l];
                    if (proj->dchi)
                        for (int x = 0; x < 3; ++x)
                            rdchi[(row * NP + l) * 3 + x] += proj->dchi[(s * np + l) * 3 + x];
                }
            }
            at.count = (int32_t)(rpack.size() - at.start);
            if (rpack.size() > (size_t)INT32_MAX / 16)
                return bail(fail(SQ_ERR_ARG, "projector tables too large"));
        }
        if (c.periodic)
            for (int a = 0; a < 3; ++a)
                if (c.max_region[a] + bbmax[a] > c.N[a])
                    return bail(fail(SQ_ERR_ARG, "region + projector support (%d + %d) exceeds the "
                                     "periodic grid (%d) on axis %d", c.max_region[a], bbmax[a],
                                     c.N[a], a));
    }

    // ---- device memory ---------------------------------------------------
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return bail(fail(SQ_ERR_HIP, "no HIP device"));
    const int64_t K1 = c.K + 1;
    sq_status st;
#define ALLOC(ptr, n)                                              \
    do {                                                           \
        if ((st = c.alloc(&(ptr), (n))) != SQ_OK) return bail(st); \
    } while (0)
#define UPLOAD(ptr, src, n)                                                 \
    do {                                                                    \
        if ((st = c.upload(&(ptr), (src), (n))) != SQ_OK) return bail(st);  \
    } while (0)
    UPLOAD(c.d_items, items.data(), items.size());
    // one work counter per launch group (one per region for the plain plan)
    ALLOC(c.d_counter, (size_t)std::max<int64_t>(64, c.p.tune == 2 ? n_nodes : 0));
    ALLOC(c.d_status, 4);
    ALLOC(c.d_scal, 1);
    if (c.prec == SQ_FP64 || c.aprec == SQ_FP64) ALLOC(c.d_D64, c.nv);
    if (c.prec == SQ_FP32_ACC64 || c.aprec == SQ_FP32_ACC64) ALLOC(c.d_D32, c.nv);
    ALLOC(c.d_mu, (size_t)(n_nodes * K1));
    ALLOC(c.d_M, K1);
    c.n_mpart = (int)std::min<int64_t>(N_PARTIAL, n_nodes);
    ALLOC(c.d_mpartial, (size_t)c.n_mpart * K1);
    if (c.n_atoms) {
        UPLOAD(c.d_atoms, atoms.data(), atoms.size());
        UPLOAD(c.d_pack, rpack.data(), rpack.size());
        UPLOAD(c.d_colidx, colidx.data(), colidx.size());
        UPLOAD(c.d_chi_full, chi64.data(), chi64.size());
        UPLOAD(c.d_cJ, cJ.data(), cJ.size());
        UPLOAD(c.d_sup_off, sup_off.data(), sup_off.size());
        UPLOAD(c.d_sup_idx, sup_idx.data(), sup_idx.size());
        if (c.prec == SQ_FP64 || c.aprec == SQ_FP64) {
            UPLOAD(c.d_chi64, rchi.data(), rchi.size());
            if (c.have_dchi) UPLOAD(c.d_dchi64, rdchi.data(), rdchi.size());
        }
        if (c.prec == SQ_FP32_ACC64 || c.aprec == SQ_FP32_ACC64) {
            std::vector<float> f(rchi.begin(), rchi.end());
            UPLOAD(c.d_chi32, f.data(), f.size());
            if (c.have_dchi) {
                std::vector<float> g(rdchi.begin(), rdchi.end());
                UPLOAD(c.d_dchi32, g.data(), g.size());
            }
        }
        // point-major view for the whole-domain operator
        const int64_t nnz = (int64_t)sup_idx.size();
        std::vector<int64_t> order(nnz);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int64_t a, int64_t b) { return sup_idx[a] < sup_idx[b]; });
        std::vector<int64_t> pt_idx, pt_off, pt_row(nnz);
        std::vector<int32_t> pt_atom(nnz);
        std::vector<int32_t> atom_of(nnz);
        for (int J = 0; J < c.n_atoms; ++J)
            for (int64_t s = sup_off[J]; s < sup_off[J + 1]; ++s) atom_of[s] = J;
        for (int64_t e = 0; e < nnz; ++e) {
            const int64_t row = order[e];
            if (e == 0 || sup_idx[row] != sup_idx[order[e - 1]]) {
                pt_idx.push_back(sup_idx[row]);
                pt_off.push_back(e);
            }
            pt_row[e] = row;
            pt_atom[e] = atom_of[row];
        }
        pt_off.push_back(nnz);
        c.n_upts = (int64_t)pt_idx.size();
        UPLOAD(c.d_pt_idx, pt_idx.data(), pt_idx.size());
        UPLOAD(c.d_pt_off, pt_off.data(), pt_off.size());
        UPLOAD(c.d_pt_row, pt_row.data(), pt_row.size());
        UPLOAD(c.d_pt_atom, pt_atom.data(), pt_atom.size());
    }
    // Lanczos and Fermi workspaces
    ALLOC(c.lz.q, c.nv);
    ALLOC(c.lz.qp, c.nv);
    ALLOC(c.lz.y, c.nv);
    ALLOC(c.lz.alpha, LANCZOS_STEPS);
    ALLOC(c.lz.beta, LANCZOS_STEPS);
    ALLOC(c.lz.partial, N_PARTIAL);
    ALLOC(c.lz.partial2, N_PARTIAL);
    ALLOC(c.lz.cp, (size_t)std::max(1, c.n_atoms) * NP);
    c.lz.n_partial = N_PARTIAL;
    ALLOC(c.fw.P, (size_t)1 << NQ_CAP_LOG2);
    ALLOC(c.fw.partial, N_PARTIAL);
    ALLOC(c.fw.ticket, 1);
    ALLOC(c.fw.cp, K1);
    ALLOC(c.fw.dp, K1);
    ALLOC(c.fw.dcp, K1);
    ALLOC(c.fw.dup, K1);
    ALLOC(c.fw.ep, K1);
    c.fw.n_partial = N_PARTIAL;
    c.fw.nq_cap_log2 = NQ_CAP_LOG2;
    if (hipMemset(c.fw.ticket, 0, sizeof(int)) != hipSuccess ||
        hipMemset(c.d_status, 0, sizeof(int32_t)) != hipSuccess ||
        hipMemset(c.d_scal, 0, sizeof(Scalars)) != hipSuccess)
        return bail(fail(SQ_ERR_HIP, "hipMemset failed"));
    // ---- launch plan -----------------------------------------------------
    // Regions of several edge buckets run either as one launch at the largest
    // bucket (small boxes leave most of a large workgroup idle) or as one
    // launch per bucket (more launches, each with its own tail).  With
    // params->tune == 0 both plans are timed here on a sample of the work
    // list and the faster one is kept (cached per geometry); otherwise the
    // split plan is used whenever there is more than one bucket.
    auto grids = [&](std::vector<Group> &gs) {
        for (Group &g : gs) {
            auto f = c.tuned_bpc.find(g.E);
            g.bpc = f != c.tuned_bpc.end() ? f->second : 0;
            set_forward_grid(c.prec, c.r, ncu, g);
        }
    };
    std::vector<Group> merged = make_groups(items, PLAN_MERGED);
    std::vector<Group> split = make_groups(items, PLAN_SPLIT);
    if ((int)split.size() > 64) return bail(fail(SQ_ERR_ARG, "too many launch groups"));
    grids(merged);
    grids(split);
    c.plan = split.size() > 1 ? PLAN_SPLIT : PLAN_MERGED;
    if (c.p.tune == 2) {
        c.plan = PLAN_PER_REGION;
        c.groups = make_groups(items, PLAN_PER_REGION);
        grids(c.groups);
    } else {
        if (split.size() > 1 && c.p.tune == 0) {
            const sq_status ts = tune_plan(c, items, ncu);
            if (ts != SQ_OK) return bail(ts);
        }
        c.groups = c.plan == PLAN_SPLIT ? split : merged;
        grids(c.groups);   // the tuner's workgroups per CU, when it ran
    }

    // nonlocal force work list: nodes where some chi_Jlm is nonzero, one
    // launch per edge bucket
    if (c.n_atoms) {
        std::vector<char> covered(c.nv, 0);
        for (int64_t g : sup_idx) covered[g] = 1;
        std::vector<Item> fitems;
        for (const Item &it : items) {
            int64_t g[3];
            for (int a = 0; a < 3; ++a) {
                g[a] = it.lo[a] + it.ctr[a];
                if (c.periodic) g[a] = ((g[a] % c.N[a]) + c.N[a]) % c.N[a];
            }
            if (covered[g[0] + (int64_t)c.N[0] * (g[1] + (int64_t)c.N[1] * g[2])]) {
                fitems.push_back(it);
                c.force_region_points += (int64_t)it.dim[0] * it.dim[1] * it.dim[2];
            }
        }
        c.n_force_nodes = (int64_t)fitems.size();
        if (!fitems.empty()) {
            UPLOAD(c.d_fitems, fitems.data(), fitems.size());
            c.fgroups = make_groups(fitems, PLAN_SPLIT);
            for (Group &g : c.fgroups) {
                if (!cc_force_supported(c.prec, g.E)) continue;
                const int occ = cc_force_blocks_per_cu(c.prec, g.E, c.r, g.maskz);
                g.grid_fwd = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)occ * ncu, g.count));
            }
        }
    }

    // adjoint: one vector slot per resident workgroup, shared by the groups
    c.adj_ok = true;
    for (const Group &g : c.groups) c.adj_ok = c.adj_ok && g.E <= adjoint_max_edge(c.aprec);
    for (const Group &g : c.groups)
        if (adjoint64_edge(c.aprec, g.E) &&
            (int64_t)c.N[0] * c.N[1] * c.N[2] > adjoint64_max_grid())
            c.adj_grid_ok = false;
    c.adj_ok = c.adj_ok && c.adj_grid_ok;
    if (c.adj_ok) {
        const bool grad = c.n_atoms > 0 && c.have_dchi;
        const int64_t esz = c.aprec == SQ_FP64 ? 8 : 4;
        // groups of the FP64 edge-27 kernel keep v_k, vt_{k+1}, the forward
        // projections and the atom list of their in-flight regions (own layout)
        auto zc = [&](const Group &g) { return adjoint64_edge(c.aprec, g.E); };
        auto agrid = [&](const Group &g, bool sa) {
            const int occ = zc(g) ? adjoint64_blocks_per_cu(g.E, c.r, grad)
                                  : adjoint_blocks_per_cu(c.aprec, g.E, c.r, sa, grad);
            return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)occ * ncu, g.count));
        };
        // stride 1 keeps every v_k of the in-flight regions (no rebuild, two
        // operator applications per step); chosen by default when that pool
        // stays below 8 GiB
        int64_t pool_sa = 0;
        for (const Group &g : c.groups)
            if (!zc(g))
                pool_sa = std::max<int64_t>(pool_sa, (int64_t)agrid(g, true) *
                                                         storeall_slot_elems(c.K, g.E) * esz);
        c.storeall = params->ckpt_every == 1 ||
                     (params->ckpt_every == 0 && pool_sa <= (int64_t)8 << 30);
        // a store-all kernel without the column projector path (never the case
        // for the supported edges, but kept well defined) rebuilds with stride 10
        if (c.storeall) c.p.ckpt_every = 10;
        c.n_ckpt = c.K >= 2 ? (c.K - 2) / c.p.ckpt_every + 1 : 1;
        c.ckpt_stride = 0;
        int max_grid = 1;
        for (Group &g : c.groups) {
            g.grid_adj = agrid(g, c.storeall);
            max_grid = std::max(max_grid, g.grid_adj);
            const int64_t e3 = (int64_t)g.E * g.E * g.E;
            // a kernel without the column projector path falls back to the
            // rebuild layout, so a store-all slot also covers that one
            int64_t st = (int64_t)c.n_ckpt * 2 * e3;
            if (c.storeall) st = std::max<int64_t>(st, storeall_slot_elems(c.K, g.E));
            if (zc(g)) st = adjoint64_slot_elems(c.K, g.E);
            c.ckpt_stride = std::max(c.ckpt_stride, st);
        }
        c.ckpt_stride = round_np(c.ckpt_stride);   // slots stay NP-vector aligned
        const size_t n = (size_t)max_grid * c.ckpt_stride;
        if (c.aprec == SQ_FP64) {
            double *q = nullptr;
            ALLOC(q, n);
            c.d_ckpt = q;
        } else {
            float *q = nullptr;
            ALLOC(q, n);
            c.d_ckpt = q;
        }
    }
#undef ALLOC
#undef UPLOAD
    if (hipDeviceSynchronize() != hipSuccess) return bail(fail(SQ_ERR_HIP, "setup sync failed"));
    *out = ctx;
    return SQ_OK;
}

sq_status sq_destroy(sq_ctx *ctx) {
    if (!ctx) return SQ_OK;
    (void)hipDeviceSynchronize();
    delete ctx;
    return SQ_OK;
}

sq_status sq_get_info(const sq_ctx *ctx, sq_info *info) {
    if (!ctx || !info) return fail(SQ_ERR_ARG, "NULL argument");
    info->n_nodes = ctx->n_nodes;
    info->order = ctx->K;
    for (int a = 0; a < 3; ++a) {
        info->vgrid[a] = ctx->N[a];
        info->max_region[a] = ctx->max_region[a];
    }
    info->n_atoms = ctx->n_atoms;
    info->region_points = ctx->region_points;
    info->workspace_bytes = ctx->bytes;
    info->n_launches = (int32_t)ctx->groups.size();
    info->forward_blocks = 0;
    for (const Group &g : ctx->groups) info->forward_blocks += g.grid_fwd;
    info->n_force_nodes = ctx->n_force_nodes;
    info->force_region_points = ctx->force_region_points;
    return SQ_OK;
}

sq_status sq_density(sq_ctx *ctx, const double *V, double lambda_min, double lambda_max,
                     double *moments, double *moment_sum, void *stream) {
    if (!ctx) return fail(SQ_ERR_ARG, "ctx is NULL");
    if (!V) return fail(SQ_ERR_ARG, "V is NULL");
    sq_ctx &c = *ctx;
    hipStream_t st = static_cast<hipStream_t>(stream);
    TRY(prepare_operator(c, V, lambda_min, lambda_max, st));
    HIP_TRY(k_fill_i32(c.d_status, 0, 1, st));
    double *mu = moments ? moments : c.d_mu;
    TRY(run_forward(c, c.groups, c.d_items, mu, st));
    HIP_TRY(k_moment_sum(mu, c.n_nodes, c.K, c.d_mpartial, c.n_mpart, c.d_M, moment_sum, st));
    c.mu_last = mu;
    c.have_density = true;
    c.have_fermi = false;
    c.have_gauss = false;
    c.last_stream = st;
    return SQ_OK;
}

sq_status sq_fermi_level(sq_ctx *ctx, double Ne_target, double tol_Ne, int32_t max_iter,
                         double *lambda_f, double *rho, double *u, double *totals, void *stream) {
    if (!ctx) return fail(SQ_ERR_ARG, "ctx is NULL");
    sq_ctx &c = *ctx;
    if (!c.have_density) return fail(SQ_ERR_STATE, "sq_fermi_level needs a preceding sq_density");
    if (!lambda_f) return fail(SQ_ERR_ARG, "lambda_f is NULL");
    if (max_iter < 0 || max_iter > 100000) return fail(SQ_ERR_ARG, "max_iter out of range");
    if (max_iter > 0 && !(tol_Ne >= 0.0)) return fail(SQ_ERR_ARG, "tol_Ne must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(k_fermi(c.fw, c.d_scal, c.d_M, c.K, c.p.kT, Ne_target, tol_Ne, max_iter, lambda_f, st));
    HIP_TRY(k_totals(c.fw, c.d_M, c.K, c.d_scal, totals, lambda_f, st));
    if (rho || u) HIP_TRY(k_contract(c.mu_last, c.n_nodes, c.K, c.fw.cp, c.fw.dp, rho, u, st));
    c.have_fermi = true;
    c.last_stream = st;
    return SQ_OK;
}

sq_status sq_entropy(sq_ctx *ctx, double *s, double *totals, void *stream) {
    if (!ctx) return fail(SQ_ERR_ARG, "ctx is NULL");
    sq_ctx &c = *ctx;
    if (!c.have_fermi)
        return fail(SQ_ERR_STATE, "sq_entropy needs sq_density and sq_fermi_level first");
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(k_entropy(c.fw, c.d_M, c.K, c.p.kT, c.d_scal, totals, st));
    if (s) HIP_TRY(k_contract(c.mu_last, c.n_nodes, c.K, c.fw.ep, c.fw.ep, s, nullptr, st));
    c.last_stream = st;
    return SQ_OK;
}

sq_status sq_density_backward(sq_ctx *ctx, const double *g_rho, const double *g_u, double *dV,
                              double *dR, void *stream) {
    if (!ctx) return fail(SQ_ERR_ARG, "ctx is NULL");
    sq_ctx &c = *ctx;
    if (!c.have_fermi)
        return fail(SQ_ERR_STATE, "sq_density_backward needs sq_density and sq_fermi_level first");
    if (!c.adj_grid_ok)
        return fail(SQ_ERR_ARG, "the FP64 adjoint of edge-%d regions supports V grids of up to "
                    "%lld points (this context: %lld)", c.E, (long long)adjoint64_max_grid(),
                    (long long)c.N[0] * c.N[1] * c.N[2]);
    if (!c.adj_ok)
        return fail(SQ_ERR_ARG, "the %s adjoint supports region edges up to %d (this context: %d)",
                    c.aprec == SQ_FP64 ? "FP64" : "FP32", adjoint_max_edge(c.aprec), c.E);
    if (dR && !(c.n_atoms > 0 && c.have_dchi))
        return fail(SQ_ERR_ARG, "dR needs projector tables with dchi");
    if (!dV && !dR) return SQ_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool grad = dR != nullptr;
    HIP_TRY(k_fill_i32(c.d_counter, 0, (int64_t)c.groups.size(), st));
    auto launch = [&](auto tag) -> sq_status {
        using T = decltype(tag);
        for (size_t g = 0; g < c.groups.size(); ++g) {
            const Group &gr = c.groups[g];
            AdjointArgs<T> a{};
            fill_region_args(c, a.g);
            a.g.items = c.d_items + gr.begin;
            a.g.n_items = gr.count;
            a.g.counter = c.d_counter + g;
            a.g.moments = nullptr;
            a.coef_c = c.fw.cp;
            a.coef_d = c.fw.dp;
            a.g_rho = g_rho;
            a.g_u = g_u;
            a.dV = dV;
            a.dR = dR;
            a.ckpt = static_cast<T *>(c.d_ckpt);
            a.ckpt_every = c.p.ckpt_every;
            a.n_ckpt = c.n_ckpt;
            a.ckpt_stride = c.ckpt_stride;
            if (adjoint64_edge(c.aprec, gr.E))
                HIP_TRY(launch_adjoint64(gr.E, c.r, grad, &a, gr.grid_adj, st));
            else
                HIP_TRY(launch_adjoint(c.aprec, gr.E, c.r, c.storeall, grad, &a, gr.grid_adj, st));
        }
        return SQ_OK;
    };
    if (c.aprec == SQ_FP64) TRY(launch(double{}));
    else TRY(launch(float{}));
    c.last_stream = st;
    return SQ_OK;
}

sq_status sq_gauss_density(sq_ctx *ctx, const double *V, double lambda_min, double lambda_max,
                           double *nodes, double *weights, void *stream) {
    if (!ctx) return fail(SQ_ERR_ARG, "ctx is NULL");
    if (!V) return fail(SQ_ERR_ARG, "V is NULL");
    if ((nodes == nullptr) != (weights == nullptr))
        return fail(SQ_ERR_ARG, "nodes and weights must both be given or both be NULL");
    sq_ctx &c = *ctx;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t nk = (size_t)c.n_nodes * (size_t)c.K;
    if (!c.d_gpart) TRY(c.alloc(&c.d_gpart, 3 * (size_t)N_PARTIAL));
    if (!nodes && !c.d_glam) {
        TRY(c.alloc(&c.d_glam, nk));
        TRY(c.alloc(&c.d_gwgt, nk));
    }
    double *L = nodes ? nodes : c.d_glam, *W = nodes ? weights : c.d_gwgt;
    int ncu = 0;
    for (Group &g : c.groups) {
        if (g.grid_gauss) continue;
        if (!ncu) {
            int dev = 0;
            HIP_TRY(hipGetDevice(&dev));
            HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        }
        const int occ = gauss_lanczos_blocks_per_cu(c.prec, g.E, c.r, g.maskz);
        g.grid_gauss = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)occ * ncu, g.count));
    }
    TRY(prepare_operator(c, V, lambda_min, lambda_max, st));
    HIP_TRY(k_fill_i32(c.d_status, 0, 1, st));
    HIP_TRY(k_fill_i32(c.d_counter, 0, (int64_t)c.groups.size(), st));
    auto sweep = [&](auto tag) -> sq_status {
        using T = decltype(tag);
        for (size_t g = 0; g < c.groups.size(); ++g) {
            RegionArgs<T> a{};
            fill_region_args(c, a);
            a.items = c.d_items + c.groups[g].begin;
            a.n_items = c.groups[g].count;
            a.counter = c.d_counter + g;
            a.moments = nullptr;
            HIP_TRY(launch_gauss_lanczos(c.prec, c.groups[g].E, c.r, c.groups[g].maskz, &a, L, W,
                                         c.groups[g].grid_gauss, st));
        }
        return SQ_OK;
    };
    if (c.prec == SQ_FP64) TRY(sweep(double{}));
    else TRY(sweep(float{}));
    HIP_TRY(k_gauss_eig(L, W, c.n_nodes, c.K, c.d_scal, c.d_status, st));
    c.glam_last = L;
    c.gwgt_last = W;
    c.have_gauss = true;
    c.have_density = false;
    c.have_fermi = false;
    c.last_stream = st;
    return SQ_OK;
}

sq_status sq_gauss_fermi_level(sq_ctx *ctx, double Ne_target, double tol_Ne, int32_t max_iter,
                               double *lambda_f, double *rho, double *u, double *s,
                               double *totals, void *stream) {
    if (!ctx) return fail(SQ_ERR_ARG, "ctx is NULL");
    sq_ctx &c = *ctx;
    if (!c.have_gauss)
        return fail(SQ_ERR_STATE, "sq_gauss_fermi_level needs a preceding sq_gauss_density");
    if (!lambda_f) return fail(SQ_ERR_ARG, "lambda_f is NULL");
    if (max_iter < 0 || max_iter > 100000) return fail(SQ_ERR_ARG, "max_iter out of range");
    if (max_iter > 0 && !(tol_Ne >= 0.0)) return fail(SQ_ERR_ARG, "tol_Ne must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nk = c.n_nodes * (int64_t)c.K;
    HIP_TRY(k_gauss_fermi(c.fw, c.d_scal, c.glam_last, c.gwgt_last, nk, c.p.kT, Ne_target, tol_Ne,
                          max_iter, lambda_f, st));
    HIP_TRY(k_gauss_fields(c.glam_last, c.gwgt_last, c.n_nodes, c.K, c.p.kT, c.d_scal, rho, u, s,
                           c.d_gpart, N_PARTIAL, totals, lambda_f, st));
    c.last_stream = st;
    return SQ_OK;
}

sq_status sq_nonlocal_force(sq_ctx *ctx, double *f_nl, void *stream) {
    if (!ctx) return fail(SQ_ERR_ARG, "ctx is NULL");
    if (!f_nl) return fail(SQ_ERR_ARG, "f_nl is NULL");
    sq_ctx &c = *ctx;
    if (!c.have_fermi)
        return fail(SQ_ERR_STATE, "sq_nonlocal_force needs sq_density and sq_fermi_level first");
    if (c.n_atoms == 0) return fail(SQ_ERR_ARG, "the context has no projectors");
    for (const Group &g : c.fgroups)
        if (!cc_force_supported(c.prec, g.E)) {
            int emax = 0;
            for (int e : {9, 13, 17, 21, 27, 32})
                if (cc_force_supported(c.prec, e)) emax = e;
            return fail(SQ_ERR_ARG, "the %s nonlocal force supports region edges up to %d (this "
                        "work list: %d)", c.prec == SQ_FP64 ? "FP64" : "FP32", emax, g.E);
        }
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(k_fill_f64(f_nl, 0.0, 3 * (int64_t)c.n_atoms, st));
    if (c.fgroups.empty()) return SQ_OK;
    ForceParams fp{};
    double w1[MAX_R + 1];
    fd_first_weights(c.r, w1);
    for (int a = 0; a < 3; ++a)
        for (int p = 0; p <= MAX_R; ++p) fp.grad[a][p] = p <= c.r ? w1[p] / c.p.h[a] : 0.0;
    fp.cp = c.fw.cp;
    fp.force = f_nl;
    HIP_TRY(k_fill_i32(c.d_counter, 0, (int64_t)c.fgroups.size(), st));
    auto launch = [&](auto tag) -> sq_status {
        using T = decltype(tag);
        for (size_t g = 0; g < c.fgroups.size(); ++g) {
            RegionArgs<T> a{};
            fill_region_args(c, a);
            a.items = c.d_fitems + c.fgroups[g].begin;
            a.n_items = c.fgroups[g].count;
            a.counter = c.d_counter + g;
            a.moments = nullptr;
            HIP_TRY(launch_cc_force(c.prec, c.fgroups[g].E, c.r, c.fgroups[g].maskz, &a, fp,
                                    c.fgroups[g].grid_fwd, st));
        }
        return SQ_OK;
    };
    if (c.prec == SQ_FP64) TRY(launch(double{}));
    else TRY(launch(float{}));
    c.last_stream = st;
    return SQ_OK;
}

sq_status sq_scf(sq_ctx *ctx, const double *b, const double *phi_bc, double Ne,
                 double lambda_min, double lambda_max, const sq_scf_params *sp, double *V,
                 double *rho, double *lambda_f, sq_scf_info *info, void *stream) {
    if (!ctx || !b || !sp || !V || !info) return fail(SQ_ERR_ARG, "NULL argument");
    sq_ctx &c = *ctx;
    const bool emb = c.p.bc == SQ_BC_EMBEDDED;
    if (!c.periodic && !emb)
        return fail(SQ_ERR_ARG, "sq_scf needs a periodic or an embedded context");
    if (emb && !phi_bc) return fail(SQ_ERR_ARG, "an embedded sq_scf needs phi_bc");
    if (emb)
        for (int a = 0; a < 3; ++a)
            if (c.p.rcut[a] < c.r)
                return fail(SQ_ERR_ARG, "an embedded sq_scf needs padding (rcut) >= the FD "
                            "radius %d on every axis", c.r);
    if (!c.all_nodes) return fail(SQ_ERR_ARG, "sq_scf needs every node of the grid (nodes == NULL)");
    if (!(sp->beta > 0.0) || !(sp->tol > 0.0) || !(sp->poisson_rtol > 0.0) ||
        !(sp->fermi_tol >= 0.0) || sp->max_iter < 1 || sp->poisson_max_iter < 1 ||
        (sp->anderson != 0 && sp->anderson != 1))
        return fail(SQ_ERR_ARG, "invalid sq_scf_params");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nv = c.nv;
    const int nb = N_PARTIAL;
    // phi, n, src, r, p, Ap, V_out, F, the previous pair V' and F', and a vector of ones
    constexpr int NVEC = 11;
    if (!c.d_scf) {
        TRY(c.alloc(&c.d_scf, (size_t)NVEC * nv));
        TRY(c.alloc(&c.d_scf_part, 2 * (size_t)nb));
        TRY(c.alloc(&c.d_scf_sc, (size_t)SC_COUNT));
        TRY(c.alloc(&c.d_scf_rho, (size_t)c.n_nodes));
        TRY(c.alloc(&c.d_scf_lf, 1));
        HIP_TRY(k_fill_f64(c.d_scf, 0.0, (int64_t)(NVEC - 1) * nv, st));
        HIP_TRY(k_fill_f64(c.d_scf + (NVEC - 1) * nv, 1.0, nv, st));
    }
    double *phi = c.d_scf, *nx = phi + nv, *src = nx + nv, *r = src + nv, *p = r + nv,
           *Ap = p + nv, *vout = Ap + nv, *F = vout + nv, *Vp = F + nv, *Fp = Vp + nv,
           *ones = Fp + nv;
    ScfGrid g{};
    for (int a = 0; a < 3; ++a) {
        g.N[a] = c.N[a];
        g.n[a] = c.p.n[a];
        g.pad[a] = emb ? c.p.rcut[a] : 0;
        g.ih2[a] = c.ih2[a];
    }
    g.r = c.r;
    g.periodic = c.periodic;
    const int64_t n_omega = (int64_t)c.p.n[0] * c.p.n[1] * c.p.n[2];
    // the Dirichlet values of an embedded problem live on phi's padding (its
    // interior starts from them too)
    if (emb) HIP_TRY(hipMemcpyAsync(phi, phi_bc, nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    for (int q = 0; q <= MAX_R; ++q) g.w[q] = c.w[q];
    double *rhoq = rho ? rho : c.d_scf_rho;
    double *lf = lambda_f ? lambda_f : c.d_scf_lf;
    double *sc = c.d_scf_sc;
    *info = sq_scf_info{};
    info->poisson_converged = 1;
    double hs[SC_COUNT];
    auto fetch = [&](void) -> sq_status {
        HIP_TRY(hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        return SQ_OK;
    };
    const double inv_h3 = 1.0 / c.h3;
    for (int it = 0; it < sp->max_iter; ++it) {
        TRY(sq_density(ctx, V, lambda_min, lambda_max, nullptr, nullptr, stream));
        TRY(sq_fermi_level(ctx, Ne, sp->fermi_tol, 200, lf, rhoq, nullptr, nullptr, stream));
        HIP_TRY(scf_source(g, rhoq, b, inv_h3, nx, src, ones, c.d_scf_part, nb, sc, st));
        HIP_TRY(scf_cg_start(g, src, phi, r, p, c.d_scf_part, nb, sc, st));
        int cgi = 0;
        double relres = 0.0;
        for (;;) {
            TRY(fetch());
            relres = hs[SC_BB] > 0.0 ? std::sqrt(std::max(hs[SC_RR], 0.0) / hs[SC_BB]) : 0.0;
            if (relres < sp->poisson_rtol || cgi >= sp->poisson_max_iter) break;
            const int chunk = std::min(10, sp->poisson_max_iter - cgi);
            for (int j = 0; j < chunk; ++j)
                HIP_TRY(scf_cg_iter(g, phi, r, p, Ap, c.d_scf_part, nb, sc, st));
            cgi += chunk;
        }
        info->poisson_iterations += cgi;
        info->poisson_relres = std::max(info->poisson_relres, relres);
        if (!(relres < sp->poisson_rtol)) info->poisson_converged = 0;
        if (!emb) HIP_TRY(scf_center(phi, nv, ones, c.d_scf_part, nb, sc, st));
        HIP_TRY(scf_vout(g, phi, nx, V, vout, F, c.d_scf_part, nb, sc, st));
        TRY(fetch());
        info->iterations = it + 1;
        info->residual = std::sqrt(std::max(hs[SC_FF], 0.0) / (double)n_omega);
        if (info->residual < sp->tol) {
            info->converged = 1;
            break;
        }
        if (it + 1 < sp->max_iter)   // V keeps the last V_in when the loop runs out
            HIP_TRY(scf_mix(V, Vp, F, Fp, nv, sp->beta, sp->anderson && it > 0, c.d_scf_part,
                            nb, sc, st));
    }
    TRY(sq_device_status(ctx));
    c.last_stream = st;
    return SQ_OK;
}

sq_status sq_device_status(sq_ctx *ctx) {
    if (!ctx) return fail(SQ_ERR_ARG, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(ctx->last_stream));
    int32_t flag = 0;
    Scalars s{};
    HIP_TRY(hipMemcpy(&flag, ctx->d_status, sizeof(flag), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&s, ctx->d_scal, sizeof(s), hipMemcpyDeviceToHost));
    if (flag & 4) return fail(SQ_ERR_NOT_CONVERGED, "a Jacobi-matrix eigensolve did not converge");
    if (flag) return fail(SQ_ERR_ARG, "a region touched more atoms than the kernel's atom table holds");
    if (s.status) return fail((sq_status)s.status, "device reported status %d", s.status);
    return SQ_OK;
}

}  // extern "C"
