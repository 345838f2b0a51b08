// Host-side driver for the AddressSanitizer / UndefinedBehaviorSanitizer run of
// the C ABI's setup code (built and run by tests/test_host_sanitizers.py).
// Every call below either fails validation or builds all host tables (work
// list, column-major projector tables, force work list) and then stops at the
// first device call when no GPU is present; with a GPU it also sets up and
// tears down a context.  Any out-of-bounds access or undefined behaviour in
// that host code aborts the process with a sanitizer report.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "sq.h"

namespace {

sq_params params(int bc, int n, int rcut) {
    sq_params p{};
    p.n[0] = n;
    p.n[1] = n - 1;
    p.n[2] = n + 1;
    p.h[0] = p.h[1] = p.h[2] = 0.5;
    p.fd_order = 4;
    p.bc = bc;
    p.rcut[0] = p.rcut[1] = p.rcut[2] = rcut;
    p.order = 8;
    p.kT = 0.1;
    p.precision = SQ_FP32_ACC64;
    p.ckpt_every = 1;
    p.adjoint_precision = SQ_FP64;
    p.tune = 1;
    return p;
}

// ball-shaped supports of radius rad nodes around a few centres on grid v[3]
struct Tables {
    std::vector<int64_t> off, idx;
    std::vector<double> chi, dchi, c;
};

Tables supports(const int v[3], int n_atoms, int rad) {
    Tables t;
    t.off.push_back(0);
    for (int j = 0; j < n_atoms; ++j) {
        const int cx = (3 + 5 * j) % v[0], cy = (2 + 3 * j) % v[1], cz = (4 + 7 * j) % v[2];
        for (int z = cz - rad; z <= cz + rad; ++z)
            for (int y = cy - rad; y <= cy + rad; ++y)
                for (int x = cx - rad; x <= cx + rad; ++x) {
                    const int dx = x - cx, dy = y - cy, dz = z - cz;
                    if (dx * dx + dy * dy + dz * dz > rad * rad) continue;
                    if (x < 0 || y < 0 || z < 0 || x >= v[0] || y >= v[1] || z >= v[2]) continue;
                    t.idx.push_back(x + (int64_t)v[0] * (y + (int64_t)v[1] * z));
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    for (int l = 0; l < 4; ++l) t.chi.push_back(std::exp(-0.3 * r2) * (l + 1));
                    for (int q = 0; q < 12; ++q) t.dchi.push_back(0.01 * (q + 1) * (dx - dy + dz));
                }
        t.off.push_back((int64_t)t.idx.size());
        for (int l = 0; l < 4; ++l) t.c.push_back(l % 2 ? -0.5 : 0.7);
    }
    return t;
}

int failures = 0;

void expect(bool ok, const char *what, sq_status st) {
    if (!ok) {
        std::printf("FAILED: %s (status %d: %s)\n", what, (int)st, sq_last_error());
        ++failures;
    }
}

sq_status setup(const sq_params &p, const Tables *t, int n_atoms, const int64_t *nodes,
                const int32_t *rc, int64_t n_nodes) {
    sq_projectors pr{};
    if (t) {
        pr.n_atoms = n_atoms;
        pr.n_proj = 4;
        pr.sup_off = t->off.data();
        pr.sup_idx = t->idx.data();
        pr.chi = t->chi.data();
        pr.dchi = t->dchi.data();
        pr.c = t->c.data();
    }
    sq_ctx *ctx = nullptr;
    const sq_status st = sq_setup(&p, t ? &pr : nullptr, nodes, rc, n_nodes, &ctx);
    if (ctx) sq_destroy(ctx);
    return st;
}

}  // namespace

int main() {
    // valid geometries in every boundary mode: host tables built, then either a
    // context (GPU present) or SQ_ERR_HIP at the first device call
    for (int bc = 0; bc < 3; ++bc) {
        const sq_params p = params(bc, 12, 2);
        int v[3] = {p.n[0], p.n[1], p.n[2]};
        if (bc == SQ_BC_EMBEDDED)
            for (int a = 0; a < 3; ++a) v[a] += 2 * p.rcut[a];
        const Tables t = supports(v, 3, 2);
        const int64_t n_omega = (int64_t)p.n[0] * p.n[1] * p.n[2];
        sq_status st = setup(p, &t, 3, nullptr, nullptr, n_omega);
        expect(st == SQ_OK || st == SQ_ERR_HIP, "valid setup, all nodes", st);
        // a node subset with uneven half-widths (several edge buckets)
        std::vector<int64_t> nodes;
        std::vector<int32_t> rc;
        for (int64_t q = 0; q < n_omega; q += 7) {
            nodes.push_back(q);
            for (int a = 0; a < 3; ++a) rc.push_back((int32_t)(q % 3));
        }
        st = setup(p, &t, 3, nodes.data(), rc.data(), (int64_t)nodes.size());
        expect(st == SQ_OK || st == SQ_ERR_HIP, "valid setup, uneven node subset", st);
    }
    // malformed projector CSR offsets: refused before any table is read
    const int64_t bad[][3] = {{0, 100, 50}, {0, 3, 2}, {0, 5, 4}, {1, 2, 3}, {0, -1, 2}};
    for (const auto &b : bad) {
        const sq_params p = params(SQ_BC_PERIODIC, 8, 2);
        Tables t;
        t.off.assign(b, b + 3);
        const int64_t nnz = b[2] > 0 ? b[2] : 0;
        t.idx.assign((size_t)nnz, 0);
        t.chi.assign((size_t)nnz * 4, 0.0);
        t.c.assign(8, 1.0);
        sq_projectors pr{};
        pr.n_atoms = 2;
        pr.n_proj = 4;
        pr.sup_off = t.off.data();
        pr.sup_idx = t.idx.data();
        pr.chi = t.chi.data();
        pr.c = t.c.data();
        sq_ctx *ctx = nullptr;
        const int64_t n_omega = (int64_t)p.n[0] * p.n[1] * p.n[2];
        const sq_status st = sq_setup(&p, &pr, nullptr, nullptr, n_omega, &ctx);
        expect(st == SQ_ERR_ARG && ctx == nullptr, "malformed sup_off refused", st);
    }
    // out-of-range support index, node index and half-width
    {
        const sq_params p = params(SQ_BC_DIRICHLET, 10, 2);
        int v[3] = {p.n[0], p.n[1], p.n[2]};
        Tables t = supports(v, 2, 2);
        t.idx[1] = (int64_t)v[0] * v[1] * v[2];
        const int64_t n_omega = (int64_t)p.n[0] * p.n[1] * p.n[2];
        expect(setup(p, &t, 2, nullptr, nullptr, n_omega) == SQ_ERR_ARG, "support index range",
               SQ_ERR_ARG);
        const int64_t nodes[2] = {0, n_omega};
        expect(setup(p, nullptr, 0, nodes, nullptr, 2) == SQ_ERR_ARG, "node index range",
               SQ_ERR_ARG);
        const int64_t one[1] = {5};
        const int32_t neg[3] = {1, -1, 1};
        expect(setup(p, nullptr, 0, one, neg, 1) == SQ_ERR_ARG, "negative half-width",
               SQ_ERR_ARG);
    }
    std::printf("%s\n", failures ? "failures" : "ok");
    return failures ? 1 : 0;
}
