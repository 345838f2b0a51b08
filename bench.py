"""Benchmark of the spectral-quadrature hot path on one MI355X.

One step = the whole path over the 64^3 Mg-like workload (96 atoms x 4
projectors, 27^3 node regions, K = 100, kT = 0.001 Ha, N_e = 192):
  spectral bounds (device FP64 Lanczos) -> scaled diagonal -> FP32 region
  recurrence with FP64 moments -> moment sum -> FP64 Fermi bisection ->
  coefficients -> pointwise rho, u -> FP64 adjoint (dV, dR).
Inputs are resident in HBM before the timed region.  Throughput is counted in
node-steps (one node advanced by one Chebyshev order; K per node per step).

Beside the headline it times, each with its error against the FP64 oracle:
the 4096 uneven clipped regions (one graph-captured persistent FP32 launch
against one FP64 launch per region), the 48^3 vacancy cell (forward +
adjoint), the embedded 128^3 defect cell (forward + bisection on all nodes,
adjoint on one GPU's share of them), and the paper's own pieces around the
path (Gauss quadrature, Clenshaw-Curtis force, entropy, SCF).

Prints one JSON line (rank 0).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12                            # bytes/s, MI355X HBM3E
PEAK_FP32_VALU = 256 * 4 * 16 * 2 * 2.4e9    # non-packed FP32 (and FP64) FMA: 78.6 TFLOP/s
PEAK_LDS = 256 * 128 * 2.4e9                 # 128 B/clk/CU: 78.6 TB/s
T0 = time.perf_counter()


def log(msg):
    print(f"[bench {time.perf_counter() - T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


# Algorithmic HBM bytes per region-point and Chebyshev step (the streaming
# model of the recurrence: read v_k, read v_{k-1}, write v_{k+1}; the adjoint
# recomputes the forward, runs the reverse recurrence, re-reads v_k and
# updates a region dV accumulator).  s = bytes per value.
def bytes_forward(s):
    return 3 * s


def bytes_adjoint(s):
    return 3 * s + 3 * s + s + 2 * s


# 9r + 4 flops per region-point and application of 2 Hs: 3r symmetric pairs
# (add + FMA), the diagonal FMA and the recurrence FMA.
def flops_app(r):
    return 9 * r + 4


# sources each profiled kernel is compiled from (the host-side API does not
# change what a kernel fetches and writes)
_REGION = ("sq_internal.h", "sq_region.h")
KERNEL_SOURCES = {
    "cheb_forward_kernel": _REGION + ("sq_forward.hip",),
    "cheb_adjoint64_kernel": _REGION + ("sq_adjoint64.h", "sq_adjoint64.hip"),
    "cheb_adjoint_kernel": _REGION + ("sq_adjoint_kernel.h", "sq_adjoint.hip",
                                      "sq_adjoint_r1.hip", "sq_adjoint_r2.hip",
                                      "sq_adjoint_r3.hip", "sq_adjoint_r4.hip",
                                      "sq_adjoint_r5.hip", "sq_adjoint_r6.hip"),
    "gauss_lanczos_kernel": _REGION + ("sq_gauss_lanczos.hip",),
    "cc_force_kernel": _REGION + ("sq_force.h", "sq_force.hip"),
}


def kernel_source_hash(kernel):
    """sha256 over the HIP sources of one profiled kernel (names and contents)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2011_13517_amd", "csrc")
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        h.update(name.encode())
        with open(os.path.join(d, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE
    summary of `workload`, or None when it is missing or was taken from other
    kernel sources."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k or k.get("source_sha256") != kernel_source_hash(kernel):
        return None
    return {"fetch_bytes": k["fetch_bytes"], "write_bytes": k["write_bytes"],
            "bytes": k["fetch_bytes"] + k["write_bytes"], "source": os.path.basename(path)}


def roofline_hbm(kernel, alg_bytes, seconds, workload, flops=None, lds_bytes=None):
    """Roofline entry of one kernel on the HBM-byte basis (algorithmic bytes per
    launch over the launch's duration), with its VALU and LDS fractions beside."""
    ach = alg_bytes / seconds
    d = dict(bound="hbm", kernel=kernel, achieved=ach / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s",
             frac=ach / PEAK_HBM, algorithmic_bytes=alg_bytes, seconds=seconds,
             traffic=recorded_traffic(kernel, workload))
    if flops is not None:
        d["valu_frac"] = flops / seconds / PEAK_FP32_VALU
    if lds_bytes is not None:
        d["lds_frac"] = lds_bytes / seconds / PEAK_LDS
    return d


def host_cpu():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def events(n):
    import torch
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def oracle_adjoint(prob, lmin, lmax, lf, g_rho, g_u, nodes, node_m):
    """Oracle (dV, dR) of sum_q (g_rho[q] rho_q + g_u[q] u_q) at fixed lambda_f:
    the Chebyshev weights a_k of Eq. (rhoFinal) and of the band-energy density."""
    import oracle as O
    K = prob.order
    c, _ = O.cheb_coeffs(O.KIND_G, lf, prob.kT, lmin, lmax, K)
    d, _ = O.cheb_coeffs(O.KIND_U, lf, prob.kT, lmin, lmax, K)
    c[0] *= 0.5
    d[0] *= 0.5
    a = 2.0 * (g_rho[:, None] * c[None, :] + g_u[:, None] * d[None, :])
    return O.adjoint(prob, lmin, lmax, a, nodes=nodes, node_m=node_m,
                     with_dR=prob.n_atoms > 0)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def adjoint_accuracy(prob, lmin, lmax, lf, n_sample, seed, dev):
    """dV and dR of the FP64 adjoint on a node subset (same kernel and edge bucket
    as the timed launch) against the oracle, with random cotangents."""
    import torch

    from paper_2011_13517_amd import sq
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(prob.n_nodes, n_sample, replace=False))
    nodes = prob.node_list()[pick]
    node_m = None if prob.node_rcut is None else prob.node_rcut[pick]
    g_rho, g_u = rng.normal(size=nodes.size), rng.normal(size=nodes.size)
    t = time.perf_counter()
    gV, dR = oracle_adjoint(prob, lmin, lmax, lf, g_rho, g_u, nodes, node_m)
    t = time.perf_counter() - t
    ctx = sq.Context(prob, precision=1, adjoint_precision=0, ckpt_every=1, nodes=nodes,
                     node_rcut=node_m)
    V = torch.tensor(prob.V, dtype=torch.float64, device=dev)
    ctx.density(V, lmin, lmax)
    lam = torch.tensor([lf], dtype=torch.float64, device=dev)
    ctx.fermi_level(max_iter=0, lambda_f=lam, want_fields=False, device=dev)
    dV = torch.zeros_like(V)
    dRg = torch.zeros((prob.n_atoms, 3), dtype=torch.float64, device=dev) \
        if prob.n_atoms else None
    ctx.backward(torch.tensor(g_rho, device=dev), torch.tensor(g_u, device=dev), dV, dRg)
    torch.cuda.synchronize()
    ctx.status()
    ctx.close()
    out = {"dV_rel": rel(dV.cpu().numpy(), gV), "sample_nodes": int(nodes.size),
           "oracle_seconds": t,
           "reference": "FP64 oracle adjoint, random cotangents, same lambda_f and bounds"}
    if prob.n_atoms:
        out["dR_rel"] = rel(dRg.cpu().numpy(), dR)
    return out


def force_leg(ctx, prob, tot, lf, dev):
    """Clenshaw-Curtis nonlocal force (sq_nonlocal_force) at the Fermi level of
    the last timed step, timed with HIP events on the current stream; its error
    against the oracle on the 4 nodes nearest to atom 0 (node-subset context)."""
    import torch

    import oracle as O
    from paper_2011_13517_amd import sq
    info = ctx.info
    f = torch.empty((ctx.n_atoms, 3), dtype=torch.float64, device=dev)
    ctx.nonlocal_force(f)
    torch.cuda.synchronize()
    e = events(2)
    e[0].record()
    ctx.nonlocal_force(f)
    e[1].record()
    torch.cuda.synchronize()
    ctx.status()
    t = e[0].elapsed_time(e[1]) * 1e-3
    nf, pts = int(info.n_force_nodes), int(info.force_region_points)
    r = prob.fd_order // 2
    log(f"nonlocal force: {nf} nodes in supports, {t:.3f} s")
    n = np.asarray(prob.n)
    pos = np.asarray(prob.atom_pos[0]) / np.asarray(prob.h)
    grid = np.stack(np.meshgrid(*(np.arange(k) for k in n), indexing="ij"), -1).reshape(-1, 3)
    d = np.abs(grid - pos[None, :])
    d = np.minimum(d, n[None, :] - d) if prob.bc == 0 else d
    idx = np.argsort((d ** 2).sum(1))[:4]
    nodes = grid[idx, 0] + n[0] * (grid[idx, 1] + n[1] * grid[idx, 2])
    om, tau = float(tot[4]), float(tot[5])
    t_o = time.perf_counter()
    f_ref = O.cc_nonlocal_force(prob, om - tau, om + tau, lf, nodes=nodes)
    t_o = time.perf_counter() - t_o
    sub = sq.Context(prob, precision=1, nodes=nodes)
    V = torch.tensor(prob.V, dtype=torch.float64, device=dev)
    sub.density(V, om - tau, om + tau)
    sub.fermi_level(max_iter=0, lambda_f=torch.tensor([lf], dtype=torch.float64, device=dev),
                    want_fields=False, device=dev)
    fs = sub.nonlocal_force(device=dev).cpu().numpy()
    sub.close()
    cpu = dict(value=nodes.size * ctx.K / t_o, unit="node-steps/s", cores=1, kind="oracle",
               sample=f"{nodes.size} nodes nearest to atom 0 ({t_o:.1f} s)")
    return {"seconds": t, "force_nodes": nf, "node_steps_per_s": nf * ctx.K / t,
            "cpu_baseline": cpu,
            "roofline": roofline_hbm("cc_force_kernel", bytes_forward(4) * pts * ctx.K, t,
                                     prob.name, flops=flops_app(r) * pts * ctx.K),
            "accuracy": {"rel_df": rel(fs, f_ref), "sample_nodes": int(nodes.size),
                         "precision": "FP32 recurrence, FP64 contraction",
                         "reference": "FP64 oracle, Eq. (NLforceSQ) on the same nodes"},
            "max_abs_f": float(f.abs().max().item())}


def scf_leg(ctx, prob, tot, dev):
    """Two iterations of the SCF loop (sq_scf) on the same cell from V_in = 0,
    with the synthetic pseudocharge (Z = 2 per atom) and the scaling bounds of
    the timed run widened by 5 Ha on each side; wall time per iteration (the
    loop synchronises at every CG check)."""
    import torch

    from paper_2011_13517_amd import synth
    b = torch.tensor(synth.pseudocharge(prob), dtype=torch.float64, device=dev)
    Vs = torch.zeros(int(np.prod(prob.vshape)), dtype=torch.float64, device=dev)
    om, tau = float(tot[4]), float(tot[5])
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, _, lf, info = ctx.scf(b, 2.0 * prob.n_atoms, Vs, om - tau - 5.0, om + tau + 5.0,
                             beta=0.3, tol=1e-6, max_iter=2, poisson_rtol=1e-10)
    torch.cuda.synchronize()
    t = time.perf_counter() - t
    log(f"SCF: {info['iterations']} iterations, {t / info['iterations']:.3f} s each, "
        f"residual {info['residual']:.3e}, {info['poisson_iterations']} CG steps")
    return {"seconds_per_iteration": t / info["iterations"], "iterations": info["iterations"],
            "residual": info["residual"], "poisson_cg_steps": info["poisson_iterations"],
            "poisson_relres": info["poisson_relres"], "lambda_f": float(lf.item()),
            "start": "V_in = 0, Gaussian pseudocharge Z = 2 per atom"}


GAUSS_ORDER = 80   # the paper's Lanczos degree beside Chebyshev degree 100


def gauss_leg(prob, V, tot, region_points, dev):
    """Gauss-quadrature density on the same workload with the paper's Lanczos
    degree (its own context): K_L Lanczos steps per node (sq_gauss_density:
    bounds as in the Chebyshev run, the Lanczos sweep, the Jacobi eigensolves)
    and sq_gauss_fermi_level (bisection and rho, u, s), timed with HIP events on
    the current stream; fields of a few nodes against the oracle's rules at the
    same lambda_f."""
    import dataclasses

    import torch

    import oracle as O
    from paper_2011_13517_amd import sq
    prob = dataclasses.replace(prob, order=GAUSS_ORDER)
    ctx = sq.Context(prob, precision=1)
    K, n = ctx.K, ctx.n_nodes
    om, tau = float(tot[4]), float(tot[5])
    lmin, lmax = om - tau, om + tau
    nodes = torch.empty((n, K), dtype=torch.float64, device=dev)
    wts = torch.empty_like(nodes)
    Ne = prob.Ne if prob.Ne is not None else 0.0
    ctx.gauss_density(V, lmin, lmax, nodes=nodes, weights=wts)
    torch.cuda.synchronize()
    e = events(3)
    e[0].record()
    ctx.gauss_density(V, lmin, lmax, nodes=nodes, weights=wts)
    e[1].record()
    lf, rho, u, s, gt = ctx.gauss_fermi_level(Ne=Ne, tol=1e-8, max_iter=200, device=dev)
    e[2].record()
    torch.cuda.synchronize()
    ctx.status()
    t_rules = e[0].elapsed_time(e[1]) * 1e-3
    t_fields = e[1].elapsed_time(e[2]) * 1e-3
    gt = gt.cpu().numpy()
    log(f"Gauss quadrature: rules {t_rules:.3f} s, Fermi level + fields {t_fields:.3f} s, "
        f"N_e={gt[0]:.10f} lambda_f={lf.item():.10f}")
    rng = np.random.default_rng(13)
    sample = np.sort(rng.choice(n, 4, replace=False))
    t_o = time.perf_counter()
    lam_o, w_o = O.gauss_rules(prob, lmin, lmax, K, nodes=prob.node_list()[sample])
    t_o = time.perf_counter() - t_o
    rho_o, u_o, s_o = O.gauss_fields(lam_o, w_o, lf.item(), prob.kT)
    rho_g = rho.cpu().numpy()
    r = prob.fd_order // 2
    ctx.close()
    return {
        "metric": "node-Lanczos-steps/s",
        "order": K,
        "value": n * K / (t_rules + t_fields),
        "seconds": {"rules": t_rules, "fermi_fields": t_fields},
        "roofline": roofline_hbm("gauss_lanczos_kernel", bytes_forward(4) * region_points * K,
                                 t_rules, prob.name, flops=flops_app(r) * region_points * K),
        "totals": {"Ne": float(gt[0]), "U": float(gt[1]), "S": float(gt[2]),
                   "U_minus_kT_S": float(gt[3]), "lambda_f": float(lf.item())},
        "accuracy": {"max_abs_drho": float(np.abs(rho_g[sample] - rho_o).max()),
                     "rel_drho": float(np.abs(rho_g[sample] - rho_o).max() / np.abs(rho_g).max()),
                     "sample_nodes": int(sample.size),
                     "reference": "FP64 oracle Gauss rules at the GPU's lambda_f"},
        "precision": "FP32 Lanczos vectors, FP64 a_k, b_k, eigensolve, bisection, fields",
        "cpu_baseline": dict(value=sample.size * K / t_o, unit="node-steps/s", cores=1,
                             kind="oracle",
                             sample=f"{sample.size} random nodes, oracle Lanczos + tridiagonal "
                                    f"eigensolve ({t_o:.1f} s)"),
    }


def config3_leg(dev):
    """The 4096 uneven Dirichlet-clipped regions (edges 11..27, K = 100): one
    persistent FP32 launch plan (the tuner's) captured into a HIP graph and
    replayed, against the plain FP64 path of one launch per region; moments of
    sampled regions against the oracle."""
    import torch

    import oracle as O
    from paper_2011_13517_amd import sq, synth
    prob = synth.config(3)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    V = torch.tensor(prob.V, dtype=torch.float64, device=dev)
    K, n = prob.order, prob.n_nodes
    out = {"workload": prob.name, "nodes": n, "order": K}

    def timed(ctx, reps, graph=False, warm=True):
        mu = torch.empty((n, K + 1), dtype=torch.float64, device=dev)
        step = lambda: ctx.density(V, lmin, lmax, moments=mu)  # noqa: E731
        if graph:
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                step()
            torch.cuda.current_stream().wait_stream(s)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                step()
            run = g.replay
        else:
            if warm:
                step()
            run = step
        torch.cuda.synchronize()
        e = events(2)
        e[0].record()
        for _ in range(reps):
            run()
        e[1].record()
        torch.cuda.synchronize()
        ctx.status()
        return e[0].elapsed_time(e[1]) * 1e-3 / reps, mu

    c32 = sq.Context(prob, precision=1)
    t32, mu32 = timed(c32, 20, graph=True)
    out["fp32_persistent_graph"] = {"seconds": t32, "launches": int(c32.info.n_launches),
                                    "node_steps_per_s": n * K / t32,
                                    "region_points": int(c32.info.region_points)}
    c32.close()
    # 4096 launches of one workgroup each (seconds per pass); the library's
    # code object is loaded by the earlier legs, so one pass is timed cold
    c64 = sq.Context(prob, precision=0, tune=2)
    t64, mu64 = timed(c64, 1, warm=False)
    out["fp64_per_region_launches"] = {"seconds": t64, "launches": int(c64.info.n_launches),
                                       "node_steps_per_s": n * K / t64}
    c64.close()
    c64p = sq.Context(prob, precision=0)
    t64p, _ = timed(c64p, 5, graph=True)
    out["fp64_persistent_graph"] = {"seconds": t64p, "launches": int(c64p.info.n_launches)}
    c64p.close()
    out["speedup_fp32_graph_vs_fp64_per_region"] = t64 / t32
    out["speedup_fp32_graph_vs_fp64_persistent"] = t64p / t32
    rng = np.random.default_rng(31)
    pick = np.sort(rng.choice(n, 16, replace=False))
    mu_ref = O.moments(prob, lmin, lmax, nodes=prob.nodes[pick], node_m=prob.node_rcut[pick])
    out["accuracy"] = {"max_abs_dmu_fp32": float(np.abs(mu32.cpu().numpy()[pick] - mu_ref).max()),
                       "max_abs_dmu_fp64": float(np.abs(mu64.cpu().numpy()[pick] - mu_ref).max()),
                       "sample_nodes": int(pick.size), "reference": "FP64 oracle moments"}
    log(f"config 3: FP32 graph {t32 * 1e3:.2f} ms, FP64 per-region {t64 * 1e3:.2f} ms "
        f"({t64 / t32:.1f}x), FP64 persistent {t64p * 1e3:.2f} ms")
    return out


def config4_leg(dev):
    """The 48^3 vacancy cell (21^3 regions, K = 80): FP32 forward + Fermi
    bisection + FP64 adjoint (dV, dR) over all nodes, HIP events."""
    import torch

    from paper_2011_13517_amd import sq, synth
    prob = synth.config(4)
    ctx = sq.Context(prob, precision=1, adjoint_precision=0, ckpt_every=1)
    V = torch.tensor(prob.V, dtype=torch.float64, device=dev)
    n, K = ctx.n_nodes, ctx.K
    g = torch.ones(n, dtype=torch.float64, device=dev)
    dV = torch.zeros_like(V)
    dR = torch.zeros((prob.n_atoms, 3), dtype=torch.float64, device=dev)
    lam = torch.zeros(1, dtype=torch.float64, device=dev)
    for rep in range(2):
        e = events(4)
        e[0].record()
        ctx.density(V)
        e[1].record()
        _, _, _, tot = ctx.fermi_level(Ne=prob.Ne, tol=1e-8, max_iter=200, lambda_f=lam,
                                       device=dev)
        e[2].record()
        ctx.backward(g, g, dV, dR)
        e[3].record()
        torch.cuda.synchronize()
    ctx.status()
    tf, tb = e[0].elapsed_time(e[1]) * 1e-3, e[2].elapsed_time(e[3]) * 1e-3
    pts = int(ctx.info.region_points)
    tot = tot.cpu().numpy()
    om, tau = float(tot[4]), float(tot[5])
    ctx.close()
    r = prob.fd_order // 2
    acc = adjoint_accuracy(prob, om - tau, om + tau, float(lam.item()), 16, 44, dev)
    log(f"config 4: forward {tf:.3f} s, adjoint {tb:.3f} s; dV rel {acc['dV_rel']:.2e}")
    return {"workload": prob.name, "nodes": n, "order": K,
            "seconds": {"forward": tf, "adjoint": tb},
            "node_steps_per_s": n * K / (tf + e[1].elapsed_time(e[2]) * 1e-3 + tb),
            "roofline_forward": roofline_hbm("cheb_forward_kernel", bytes_forward(4) * pts * K,
                                             tf, prob.name, flops=flops_app(r) * pts * K),
            "roofline_adjoint": roofline_hbm("cheb_adjoint_kernel", bytes_adjoint(8) * pts * K,
                                             tb, prob.name,
                                             flops=(2 * K - 2) * flops_app(r) * pts),
            "adjoint_accuracy": acc, "Ne_error": float(tot[0] - prob.Ne)}


def config5_leg(dev, adjoint_stride, cpu_sample):
    """The embedded 128^3 defect cell (154^3 padded grid, 766 atoms, 27^3
    regions, K = 120): device bounds + FP32 forward + FP64 bisection to
    |dN_e| < 1e-8 on all 2,097,152 nodes, and the FP64 adjoint on one GPU's
    share of the nodes (every adjoint_stride-th node), HIP events; the oracle on
    a stratified sample of the same nodes."""
    import torch

    import oracle as O
    from paper_2011_13517_amd import sq, synth
    t_syn = time.perf_counter()
    prob = synth.config(5)
    t_syn = time.perf_counter() - t_syn
    log(f"config 5 inputs built in {t_syn:.1f} s")
    ctx = sq.Context(prob, precision=1)
    V = torch.tensor(prob.V, dtype=torch.float64, device=dev)
    n, K = ctx.n_nodes, ctx.K
    pts = int(ctx.info.region_points)
    lam = torch.zeros(1, dtype=torch.float64, device=dev)
    mu = torch.empty((n, K + 1), dtype=torch.float64, device=dev)
    ctx.density(V, moments=mu)   # warm-up (tuner, code objects)
    torch.cuda.synchronize()
    e = events(3)
    e[0].record()
    ctx.density(V, moments=mu)
    e[1].record()
    _, rho, _, tot = ctx.fermi_level(Ne=prob.Ne, tol=1e-8, max_iter=200, lambda_f=lam,
                                     device=dev)
    e[2].record()
    torch.cuda.synchronize()
    ctx.status()
    tf, tfe = e[0].elapsed_time(e[1]) * 1e-3, e[1].elapsed_time(e[2]) * 1e-3
    tot = tot.cpu().numpy()
    om, tau = float(tot[4]), float(tot[5])
    lf = float(lam.item())
    log(f"config 5: forward {tf:.3f} s, bisection + fields {tfe:.3f} s, "
        f"N_e - target {tot[0] - prob.Ne:.2e}")
    # stratified oracle sample: the 8 corners of Omega (regions in the padding),
    # nodes nearest the Al solutes and random interior nodes
    rng = np.random.default_rng(55)
    n0, n1, n2 = prob.n
    corners = [i + n0 * (j + n1 * k) for i in (0, n0 - 1) for j in (0, n1 - 1)
               for k in (0, n2 - 1)]
    sample = np.unique(np.concatenate([corners, rng.choice(n, cpu_sample, replace=False)]))
    t_o = time.perf_counter()
    mu_ref = O.moments(prob, om - tau, om + tau, nodes=sample)
    t_o = time.perf_counter() - t_o
    c, _ = O.cheb_coeffs(O.KIND_G, lf, prob.kT, om - tau, om + tau, K)
    rho_ref, _ = O.contract(mu_ref, c, c)
    rho_g = rho.cpu().numpy()
    mu_s = mu[torch.tensor(sample, device=dev)].cpu().numpy()
    ctx.close()
    del mu, rho
    # adjoint on one GPU's share of the nodes
    nodes = np.arange(0, n, adjoint_stride, dtype=np.int64)
    actx = sq.Context(prob, precision=1, adjoint_precision=0, ckpt_every=1, nodes=nodes)
    actx.density(V, om - tau, om + tau)
    actx.fermi_level(max_iter=0, lambda_f=lam, want_fields=False, device=dev)
    g = torch.ones(nodes.size, dtype=torch.float64, device=dev)
    dV = torch.zeros_like(V)
    dR = torch.zeros((prob.n_atoms, 3), dtype=torch.float64, device=dev)
    e = events(2)
    e[0].record()
    actx.backward(g, g, dV, dR)
    e[1].record()
    torch.cuda.synchronize()
    actx.status()
    tb = e[0].elapsed_time(e[1]) * 1e-3
    apts = int(actx.info.region_points)
    actx.close()
    acc = adjoint_accuracy(prob, om - tau, om + tau, lf, 12, 57, dev)
    log(f"config 5: adjoint on {nodes.size} nodes {tb:.3f} s; dV rel {acc['dV_rel']:.2e}")
    r = prob.fd_order // 2
    t_step = tf + tfe + tb * adjoint_stride
    return {
        "workload": prob.name, "nodes": n, "order": K, "atoms": prob.n_atoms, "Ne": prob.Ne,
        "seconds": {"forward": tf, "fermi_fields": tfe,
                    "adjoint_share": tb, "adjoint_share_nodes": int(nodes.size),
                    "step_estimate": t_step},
        "node_steps_per_s_forward": n * K / (tf + tfe),
        "node_steps_per_s_step_estimate": n * K / t_step,
        "roofline_forward": roofline_hbm("cheb_forward_kernel", bytes_forward(4) * pts * K, tf,
                                         prob.name, flops=flops_app(r) * pts * K),
        "roofline_adjoint": roofline_hbm("cheb_adjoint64_kernel", bytes_adjoint(8) * apts * K,
                                         tb, prob.name,
                                         flops=(2 * K - 2) * flops_app(r) * apts),
        "Ne_error": float(tot[0] - prob.Ne), "lambda_f": lf,
        "accuracy": {"max_abs_drho": float(np.abs(rho_g[sample] - rho_ref).max()),
                     "rel_drho": float(np.abs(rho_g[sample] - rho_ref).max() /
                                       np.abs(rho_g).max()),
                     "max_abs_dmu": float(np.abs(mu_s - mu_ref).max()),
                     "sample_nodes": int(sample.size), "reference": "FP64 oracle"},
        "adjoint_accuracy": acc,
        "cpu_baseline": dict(value=sample.size * K / t_o, unit="node-steps/s",
                             cores=O.num_threads(), kind="oracle",
                             sample=f"{sample.size} nodes (8 corners + random), oracle moments "
                                    f"({t_o:.1f} s)"),
        "note": "the adjoint is timed on every %d-th node (one GPU's share of the cell split %d "
                "ways); step_estimate scales it to all nodes" % (adjoint_stride, adjoint_stride),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-force", action="store_true",
                    help="skip the Clenshaw-Curtis nonlocal-force leg")
    ap.add_argument("--no-scf", action="store_true", help="skip the SCF-loop leg")
    ap.add_argument("--no-gauss", action="store_true",
                    help="skip the Gauss-quadrature (LSSGQ) leg")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the legs of the 4096-region, 48^3 and embedded 128^3 workloads")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the oracle comparisons of the main workload (they launch the "
                         "timed kernels again on small node subsets; profiling runs use this so "
                         "that per-kernel averages are those of the timed launches)")
    ap.add_argument("--local-only", action="store_true",
                    help="the workload without its atoms (local Hamiltonian only): a profiling "
                         "aid that times the stencil and diagonal apart from the projector block")
    ap.add_argument("--c5-adjoint-stride", type=int, default=8)
    ap.add_argument("--cpu-sample", type=int, default=2048)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run three device-to-device copies of MIB MiB (a kernel of "
                         "known HBM traffic that scales FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(this build has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2011_13517_amd import sq, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    prob = synth.config(args.config)
    if args.local_only:
        prob = synth.without_projectors(prob)
    log(f"workload {prob.name}: {prob.n_nodes} nodes, K={prob.order}, atoms={prob.n_atoms}")
    # FP32 forward; FP64 adjoint keeping every v_k of its in-flight regions
    ctx = sq.Context(prob, precision=1, adjoint_precision=0, ckpt_every=1)
    info = ctx.info
    K = ctx.K
    n_nodes = ctx.n_nodes
    region_points = int(info.region_points)
    V = torch.tensor(prob.V, dtype=torch.float64, device=dev)
    g_rho = torch.ones(n_nodes, dtype=torch.float64, device=dev)
    g_u = torch.ones(n_nodes, dtype=torch.float64, device=dev)
    dV = torch.zeros_like(V)
    dR = torch.zeros((max(prob.n_atoms, 1), 3), dtype=torch.float64, device=dev)
    mu = torch.empty((n_nodes, K + 1), dtype=torch.float64, device=dev)
    M = torch.empty(K + 1, dtype=torch.float64, device=dev)
    lam = torch.zeros(1, dtype=torch.float64, device=dev)
    Ne = prob.Ne if prob.Ne is not None else 0.0
    max_iter = 200 if prob.Ne is not None else 0
    if max_iter == 0:
        lam.fill_(prob.lambda_f)
    ev = {k: events(2) for k in ("fwd", "bwd")}
    times = {"fwd": [], "bwd": []}

    def step(timed):
        if timed:
            ev["fwd"][0].record()
        ctx.density(V, math.nan, math.nan, moments=mu, moment_sum=M)
        if timed:
            ev["fwd"][1].record()
        out = ctx.fermi_level(Ne=Ne, tol=1e-8, max_iter=max_iter, lambda_f=lam, device=dev)
        if timed:
            ev["bwd"][0].record()
        ctx.backward(g_rho, g_u, dV, dR if prob.n_atoms else None)
        if timed:
            ev["bwd"][1].record()
        return out

    for w in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        out = step(True)
        torch.cuda.synchronize()
        times["fwd"].append(ev["fwd"][0].elapsed_time(ev["fwd"][1]) * 1e-3)
        times["bwd"].append(ev["bwd"][0].elapsed_time(ev["bwd"][1]) * 1e-3)
        log(f"step {s + 1}/{args.steps}: forward {times['fwd'][-1]:.3f} s, "
            f"adjoint {times['bwd'][-1]:.3f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    value = n_nodes * K * args.steps / wall
    lam_v, rho, u, tot = out
    tot = tot.cpu().numpy()
    ctx.status()
    log(f"timed {args.steps} steps in {wall:.3f} s -> {value:.4e} node-steps/s; "
        f"N_e={tot[0]:.10f} lambda_f={lam_v.item():.10f} iters={int(tot[6])}")

    r = prob.fd_order // 2
    t_fwd = float(np.mean(times["fwd"]))
    t_bwd = float(np.mean(times["bwd"]))
    # LDS bytes of the local part: 4r neighbour values read per point and step
    rf = roofline_hbm("cheb_forward_kernel", bytes_forward(4) * region_points * K, t_fwd,
                      prob.name, flops=flops_app(r) * region_points * K,
                      lds_bytes=4 * r * 4 * region_points * K)
    rb = roofline_hbm("cheb_adjoint64_kernel", bytes_adjoint(8) * region_points * K, t_bwd,
                      prob.name, flops=(2 * K - 2) * flops_app(r) * region_points,
                      lds_bytes=2 * 4 * r * 8 * region_points * K)
    dominant, other = (rb, rf) if t_bwd >= t_fwd else (rf, rb)

    extra = {}
    tot_om, tot_tau = float(tot[4]), float(tot[5])
    lmin, lmax = tot_om - tot_tau, tot_om + tot_tau
    # entropy and band free energy from the last step's moments (Eq. (sq))
    s_q = torch.empty(n_nodes, dtype=torch.float64, device=dev)
    s_tot = torch.empty(2, dtype=torch.float64, device=dev)
    e = events(2)
    e[0].record()
    ctx.entropy(s_q, s_tot)
    e[1].record()
    torch.cuda.synchronize()
    s_tot = s_tot.cpu().numpy()
    extra["entropy"] = {"seconds": e[0].elapsed_time(e[1]) * 1e-3, "S": float(s_tot[0]),
                        "U_minus_kT_S": float(s_tot[1])}
    if not args.no_force and prob.n_atoms:
        extra["cc_force"] = force_leg(ctx, prob, tot, lam_v.item(), dev)
    rho_np = rho.cpu().numpy()
    mu_np = mu.cpu().numpy()
    ctx.close()
    del mu
    if not args.no_gauss:
        extra["lssgq"] = gauss_leg(prob, V, tot, region_points, dev)
    if not args.no_scf and prob.bc == 0 and prob.nodes is None and prob.n_atoms:
        sctx = sq.Context(prob, precision=1)
        extra["scf"] = scf_leg(sctx, prob, tot, dev)
        sctx.close()

    # accuracy against the FP64 oracle on sampled nodes
    import oracle as O
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(n_nodes, args.cpu_sample, replace=False))
    acc = None
    t_oracle_fwd = 0.0
    if not args.no_accuracy or not args.no_cpu_baseline:
        t_o = time.perf_counter()
        mu_ref = O.moments(prob, lmin, lmax, nodes=prob.node_list()[sample])
        t_oracle_fwd = time.perf_counter() - t_o
        c, _ = O.cheb_coeffs(O.KIND_G, lam_v.item(), prob.kT, lmin, lmax, K)
        rho_ref, _ = O.contract(mu_ref, c, c)
        drho = np.abs(rho_np[sample] - rho_ref)
        acc = dict(max_abs_drho=float(drho.max()),
                   rel_drho=float(drho.max() / np.abs(rho_np).max()),
                   max_abs_dmu=float(np.abs(mu_np[sample] - mu_ref).max()),
                   sample_nodes=int(sample.size), reference="FP64 oracle")
        log(f"accuracy vs oracle on {sample.size} nodes: max|drho| {drho.max():.3e}")
    if prob.n_atoms and not args.no_accuracy:
        extra["adjoint_accuracy"] = adjoint_accuracy(prob, lmin, lmax, lam_v.item(), 24, 22, dev)
        log(f"adjoint accuracy: dV rel {extra['adjoint_accuracy']['dV_rel']:.2e}, "
            f"dR rel {extra['adjoint_accuracy']['dR_rel']:.2e}")

    cpu = None
    if not args.no_cpu_baseline:
        a = np.ones((sample.size, K + 1))
        t_o = time.perf_counter()
        O.adjoint(prob, lmin, lmax, a, nodes=prob.node_list()[sample])
        t_oracle_bwd = time.perf_counter() - t_o
        t_cpu = t_oracle_fwd + t_oracle_bwd
        cores = O.num_threads()
        # one core, on a smaller sample of the same nodes
        one = sample[:64]
        O.set_num_threads(1)
        t1 = time.perf_counter()
        O.moments(prob, lmin, lmax, nodes=prob.node_list()[one])
        O.adjoint(prob, lmin, lmax, np.ones((one.size, K + 1)), nodes=prob.node_list()[one])
        t1 = time.perf_counter() - t1
        O.set_num_threads(cores)
        cpu = dict(value=sample.size * K / t_cpu, unit="node-steps/s", cores=cores,
                   kind="oracle", host_cpu=host_cpu(),
                   single_core_value=one.size * K / t1,
                   sample=f"{sample.size} random nodes of the same workload: oracle moments "
                          f"({t_oracle_fwd:.1f} s) + oracle adjoint ({t_oracle_bwd:.1f} s) on "
                          f"{cores} threads; {one.size} of them on 1 thread ({t1:.1f} s)")
        log(f"cpu baseline {cpu['value']:.3e} node-steps/s on {cores} threads, "
            f"{cpu['single_core_value']:.3e} on 1")

    if not args.no_fp64:
        ctx64 = sq.Context(prob, precision=0)
        mu64 = torch.empty((n_nodes, K + 1), dtype=torch.float64, device=dev)
        ctx64.density(V, lmin, lmax, moments=mu64)
        torch.cuda.synchronize()
        e = events(2)
        e[0].record()
        ctx64.density(V, lmin, lmax, moments=mu64)
        e[1].record()
        torch.cuda.synchronize()
        t64 = e[0].elapsed_time(e[1]) * 1e-3
        ctx64.close()
        del mu64
        extra["fp64_forward"] = dict(seconds=t64, node_steps_per_s=n_nodes * K / t64,
                                     fp32_speedup=t64 / t_fwd)
        log(f"FP64 forward {t64:.3f} s vs FP32 forward {t_fwd:.3f} s")
        # the FP32 adjoint variant (not the timed one: its gradient misses 1e-5)
        c32 = sq.Context(prob, precision=1, adjoint_precision=1, ckpt_every=1)
        c32.density(V, lmin, lmax)
        c32.fermi_level(max_iter=0, lambda_f=lam_v, want_fields=False, device=dev)
        c32.backward(g_rho, g_u, dV, dR if prob.n_atoms else None)
        torch.cuda.synchronize()
        e = events(2)
        e[0].record()
        c32.backward(g_rho, g_u, dV, dR if prob.n_atoms else None)
        e[1].record()
        torch.cuda.synchronize()
        c32.close()
        extra["fp32_adjoint_variant"] = {"seconds": e[0].elapsed_time(e[1]) * 1e-3,
                                         "note": "FP32 vectors; gradient error 1e-5..5e-4 "
                                                 "relative, so not the timed adjoint"}

    if not args.no_configs and args.config == 2:
        extra["config3"] = config3_leg(dev)
        extra["config4"] = config4_leg(dev)
        extra["config5"] = config5_leg(dev, args.c5_adjoint_stride, args.cpu_sample)

    line = {
        "metric": "SQ grid-node·Chebyshev-steps/s at 1 GPU; max |Δρ| vs FP64 oracle",
        "value": value,
        "unit": "node-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": prob.name,
            "grid": list(prob.n), "h": list(prob.h), "fd_order": prob.fd_order,
            "nodes": n_nodes, "region": list(info.max_region), "order": K, "kT": prob.kT,
            "atoms": prob.n_atoms, "Ne": prob.Ne, "region_points": region_points,
            "precision": "FP32 recurrence, FP64 moments/coefficients/bisection",
            "adjoint_precision": "FP64 vectors and accumulation",
            "step": "Lanczos bounds + forward + Fermi bisection + rho,u + adjoint (dV, dR)",
        },
        "roofline": dominant,
        "roofline_other": other,
        "times_s": {"forward_mean": t_fwd, "adjoint_mean": t_bwd},
        "region_point_steps_per_s": region_points * K * args.steps / wall,
        "accuracy": acc,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    log("done")
    print(json.dumps(line))


if __name__ == "__main__":
    main()
