"""Benchmark of the spectral-quadrature hot path on one MI355X.

One step = the whole path over the 64^3 Mg-like workload (96 atoms x 4
projectors, 27^3 node regions, K = 100, kT = 0.001 Ha, N_e = 192):
  spectral bounds (device FP64 Lanczos) -> scaled diagonal -> FP32 region
  recurrence with FP64 moments -> moment sum -> FP64 Fermi bisection ->
  coefficients -> pointwise rho, u -> adjoint (dV, dR).
Inputs are resident in HBM before the timed region.  Throughput is counted in
node-steps (one node advanced by one Chebyshev order; K per node per step).

Prints one JSON line (rank 0).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VALU = 256 * 4 * 16 * 2 * 2.4e9   # non-packed FP32 FMA: 78.6 TFLOP/s
PEAK_HBM = 8.0e12


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# sources each profiled kernel is compiled from (the host-side API does not
# change what a kernel fetches and writes)
_REGION = ("sq_internal.h", "sq_region.h")
KERNEL_SOURCES = {
    "cheb_forward_kernel": _REGION + ("sq_forward.hip",),
    "cheb_adjoint_kernel": _REGION + ("sq_adjoint_kernel.h", "sq_adjoint.hip",
                                      "sq_adjoint_r1.hip", "sq_adjoint_r2.hip",
                                      "sq_adjoint_r3.hip", "sq_adjoint_r4.hip",
                                      "sq_adjoint_r5.hip", "sq_adjoint_r6.hip"),
    "gauss_lanczos_kernel": _REGION + ("sq_gauss_lanczos.hip",),
    "gauss_eig_kernel": ("sq_internal.h", "sq_kernels.h", "sq_gauss.hip"),
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


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE
    summary, or None when it is missing or was taken from other kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_c2_periodic64_r6_K100.json")
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


def force_leg(ctx, prob, f_app, tot, lf, dev):
    """Clenshaw-Curtis nonlocal force (sq_nonlocal_force) at the Fermi level of
    the last timed step, timed with HIP events on the current stream."""
    import torch
    info = ctx.info
    f = torch.empty((ctx.n_atoms, 3), dtype=torch.float64, device=dev)
    ctx.nonlocal_force(f)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.nonlocal_force(f)
    e1.record()
    torch.cuda.synchronize()
    ctx.status()
    t = e0.elapsed_time(e1) * 1e-3
    nf, pts = int(info.n_force_nodes), int(info.force_region_points)
    achieved = pts * ctx.K * f_app / t / 1e12
    log(f"nonlocal force: {nf} nodes in supports, {t:.3f} s")
    # the oracle on the 4 nodes nearest to atom 0 (all inside its support)
    import oracle as O
    n = np.asarray(prob.n)
    pos = np.asarray(prob.atom_pos[0]) / np.asarray(prob.h)
    grid = np.stack(np.meshgrid(*(np.arange(k) for k in n), indexing="ij"), -1).reshape(-1, 3)
    d = np.abs(grid - pos[None, :])
    d = np.minimum(d, n[None, :] - d) if prob.bc == 0 else d
    idx = np.argsort((d ** 2).sum(1))[:4]
    nodes = grid[idx, 0] + n[0] * (grid[idx, 1] + n[1] * grid[idx, 2])
    om, tau = float(tot[4]), float(tot[5])
    t_o = time.perf_counter()
    O.cc_nonlocal_force(prob, om - tau, om + tau, lf, nodes=nodes)
    t_o = time.perf_counter() - t_o
    cpu = dict(value=nodes.size * ctx.K / t_o, unit="node-steps/s", cores=1,
               kind="oracle", sample=f"{nodes.size} nodes nearest to atom 0 ({t_o:.1f} s)")
    return {"seconds": t, "force_nodes": nf, "node_steps_per_s": nf * ctx.K / t,
            "cpu_baseline": cpu,
            "roofline": dict(bound="alu", kernel="cc_force_kernel", achieved=achieved,
                             peak=PEAK_FP32_VALU / 1e12, unit="TFLOP/s",
                             frac=achieved / (PEAK_FP32_VALU / 1e12),
                             traffic=recorded_traffic("cc_force_kernel")),
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


def gauss_leg(ctx, prob, V, tot, f_app, region_points, dev):
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
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
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
    achieved = region_points * K * f_app / t_rules / 1e12
    ctx.close()
    return {
        "metric": "node-Lanczos-steps/s",
        "order": K,
        "value": n * K / (t_rules + t_fields),
        "seconds": {"rules": t_rules, "fermi_fields": t_fields},
        "roofline": dict(bound="alu", kernel="gauss_lanczos_kernel + gauss_eig_kernel",
                         achieved=achieved, peak=PEAK_FP32_VALU / 1e12, unit="TFLOP/s",
                         frac=achieved / (PEAK_FP32_VALU / 1e12),
                         traffic=recorded_traffic("gauss_lanczos_kernel")),
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
    log(f"workload {prob.name}: {prob.n_nodes} nodes, K={prob.order}, atoms={prob.n_atoms}")
    # adjoint keeps every v_k of its in-flight regions (ckpt_every = 1)
    ctx = sq.Context(prob, precision=1, adjoint_precision=1, ckpt_every=1)
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
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for k in ("fwd", "bwd")}
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

    # roofline of the two region kernels.  Algorithmic flops of one application of
    # w = 2 Hs v - u at one region point: 3r symmetric pairs (add + FMA) = 9r, the
    # diagonal FMA and the recurrence FMA = 4 (the nonlocal term is not counted).
    # Forward: K applications.  Adjoint (store-all): K-1 forward applications to
    # store v_0..v_{K-1}, K-1 adjoint applications and K FMAs into dV.
    r = prob.fd_order // 2
    f_app = 9 * r + 4
    flops_fwd = region_points * K * f_app
    flops_bwd = region_points * ((2 * K - 2) * f_app + 2 * K)
    t_fwd = float(np.mean(times["fwd"]))
    t_bwd = float(np.mean(times["bwd"]))
    rf = dict(bound="alu", achieved=flops_fwd / t_fwd / 1e12, peak=PEAK_FP32_VALU / 1e12,
              unit="TFLOP/s", traffic=None)
    rb = dict(bound="alu", achieved=flops_bwd / t_bwd / 1e12, peak=PEAK_FP32_VALU / 1e12,
              unit="TFLOP/s", traffic=None)
    for d in (rf, rb):
        d["frac"] = d["achieved"] / d["peak"]
    rf["kernel"], rb["kernel"] = "cheb_forward_kernel", "cheb_adjoint_kernel"
    rf["traffic"] = recorded_traffic("cheb_forward_kernel")
    rb["traffic"] = recorded_traffic("cheb_adjoint_kernel")
    dominant, other = (rb, rf) if t_bwd >= t_fwd else (rf, rb)

    # accuracy against the FP64 oracle on sampled nodes
    extra = {}
    # entropy and band free energy from the last step's moments (Eq. (sq))
    s_q = torch.empty(n_nodes, dtype=torch.float64, device=dev)
    s_tot = torch.empty(2, dtype=torch.float64, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.entropy(s_q, s_tot)
    e1.record()
    torch.cuda.synchronize()
    s_tot = s_tot.cpu().numpy()
    extra["entropy"] = {"seconds": e0.elapsed_time(e1) * 1e-3, "S": float(s_tot[0]),
                        "U_minus_kT_S": float(s_tot[1])}
    if not args.no_force and prob.n_atoms:
        extra["cc_force"] = force_leg(ctx, prob, f_app, tot, lam_v.item(), dev)
    if not args.no_gauss:
        extra["lssgq"] = gauss_leg(ctx, prob, V, tot, f_app, region_points, dev)
    if not args.no_scf and prob.bc == 0 and prob.nodes is None and prob.n_atoms:
        extra["scf"] = scf_leg(ctx, prob, tot, dev)
    rho_np = rho.cpu().numpy()
    tot_om, tot_tau = float(tot[4]), float(tot[5])
    lmin, lmax = tot_om - tot_tau, tot_om + tot_tau
    import oracle as O
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(n_nodes, args.cpu_sample, replace=False))
    t_o = time.perf_counter()
    mu_ref = O.moments(prob, lmin, lmax, nodes=prob.node_list()[sample])
    t_oracle_fwd = time.perf_counter() - t_o
    c, _ = O.cheb_coeffs(O.KIND_G, lam_v.item(), prob.kT, lmin, lmax, K)
    rho_ref, _ = O.contract(mu_ref, c, c)
    drho = np.abs(rho_np[sample] - rho_ref)
    extra["accuracy"] = dict(max_abs_drho=float(drho.max()),
                             rel_drho=float(drho.max() / np.abs(rho_np).max()),
                             max_abs_dmu=float(np.abs(mu.cpu().numpy()[sample] - mu_ref).max()),
                             sample_nodes=int(sample.size), reference="FP64 oracle")
    log(f"accuracy vs oracle on {sample.size} nodes: max|drho| {drho.max():.3e}")

    cpu = None
    if not args.no_cpu_baseline:
        a = np.ones((sample.size, K + 1))
        t_o = time.perf_counter()
        O.adjoint(prob, lmin, lmax, a, nodes=prob.node_list()[sample])
        t_oracle_bwd = time.perf_counter() - t_o
        t_cpu = t_oracle_fwd + t_oracle_bwd
        cpu = dict(value=sample.size * K / t_cpu, unit="node-steps/s", cores=O.num_threads(),
                   kind="oracle",
                   sample=f"{sample.size} random nodes of the same workload: oracle moments "
                          f"({t_oracle_fwd:.1f} s) + oracle adjoint ({t_oracle_bwd:.1f} s)")
        log(f"cpu baseline {cpu['value']:.3e} node-steps/s on {cpu['cores']} threads")

    if not args.no_fp64:
        ctx64 = sq.Context(prob, precision=0)
        mu64 = torch.empty_like(mu)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ctx64.density(V, lmin, lmax, moments=mu64)
        torch.cuda.synchronize()
        e0.record()
        ctx64.density(V, lmin, lmax, moments=mu64)
        e1.record()
        torch.cuda.synchronize()
        t64 = e0.elapsed_time(e1) * 1e-3
        ctx64.close()
        extra["fp64_forward"] = dict(seconds=t64, node_steps_per_s=n_nodes * K / t64,
                                     fp32_speedup=t64 / t_fwd)
        log(f"FP64 forward {t64:.3f} s vs FP32 forward {t_fwd:.3f} s")

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
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": prob.name,
            "grid": list(prob.n), "h": list(prob.h), "fd_order": prob.fd_order,
            "nodes": n_nodes, "region": list(info.max_region), "order": K, "kT": prob.kT,
            "atoms": prob.n_atoms, "Ne": prob.Ne, "region_points": region_points,
            "precision": "FP32 recurrence, FP64 moments/coefficients/bisection",
            "adjoint_precision": "FP32 vectors, FP64 dV/dR accumulation",
            "step": "Lanczos bounds + forward + Fermi bisection + rho,u + adjoint (dV, dR)",
        },
        "roofline": dominant,
        "roofline_other": other,
        "times_s": {"forward_mean": t_fwd, "adjoint_mean": t_bwd},
        "region_point_steps_per_s": region_points * K * args.steps / wall,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
