"""torch.autograd.Function wrapper and HIP-graph replay of the whole path.

SQDensity: rho, u from the C ABI against the FP64 oracle, and autograd
gradients (dV, dR) against the oracle adjoint (FP64 context: 1e-10).
Graph: sq_density (device Lanczos) + sq_fermi_level + sq_density_backward
captured once and replayed with new potentials between replays; every replay
is checked against an eager run on the same input (the projector dot products
and dV, dR are reduced with atomics whose order varies between runs, so the
comparison allows 1e-11 (FP64) or 2e-5 (FP32) of the scale).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2011_13517_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _problem():
    return synth.small_problem(61, n=(12, 13, 12), rcut=(2, 2, 3), n_atoms=3, rc=1.4, order=14,
                               kT=0.2, fd_order=6)


def test_sqdensity_autograd_vs_oracle():
    from paper_2011_13517_amd import sq
    print("[case] SQDensity autograd", flush=True)
    prob = _problem()
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    lf = 0.5 * (lmin + lmax) - 0.25 * (lmax - lmin)
    ctx = sq.Context(prob, precision=0)
    V = torch.tensor(prob.V, dtype=torch.float64, device="cuda", requires_grad=True)
    R = torch.zeros((prob.n_atoms, 3), dtype=torch.float64, device="cuda", requires_grad=True)
    lam_in = torch.tensor([lf], dtype=torch.float64, device="cuda")
    rho, u, lam = sq.SQDensity.apply(V, R, ctx, 0.0, 0.0, 0, (lmin, lmax), lam_in)
    rng = np.random.default_rng(9)
    g_rho, g_u = rng.normal(size=prob.n_nodes), rng.normal(size=prob.n_nodes)
    y = (rho * torch.tensor(g_rho, device="cuda")).sum() + \
        (u * torch.tensor(g_u, device="cuda")).sum()
    y.backward()
    mu = O.moments(prob, lmin, lmax)
    c, _ = O.cheb_coeffs(O.KIND_G, lf, prob.kT, lmin, lmax, prob.order)
    d, _ = O.cheb_coeffs(O.KIND_U, lf, prob.kT, lmin, lmax, prob.order)
    rho_ref, u_ref = O.contract(mu, c, d)
    assert np.abs(rho.detach().cpu().numpy() - rho_ref).max() <= 1e-10 * np.abs(rho_ref).max()
    assert np.abs(u.detach().cpu().numpy() - u_ref).max() <= 1e-10 * np.abs(u_ref).max()
    cp, dp = c.copy(), d.copy()
    cp[0] *= 0.5
    dp[0] *= 0.5
    a = 2.0 * (g_rho[:, None] * cp[None, :] + g_u[:, None] * dp[None, :])
    gV, dR = O.adjoint(prob, lmin, lmax, a)
    dV = V.grad.cpu().numpy()
    assert np.abs(dV - gV).max() <= 1e-10 * np.abs(gV).max()
    assert np.abs(R.grad.cpu().numpy() - dR).max() <= 1e-10 * np.abs(dR).max()
    # a second forward on the same context invalidates the first graph's backward
    rho2, u2, _ = sq.SQDensity.apply(V, R, ctx, 0.0, 0.0, 0, (lmin, lmax), lam_in)
    with pytest.raises(RuntimeError, match="another forward"):
        rho.sum().backward()
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_matches_eager(precision):
    from paper_2011_13517_amd import sq
    print(f"[case] graph replay precision={precision}", flush=True)
    prob = _problem()
    Ne = 0.5 * prob.n_nodes * 2 * 0.3
    ctx = sq.Context(prob, precision=precision)
    dev = torch.device("cuda")
    n, K = ctx.n_nodes, ctx.K
    V0 = torch.tensor(prob.V, dtype=torch.float64, device=dev)
    V = V0.clone()
    mu = torch.empty((n, K + 1), dtype=torch.float64, device=dev)
    M = torch.empty(K + 1, dtype=torch.float64, device=dev)
    lam = torch.zeros(1, dtype=torch.float64, device=dev)
    rho = torch.empty(n, dtype=torch.float64, device=dev)
    u = torch.empty(n, dtype=torch.float64, device=dev)
    tot = torch.empty(8, dtype=torch.float64, device=dev)
    g = torch.ones(n, dtype=torch.float64, device=dev)
    dV = torch.zeros_like(V)
    dR = torch.zeros((prob.n_atoms, 3), dtype=torch.float64, device=dev)

    def step():
        ctx.density(V, math.nan, math.nan, moments=mu, moment_sum=M)
        ctx.fermi_level(Ne=Ne, tol=1e-9, max_iter=200, lambda_f=lam, rho=rho, u=u, totals=tot)
        dV.zero_()
        dR.zero_()
        ctx.backward(g, g, dV, dR)

    def snapshot():
        torch.cuda.synchronize()
        return [t.clone() for t in (mu, M, lam, rho, u, tot, dV, dR)]

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()                      # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    rng = np.random.default_rng(3)
    for rep in range(3):
        pert = torch.tensor(rng.uniform(-0.05, 0.05, size=prob.V.shape), device=dev)
        V.copy_(V0 + pert)
        graph.replay()
        got = snapshot()
        step()                      # eager on the same input
        ref = snapshot()
        assert ctx.status() == 0
        # mu, M, lambda_f, rho, u, totals, dV, dR: the projector dot products and
        # dV / dR are reduced with atomics, so the summation order may differ
        # between runs; a stale input would differ by O(0.05)
        tol = 1e-11 if precision == 0 else 2e-5
        for i, (a, b) in enumerate(zip(got, ref)):
            if i == 5:
                a, b = a[:6], b[:6]          # iteration count and status may differ by one step
            scale = max(b.abs().max().item(), 1.0)
            assert (a - b).abs().max().item() <= tol * scale, (rep, i)
        assert abs(got[5][0].item() - Ne) < 1e-8
    ctx.close()


def test_graph_replay_gauss_and_force():
    """The Gauss-quadrature rules, their Fermi level and fields, and the
    Clenshaw-Curtis nonlocal force captured in one HIP graph (after an eager
    warm-up that makes the one-time allocations) and replayed on changed inputs,
    each replay checked against the eager result (FP64)."""
    from paper_2011_13517_amd import sq
    print("[case] graph replay gauss + force", flush=True)
    prob = _problem()
    Ne = 0.3 * prob.n_nodes
    ctx = sq.Context(prob, precision=0)
    dev = torch.device("cuda")
    n, K = ctx.n_nodes, ctx.K
    V0 = torch.tensor(prob.V, dtype=torch.float64, device=dev)
    V = V0.clone()
    mu = torch.empty((n, K + 1), dtype=torch.float64, device=dev)
    lam = torch.zeros(1, dtype=torch.float64, device=dev)
    glam = torch.zeros(1, dtype=torch.float64, device=dev)
    nodes = torch.empty((n, K), dtype=torch.float64, device=dev)
    wts = torch.empty_like(nodes)
    rho, u, s = (torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3))
    tot = torch.empty(8, dtype=torch.float64, device=dev)
    f = torch.empty((prob.n_atoms, 3), dtype=torch.float64, device=dev)

    def step():
        ctx.density(V, math.nan, math.nan, moments=mu)
        ctx.fermi_level(Ne=Ne, tol=1e-9, max_iter=200, lambda_f=lam, want_fields=False)
        ctx.nonlocal_force(f)
        ctx.gauss_density(V, math.nan, math.nan, nodes=nodes, weights=wts)
        ctx.gauss_fermi_level(Ne=Ne, tol=1e-9, max_iter=200, lambda_f=glam, rho=rho, u=u, s=s,
                              totals=tot)

    def snapshot():
        torch.cuda.synchronize()
        return [t.clone() for t in (nodes, wts, glam, rho, u, s, tot, f)]

    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        step()
    torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    rng = np.random.default_rng(5)
    for rep in range(3):
        pert = torch.tensor(rng.uniform(-0.05, 0.05, size=prob.V.shape), device=dev)
        V.copy_(V0 + pert)
        graph.replay()
        got = snapshot()
        step()
        ref = snapshot()
        assert ctx.status() == 0
        # projector dot products (both sweeps) and the force sums use atomics, so
        # low-order bits may differ; a stale input would differ by O(0.05)
        for i, (a, b) in enumerate(zip(got, ref)):
            if i == 6:
                a, b = a[:6], b[:6]
            tol = 1e-11
            scale = max(b.abs().max().item(), 1.0)
            assert (a - b).abs().max().item() <= tol * scale, (rep, i)
        assert abs(got[6][0].item() - Ne) < 1e-8
    ctx.close()


def test_graph_replay_config3_split_plan():
    """Config 3 (4096 uneven Dirichlet-clipped regions, K = 100, FP32) with one
    persistent launch per edge bucket (several work counters and launches):
    sq_density + sq_fermi_level (fixed lambda_f) captured once and replayed with
    new potentials; every replay against an eager run on the same input, and the
    replay of the unperturbed potential against the oracle on sampled nodes."""
    from paper_2011_13517_amd import sq
    print("[case] graph replay config3 split plan", flush=True)
    prob = synth.config(3)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    ctx = sq.Context(prob, precision=1, tune=1)
    assert ctx.info.n_launches > 1
    dev = torch.device("cuda")
    n, K = ctx.n_nodes, ctx.K
    V0 = torch.tensor(prob.V, dtype=torch.float64, device=dev)
    V = V0.clone()
    mu = torch.empty((n, K + 1), dtype=torch.float64, device=dev)
    M = torch.empty(K + 1, dtype=torch.float64, device=dev)
    lam = torch.tensor([prob.lambda_f], dtype=torch.float64, device=dev)
    rho = torch.empty(n, dtype=torch.float64, device=dev)
    u = torch.empty(n, dtype=torch.float64, device=dev)
    tot = torch.empty(8, dtype=torch.float64, device=dev)

    def step():
        ctx.density(V, lmin, lmax, moments=mu, moment_sum=M)
        ctx.fermi_level(max_iter=0, lambda_f=lam, rho=rho, u=u, totals=tot)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    rng = np.random.default_rng(7)
    for rep in range(3):
        pert = 0.0 if rep == 0 else 0.05
        V.copy_(V0 + torch.tensor(rng.uniform(-pert, pert, size=prob.V.shape), device=dev))
        graph.replay()
        torch.cuda.synchronize()
        got = [t.clone() for t in (mu, rho, u)]
        step()
        torch.cuda.synchronize()
        assert ctx.status() == 0
        for a, b in zip(got, (mu, rho, u)):
            # FP32 projector sums use LDS atomics (order may vary); a stale input
            # would differ by O(0.05)
            assert (a - b).abs().max().item() <= 2e-5 * max(b.abs().max().item(), 1.0)
        if rep == 0:
            pick = np.sort(rng.choice(n, 12, replace=False))
            mu_ref = O.moments(prob, lmin, lmax, nodes=prob.nodes[pick],
                               node_m=prob.node_rcut[pick])
            assert np.abs(got[0].cpu().numpy()[pick] - mu_ref).max() < K * 2.0 ** -24 * 8
    ctx.close()


def test_graph_replay_edge27_fp64_adjoint():
    """The benchmarked sequence on 512 random nodes of the 64^3 workload (27^3
    regions, r = 6, 96 atoms, K = 100): device bounds + FP32 forward + Fermi
    level (fixed lambda_f) + the FP64 edge-27 adjoint (dV, dR), captured once and
    replayed with new potentials; every replay against an eager run on the same
    input (the adjoint itself is held to the oracle in test_gpu_adjoint.py)."""
    from paper_2011_13517_amd import sq
    print("[case] graph replay edge27 fp64 adjoint", flush=True)
    prob = synth.config(2)
    rng = np.random.default_rng(27)
    nodes = np.sort(rng.choice(prob.n_nodes, 512, replace=False)).astype(np.int64)
    ctx = sq.Context(prob, precision=1, nodes=nodes, adjoint_precision=0, ckpt_every=1)
    assert tuple(ctx.info.max_region) == (27, 27, 27)
    dev = torch.device("cuda")
    n, K = ctx.n_nodes, ctx.K
    V0 = torch.tensor(prob.V, dtype=torch.float64, device=dev)
    V = V0.clone()
    mu = torch.empty((n, K + 1), dtype=torch.float64, device=dev)
    M = torch.empty(K + 1, dtype=torch.float64, device=dev)
    lam = torch.tensor([0.0973], dtype=torch.float64, device=dev)
    rho = torch.empty(n, dtype=torch.float64, device=dev)
    u = torch.empty(n, dtype=torch.float64, device=dev)
    tot = torch.empty(8, dtype=torch.float64, device=dev)
    g_rho = torch.tensor(rng.normal(size=n), dtype=torch.float64, device=dev)
    g_u = torch.tensor(rng.normal(size=n), dtype=torch.float64, device=dev)
    dV = torch.zeros_like(V)
    dR = torch.zeros((prob.n_atoms, 3), dtype=torch.float64, device=dev)

    def step():
        ctx.density(V, math.nan, math.nan, moments=mu, moment_sum=M)
        ctx.fermi_level(max_iter=0, lambda_f=lam, rho=rho, u=u, totals=tot)
        dV.zero_()
        dR.zero_()
        ctx.backward(g_rho, g_u, dV, dR)

    def snapshot():
        torch.cuda.synchronize()
        return [t.clone() for t in (mu, rho, u, dV, dR)]

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        pert = 0.0 if rep == 0 else 0.05
        V.copy_(V0 + torch.tensor(rng.uniform(-pert, pert, size=prob.V.shape), device=dev))
        graph.replay()
        got = snapshot()
        step()
        ref = snapshot()
        assert ctx.status() == 0
        # projections and dV / dR are reduced with atomics (order may differ);
        # a stale input would differ by O(0.05)
        for i, (a, b) in enumerate(zip(got, ref)):
            tol = 2e-5 if i < 3 else 1e-11
            scale = max(b.abs().max().item(), 1e-300)
            assert (a - b).abs().max().item() <= tol * scale, (rep, i)
        assert dR.abs().max().item() > 0
    ctx.close()
