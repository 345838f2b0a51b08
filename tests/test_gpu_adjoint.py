"""Adjoint (sq_density_backward) through the C ABI against the FP64 oracle.

Tolerances: the FP64 adjoint (the default adjoint_precision, also behind an FP32
forward context, and the precision the benchmark times) within 1e-10 max-norm
relative of the oracle, at every region edge including 27.  The optional FP32
adjoint (FP32 primal and adjoint vectors) within 1e-5 at small K; at K = 80..100
the gradient sum dV(x) = sum_k alpha_k vt_{k+1}(x) v_k(x) cancels by three to
four orders of magnitude, and FP32 rounding of any one of v_k, vt_k or the sum
(2^-24 per step over 2K steps) leaves 1e-5..5e-4 max-norm relative error, so
that variant is held to 1e-3 and is not the benchmarked one.  Finite
differences always use the FP64 forward pass: a fourth-order central difference
at delta = 1e-4 Ha agrees with the adjoint to ~3e-8 relative (truncation
delta^4 and rounding eps |y| / delta both below that), held to 2e-7.
"""
import numpy as np
import pytest

import oracle as O
from paper_2011_13517_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cotangents(n, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=n), rng.normal(size=n)


def oracle_adjoint(prob, lmin, lmax, lf, g_rho, g_u, nodes=None, node_m=None):
    K = prob.order
    c, _ = O.cheb_coeffs(O.KIND_G, lf, prob.kT, lmin, lmax, K)
    d, _ = O.cheb_coeffs(O.KIND_U, lf, prob.kT, lmin, lmax, K)
    c[0] *= 0.5
    d[0] *= 0.5
    a = 2.0 * (g_rho[:, None] * c[None, :] + g_u[:, None] * d[None, :])
    return O.adjoint(prob, lmin, lmax, a, nodes=nodes, node_m=node_m,
                     with_dR=prob.n_atoms > 0)


def gpu_adjoint(prob, lmin, lmax, lf, g_rho, g_u, precision, nodes=None, node_rcut=None,
                ckpt_every=0, with_dR=True, adjoint_precision=0):
    from paper_2011_13517_amd import sq
    ctx = sq.Context(prob, precision=precision, nodes=nodes, node_rcut=node_rcut,
                     ckpt_every=ckpt_every, adjoint_precision=adjoint_precision)
    V = torch.tensor(prob.V, dtype=torch.float64, device="cuda")
    ctx.density(V, lmin, lmax)
    lam = torch.tensor([lf], dtype=torch.float64, device="cuda")
    ctx.fermi_level(max_iter=0, lambda_f=lam, want_fields=False)
    gr = torch.tensor(g_rho, dtype=torch.float64, device="cuda")
    gu = torch.tensor(g_u, dtype=torch.float64, device="cuda")
    dV = torch.zeros_like(V)
    dR = torch.zeros((prob.n_atoms, 3), dtype=torch.float64, device="cuda") \
        if (with_dR and prob.n_atoms) else None
    ctx.backward(gr, gu, dV, dR)
    torch.cuda.synchronize()
    ctx.status()
    ctx.close()
    return dV.cpu().numpy(), (dR.cpu().numpy() if dR is not None else None)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("bc", [synth.BC_PERIODIC, synth.BC_DIRICHLET, synth.BC_EMBEDDED])
# ckpt 1 keeps every v_k (store-all), 0 picks store-all when it fits, C > 1 rebuilds
@pytest.mark.parametrize("precision,aprec,ckpt", [(0, 0, 3), (0, 0, 1), (1, 1, 2), (1, 1, 10),
                                                  (1, 1, 1), (1, 0, 4), (1, 0, 0)])
def test_adjoint_small(bc, precision, aprec, ckpt):
    print(f"[case] adjoint small bc={bc} precision={precision}/{aprec} ckpt={ckpt}", flush=True)
    prob = synth.small_problem(51 + bc, n=(13, 14, 12), bc=bc, rcut=(2, 3, 2), n_atoms=4, rc=1.4,
                               order=13, kT=0.2, fd_order=6)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    lf = 0.5 * (lmin + lmax) - 0.3 * (lmax - lmin)
    n = prob.n_nodes
    g_rho, g_u = _cotangents(n, 1)
    gV, dR = oracle_adjoint(prob, lmin, lmax, lf, g_rho, g_u)
    dV_g, dR_g = gpu_adjoint(prob, lmin, lmax, lf, g_rho, g_u, precision, ckpt_every=ckpt,
                             adjoint_precision=aprec)
    tol = 1e-10 if aprec == 0 else 1e-5
    assert rel(dV_g, gV) < tol
    assert rel(dR_g, dR) < tol


def test_adjoint_accumulates_and_dV_only():
    prob = synth.small_problem(55, n=(12, 12, 12), rcut=(2, 2, 2), n_atoms=2, rc=1.3, order=9,
                               kT=0.2)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    lf = 0.5 * (lmin + lmax)
    g_rho, g_u = _cotangents(prob.n_nodes, 2)
    gV, _ = oracle_adjoint(prob, lmin, lmax, lf, g_rho, g_u)
    dV_g, dR_g = gpu_adjoint(prob, lmin, lmax, lf, g_rho, g_u, 0, with_dR=False)
    assert dR_g is None and rel(dV_g, gV) < 1e-10


def _fd_directional(prob, lmin, lmax, lf, g_rho, g_u, nodes, dvec, delta=1e-4):
    """Fourth-order central difference of y = sum g_rho rho + g_u u along dvec,
    from the FP64 forward pass on the node subset."""
    from paper_2011_13517_amd import sq
    ys = {}
    for s in (2, 1, -1, -2):
        ctx = sq.Context(prob, precision=0, nodes=nodes)
        V = torch.tensor(prob.V + s * delta * dvec, dtype=torch.float64, device="cuda")
        ctx.density(V, lmin, lmax)
        lam = torch.tensor([lf], dtype=torch.float64, device="cuda")
        _, rho, u, _ = ctx.fermi_level(max_iter=0, lambda_f=lam)
        ys[s] = float((g_rho * rho.cpu().numpy()).sum() + (g_u * u.cpu().numpy()).sum())
        ctx.close()
    return (-ys[2] + 8 * ys[1] - 8 * ys[-1] + ys[-2]) / (12 * delta)


def test_adjoint_config4_nodes_vs_oracle_and_fd():
    """Config 4 geometry (48^3, 21^3 regions, K = 80, 63 atoms, one vacancy) on a
    node subset: FP64 adjoint (FP64 and FP32 forward contexts) vs oracle at 1e-10,
    the optional FP32 adjoint at its bound, and a central difference of the FP64
    forward pass along a random potential direction (delta = 1e-4 Ha)."""
    print("[case] adjoint config4 subset", flush=True)
    prob = synth.config(4)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    lf = -0.05
    rng = np.random.default_rng(4)
    nodes = np.sort(rng.choice(prob.n_nodes, 24, replace=False))
    g_rho, g_u = _cotangents(nodes.size, 3)
    gV, dR = oracle_adjoint(prob, lmin, lmax, lf, g_rho, g_u, nodes=nodes)
    dV64, dR64 = gpu_adjoint(prob, lmin, lmax, lf, g_rho, g_u, 0, nodes=nodes)
    dVm, dRm = gpu_adjoint(prob, lmin, lmax, lf, g_rho, g_u, 1, nodes=nodes, adjoint_precision=0)
    dV32, dR32 = gpu_adjoint(prob, lmin, lmax, lf, g_rho, g_u, 1, nodes=nodes,
                             adjoint_precision=1)
    assert rel(dV64, gV) < 1e-10 and rel(dR64, dR) < 1e-10
    assert rel(dVm, gV) < 1e-10 and rel(dRm, dR) < 1e-10
    print(f"FP32 adjoint at K=80: dV rel {rel(dV32, gV):.2e}, dR rel {rel(dR32, dR):.2e}")
    assert rel(dV32, gV) < 1e-3 and rel(dR32, dR) < 1e-3
    dvec = np.zeros(prob.V.size)
    pts = rng.choice(np.flatnonzero(gV != 0), 512, replace=False)
    dvec[pts] = rng.uniform(-1, 1, 512)
    fd = _fd_directional(prob, lmin, lmax, lf, g_rho, g_u, nodes, dvec)
    ad = float(dV64 @ dvec)
    print(f"directional derivative: fd {fd:.12e} adjoint {ad:.12e}")
    assert abs(fd - ad) < 2e-7 * abs(ad), (fd, ad)


def test_adjoint_config2_bench_launch():
    """The benchmarked configuration (64^3, 27^3 regions, 12th-order FD, K = 100,
    96 atoms) with the adjoint in the precision the benchmark times (FP64, the
    edge-27 kernel) behind the FP32 forward context: sampled nodes against the
    FP64 oracle at 1e-10 for dV and dR, and a central difference of the FP64
    forward pass along a random potential direction."""
    print("[case] adjoint config2 sample FP64 edge 27", flush=True)
    prob = synth.config(2)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    lf = 0.5 * (lmin + lmax) - 0.4 * (lmax - lmin)
    rng = np.random.default_rng(22)
    nodes = np.sort(rng.choice(prob.n_nodes, 12, replace=False))
    g_rho, g_u = _cotangents(nodes.size, 5)
    gV, dR = oracle_adjoint(prob, lmin, lmax, lf, g_rho, g_u, nodes=nodes)
    dV, dRg = gpu_adjoint(prob, lmin, lmax, lf, g_rho, g_u, 1, nodes=nodes, ckpt_every=1,
                          adjoint_precision=0)
    print(f"FP64 adjoint at K=100, 27^3: dV rel {rel(dV, gV):.2e}, dR rel {rel(dRg, dR):.2e}")
    assert rel(dV, gV) < 1e-10 and rel(dRg, dR) < 1e-10
    dvec = np.zeros(prob.V.size)
    pts = rng.choice(np.flatnonzero(gV != 0), 512, replace=False)
    dvec[pts] = rng.uniform(-1, 1, 512)
    fd = _fd_directional(prob, lmin, lmax, lf, g_rho, g_u, nodes, dvec)
    ad = float(dV @ dvec)
    print(f"directional derivative: fd {fd:.12e} adjoint {ad:.12e}")
    assert abs(fd - ad) < 2e-7 * abs(ad), (fd, ad)


@pytest.mark.parametrize("ckpt", [0, 7])
def test_fp32_adjoint_config2(ckpt):
    """The optional FP32 adjoint at edge 27 (store-all by default; rebuild with
    ckpt 7) on sampled nodes against the FP64 oracle, at the FP32 gradient bound
    of 1e-3 (see the module docstring)."""
    print(f"[case] FP32 adjoint config2 sample ckpt={ckpt}", flush=True)
    prob = synth.config(2)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    lf = 0.5 * (lmin + lmax) - 0.4 * (lmax - lmin)
    rng = np.random.default_rng(22)
    nodes = np.sort(rng.choice(prob.n_nodes, 12, replace=False))
    g_rho, g_u = _cotangents(nodes.size, 5)
    gV, dR = oracle_adjoint(prob, lmin, lmax, lf, g_rho, g_u, nodes=nodes)
    dV32, dR32 = gpu_adjoint(prob, lmin, lmax, lf, g_rho, g_u, 1, nodes=nodes, ckpt_every=ckpt,
                             adjoint_precision=1)
    print(f"FP32 adjoint at K=100, 27^3: dV rel {rel(dV32, gV):.2e}, dR rel {rel(dR32, dR):.2e}")
    assert rel(dV32, gV) < 1e-3 and rel(dR32, dR) < 1e-3


def test_adjoint_config5_embedded_nodes():
    """Embedded 128^3 workload (V and projectors on the 154^3 padded grid, K = 120):
    the FP64 edge-27 adjoint on sampled nodes, the corners of Omega (regions
    reaching into the padding) among them, against the oracle at 1e-10."""
    print("[case] adjoint config5 embedded sample", flush=True)
    prob = synth.config(5)
    lmin, lmax = O.gershgorin(prob)
    n0, n1, n2 = prob.n
    corners = [i + n0 * (j + n1 * k) for i in (0, n0 - 1) for j in (0, n1 - 1)
               for k in (0, n2 - 1)]
    rng = np.random.default_rng(57)
    nodes = np.unique(np.concatenate([corners, rng.choice(prob.n_nodes, 8, replace=False)]))
    lf = 0.5 * (lmin + lmax) - 0.45 * (lmax - lmin)
    g_rho, g_u = _cotangents(nodes.size, 7)
    gV, dR = oracle_adjoint(prob, lmin, lmax, lf, g_rho, g_u, nodes=nodes)
    dV, dRg = gpu_adjoint(prob, lmin, lmax, lf, g_rho, g_u, 1, nodes=nodes, adjoint_precision=0)
    print(f"config 5 FP64 adjoint: dV rel {rel(dV, gV):.2e}, dR rel {rel(dRg, dR):.2e}")
    assert np.abs(dR).max() > 0
    assert rel(dV, gV) < 1e-10 and rel(dRg, dR) < 1e-10


@pytest.mark.parametrize("order", [1, 2, 11, 12])
def test_fp64_adjoint_edge27_clipped_boxes(order):
    """The FP64 edge-27 kernel on ragged Dirichlet-clipped boxes (edges 14..27 per
    axis, some in the 27 bucket with dz < 27), K = 1 (no recurrence step), K = 2
    (one), odd and even K, dV + dR and dV alone, against the oracle at 1e-10."""
    print(f"[case] FP64 adjoint edge27 clipped K={order}", flush=True)
    prob = synth.small_problem(81, n=(30, 28, 32), h=(0.5, 0.5, 0.5), bc=synth.BC_DIRICHLET,
                               rcut=(13, 13, 13), n_atoms=6, rc=1.4, order=order, kT=0.2,
                               fd_order=6)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    lf = 0.5 * (lmin + lmax) - 0.3 * (lmax - lmin)
    n0, n1, n2 = prob.n
    rng = np.random.default_rng(order)
    picks = [0, n0 - 1 + n0 * (n1 - 1) * n2 // n2, (n0 // 2) + n0 * ((n1 // 2) + n1 * (n2 // 2))]
    nodes = np.unique(np.concatenate([picks, rng.choice(prob.n_nodes, 9, replace=False)]))
    g_rho, g_u = _cotangents(nodes.size, 11)
    gV, dR = oracle_adjoint(prob, lmin, lmax, lf, g_rho, g_u, nodes=nodes)
    dV, dRg = gpu_adjoint(prob, lmin, lmax, lf, g_rho, g_u, 1, nodes=nodes, adjoint_precision=0)
    assert rel(dV, gV) < 1e-10 and rel(dRg, dR) < 1e-10
    dV2, none = gpu_adjoint(prob, lmin, lmax, lf, g_rho, g_u, 0, nodes=nodes, with_dR=False)
    assert none is None and rel(dV2, gV) < 1e-10


def test_fp64_adjoint_edge27_too_many_atoms_reports_error():
    """A 27^3 FP64 region whose box meets more atoms than the edge-27 kernel's atom
    table holds (48): the adjoint must report SQ_ERR_ARG through the status word,
    not return a truncated gradient.  60 small supports (r_c = 0.6 bohr) packed in
    a 15-bohr cell keep every pencil below the column-entry limit, so the atom table
    is the only limit hit; the FP32 forward (128-atom table) runs as usual."""
    print("[case] FP64 adjoint edge27 with 60 atoms in one box", flush=True)
    prob = synth.small_problem(91, n=(30, 30, 30), h=(0.5, 0.5, 0.5), bc=synth.BC_PERIODIC,
                               rcut=(13, 13, 13), n_atoms=60, rc=0.6, order=4, kT=0.2,
                               fd_order=4)
    lmin, lmax = O.gershgorin(prob)
    lf = 0.5 * (lmin + lmax)
    nodes = np.array([0, 4321, 13000], dtype=np.int64)
    g_rho, g_u = _cotangents(nodes.size, 3)
    with pytest.raises(RuntimeError, match="more atoms"):
        gpu_adjoint(prob, lmin, lmax, lf, g_rho, g_u, 1, nodes=nodes, adjoint_precision=0)
