"""Spectral Gauss quadrature (LSSGQ) through the C ABI against the FP64 oracle.

sq_gauss_density (per-node Lanczos on the GPU, FP64 Jacobi eigensolve) and
sq_gauss_fermi_level (bisection of Eq. (Ne) over the rules, fields of Eqs.
(rhoq), (uq), (sq)) against oracle.gauss_rules / gauss_fermi_level /
gauss_fields on the same seeded inputs.

Tolerances: FP64 recurrence, nodes within 1e-10 tau and weights within 1e-10,
fields within 1e-10 of their max norm; FP32 recurrence (FP64 a_k, b_k), nodes
within 1e-5 tau, weights within 1e-5, fields within 1e-5 of their max norm.
Node-by-node comparison needs the two Lanczos runs to stay close, which holds
while orthogonality is not lost (small K here); at the full size the fields
and properties that hold at any K are compared instead.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2011_13517_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu(prob, precision, lmin, lmax, Ne=None, lf=None, nodes=None, node_rcut=None):
    from paper_2011_13517_amd import sq
    ctx = sq.Context(prob, precision=precision, nodes=nodes, node_rcut=node_rcut)
    V = torch.tensor(prob.V, dtype=torch.float64, device="cuda")
    lam, w = ctx.gauss_density(V, lmin, lmax)
    out = {}
    if Ne is not None or lf is not None:
        lfd = torch.tensor([0.0 if lf is None else lf], dtype=torch.float64, device="cuda")
        lfo, rho, u, s, tot = ctx.gauss_fermi_level(Ne=Ne or 0.0, tol=1e-10,
                                                    max_iter=200 if lf is None else 0,
                                                    lambda_f=lfd)
        torch.cuda.synchronize()
        out.update(lf=float(lfo.item()), rho=rho.cpu().numpy(), u=u.cpu().numpy(),
                   s=s.cpu().numpy(), tot=tot.cpu().numpy())
    torch.cuda.synchronize()
    ctx.status()
    out.update(lam=lam.cpu().numpy(), w=w.cpu().numpy())
    ctx.close()
    return out


def _tols(precision):
    return (1e-10, 1e-10) if precision == 0 else (1e-5, 1e-5)


@pytest.mark.parametrize("bc", [synth.BC_PERIODIC, synth.BC_DIRICHLET, synth.BC_EMBEDDED])
@pytest.mark.parametrize("precision", [0, 1])
def test_gauss_rules_and_fields_small(bc, precision):
    """Every node of a 13x12x14 grid (boxes clipped at the walls, several
    tiles), K = 12: nodes, weights, lambda_f and the three fields."""
    print(f"[case] gauss small bc={bc} precision={precision}", flush=True)
    prob = synth.small_problem(81 + bc, n=(13, 12, 14), bc=bc, rcut=(2, 3, 2), n_atoms=4,
                               rc=1.4, order=12, kT=0.2, fd_order=6)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    tau = 0.5 * (lmax - lmin)
    Ne = 0.3 * prob.n_nodes
    g = _gpu(prob, precision, lmin, lmax, Ne=Ne)
    lam, w = O.gauss_rules(prob, lmin, lmax, prob.order)
    lf, _ = O.gauss_fermi_level(lam, w, prob.kT, lmin, lmax, Ne, tol=1e-10)
    rho, u, s = O.gauss_fields(lam, w, lf, prob.kT)
    tn, tf = _tols(precision)
    assert np.abs(g["lam"] - lam).max() <= tn * tau
    assert np.abs(g["w"] - w).max() <= tn
    assert abs(g["lf"] - lf) <= (1e-9 if precision == 0 else 1e-5) * tau
    # fields at the GPU's lambda_f (bisection stops may differ in the last bits)
    rho2, u2, s2 = O.gauss_fields(lam, w, g["lf"], prob.kT)
    for a, b in ((g["rho"], rho2), (g["u"], u2), (g["s"], s2)):
        assert np.abs(a - b).max() <= tf * np.abs(b).max()
    assert abs(g["tot"][0] - Ne) <= 1e-9 * Ne
    assert abs(g["tot"][1] - g["u"].sum()) <= 1e-12 * np.abs(g["u"]).sum()
    assert abs(g["tot"][2] - g["s"].sum()) <= 1e-12 * np.abs(g["s"]).sum() + 1e-300
    assert abs(g["tot"][3] - (g["tot"][1] - prob.kT * g["tot"][2])) <= 1e-12 * abs(g["tot"][3])
    assert g["tot"][7] == 0
    del rho, u, s


@pytest.mark.parametrize("K", [1, 2, 5])
def test_gauss_short_rules(K):
    """K = 1 gives the single node H_qq with weight 1; K = 2 and 5 node by node."""
    print(f"[case] gauss short K={K}", flush=True)
    prob = synth.small_problem(5, n=(10, 9, 11), rcut=(2, 2, 2), n_atoms=3, rc=1.3, order=K,
                               kT=0.3, fd_order=4)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    g = _gpu(prob, 0, lmin, lmax)
    lam, w = O.gauss_rules(prob, lmin, lmax, K)
    tau = 0.5 * (lmax - lmin)
    assert np.abs(g["lam"] - lam).max() <= 1e-10 * tau
    assert np.abs(g["w"] - w).max() <= 1e-10
    if K == 1:
        assert np.all(g["w"] == 1.0)


def test_gauss_closed_krylov_space():
    """K = 40 on 3x3x3 boxes (27 points): the Krylov space closes (or loses
    orthogonality) before K; the rule is still the node's spectral measure, so
    the fields agree with the oracle's and with the dense eigendecomposition."""
    print("[case] gauss closed Krylov space", flush=True)
    prob = synth.small_problem(14, n=(7, 7, 7), rcut=(1, 1, 1), n_atoms=2, rc=1.2, order=40,
                               kT=0.4)
    lmin, lmax = O.gershgorin(prob)
    omega, tau = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    lf = omega - 0.2 * tau
    g = _gpu(prob, 0, lmin, lmax, lf=lf)
    lam, w = O.gauss_rules(prob, lmin, lmax, 40)
    rho, u, s = O.gauss_fields(lam, w, lf, prob.kT)
    assert np.abs(g["rho"] - rho).max() <= 1e-10 * np.abs(rho).max()
    assert np.abs(g["u"] - u).max() <= 1e-10 * np.abs(u).max()
    H, dims, ctr = O.node_dense(prob, 100, (1, 1, 1), lmin, lmax)
    ev, U = np.linalg.eigh(H)
    occ = 1.0 / (1.0 + np.exp((ev * tau + omega - lf) / prob.kT))
    assert abs(g["rho"][100] - 2.0 * np.sum(U[ctr] ** 2 * occ)) < 1e-10
    assert np.abs(g["w"].sum(1) - 1.0).max() < 1e-12


def test_gauss_uneven_regions():
    """Per-node region widths (uneven boxes in several edge buckets and launch
    groups), FP64, node by node on a subset."""
    print("[case] gauss uneven regions", flush=True)
    base = synth.small_problem(23, n=(20, 18, 22), rcut=(4, 4, 4), n_atoms=6, rc=1.4, order=10,
                               kT=0.2, fd_order=6)
    rng = np.random.default_rng(4)
    nodes = np.sort(rng.choice(int(np.prod(base.n)), 60, replace=False)).astype(np.int64)
    nr = rng.integers(1, 5, size=(60, 3)).astype(np.int32)
    lmin, lmax = O.lanczos_bounds(base, steps=60)
    g = _gpu(base, 0, lmin, lmax, nodes=nodes, node_rcut=nr)
    lam, w = O.gauss_rules(base, lmin, lmax, base.order, nodes=nodes, node_m=nr)
    tau = 0.5 * (lmax - lmin)
    assert np.abs(g["lam"] - lam).max() <= 1e-10 * tau
    assert np.abs(g["w"] - w).max() <= 1e-10


def test_gauss_config2_sampled_fp32():
    """64^3 grid, 27^3 regions, 96 atoms, K = 80 (the paper's Lanczos order),
    FP32 vectors: properties at every node (weights sum to 1, nodes inside the
    bounds, N_e met) and the fields of sampled nodes against the oracle's rules
    at the GPU's lambda_f."""
    print("[case] gauss config2", flush=True)
    prob = dataclasses.replace(synth.config(2), order=80)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    Ne = 192.0
    g = _gpu(prob, 1, lmin, lmax, Ne=Ne)
    assert np.abs(g["w"].sum(1) - 1.0).max() < 1e-5
    assert g["lam"].min() >= lmin - 1e-6 * (lmax - lmin)
    assert g["lam"].max() <= lmax + 1e-6 * (lmax - lmin)
    assert np.all(np.diff(g["lam"], axis=1) >= 0)
    assert abs(g["tot"][0] - Ne) <= 1e-8 * Ne
    rng = np.random.default_rng(12)
    sample = np.sort(rng.choice(prob.n_nodes, 6, replace=False))
    lam, w = O.gauss_rules(prob, lmin, lmax, prob.order, nodes=sample)
    rho, u, s = O.gauss_fields(lam, w, g["lf"], prob.kT)
    assert np.abs(g["rho"][sample] - rho).max() <= 1e-5 * np.abs(g["rho"]).max()
    assert np.abs(g["u"][sample] - u).max() <= 1e-5 * np.abs(g["u"]).max()
    assert np.abs(g["s"][sample] - s).max() <= 1e-5 * max(np.abs(g["s"]).max(), 1e-12)


def test_gauss_state_errors():
    """Fermi level before any Gauss sweep, and after sq_density replaced it."""
    from paper_2011_13517_amd import sq
    from paper_2011_13517_amd._lib import SQError
    prob = synth.small_problem(3, n=(8, 8, 8), rcut=(1, 1, 1), order=4)
    ctx = sq.Context(prob, precision=0)
    with pytest.raises(SQError):
        ctx.gauss_fermi_level(Ne=1.0)
    V = torch.tensor(prob.V, dtype=torch.float64, device="cuda")
    lmin, lmax = O.gershgorin(prob)
    ctx.gauss_density(V, lmin, lmax)
    ctx.density(V, lmin, lmax)
    with pytest.raises(SQError):
        ctx.gauss_fermi_level(Ne=1.0)
    ctx.close()


def test_gauss_rules_integrate_gpu_moments():
    """Gauss exactness on the GPU alone: the K-point rules of sq_gauss_density
    integrate T_j exactly for j <= 2K - 1, so sum_k w_k T_j(theta_k) equals the
    Chebyshev moments mu_j of sq_density on the same regions (FP64)."""
    from paper_2011_13517_amd import sq
    print("[case] gauss rules vs GPU moments", flush=True)
    K = 8
    prob = synth.small_problem(17, n=(11, 12, 10), rcut=(2, 2, 2), n_atoms=3, rc=1.3, order=K,
                               kT=0.2, fd_order=6)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    om, tau = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    g = _gpu(prob, 0, lmin, lmax)
    ctx = sq.Context(dataclasses.replace(prob, order=2 * K + 1), precision=0)
    V = torch.tensor(prob.V, dtype=torch.float64, device="cuda")
    mu, _ = ctx.density(V, lmin, lmax)
    torch.cuda.synchronize()
    mu = mu.cpu().numpy()
    ctx.close()
    th = np.arccos(np.clip((g["lam"] - om) / tau, -1.0, 1.0))
    for j in range(2 * K):
        got = np.sum(g["w"] * np.cos(j * th), axis=1)
        assert np.abs(got - mu[:, j]).max() <= 1e-10, j
    assert np.abs(np.sum(g["w"] * np.cos(2 * K * th), axis=1) - mu[:, 2 * K]).max() > 1e-8


def test_gauss_fp64_edge27_wave_per_atom_path():
    """FP64 at edge 27: the box and the column tables do not share the LDS, so the
    Lanczos sweep takes the wave-per-atom projector path; node by node against the
    oracle on a subset of the 64^3 workload (K = 6)."""
    print("[case] gauss fp64 edge 27", flush=True)
    prob = dataclasses.replace(synth.config(2), order=6)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    rng = np.random.default_rng(21)
    nodes = np.sort(rng.choice(prob.n_nodes, 24, replace=False)).astype(np.int64)
    g = _gpu(prob, 0, lmin, lmax, nodes=nodes)
    lam, w = O.gauss_rules(prob, lmin, lmax, prob.order, nodes=nodes)
    tau = 0.5 * (lmax - lmin)
    assert np.abs(g["lam"] - lam).max() <= 1e-10 * tau
    assert np.abs(g["w"] - w).max() <= 1e-10
