"""Parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances
* FP64 path: moments within 1e-12 absolute (|mu_k| <= 1, K <= 100 steps of
  O(1e-16) rounding), densities within 1e-10 max-norm relative.
* FP32 path: each step rounds every vector entry to 2^-24 relative; the
  propagated error of mu_k stays below K * 2^-24 * 8 (row sum of |2 Hs| <= 4
  plus v_{k-1}); densities within 1e-5 max-norm relative,
  max_q |rho_q - rho_q^ref| / max_q |rho_q^ref|.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2011_13517_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _sq():
    from paper_2011_13517_amd import sq
    return sq


def fp32_mu_tol(K):
    return K * 2.0 ** -24 * 8


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gpu_forward(prob, lmin, lmax, precision, nodes=None, node_rcut=None, Ne=None, lf=None,
                tol=1e-10, tune=0, info=None):
    sq = _sq()
    ctx = sq.Context(prob, precision=precision, nodes=nodes, node_rcut=node_rcut, tune=tune)
    if info is not None:
        info.append(ctx.info)
    V = torch.tensor(prob.V, dtype=torch.float64, device="cuda")
    mu, M = ctx.density(V, lmin, lmax)
    if Ne is not None:
        lam, rho, u, tot = ctx.fermi_level(Ne=Ne, tol=tol, max_iter=200)
    else:
        lam = torch.tensor([lf], dtype=torch.float64, device="cuda")
        lam, rho, u, tot = ctx.fermi_level(max_iter=0, lambda_f=lam)
    torch.cuda.synchronize()
    out = dict(mu=mu.cpu().numpy(), M=M.cpu().numpy(), lf=float(lam.item()),
               rho=rho.cpu().numpy(), u=u.cpu().numpy(), tot=tot.cpu().numpy())
    ctx.status()
    ctx.close()
    return out


def oracle_fields(mu, lf, kT, lmin, lmax, K):
    c, _ = O.cheb_coeffs(O.KIND_G, lf, kT, lmin, lmax, K)
    d, _ = O.cheb_coeffs(O.KIND_U, lf, kT, lmin, lmax, K)
    return O.contract(mu, c, d)


@pytest.mark.parametrize("bc", [synth.BC_PERIODIC, synth.BC_DIRICHLET, synth.BC_EMBEDDED])
@pytest.mark.parametrize("precision", [0, 1])
def test_small_all_nodes(bc, precision):
    """Several tiles of small regions, projectors, ragged Dirichlet boxes."""
    print(f"[case] small bc={bc} precision={precision}", flush=True)
    prob = synth.small_problem(31 + bc, n=(14, 13, 12), bc=bc, rcut=(3, 2, 2), n_atoms=4, rc=1.4,
                               order=24, kT=0.15, fd_order=6)
    lmin, lmax = O.lanczos_bounds(prob, steps=80)
    mu_ref = O.moments(prob, lmin, lmax)
    Ne = 0.3 * mu_ref.shape[0]
    M_ref = mu_ref.sum(0)
    lf_ref, _ = O.fermi_level(M_ref, prob.kT, lmin, lmax, Ne, tol=1e-11)
    rho_ref, u_ref = oracle_fields(mu_ref, lf_ref, prob.kT, lmin, lmax, prob.order)
    g = gpu_forward(prob, lmin, lmax, precision, Ne=Ne, tol=1e-11)
    if precision == 0:
        assert np.abs(g["mu"] - mu_ref).max() < 1e-12
        assert abs(g["lf"] - lf_ref) < 1e-9
        assert rel_err(g["rho"], rho_ref) < 1e-10
        assert rel_err(g["u"], u_ref) < 1e-10
    else:
        assert np.abs(g["mu"] - mu_ref).max() < fp32_mu_tol(prob.order)
        assert rel_err(g["rho"], rho_ref) < 1e-5
    assert abs(g["tot"][0] - Ne) < 1e-9 * Ne
    assert g["tot"][7] == 0


def test_config1_fp64_full():
    print("[case] config1 fp64 full", flush=True)
    prob = synth.config(1)
    lmin, lmax = O.lanczos_bounds(prob, steps=120)
    mu_ref = O.moments(prob, lmin, lmax)
    lf_ref, _ = O.fermi_level(mu_ref.sum(0), prob.kT, lmin, lmax, prob.Ne, tol=1e-11)
    rho_ref, u_ref = oracle_fields(mu_ref, lf_ref, prob.kT, lmin, lmax, prob.order)
    g = gpu_forward(prob, lmin, lmax, 0, Ne=prob.Ne, tol=1e-11)
    assert np.abs(g["mu"] - mu_ref).max() < 1e-12
    assert abs(g["lf"] - lf_ref) < 1e-9
    assert rel_err(g["rho"], rho_ref) < 1e-10
    assert rel_err(g["u"], u_ref) < 1e-10
    assert abs(g["rho"].sum() - prob.Ne) < 1e-9
    # totals: N_e, U and the lambda_f derivatives against the oracle's coefficients
    dc, _ = O.cheb_coeffs(O.KIND_DG, lf_ref, prob.kT, lmin, lmax, prob.order)
    M = mu_ref.sum(0)
    dne = 2 * (0.5 * dc[0] * M[0] + dc[1:] @ M[1:])
    assert abs(g["tot"][2] - dne) < 1e-8 * abs(dne)
    assert abs(g["tot"][1] - u_ref.sum()) < 1e-9 * abs(u_ref.sum())


def test_config1_fp32_full():
    print("[case] config1 fp32 full", flush=True)
    prob = synth.config(1)
    lmin, lmax = O.lanczos_bounds(prob, steps=120)
    mu_ref = O.moments(prob, lmin, lmax)
    lf_ref, _ = O.fermi_level(mu_ref.sum(0), prob.kT, lmin, lmax, prob.Ne, tol=1e-11)
    rho_ref, _ = oracle_fields(mu_ref, lf_ref, prob.kT, lmin, lmax, prob.order)
    g = gpu_forward(prob, lmin, lmax, 1, Ne=prob.Ne, tol=1e-11)
    assert np.abs(g["mu"] - mu_ref).max() < fp32_mu_tol(prob.order)
    assert rel_err(g["rho"], rho_ref) < 1e-5


def _sample_nodes(prob, n, seed):
    rng = np.random.default_rng(seed)
    total = prob.n_nodes
    return np.unique(np.concatenate([[0, total - 1], rng.choice(total, n, replace=False)]))


@pytest.mark.parametrize("precision", [0, 1])
def test_config2_sampled(precision):
    """Full 64^3 / 27^3 / K=100 workload on the GPU; the oracle on sampled nodes.
    lambda_f: the oracle's own bisection on the GPU FP64 aggregate moments
    (the oracle cannot afford all 262144 nodes inside a test)."""
    print(f"[case] config2 precision={precision}", flush=True)
    prob = synth.config(2)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    g = gpu_forward(prob, lmin, lmax, precision, Ne=prob.Ne, tol=1e-9)
    sample = _sample_nodes(prob, 10, 5)
    mu_ref = O.moments(prob, lmin, lmax, nodes=sample)
    assert np.all(np.abs(g["mu"][:, 0] - 1.0) == 0)
    if precision == 0:
        assert np.abs(g["mu"][sample] - mu_ref).max() < 1e-12
        lf_o, _ = O.fermi_level(g["M"], prob.kT, lmin, lmax, prob.Ne, tol=1e-9)
        assert abs(g["lf"] - lf_o) < 1e-9
    else:
        assert np.abs(g["mu"][sample] - mu_ref).max() < fp32_mu_tol(prob.order)
    rho_ref, u_ref = oracle_fields(mu_ref, g["lf"], prob.kT, lmin, lmax, prob.order)
    scale = np.abs(g["rho"]).max()
    err = np.abs(g["rho"][sample] - rho_ref).max() / scale
    assert err < (1e-10 if precision == 0 else 1e-5), err
    assert abs(g["tot"][0] - prob.Ne) < 1e-8 * prob.Ne


@pytest.mark.parametrize("precision,tune", [(0, 0), (1, 0), (1, 1), (0, 2)])
def test_config3_uneven_clipped(precision, tune):
    """4096 uneven Dirichlet-clipped regions (edges 11..27 before clipping):
    the launch plan the tuner picks (tune 0), one persistent launch per edge
    bucket (tune 1), and one launch per region (tune 2, the plain path)."""
    print(f"[case] config3 precision={precision} tune={tune}", flush=True)
    prob = synth.config(3)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    info = []
    g = gpu_forward(prob, lmin, lmax, precision, lf=prob.lambda_f, tune=tune, info=info)
    print(f"persistent launches per pass: {info[0].n_launches}")
    if tune == 1:
        assert info[0].n_launches > 1
    elif tune == 2:
        assert info[0].n_launches == prob.n_nodes
    else:
        assert info[0].n_launches >= 1
    nodes, widths = prob.nodes, prob.node_rcut
    # sample: the smallest and largest boxes, clipped and interior ones
    sizes = []
    for q in range(nodes.size):
        _, dim, _ = O.node_box(prob, nodes[q], widths[q])
        sizes.append(int(np.prod(dim)))
    sizes = np.array(sizes)
    order = np.argsort(sizes)
    rng = np.random.default_rng(3)
    pick = np.unique(np.concatenate([order[:4], order[-4:], rng.choice(nodes.size, 8, False)]))
    mu_ref = O.moments(prob, lmin, lmax, nodes=nodes[pick], node_m=widths[pick])
    tol = 1e-12 if precision == 0 else fp32_mu_tol(prob.order)
    assert np.abs(g["mu"][pick] - mu_ref).max() < tol
    rho_ref, _ = oracle_fields(mu_ref, prob.lambda_f, prob.kT, lmin, lmax, prob.order)
    err = np.abs(g["rho"][pick] - rho_ref).max() / np.abs(g["rho"]).max()
    assert err < (1e-10 if precision == 0 else 1e-5)


def test_device_lanczos_bounds():
    """NaN bounds: FP64 Lanczos on the device, same start vector as the oracle's."""
    print("[case] lanczos", flush=True)
    sq = _sq()
    for prob in (synth.small_problem(41, n=(10, 10, 10), rcut=(2, 2, 2), n_atoms=3, rc=1.3),
                 synth.small_problem(42, n=(8, 6, 7), bc=synth.BC_DIRICHLET, rcut=(2, 2, 2))):
        ctx = sq.Context(prob, precision=0)
        V = torch.tensor(prob.V, dtype=torch.float64, device="cuda")
        ctx.density(V)
        lam, _, _, tot = ctx.fermi_level(max_iter=0, lambda_f=torch.zeros(1, dtype=torch.float64,
                                                                            device="cuda"))
        tot = tot.cpu().numpy()
        ctx.close()
        om, tau = tot[4], tot[5]
        lo_o, hi_o = O.lanczos_bounds(prob, steps=100, seed=0x5EED, margin=0.01)
        assert abs((om - tau) - lo_o) < 1e-8 * (hi_o - lo_o)
        assert abs((om + tau) - hi_o) < 1e-8 * (hi_o - lo_o)
        N = int(np.prod(prob.vshape))
        H = np.stack([O.apply_full(prob, np.eye(N)[j]) for j in range(N)], 1)
        ev = np.linalg.eigvalsh(H)
        assert om - tau < ev[0] and ev[-1] < om + tau


def test_fermi_not_bracketed_reports_status():
    print("[case] not bracketed", flush=True)
    sq = _sq()
    prob = synth.small_problem(43, n=(6, 6, 6), rcut=(1, 1, 1), order=10, kT=0.2,
                               with_projectors=False)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    ctx = sq.Context(prob, precision=0)
    V = torch.tensor(prob.V, dtype=torch.float64, device="cuda")
    ctx.density(V, lmin, lmax)
    lam, _, _, tot = ctx.fermi_level(Ne=2.0 * 216 + 1.0, tol=1e-10, max_iter=100)
    torch.cuda.synchronize()
    assert tot[7].item() == -4
    assert math.isnan(lam.item())
    from paper_2011_13517_amd._lib import SQError
    with pytest.raises(SQError):
        ctx.status()
    ctx.close()


def test_fermi_max_iter_exhausted_reports_not_converged():
    """A bisection cut off after 3 midpoints (|N_e - target| still above tol)
    returns the oracle's third midpoint with status SQ_ERR_NOT_CONVERGED in
    totals[7] and in sq_device_status; a following solve with room to converge
    on the same moments reports SQ_OK again."""
    print("[case] max_iter exhausted", flush=True)
    sq = _sq()
    prob = synth.small_problem(45, n=(8, 8, 8), rcut=(2, 2, 2), order=16, kT=0.1,
                               with_projectors=False)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    mu_ref = O.moments(prob, lmin, lmax)
    Ne = 0.4 * mu_ref.shape[0]
    lf_o, it_o, conv_o = O.fermi_level(mu_ref.sum(0), prob.kT, lmin, lmax, Ne, tol=1e-12,
                                       max_iter=3, with_status=True)
    assert not conv_o and it_o == 3
    ctx = sq.Context(prob, precision=0)
    V = torch.tensor(prob.V, dtype=torch.float64, device="cuda")
    ctx.density(V, lmin, lmax)
    lam, _, _, tot = ctx.fermi_level(Ne=Ne, tol=1e-12, max_iter=3)
    torch.cuda.synchronize()
    assert tot[7].item() == -4 and tot[6].item() == 3
    assert abs(lam.item() - lf_o) < 1e-12 * (lmax - lmin)
    from paper_2011_13517_amd._lib import SQError
    with pytest.raises(SQError):
        ctx.status()
    lam, _, _, tot = ctx.fermi_level(Ne=Ne, tol=1e-9, max_iter=200)
    torch.cuda.synchronize()
    ctx.status()
    assert tot[7].item() == 0 and abs(tot[0].item() - Ne) < 1e-9
    ctx.close()


def test_edge_cases_single_node_and_thin_boxes():
    """K = 1, a single node, zero-width axes and anisotropic spacing."""
    print("[case] edge cases", flush=True)
    prob = synth.small_problem(44, n=(9, 10, 8), h=(0.5, 0.6, 0.7), rcut=(0, 2, 1), n_atoms=2,
                               rc=1.2, order=1, fd_order=4)
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    for precision in (0, 1):
        for nodes in ([17], None):
            g = gpu_forward(prob, lmin, lmax, precision, nodes=nodes, lf=0.0)
            ref = O.moments(prob, lmin, lmax, nodes=nodes)
            tol = 1e-13 if precision == 0 else 1e-6
            assert np.abs(g["mu"] - ref).max() < tol


def test_config5_embedded_full_fp32_sampled():
    """Embedded 128^3 domain (V and projectors on the 154^3 padded grid, 1791
    projector atoms, K = 120): all 2,097,152 nodes in one FP32 launch with the
    FP64 bisection on N_e = 1534; sampled nodes (corners of Omega, whose
    regions reach into the padding, and random interior nodes) against the
    oracle.  Gershgorin bounds from the oracle are passed to both sides."""
    print("[case] config5 embedded FP32 full", flush=True)
    sq = _sq()
    prob = synth.config(5)
    lmin, lmax = O.gershgorin(prob)
    n0, n1, n2 = prob.n
    corners = [i + n0 * (j + n1 * k) for i in (0, n0 - 1) for j in (0, n1 - 1)
               for k in (0, n2 - 1)]
    rng = np.random.default_rng(55)
    sample = np.unique(np.concatenate([corners, rng.choice(prob.n_nodes, 10, replace=False)]))
    ctx = sq.Context(prob, precision=1)
    V = torch.tensor(prob.V, dtype=torch.float64, device="cuda")
    mu, M = ctx.density(V, lmin, lmax)
    lam, rho, u, tot = ctx.fermi_level(Ne=prob.Ne, tol=1e-8, max_iter=200)
    torch.cuda.synchronize()
    ctx.status()
    idx = torch.tensor(sample, device="cuda")
    mu_s = mu[idx].cpu().numpy()
    rho_all = rho.cpu().numpy()
    tot = tot.cpu().numpy()
    lf = float(lam.item())
    ctx.close()
    mu_ref = O.moments(prob, lmin, lmax, nodes=sample)
    assert np.abs(mu_s - mu_ref).max() < fp32_mu_tol(prob.order)
    rho_ref, _ = oracle_fields(mu_ref, lf, prob.kT, lmin, lmax, prob.order)
    assert np.abs(rho_all[sample] - rho_ref).max() / np.abs(rho_all).max() < 1e-5
    # the config's bisection tolerance, absolute: |N_e(lambda_f) - N_e| < 1e-8
    assert abs(tot[0] - prob.Ne) < 1e-8, tot[0] - prob.Ne
    assert tot[7] == 0
    assert abs(rho_all.sum() - prob.Ne) < 1e-6 * prob.Ne


def test_config5_embedded_fp64_nodes():
    """Embedded workload, FP64 path on a node subset (including the corners of
    Omega) against the oracle at the FP64 tolerances."""
    print("[case] config5 embedded FP64 subset", flush=True)
    prob = synth.config(5)
    lmin, lmax = O.gershgorin(prob)
    n0, n1, n2 = prob.n
    corners = [i + n0 * (j + n1 * k) for i in (0, n0 - 1) for j in (0, n1 - 1)
               for k in (0, n2 - 1)]
    rng = np.random.default_rng(56)
    nodes = np.unique(np.concatenate([corners, rng.choice(prob.n_nodes, 24, replace=False)]))
    lf = 0.5 * (lmin + lmax) - 0.45 * (lmax - lmin)
    g = gpu_forward(prob, lmin, lmax, 0, nodes=nodes, lf=lf)
    mu_ref = O.moments(prob, lmin, lmax, nodes=nodes)
    assert np.abs(g["mu"] - mu_ref).max() < 1e-12
    rho_ref, u_ref = oracle_fields(mu_ref, lf, prob.kT, lmin, lmax, prob.order)
    assert rel_err(g["rho"], rho_ref) < 1e-10
    assert rel_err(g["u"], u_ref) < 1e-10
