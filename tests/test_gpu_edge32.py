"""The largest FP32 edge bucket (32): boxes of edge 28..32 run the edge-32
kernel instances of the Chebyshev forward sweep, the Gauss Lanczos sweep and
the nonlocal force; checked against the oracle on a few nodes whose boxes are
31 nodes long in x (Dirichlet grid, so the boxes of the end nodes are clipped)."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2011_13517_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _problem():
    prob = synth.small_problem(32, n=(36, 8, 9), bc=synth.BC_DIRICHLET, rcut=(15, 2, 2),
                               n_atoms=4, rc=1.4, order=10, kT=0.2, fd_order=6)
    nodes = np.array([17 + 36 * (4 + 8 * 4), 16 + 36 * (3 + 8 * 5), 2 + 36 * (4 + 8 * 4),
                      35 + 36 * (7 + 8 * 8), 18 + 36 * (0 + 8 * 1)], dtype=np.int64)
    return prob, nodes


def test_edge32_forward_gauss_force_fp32():
    from paper_2011_13517_amd import sq
    print("[case] edge 32 fp32", flush=True)
    prob, nodes = _problem()
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    ctx = sq.Context(prob, precision=1, nodes=nodes)
    assert int(ctx.info.max_region[0]) == 31
    V = torch.tensor(prob.V, dtype=torch.float64, device="cuda")
    mu, _ = ctx.density(V, lmin, lmax)
    lf = 0.5 * (lmin + lmax) - 0.3 * (lmax - lmin)
    ctx.fermi_level(max_iter=0, lambda_f=torch.tensor([lf], dtype=torch.float64, device="cuda"),
                    want_fields=False)
    f = ctx.nonlocal_force().cpu().numpy()
    lam, w = ctx.gauss_density(V, lmin, lmax)
    torch.cuda.synchronize()
    ctx.status()
    mu, lam, w = mu.cpu().numpy(), lam.cpu().numpy(), w.cpu().numpy()
    ctx.close()
    mu_ref = O.moments(prob, lmin, lmax, nodes=nodes)
    assert np.abs(mu - mu_ref).max() <= 1e-5
    f_ref = O.cc_nonlocal_force(prob, lmin, lmax, lf, nodes=nodes)
    # two of the four atoms have supports crossing these boxes (max |f| = 0.26 on the CPU)
    assert np.abs(f_ref).max() > 1e-2
    assert np.abs(f - f_ref).max() <= 1e-4 * np.abs(f_ref).max()
    lam_ref, w_ref = O.gauss_rules(prob, lmin, lmax, prob.order, nodes=nodes)
    tau = 0.5 * (lmax - lmin)
    assert np.abs(lam - lam_ref).max() <= 1e-5 * tau
    assert np.abs(w - w_ref).max() <= 1e-5
