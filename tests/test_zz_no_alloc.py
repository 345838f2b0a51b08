"""sq_fermi_level_noalloc through the C ABI against sq_fermi_level on the same
moment sums: the same lambda_f, totals and coefficients (the two run the same
kernels, so the results agree to the last bit; held to 1e-12), on two calls in a
row, the second with a smaller input (lower degree K, another cell); and the
host-side rejection of sizes beyond the static scratch."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
from paper_2011_13517_amd import _lib as L
from paper_2011_13517_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _p(t):
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _case(prob, Ne):
    from paper_2011_13517_amd import sq
    lmin, lmax = O.lanczos_bounds(prob, steps=60)
    K = prob.order
    ctx = sq.Context(prob, precision=0)
    V = torch.tensor(prob.V, dtype=torch.float64, device="cuda")
    M = torch.empty(K + 1, dtype=torch.float64, device="cuda")
    ctx.density(V, lmin, lmax, moment_sum=M)
    lf_ref, _, _, tot_ref = ctx.fermi_level(Ne=Ne, tol=1e-11, max_iter=200, want_fields=False)
    torch.cuda.synchronize()
    ctx.status()
    lf = torch.full((1,), -7.0, dtype=torch.float64, device="cuda")
    coef = torch.full((4, K + 1), np.nan, dtype=torch.float64, device="cuda")
    tot = torch.full((8,), np.nan, dtype=torch.float64, device="cuda")
    st = L.lib().sq_fermi_level_noalloc(_p(M), K, lmin, lmax, prob.kT, Ne, 1e-11, 200, _p(lf),
                                        _p(coef), _p(tot), _stream())
    assert st == L.SQ_OK, L.sq_last_error()
    torch.cuda.synchronize()
    ctx.close()
    lf_v, lf_r = lf.item(), lf_ref.item()
    tot, tot_ref = tot.cpu().numpy(), tot_ref.cpu().numpy()
    print(f"K={K}: lambda_f noalloc {lf_v:.15f} context {lf_r:.15f}")
    assert abs(lf_v - lf_r) <= 1e-12 * (lmax - lmin)
    assert np.all(np.abs(tot - tot_ref) <= 1e-12 * np.maximum(np.abs(tot_ref), 1.0))
    assert tot[7] == 0.0
    # the coefficients against the oracle's at the same Fermi level
    c, _ = O.cheb_coeffs(O.KIND_G, lf_v, prob.kT, lmin, lmax, K)
    d, _ = O.cheb_coeffs(O.KIND_U, lf_v, prob.kT, lmin, lmax, K)
    c[0] *= 0.5
    d[0] *= 0.5
    cf = coef.cpu().numpy()
    assert np.abs(cf[0] - c).max() < 1e-12 and np.abs(cf[1] - d).max() < 1e-11 * np.abs(d).max()
    lf_o, _ = O.fermi_level(M.cpu().numpy(), prob.kT, lmin, lmax, Ne, tol=1e-11)
    assert abs(lf_v - lf_o) < 1e-9


def test_noalloc_fermi_level_matches_context_two_calls():
    big = synth.small_problem(91, n=(12, 11, 10), rcut=(3, 2, 2), n_atoms=3, rc=1.3, order=40,
                              kT=0.05, fd_order=6)
    small = synth.small_problem(92, n=(10, 9, 10), rcut=(2, 2, 2), n_atoms=2, rc=1.0, order=16,
                                kT=0.1)
    _case(big, 0.3 * big.n_nodes)
    _case(small, 0.25 * small.n_nodes)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    M = torch.zeros(601, dtype=torch.float64, device="cuda")
    lf = torch.zeros(1, dtype=torch.float64, device="cuda")
    lib = L.lib()
    # degree above 512
    assert lib.sq_fermi_level_noalloc(_p(M), 600, -1.0, 1.0, 0.1, 1.0, 1e-9, 10, _p(lf), None,
                                      None, _stream()) == L.SQ_ERR_ARG
    # smearing that needs more than 2^20 rule points
    assert lib.sq_fermi_level_noalloc(_p(M), 10, -50.0, 50.0, 1e-5, 1.0, 1e-9, 10, _p(lf), None,
                                      None, _stream()) == L.SQ_ERR_ARG
    assert b"2^20" in lib.sq_last_error()
