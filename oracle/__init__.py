"""CPU oracle of the spectral-quadrature density path (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only users.  The product library never
imports, links or runs anything under ``oracle/``.

The arithmetic of the density path lives in plain C (``sq_oracle.c``, FP64, one
routine per step of the method); this module marshals numpy arrays into it.
The Gauss-quadrature rules (Lanczos on top of the C operator, with the
tridiagonal eigensolve as a library call) and the Clenshaw-Curtis nonlocal
force (the C operator for the recurrence, numpy for the box gradient and the
projections) are written here in numpy, FP64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sq_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (it is CPU code; no GPU toolchain involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double * 3), ("r", C.c_int32),
                ("bc", C.c_int32), ("pad", C.c_int32 * 3), ("n_atoms", C.c_int32),
                ("n_proj", C.c_int32), ("sup_off", C.c_void_p), ("sup_idx", C.c_void_p),
                ("chi", C.c_void_p), ("dchi", C.c_void_p), ("c", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P, D, I64, I32, VP = C.POINTER(_Problem), C.c_double, C.c_int64, C.c_int32, C.c_void_p
        L.orc_fd_weights.argtypes = [C.c_int, VP]
        L.orc_moments.argtypes = [P, VP, D, D, VP, VP, VP, I64, C.c_int, VP]
        L.orc_moments.restype = C.c_int
        L.orc_apply_node.argtypes = [P, VP, I64, VP, D, D, VP, VP, VP, VP]
        L.orc_apply_node.restype = C.c_int
        L.orc_node_box.argtypes = [P, I64, VP, VP, VP, VP]
        L.orc_node_box.restype = C.c_int
        L.orc_cheb_coeffs.argtypes = [C.c_int, D, D, D, D, C.c_int, VP]
        L.orc_cheb_coeffs.restype = I64
        L.orc_contract.argtypes = [VP, I64, C.c_int, VP, VP, VP, VP]
        L.orc_electron_count.argtypes = [VP, C.c_int, D, D, D, D]
        L.orc_electron_count.restype = D
        L.orc_fermi_level.argtypes = [VP, C.c_int, D, D, D, D, D, C.c_int, VP, VP]
        L.orc_fermi_level.restype = C.c_int
        L.orc_adjoint.argtypes = [P, VP, D, D, VP, VP, VP, I64, C.c_int, VP, VP, VP]
        L.orc_adjoint.restype = C.c_int
        L.orc_apply_full.argtypes = [P, VP, VP, VP]
        L.orc_lanczos.argtypes = [P, VP, C.c_int, C.c_uint64, VP, VP]
        L.orc_lanczos.restype = C.c_int
        L.orc_gershgorin.argtypes = [P, VP, VP, VP]
        L.orc_splitmix_uniform.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_splitmix_uniform.restype = D
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_splitmix64.restype = C.c_uint64
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Bound:
    """A problem marshalled for the C side (keeps the arrays alive)."""

    def __init__(self, prob):
        self.keep = []

        def arr(x, dt):
            if x is None:
                return None
            y = np.ascontiguousarray(x, dtype=dt)
            self.keep.append(y)
            return y

        s = _Problem()
        s.n[:] = [int(x) for x in prob.n]
        s.h[:] = [float(x) for x in prob.h]
        s.r = prob.fd_order // 2
        s.bc = prob.bc
        s.pad[:] = [int(x) for x in prob.pad]
        s.n_atoms = int(prob.n_atoms)
        s.n_proj = int(prob.n_proj)
        if prob.n_atoms:
            s.sup_off = _ptr(arr(prob.sup_off, np.int64))
            s.sup_idx = _ptr(arr(prob.sup_idx, np.int64))
            s.chi = _ptr(arr(prob.chi, np.float64))
            s.dchi = _ptr(arr(prob.dchi, np.float64))
            s.c = _ptr(arr(prob.c, np.float64))
        self.s = s
        self.V = arr(prob.V, np.float64)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's node loops from now on (timing only)."""
    lib().orc_set_num_threads(int(n))


def fd_weights(r: int) -> np.ndarray:
    w = np.zeros(r + 1)
    lib().orc_fd_weights(r, w.ctypes.data)
    return w


def _nodes_and_widths(prob, nodes, node_m):
    nodes = prob.node_list() if nodes is None else np.asarray(nodes, np.int64)
    if node_m is None:
        node_m = prob.node_widths() if (prob.nodes is not None and nodes is prob.nodes) else None
    mdef = np.asarray(prob.rcut, np.int32)
    nm = None if node_m is None else np.ascontiguousarray(node_m, dtype=np.int32)
    return np.ascontiguousarray(nodes), nm, mdef


def moments(prob, lmin, lmax, nodes=None, node_m=None, V=None, K=None) -> np.ndarray:
    """mu[q, k] = e_q^T T_k(Hs_q) e_q for the given nodes (default: the problem's)."""
    b = _Bound(prob)
    Vv = b.V if V is None else np.ascontiguousarray(V, np.float64)
    K = prob.order if K is None else K
    nodes, nm, mdef = _nodes_and_widths(prob, nodes, node_m)
    mu = np.zeros((nodes.size, K + 1))
    rc = lib().orc_moments(C.byref(b.s), Vv.ctypes.data, float(lmin), float(lmax),
                           nodes.ctypes.data, _ptr(nm), mdef.ctypes.data, nodes.size, K,
                           mu.ctypes.data)
    if rc:
        raise ValueError("oracle: invalid node region or parameters")
    return mu


def apply_node(prob, node, m, lmin, lmax, v=None, V=None):
    """(dims, centre index, Hs_q v) for one node; v flattened over the box (x fastest)."""
    b = _Bound(prob)
    Vv = b.V if V is None else np.ascontiguousarray(V, np.float64)
    m = np.ascontiguousarray(m, np.int32)
    dim = np.zeros(3, np.int32)
    ctr = np.zeros(1, np.int64)
    out = None
    if v is not None:
        v = np.ascontiguousarray(v, np.float64)
        out = np.zeros_like(v)
    rc = lib().orc_apply_node(C.byref(b.s), Vv.ctypes.data, int(node), m.ctypes.data,
                              float(lmin), float(lmax), _ptr(v), _ptr(out), dim.ctypes.data,
                              ctr.ctypes.data)
    if rc:
        raise ValueError("oracle: invalid node region")
    return tuple(int(x) for x in dim), int(ctr[0]), out


def node_dense(prob, node, m, lmin, lmax, V=None):
    """Dense Hs_q assembled column by column from the matrix-free product."""
    dims, ctr, _ = apply_node(prob, node, m, lmin, lmax, V=V)
    npts = dims[0] * dims[1] * dims[2]
    H = np.zeros((npts, npts))
    e = np.zeros(npts)
    for j in range(npts):
        e[:] = 0.0
        e[j] = 1.0
        H[:, j] = apply_node(prob, node, m, lmin, lmax, e, V=V)[2]
    return H, dims, ctr


def node_box(prob, node, m):
    b = _Bound(prob)
    m = np.ascontiguousarray(m, np.int32)
    lo = np.zeros(3, np.int64)
    dim = np.zeros(3, np.int32)
    ctr = np.zeros(3, np.int32)
    if lib().orc_node_box(C.byref(b.s), int(node), m.ctypes.data, lo.ctypes.data,
                          dim.ctypes.data, ctr.ctypes.data):
        raise ValueError("oracle: invalid node region")
    return lo, dim, ctr


KIND_G, KIND_U, KIND_DG, KIND_DU, KIND_S = 0, 1, 2, 3, 4


def cheb_coeffs(kind, lambda_f, kT, lmin, lmax, K):
    """c_k (kind 0), d_k (kind 1), their lambda_f derivatives (kinds 2, 3) and the
    coefficients of the entropy integrand g log g + (1-g) log(1-g) (kind 4)."""
    omega, tau = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    out = np.zeros(K + 1)
    N = lib().orc_cheb_coeffs(kind, (lambda_f - omega) / tau, kT / tau, tau, omega, K,
                              out.ctypes.data)
    return out, int(N)


def contract(mu, c, d):
    mu = np.ascontiguousarray(mu, np.float64)
    n, K1 = mu.shape
    rho, u = np.zeros(n), np.zeros(n)
    lib().orc_contract(mu.ctypes.data, n, K1 - 1, np.ascontiguousarray(c).ctypes.data,
                       np.ascontiguousarray(d).ctypes.data, rho.ctypes.data, u.ctypes.data)
    return rho, u


def entropy(mu, lambda_f, kT, lmin, lmax):
    """Pointwise entropy, Eq. (sq), in units of k_B: s^q = -2 int s(lambda) dmu_q with
    s = g log g + (1-g) log(1-g), evaluated with the Chebyshev rule as
    -2 (e_0 mu_0 / 2 + sum_k e_k mu_k).  Returns (s, e)."""
    mu = np.ascontiguousarray(mu, np.float64)
    e, _ = cheb_coeffs(KIND_S, lambda_f, kT, lmin, lmax, mu.shape[1] - 1)
    f, _ = contract(mu, e, e)
    return -f, e


def electron_count(M, lambda_f, kT, lmin, lmax):
    M = np.ascontiguousarray(M, np.float64)
    return float(lib().orc_electron_count(M.ctypes.data, M.size - 1, float(lambda_f), float(kT),
                                          float(lmin), float(lmax)))


class NotBracketed(RuntimeError):
    pass


def fermi_level(M, kT, lmin, lmax, Ne, tol=1e-10, max_iter=200, with_status=False):
    """Bisection of Eq. (Ne) on the moment sums M.  Returns (lambda_f, iterations),
    plus a converged flag (|N_e(lambda_f) - Ne| < tol reached before a 4-ulp bracket
    or max_iter midpoints) when with_status is set."""
    M = np.ascontiguousarray(M, np.float64)
    lf = np.zeros(1)
    it = np.zeros(1, np.int32)
    rc = lib().orc_fermi_level(M.ctypes.data, M.size - 1, float(kT), float(lmin), float(lmax),
                               float(Ne), float(tol), int(max_iter), lf.ctypes.data,
                               it.ctypes.data)
    if rc == -4:
        raise NotBracketed("electron count not bracketed by [lambda_min, lambda_max]")
    if with_status:
        return float(lf[0]), int(it[0]), rc == 0
    return float(lf[0]), int(it[0])


# --------------------------------------------------------------------------- #
# Gauss quadrature of the local spectral measure (LSSGQ), Eq. (Lanczos)
# --------------------------------------------------------------------------- #
def gauss_rules(prob, lmin, lmax, K, nodes=None, node_m=None, V=None):
    """K-point Gauss rule of the spectral measure of e_q for every node.

    Eq. (Lanczos) on the node Hamiltonian, scaled as in Section 2.2 (the rule
    of H_q is the rule of Hs_q mapped back): v_0 = e_q, b_0 = 0,
      a_{k+1} = (Hs v_k, v_k),  b_{k+1} v_{k+1} = (Hs - a_{k+1}) v_k - b_k v_{k-1},
    no reorthogonalisation.  The Jacobi matrix has a_1..a_K on the diagonal and
    b_1..b_{K-1} beside it; its eigenvalues are the nodes (returned unscaled,
    lambda = tau theta + omega) and the squared first components of its
    normalised eigenvectors the weights (the paper's text swaps the two
    symbols).  A Krylov space that closes before K steps (b = 0) gives the exact
    shorter rule, padded with zero weights.  The tridiagonal eigensolve is a
    library step (scipy.linalg.eigh_tridiagonal).  Returns (nodes, weights),
    each [n_nodes, K]."""
    from scipy.linalg import eigh_tridiagonal
    b = _Bound(prob)
    Vv = b.V if V is None else np.ascontiguousarray(V, np.float64)
    nodes, nm, mdef = _nodes_and_widths(prob, nodes, node_m)
    omega, tau = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    lam = np.zeros((nodes.size, K))
    wgt = np.zeros((nodes.size, K))
    for i, q in enumerate(nodes):
        m = mdef if nm is None else nm[i]
        dims, ctr, _ = apply_node(prob, q, m, lmin, lmax, V=Vv)
        v = np.zeros(int(np.prod(dims)))
        v[ctr] = 1.0
        vp = np.zeros_like(v)
        bk = 0.0
        a_list, b_list = [], []
        for k in range(K):
            w = apply_node(prob, q, m, lmin, lmax, v, V=Vv)[2]
            ak = float(v @ w)
            w = w - ak * v - bk * vp
            a_list.append(ak)
            if k == K - 1:
                break
            bn = float(np.sqrt(w @ w))
            if bn <= 1e-14:
                break
            b_list.append(bn)
            vp, v, bk = v, w / bn, bn
        theta, U = eigh_tridiagonal(np.array(a_list), np.array(b_list))
        n = len(a_list)
        lam[i, :n] = tau * theta + omega
        wgt[i, :n] = U[0, :] ** 2
        lam[i, n:] = lam[i, n - 1] if n else omega
    return lam, wgt


def _fermi_fn(lam, lf, kT):
    return 0.5 * (1.0 - np.tanh((lam - lf) / (2.0 * kT)))


def gauss_fields(lam, wgt, lf, kT):
    """rho^q, u^q and s^q (units of k_B) of Eqs. (rhoq), (uq), (sq) from the rules:
    2 sum_k w_k g, 2 sum_k w_k lambda_k g, -2 sum_k w_k (g log g + (1-g) log(1-g))."""
    g = _fermi_fn(lam, lf, kT)
    t = np.abs(lam - lf) / kT
    e = np.exp(-t)
    sfn = -(t * e / (1.0 + e) + np.log1p(e))
    rho = 2.0 * np.sum(wgt * g, axis=1)
    u = 2.0 * np.sum(wgt * lam * g, axis=1)
    s = -2.0 * np.sum(wgt * sfn, axis=1)
    return rho, u, s


def gauss_fermi_level(lam, wgt, kT, lmin, lmax, Ne, tol=1e-10, max_iter=200,
                      with_status=False):
    """Bisection of Eq. (Ne) with the Gauss rules: N_e(lambda_f) = 2 sum_q sum_k w g,
    on [lmin, lmax] with the same rule as fermi_level (mid = lo + (hi - lo)/2, lo =
    mid when N_e(mid) < target, stop at |N_e - target| < tol or a 4-ulp bracket)."""
    ne = lambda x: float(2.0 * np.sum(wgt * _fermi_fn(lam, x, kT)))
    lo, hi = float(lmin), float(lmax)
    if ne(lo) > Ne or ne(hi) < Ne:
        raise NotBracketed("electron count not bracketed by [lambda_min, lambda_max]")
    mid = lo + 0.5 * (hi - lo)
    it = 0
    converged = False
    for it in range(1, max_iter + 1):
        mid = lo + 0.5 * (hi - lo)
        n_mid = ne(mid)
        if abs(n_mid - Ne) < tol:
            converged = True
            break
        if n_mid < Ne:
            lo = mid
        else:
            hi = mid
        if hi - lo < 4.0 * np.finfo(float).eps * max(abs(lo), abs(hi)):
            break
    if with_status:
        return mid, it, converged
    return mid, it


# --------------------------------------------------------------------------- #
# Nonlocal force by the Clenshaw-Curtis quadrature, Eq. (NLforceSQ)
# --------------------------------------------------------------------------- #
def fd_first_weights(r):
    """Central first-derivative weights of radius r (Section 3's FD gradient):
    f'(x) ~ sum_p w_p (f(x + p h) - f(x - p h)) / h with
    w_p = (-1)^(p+1) (r!)^2 / (p (r-p)! (r+p)!)."""
    from math import factorial
    return np.array([0.0] + [(-1.0) ** (p + 1) * factorial(r) ** 2 /
                             (p * factorial(r - p) * factorial(r + p)) for p in range(1, r + 1)])


def _box_grad(gam, dims, h, r, axis):
    """d/dx_axis of a box function (flattened x fastest) by the radius-r central
    stencil, with the function taken as zero outside the box."""
    G = gam.reshape(dims[2], dims[1], dims[0])     # [z][y][x]
    ax = 2 - axis
    wp = fd_first_weights(r)
    out = np.zeros_like(G)
    n = G.shape[ax]
    for p in range(1, r + 1):
        if p >= n:
            break
        up = np.zeros_like(G)
        dn = np.zeros_like(G)
        sl_dst = [slice(None)] * 3
        sl_src = [slice(None)] * 3
        sl_dst[ax], sl_src[ax] = slice(0, n - p), slice(p, n)
        up[tuple(sl_dst)] = G[tuple(sl_src)]          # f(x + p)
        sl_dst[ax], sl_src[ax] = slice(p, n), slice(0, n - p)
        dn[tuple(sl_dst)] = G[tuple(sl_src)]          # f(x - p)
        out += wp[p] * (up - dn)
    return (out / h[axis]).reshape(-1)


def box_projectors(prob, lo, dims):
    """{atom: (box indices [m], chi [m, n_proj])} for the atoms whose support meets
    the box (support points mapped into box coordinates; periodic grids wrap)."""
    N = prob.vshape
    out = {}
    for J in range(prob.n_atoms):
        s0, s1 = int(prob.sup_off[J]), int(prob.sup_off[J + 1])
        idx = prob.sup_idx[s0:s1]
        g = np.stack([idx % N[0], (idx // N[0]) % N[1], idx // (N[0] * N[1])], axis=1)
        t = g - np.asarray(lo)[None, :]
        if prob.bc == 0:
            t = np.mod(t, np.asarray(N)[None, :])
        inside = np.all((t >= 0) & (t < np.asarray(dims)[None, :]), axis=1)
        if not inside.any():
            continue
        t = t[inside]
        bi = t[:, 0] + dims[0] * (t[:, 1] + dims[1] * t[:, 2])
        out[J] = (bi, prob.chi[s0:s1][inside])
    return out


def cc_nonlocal_force(prob, lmin, lmax, lambda_f, nodes=None, node_m=None, V=None):
    """f_J,nl = -4 sum_q e_q^T V_J^q grad_h (sum'_k c_k v_k^q), Eq. (NLforceSQ) in
    its discrete form (Section 3), for every atom: [n_atoms, 3].

    v_k^q: Eq. (Chebyshev) on the node's region (the same box and truncated
    Hamiltonian as the moments); c_k: Eq. (ChebyshevWeights) at lambda_f with
    c_0 halved; grad_h: the radius-r central stencil on the box with zero
    outside it; e_q^T V_J^q f = h1 h2 h3 sum_lm c_Jl chi_Jlm(q) (chi_Jlm . f)
    over the box.  Nodes outside every support contribute nothing."""
    b = _Bound(prob)
    Vv = b.V if V is None else np.ascontiguousarray(V, np.float64)
    nodes, nm, mdef = _nodes_and_widths(prob, nodes, node_m)
    K = prob.order
    c, _ = cheb_coeffs(KIND_G, lambda_f, prob.kT, lmin, lmax, K)
    cp = c.copy()
    cp[0] *= 0.5
    h3 = float(np.prod(prob.h))
    f = np.zeros((prob.n_atoms, 3))
    for i, q in enumerate(nodes):
        m = mdef if nm is None else nm[i]
        lo, dims, ctr3 = node_box(prob, q, m)
        projs = box_projectors(prob, lo, dims)
        ctr = int(ctr3[0] + dims[0] * (ctr3[1] + dims[1] * ctr3[2]))
        at_q = {J: chi[bi == ctr].sum(axis=0) for J, (bi, chi) in projs.items()
                if np.any(bi == ctr)}
        if not at_q:
            continue
        v0 = np.zeros(int(np.prod(dims)))
        v0[ctr] = 1.0
        gam = cp[0] * v0
        vp, v = v0, apply_node(prob, q, m, lmin, lmax, v0, V=Vv)[2]
        gam = gam + cp[1] * v
        for k in range(1, K):
            vn = 2.0 * apply_node(prob, q, m, lmin, lmax, v, V=Vv)[2] - vp
            vp, v = v, vn
            gam = gam + cp[k + 1] * v
        for a in range(3):
            dg = _box_grad(gam, dims, prob.h, prob.r, a)
            for J, chq in at_q.items():
                bi, chi = projs[J]
                proj = chi.T @ dg[bi]                      # chi_Jlm . d_a gamma
                f[J, a] += -4.0 * h3 * np.sum(prob.c[J] * chq * proj)
    return f


# --------------------------------------------------------------------------- #
# SCF outer loop (Section 3's flowchart): Poisson, LDA exchange-correlation,
# mixing of the effective potential -- periodic cells only
# --------------------------------------------------------------------------- #
def fd_laplacian_symbol(n, h, r):
    """Eigenvalues of the periodic FD Laplacian (Section 3's stencil) on the
    discrete Fourier modes, [n2][n1][n0]: sum_a (w_0 + 2 sum_p w_p cos(2 pi p k_a / n_a)) / h_a^2."""
    w = fd_weights(r)
    parts = []
    for a in range(3):
        k = np.arange(n[a])
        s = np.full(n[a], w[0])
        for p in range(1, r + 1):
            s = s + 2.0 * w[p] * np.cos(2.0 * np.pi * p * k / n[a])
        parts.append(s / (h[a] * h[a]))
    return parts[2][:, None, None] + parts[1][None, :, None] + parts[0][None, None, :]


def poisson_periodic(f, n, h, r):
    """phi with -Lap_h phi = 4 pi f on the periodic grid, Eq. (Poisson) with the FD
    Laplacian; f is projected to zero mean (the neutral cell) and phi has zero
    mean.  Solved exactly in the discrete Fourier basis (an FFT as library step)."""
    F = np.fft.fftn(np.asarray(f, np.float64).reshape(n[2], n[1], n[0]))
    L = fd_laplacian_symbol(n, h, r)
    F[0, 0, 0] = 0.0
    L[0, 0, 0] = 1.0
    return np.real(np.fft.ifftn(-4.0 * np.pi * F / L)).reshape(-1)


def poisson_dirichlet(f, phi_bc, prob):
    """phi on the padded grid Omega' of an embedded problem: -Lap_h phi = 4 pi f at
    the nodes of Omega, phi = phi_bc on the padding (Dirichlet values from the
    surrounding crystal; the padding must be at least the FD radius deep).  The
    interior system is assembled as a sparse matrix and solved directly (a
    library step)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    N, pad, n, r = prob.vshape, prob.pad, prob.n, prob.r
    w = fd_weights(r)
    mats = []
    for a in range(3):
        m = sp.lil_matrix((N[a], N[a]))
        for i in range(N[a]):
            m[i, i] += w[0]
            for p in range(1, r + 1):
                if i + p < N[a]:
                    m[i, i + p] += w[p]
                if i - p >= 0:
                    m[i, i - p] += w[p]
        mats.append(m.tocsr() / (prob.h[a] * prob.h[a]))
    I = [sp.identity(k, format="csr") for k in N]
    L = (sp.kron(I[2], sp.kron(I[1], mats[0])) + sp.kron(I[2], sp.kron(mats[1], I[0]))
         + sp.kron(mats[2], sp.kron(I[1], I[0]))).tocsr()
    zz, yy, xx = np.meshgrid(*(np.arange(k) for k in N[::-1]), indexing="ij")
    inside = ((xx >= pad[0]) & (xx < pad[0] + n[0]) & (yy >= pad[1]) & (yy < pad[1] + n[1])
              & (zz >= pad[2]) & (zz < pad[2] + n[2])).ravel()
    ii, bb = np.flatnonzero(inside), np.flatnonzero(~inside)
    phi = np.array(phi_bc, np.float64)
    rhs = 4.0 * np.pi * np.asarray(f, np.float64)[ii] + L[ii][:, bb] @ phi[bb]
    phi[ii] = spl.spsolve((-L[ii][:, ii]).tocsc(), rhs)
    return phi


def embed_nodes(prob):
    """Linear indices on Omega' of the nodes of Omega (x fastest)."""
    N, pad, n = prob.vshape, prob.pad, prob.n
    zz, yy, xx = np.meshgrid(*(np.arange(k) for k in n[::-1]), indexing="ij")
    return ((xx + pad[0]) + N[0] * ((yy + pad[1]) + N[1] * (zz + pad[2]))).ravel()


PW92 = dict(A=0.031091, a1=0.21370, b1=7.5957, b2=3.5876, b3=1.6382, b4=0.49294)


def lda_pw92(n):
    """LDA exchange-correlation energy per electron and potential, unpolarised:
    Slater exchange e_x = -(3/4)(3 n / pi)^(1/3), v_x = (4/3) e_x, and the
    Perdew-Wang (1992) fit of the Ceperley-Alder correlation,
    e_c = -2A(1 + a1 rs) ln(1 + 1 / (2A(b1 rs^1/2 + b2 rs + b3 rs^3/2 + b4 rs^2))),
    v_c = e_c - (rs / 3) de_c/drs, rs = (3 / (4 pi n))^(1/3).  Zero where n <= 0."""
    n = np.asarray(n, np.float64)
    exc = np.zeros_like(n)
    vxc = np.zeros_like(n)
    m = n > 0.0
    x = n[m]
    ex = -0.75 * np.cbrt(3.0 * x / np.pi)
    rs = np.cbrt(3.0 / (4.0 * np.pi * x))
    c = PW92
    sr = np.sqrt(rs)
    q0 = -2.0 * c["A"] * (1.0 + c["a1"] * rs)
    q1 = 2.0 * c["A"] * (c["b1"] * sr + c["b2"] * rs + c["b3"] * rs * sr + c["b4"] * rs * rs)
    dq1 = c["A"] * (c["b1"] / sr + 2.0 * c["b2"] + 3.0 * c["b3"] * sr + 4.0 * c["b4"] * rs)
    lg = np.log1p(1.0 / q1)
    ec = q0 * lg
    dec = -2.0 * c["A"] * c["a1"] * lg - q0 * dq1 / (q1 * q1 + q1)
    exc[m] = ex + ec
    vxc[m] = 4.0 / 3.0 * ex + ec - rs / 3.0 * dec
    return exc, vxc


def scf(prob, b, Ne, V0, lmin, lmax, beta=0.3, tol=1e-6, max_iter=30, anderson=True,
        fermi_tol=1e-10, phi_bc=None):
    """Fixed-point iteration on the effective potential (Section 3's flowchart):
    V_in -> moments (Eq. (Chebyshev)) -> lambda_f (Eq. (Ne)) -> rho^q (Eq. (rhoq))
    -> n = rho^q / (h1 h2 h3) -> phi of Eq. (Poisson) with source n + b -> V_out =
    phi + v_xc(n) -> mixing.  Mixing: F = V_out - V_in; the first step is linear,
    V <- V + beta F; later steps are Anderson with one previous pair,
    g = F.(F - F') / |F - F'|^2, V <- (V - g (V - V')) + beta (F - g (F - F')).
    Stops when the RMS of F is below tol.  Every node of the periodic cell is a
    quadrature node; (lmin, lmax) stay fixed, or with both None they are
    re-estimated for every V_in by lanczos_bounds (100 steps, the 0x5EED start
    vector, 1% margin).  Embedded problems (V, b and phi_bc on Omega') solve the
    Dirichlet problem of poisson_dirichlet with phi_bc on the padding and update
    V only at the nodes of Omega (the padding keeps the surrounding crystal's
    values); the RMS of F is over the nodes of Omega.  Returns one record per
    iteration."""
    V = np.array(V0, np.float64)
    fixed = lmin is not None
    emb = prob.bc == 2
    if emb:
        idx = embed_nodes(prob)
        n_omega = idx.size
    h3 = float(np.prod(prob.h))
    Vp = Fp = None
    recs = []
    for it in range(max_iter):
        if not fixed:
            lmin, lmax = lanczos_bounds(prob, steps=100, seed=0x5EED, margin=0.01, V=V)
        mu = moments(prob, lmin, lmax, V=V)
        lf, _ = fermi_level(mu.sum(0), prob.kT, lmin, lmax, Ne, tol=fermi_tol)
        cg, _ = cheb_coeffs(KIND_G, lf, prob.kT, lmin, lmax, prob.order)
        rho_q, _ = contract(mu, cg, cg)
        if emb:
            n_x = np.zeros_like(V)
            n_x[idx] = rho_q / h3
            phi = poisson_dirichlet(n_x + b, phi_bc, prob)
            _, vxc = lda_pw92(n_x)
            Vout = V.copy()
            Vout[idx] = phi[idx] + vxc[idx]
            F = Vout - V
            res = float(np.sqrt(np.sum(F * F) / n_omega))
        else:
            n_x = rho_q / h3
            phi = poisson_periodic(n_x + b, prob.n, prob.h, prob.r)
            _, vxc = lda_pw92(n_x)
            Vout = phi + vxc
            F = Vout - V
            res = float(np.sqrt(np.mean(F * F)))
        recs.append(dict(V_in=V.copy(), V_out=Vout, rho=rho_q, lambda_f=lf, residual=res))
        if res < tol:
            break
        if Fp is None or not anderson:
            Vn = V + beta * F
        else:
            dV, dF = V - Vp, F - Fp
            g = float(F @ dF) / float(dF @ dF)
            Vn = (V - g * dV) + beta * (F - g * dF)
        Vp, Fp = V, F
        V = Vn
    return recs


def adjoint(prob, lmin, lmax, a, nodes=None, node_m=None, V=None, with_dR=True):
    """(dV, dR) of y = sum_q sum_k a[q,k] mu_k^q at fixed lambda_f, omega, tau."""
    b = _Bound(prob)
    Vv = b.V if V is None else np.ascontiguousarray(V, np.float64)
    nodes, nm, mdef = _nodes_and_widths(prob, nodes, node_m)
    a = np.ascontiguousarray(a, np.float64)
    K = a.shape[1] - 1
    gV = np.zeros(Vv.size)
    dR = np.zeros((max(prob.n_atoms, 1), 3)) if with_dR else None
    rc = lib().orc_adjoint(C.byref(b.s), Vv.ctypes.data, float(lmin), float(lmax),
                           nodes.ctypes.data, _ptr(nm), mdef.ctypes.data, nodes.size, K,
                           a.ctypes.data, gV.ctypes.data, _ptr(dR))
    if rc:
        raise ValueError("oracle: invalid node region or parameters")
    return gV, (dR[:prob.n_atoms] if with_dR else None)


def apply_full(prob, v, V=None):
    b = _Bound(prob)
    Vv = b.V if V is None else np.ascontiguousarray(V, np.float64)
    v = np.ascontiguousarray(v, np.float64)
    out = np.zeros_like(v)
    lib().orc_apply_full(C.byref(b.s), Vv.ctypes.data, v.ctypes.data, out.ctypes.data)
    return out


def splitmix64(seed, i):
    return int(lib().orc_splitmix64(seed, i))


def splitmix_uniform(seed, n):
    L = lib()
    return np.array([L.orc_splitmix_uniform(seed, i) for i in range(n)])


def lanczos_tridiag(prob, steps, seed, V=None):
    b = _Bound(prob)
    Vv = b.V if V is None else np.ascontiguousarray(V, np.float64)
    al, be = np.zeros(steps), np.zeros(max(steps - 1, 1))
    lib().orc_lanczos(C.byref(b.s), Vv.ctypes.data, steps, seed, al.ctypes.data, be.ctypes.data)
    return al, be[:steps - 1]


def lanczos_bounds(prob, steps=120, seed=0x5EED, margin=0.01, V=None):
    """Extreme Ritz values of the whole-domain H, widened by margin * width each side."""
    from scipy.linalg import eigvalsh_tridiagonal
    al, be = lanczos_tridiag(prob, steps, seed, V=V)
    ev = eigvalsh_tridiagonal(al, be)
    lo, hi = float(ev[0]), float(ev[-1])
    wdt = hi - lo
    return lo - margin * wdt, hi + margin * wdt


def gershgorin(prob, V=None):
    b = _Bound(prob)
    Vv = b.V if V is None else np.ascontiguousarray(V, np.float64)
    lo, hi = np.zeros(1), np.zeros(1)
    lib().orc_gershgorin(C.byref(b.s), Vv.ctypes.data, lo.ctypes.data, hi.ctypes.data)
    return float(lo[0]), float(hi[0])
