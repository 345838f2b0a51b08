"""Torch-facing wrapper of libsq: device tensors in, device tensors out.

PyTorch only provides device memory and the current HIP stream; every step of
the spectral-quadrature path runs in the HIP library behind the C ABI.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional

import numpy as np
import torch

from . import _lib as L
from .synth import Problem


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype=torch.float64):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous CUDA {dtype} tensor")
    return t


class Context:
    """A spectral-quadrature context for one problem geometry (sq_setup)."""

    def __init__(self, prob: Problem, precision: Optional[int] = None, nodes=None,
                 node_rcut=None, ckpt_every: int = 0, adjoint_precision: int = L.SQ_FP64,
                 tune: int = 0):
        p = L.sq_params()
        p.n[:] = [int(x) for x in prob.n]
        p.h[:] = [float(x) for x in prob.h]
        p.fd_order = int(prob.fd_order)
        p.bc = int(prob.bc)
        p.rcut[:] = [int(x) for x in prob.rcut]
        p.order = int(prob.order)
        p.kT = float(prob.kT)
        p.precision = int(prob.precision if precision is None else precision)
        p.ckpt_every = int(ckpt_every)
        p.adjoint_precision = int(adjoint_precision)
        p.tune = int(tune)
        self.params = p
        self.prob = prob
        self._keep = []
        proj = None
        if prob.n_atoms:
            def arr(x, dt):
                y = np.ascontiguousarray(x, dtype=dt)
                self._keep.append(y)
                return y.ctypes.data

            proj = L.sq_projectors()
            proj.n_atoms = int(prob.n_atoms)
            proj.n_proj = int(prob.n_proj)
            proj.sup_off = arr(prob.sup_off, np.int64)
            proj.sup_idx = arr(prob.sup_idx, np.int64)
            proj.chi = arr(prob.chi, np.float64)
            proj.dchi = arr(prob.dchi, np.float64) if prob.dchi is not None else None
            proj.c = arr(prob.c, np.float64)
        if nodes is None and prob.nodes is not None:
            nodes, node_rcut = prob.nodes, prob.node_rcut
        if nodes is not None:
            nodes = np.ascontiguousarray(nodes, dtype=np.int64)
            n_nodes = nodes.size
            nptr = C.c_void_p(nodes.ctypes.data)
        else:
            n_nodes = int(np.prod(prob.n))
            nptr = None
        rptr = None
        if node_rcut is not None:
            node_rcut = np.ascontiguousarray(node_rcut, dtype=np.int32)
            rptr = C.c_void_p(node_rcut.ctypes.data)
        self.ctx = L.sq_setup(p, proj, nptr, rptr, n_nodes)
        self.info = L.sq_get_info(self.ctx)
        self.n_nodes = int(self.info.n_nodes)
        self.K = int(self.info.order)
        self.n_atoms = int(self.info.n_atoms)
        self._keep = []

    # -- forward -------------------------------------------------------------
    def density(self, V: torch.Tensor, lambda_min: float = math.nan,
                lambda_max: float = math.nan, moments: Optional[torch.Tensor] = None,
                moment_sum: Optional[torch.Tensor] = None):
        """sq_density: moments [n_nodes, K+1] and their sum [K+1] (FP64, device)."""
        _dev(V)
        dev = V.device
        if moments is None:
            moments = torch.empty((self.n_nodes, self.K + 1), dtype=torch.float64, device=dev)
        if moment_sum is None:
            moment_sum = torch.empty(self.K + 1, dtype=torch.float64, device=dev)
        L.sq_density(self.ctx, _ptr(V), float(lambda_min), float(lambda_max), _ptr(moments),
                     _ptr(moment_sum), _stream())
        self.generation = getattr(self, "generation", 0) + 1
        # sq_fermi_level contracts these moments later: keep the buffer alive
        # (the generation counter lets SQDensity detect a stale backward)
        self._moments = moments
        return moments, moment_sum

    def fermi_level(self, Ne: float = 0.0, tol: float = 1e-10, max_iter: int = 200,
                    lambda_f: Optional[torch.Tensor] = None, want_fields: bool = True,
                    device=None, rho: Optional[torch.Tensor] = None,
                    u: Optional[torch.Tensor] = None, totals: Optional[torch.Tensor] = None):
        """sq_fermi_level: (lambda_f[1], rho[n], u[n], totals[8]) on the device
        (outputs are allocated unless given)."""
        dev = device or torch.device("cuda")
        if lambda_f is None:
            lambda_f = torch.zeros(1, dtype=torch.float64, device=dev)
        if want_fields and rho is None:
            rho = torch.empty(self.n_nodes, dtype=torch.float64, device=dev)
        if want_fields and u is None:
            u = torch.empty(self.n_nodes, dtype=torch.float64, device=dev)
        if totals is None:
            totals = torch.empty(8, dtype=torch.float64, device=dev)
        L.sq_fermi_level(self.ctx, float(Ne), float(tol), int(max_iter), _ptr(lambda_f),
                         _ptr(rho), _ptr(u), _ptr(totals), _stream())
        return lambda_f, rho, u, totals

    def entropy(self, s: Optional[torch.Tensor] = None, totals: Optional[torch.Tensor] = None,
                device=None):
        """sq_entropy: pointwise entropy s^q (units of k_B) and {S, U - kT S}."""
        dev = device or torch.device("cuda")
        if s is None:
            s = torch.empty(self.n_nodes, dtype=torch.float64, device=dev)
        if totals is None:
            totals = torch.empty(2, dtype=torch.float64, device=dev)
        L.sq_entropy(self.ctx, _ptr(s), _ptr(totals), _stream())
        return s, totals

    # -- Gauss quadrature (LSSGQ) ---------------------------------------------
    def gauss_density(self, V: torch.Tensor, lambda_min: float = math.nan,
                      lambda_max: float = math.nan, nodes: Optional[torch.Tensor] = None,
                      weights: Optional[torch.Tensor] = None):
        """sq_gauss_density: Gauss nodes and weights [n_nodes, K] (FP64, device)."""
        _dev(V)
        dev = V.device
        if nodes is None:
            nodes = torch.empty((self.n_nodes, self.K), dtype=torch.float64, device=dev)
        if weights is None:
            weights = torch.empty((self.n_nodes, self.K), dtype=torch.float64, device=dev)
        L.sq_gauss_density(self.ctx, _ptr(V), float(lambda_min), float(lambda_max), _ptr(nodes),
                           _ptr(weights), _stream())
        # sq_gauss_fermi_level reads these rules later: keep them alive
        self._rules = (nodes, weights)
        return nodes, weights

    def gauss_fermi_level(self, Ne: float = 0.0, tol: float = 1e-10, max_iter: int = 200,
                          lambda_f: Optional[torch.Tensor] = None, want_fields: bool = True,
                          device=None, rho: Optional[torch.Tensor] = None,
                          u: Optional[torch.Tensor] = None, s: Optional[torch.Tensor] = None,
                          totals: Optional[torch.Tensor] = None):
        """sq_gauss_fermi_level: (lambda_f[1], rho[n], u[n], s[n], totals[8]) with
        totals = {N_e, U, S, U - kT S, omega, tau, iterations, status} (outputs are
        allocated unless given)."""
        dev = device or torch.device("cuda")
        if lambda_f is None:
            lambda_f = torch.zeros(1, dtype=torch.float64, device=dev)
        if want_fields:
            rho, u, s = (t if t is not None else
                         torch.empty(self.n_nodes, dtype=torch.float64, device=dev)
                         for t in (rho, u, s))
        if totals is None:
            totals = torch.empty(8, dtype=torch.float64, device=dev)
        L.sq_gauss_fermi_level(self.ctx, float(Ne), float(tol), int(max_iter), _ptr(lambda_f),
                               _ptr(rho), _ptr(u), _ptr(s), _ptr(totals), _stream())
        return lambda_f, rho, u, s, totals

    def nonlocal_force(self, f: Optional[torch.Tensor] = None, device=None):
        """sq_nonlocal_force: Clenshaw-Curtis nonlocal force [n_atoms, 3] (FP64)."""
        dev = device or torch.device("cuda")
        if f is None:
            f = torch.empty((max(self.n_atoms, 1), 3), dtype=torch.float64, device=dev)
        L.sq_nonlocal_force(self.ctx, _ptr(f), _stream())
        return f[:self.n_atoms]

    def scf(self, b: torch.Tensor, Ne: float, V: torch.Tensor, lambda_min: float = math.nan,
            lambda_max: float = math.nan, beta: float = 0.3, tol: float = 1e-6,
            fermi_tol: float = 1e-10, poisson_rtol: float = 1e-12, max_iter: int = 50,
            anderson: bool = True, poisson_max_iter: int = 2000,
            rho: Optional[torch.Tensor] = None, lambda_f: Optional[torch.Tensor] = None,
            phi_bc: Optional[torch.Tensor] = None):
        """sq_scf: runs the SCF loop in place on V (FP64, V grid); phi_bc carries the
        Dirichlet values of embedded regions.  Returns (V, rho[n], lambda_f[1],
        info dict)."""
        _dev(V)
        _dev(b)
        if phi_bc is not None:
            _dev(phi_bc)
        dev = V.device
        if rho is None:
            rho = torch.empty(self.n_nodes, dtype=torch.float64, device=dev)
        if lambda_f is None:
            lambda_f = torch.zeros(1, dtype=torch.float64, device=dev)
        p = L.sq_scf_params(beta=float(beta), tol=float(tol), fermi_tol=float(fermi_tol),
                            poisson_rtol=float(poisson_rtol), max_iter=int(max_iter),
                            anderson=int(bool(anderson)), poisson_max_iter=int(poisson_max_iter))
        info = L.sq_scf(self.ctx, _ptr(b), _ptr(phi_bc), float(Ne), float(lambda_min),
                        float(lambda_max), p, _ptr(V), _ptr(rho), _ptr(lambda_f), _stream())
        out = {k: getattr(info, k) for k, _ in L.sq_scf_info._fields_}
        return V, rho, lambda_f, out

    def backward(self, g_rho: Optional[torch.Tensor], g_u: Optional[torch.Tensor],
                 dV: Optional[torch.Tensor] = None, dR: Optional[torch.Tensor] = None):
        """sq_density_backward: accumulates into dV (V grid) and dR [n_atoms, 3]."""
        L.sq_density_backward(self.ctx, _ptr(g_rho), _ptr(g_u), _ptr(dV), _ptr(dR), _stream())
        return dV, dR

    def status(self):
        return L.sq_device_status(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            L.sq_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SQDensity(torch.autograd.Function):
    """(V, R) -> (rho, u, lambda_f) through the HIP library, differentiable in V and R.

    forward: sq_density (device Lanczos bounds unless given) and sq_fermi_level.
    backward: sq_density_backward, i.e. the adjoint of the Chebyshev recurrence
    (Eqs. (Chebyshev), (rhoq), (uq)) at fixed lambda_f, omega and tau: the
    returned dV and dR are partial derivatives with the Fermi level held fixed;
    the cotangent of lambda_f is not propagated.

    R is a [n_atoms, 3] tensor standing for the atom positions the projector
    tables of the context were built at; the forward pass does not read its
    values, the backward pass returns dy/dR_J through chi(x - R_J).

        rho, u, lam = SQDensity.apply(V, R, context, Ne, tol, max_iter)
    """

    @staticmethod
    def forward(fctx, V, R, context: "Context", Ne: float = 0.0, tol: float = 1e-10,
                max_iter: int = 200, bounds=(math.nan, math.nan),
                lambda_f: Optional[torch.Tensor] = None):
        _dev(V)
        context.density(V, float(bounds[0]), float(bounds[1]))
        lam = lambda_f.clone() if lambda_f is not None else None
        lam, rho, u, totals = context.fermi_level(Ne=Ne, tol=tol, max_iter=max_iter,
                                                  lambda_f=lam, device=V.device)
        fctx.context = context
        fctx.generation = context.generation
        fctx.V_shape = V.shape
        fctx.has_R = R is not None
        fctx.mark_non_differentiable(lam)
        fctx.totals = totals
        return rho, u, lam

    @staticmethod
    def backward(fctx, g_rho, g_u, g_lam):
        context = fctx.context
        if context.generation != fctx.generation:
            raise RuntimeError("SQDensity.backward: the context ran another forward pass since "
                               "this one; the adjoint needs the state of its own forward pass")
        dev = g_rho.device if g_rho is not None else g_u.device
        gr = g_rho.contiguous() if g_rho is not None else None
        gu = g_u.contiguous() if g_u is not None else None
        dV = torch.zeros(fctx.V_shape, dtype=torch.float64, device=dev) \
            if fctx.needs_input_grad[0] else None
        dR = None
        if fctx.has_R and fctx.needs_input_grad[1] and context.n_atoms:
            dR = torch.zeros((context.n_atoms, 3), dtype=torch.float64, device=dev)
        if dV is not None or dR is not None:
            context.backward(gr, gu, dV, dR)
        return (dV, dR) + (None,) * 7
