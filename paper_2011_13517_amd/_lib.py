"""ctypes binding of libsq.so: the C ABI of include/sq.h, names unchanged.

Argument marshalling only; every step of the computation runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# SQ_LIB names a variant build of the same library (build.py --name) for A/B
# measurements; it must exist like the default one
LIB_PATH = os.environ.get("SQ_LIB") or os.path.join(HERE, "libsq.so")

SQ_OK, SQ_ERR_ARG, SQ_ERR_HIP, SQ_ERR_OOM = 0, -1, -2, -3
SQ_ERR_NOT_CONVERGED, SQ_ERR_SPECTRUM, SQ_ERR_STATE = -4, -5, -6
SQ_BC_PERIODIC, SQ_BC_DIRICHLET, SQ_BC_EMBEDDED = 0, 1, 2
SQ_FP64, SQ_FP32_ACC64 = 0, 1

STATUS_NAMES = {0: "SQ_OK", -1: "SQ_ERR_ARG", -2: "SQ_ERR_HIP", -3: "SQ_ERR_OOM",
                -4: "SQ_ERR_NOT_CONVERGED", -5: "SQ_ERR_SPECTRUM", -6: "SQ_ERR_STATE"}

# every entry point declared in include/sq.h
EXPORTS = ("sq_setup", "sq_destroy", "sq_last_error", "sq_get_info", "sq_density",
           "sq_fermi_level", "sq_entropy", "sq_gauss_density", "sq_gauss_fermi_level", "sq_nonlocal_force", "sq_scf",
           "sq_density_backward", "sq_device_status", "sq_fermi_level_noalloc")


class sq_params(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double * 3), ("fd_order", C.c_int32),
                ("bc", C.c_int32), ("rcut", C.c_int32 * 3), ("order", C.c_int32),
                ("kT", C.c_double), ("precision", C.c_int32), ("ckpt_every", C.c_int32),
                ("adjoint_precision", C.c_int32), ("tune", C.c_int32)]


class sq_projectors(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("n_proj", C.c_int32), ("sup_off", C.c_void_p),
                ("sup_idx", C.c_void_p), ("chi", C.c_void_p), ("dchi", C.c_void_p),
                ("c", C.c_void_p)]


class sq_scf_params(C.Structure):
    _fields_ = [("beta", C.c_double), ("tol", C.c_double), ("fermi_tol", C.c_double),
                ("poisson_rtol", C.c_double), ("max_iter", C.c_int32), ("anderson", C.c_int32),
                ("poisson_max_iter", C.c_int32), ("pad_", C.c_int32)]


class sq_scf_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32),
                ("poisson_iterations", C.c_int32), ("poisson_converged", C.c_int32),
                ("residual", C.c_double), ("poisson_relres", C.c_double)]


class sq_info(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("order", C.c_int32), ("vgrid", C.c_int32 * 3),
                ("n_atoms", C.c_int32), ("max_region", C.c_int32 * 3),
                ("region_points", C.c_int64), ("workspace_bytes", C.c_int64),
                ("n_launches", C.c_int32), ("forward_blocks", C.c_int32),
                ("n_force_nodes", C.c_int64), ("force_region_points", C.c_int64)]


class SQError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libsq.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: the HIP library has not been built "
                               "(run __graft_entry__.build()); there is no fallback path")
        L = C.CDLL(LIB_PATH)
        VP, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.sq_setup.argtypes = [C.POINTER(sq_params), C.POINTER(sq_projectors), VP, VP, I64,
                               C.POINTER(VP)]
        L.sq_setup.restype = C.c_int
        L.sq_destroy.argtypes = [VP]
        L.sq_destroy.restype = C.c_int
        L.sq_last_error.argtypes = []
        L.sq_last_error.restype = C.c_char_p
        L.sq_get_info.argtypes = [VP, C.POINTER(sq_info)]
        L.sq_get_info.restype = C.c_int
        L.sq_density.argtypes = [VP, VP, D, D, VP, VP, VP]
        L.sq_density.restype = C.c_int
        L.sq_fermi_level.argtypes = [VP, D, D, I32, VP, VP, VP, VP, VP]
        L.sq_fermi_level.restype = C.c_int
        L.sq_entropy.argtypes = [VP, VP, VP, VP]
        L.sq_entropy.restype = C.c_int
        L.sq_gauss_density.argtypes = [VP, VP, D, D, VP, VP, VP]
        L.sq_gauss_density.restype = C.c_int
        L.sq_gauss_fermi_level.argtypes = [VP, D, D, I32, VP, VP, VP, VP, VP, VP]
        L.sq_gauss_fermi_level.restype = C.c_int
        L.sq_nonlocal_force.argtypes = [VP, VP, VP]
        L.sq_nonlocal_force.restype = C.c_int
        L.sq_scf.argtypes = [VP, VP, VP, D, D, D, C.POINTER(sq_scf_params), VP, VP, VP,
                             C.POINTER(sq_scf_info), VP]
        L.sq_scf.restype = C.c_int
        L.sq_density_backward.argtypes = [VP, VP, VP, VP, VP, VP]
        L.sq_density_backward.restype = C.c_int
        L.sq_device_status.argtypes = [VP]
        L.sq_device_status.restype = C.c_int
        L.sq_fermi_level_noalloc.argtypes = [VP, I32, D, D, D, D, D, I32, VP, VP, VP, VP]
        L.sq_fermi_level_noalloc.restype = C.c_int
        _lib = L
    return _lib


def check(status):
    if status != SQ_OK:
        raise SQError(status, lib().sq_last_error().decode(errors="replace"))
    return status


def sq_setup(params, projectors, nodes_ptr, node_rcut_ptr, n_nodes):
    ctx = C.c_void_p()
    check(lib().sq_setup(C.byref(params), C.byref(projectors) if projectors is not None else None,
                         nodes_ptr, node_rcut_ptr, n_nodes, C.byref(ctx)))
    return ctx


def sq_destroy(ctx):
    return check(lib().sq_destroy(ctx))


def sq_last_error():
    return lib().sq_last_error().decode(errors="replace")


def sq_get_info(ctx):
    info = sq_info()
    check(lib().sq_get_info(ctx, C.byref(info)))
    return info


def sq_density(ctx, V_ptr, lambda_min, lambda_max, moments_ptr, moment_sum_ptr, stream):
    return check(lib().sq_density(ctx, V_ptr, lambda_min, lambda_max, moments_ptr,
                                  moment_sum_ptr, stream))


def sq_fermi_level(ctx, Ne_target, tol_Ne, max_iter, lambda_f_ptr, rho_ptr, u_ptr, totals_ptr,
                   stream):
    return check(lib().sq_fermi_level(ctx, Ne_target, tol_Ne, max_iter, lambda_f_ptr, rho_ptr,
                                      u_ptr, totals_ptr, stream))


def sq_entropy(ctx, s_ptr, totals_ptr, stream):
    return check(lib().sq_entropy(ctx, s_ptr, totals_ptr, stream))


def sq_gauss_density(ctx, V_ptr, lmin, lmax, nodes_ptr, weights_ptr, stream):
    return check(lib().sq_gauss_density(ctx, V_ptr, lmin, lmax, nodes_ptr, weights_ptr, stream))


def sq_gauss_fermi_level(ctx, Ne, tol, max_iter, lf_ptr, rho_ptr, u_ptr, s_ptr, totals_ptr,
                         stream):
    return check(lib().sq_gauss_fermi_level(ctx, Ne, tol, max_iter, lf_ptr, rho_ptr, u_ptr,
                                            s_ptr, totals_ptr, stream))


def sq_nonlocal_force(ctx, f_ptr, stream):
    return check(lib().sq_nonlocal_force(ctx, f_ptr, stream))


def sq_scf(ctx, b_ptr, phi_bc_ptr, Ne, lmin, lmax, params, V_ptr, rho_ptr, lf_ptr, stream):
    info = sq_scf_info()
    check(lib().sq_scf(ctx, b_ptr, phi_bc_ptr, Ne, lmin, lmax, C.byref(params), V_ptr, rho_ptr,
                       lf_ptr, C.byref(info), stream))
    return info


def sq_density_backward(ctx, g_rho_ptr, g_u_ptr, dV_ptr, dR_ptr, stream):
    return check(lib().sq_density_backward(ctx, g_rho_ptr, g_u_ptr, dV_ptr, dR_ptr, stream))


def sq_device_status(ctx):
    return check(lib().sq_device_status(ctx))
