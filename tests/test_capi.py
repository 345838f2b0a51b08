"""The C-ABI library loads and exports what include/sq.h declares; host-side
argument validation fails with SQ_ERR_ARG before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2011_13517_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sq_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libsq.so is not built (run __graft_entry__.build())")
    return L.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert set(names) == set(L.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def _params(**kw):
    p = L.sq_params()
    p.n[:] = [8, 8, 8]
    p.h[:] = [0.5, 0.5, 0.5]
    p.fd_order = 4
    p.bc = 0
    p.rcut[:] = [2, 2, 2]
    p.order = 10
    p.kT = 0.1
    p.precision = 0
    p.ckpt_every = 0
    for k, v in kw.items():
        if isinstance(getattr(p, k), C.Array):
            getattr(p, k)[:] = v
        else:
            setattr(p, k, v)
    return p


@pytest.mark.parametrize("kw", [dict(fd_order=3), dict(fd_order=14), dict(order=0),
                                dict(kT=0.0), dict(bc=7), dict(precision=5), dict(h=[0.5, 0, 0.5]),
                                dict(n=[8, 0, 8]), dict(rcut=[-1, 2, 2]), dict(ckpt_every=-1),
                                dict(adjoint_precision=3), dict(tune=3), dict(tune=-1)])
def test_invalid_params_rejected(lib, kw):
    ctx = C.c_void_p()
    st = lib.sq_setup(C.byref(_params(**kw)), None, None, None, 512, C.byref(ctx))
    assert st == L.SQ_ERR_ARG
    assert ctx.value is None
    assert len(L.sq_last_error()) > 0


def test_null_arguments_rejected(lib):
    assert lib.sq_setup(None, None, None, None, 0, None) == L.SQ_ERR_ARG
    assert lib.sq_density(None, None, 0.0, 1.0, None, None, None) == L.SQ_ERR_ARG
    assert lib.sq_fermi_level(None, 1.0, 1e-8, 10, None, None, None, None, None) == L.SQ_ERR_ARG
    assert lib.sq_density_backward(None, None, None, None, None, None) == L.SQ_ERR_ARG
    assert lib.sq_get_info(None, None) == L.SQ_ERR_ARG
    assert lib.sq_entropy(None, None, None, None) == L.SQ_ERR_ARG
    assert lib.sq_gauss_density(None, None, 0.0, 1.0, None, None, None) == L.SQ_ERR_ARG
    assert lib.sq_gauss_fermi_level(None, 1.0, 1e-8, 10, None, None, None, None, None,
                                    None) == L.SQ_ERR_ARG
    assert lib.sq_nonlocal_force(None, None, None) == L.SQ_ERR_ARG
    sp = L.sq_scf_params(beta=0.3, tol=1e-6, fermi_tol=1e-10, poisson_rtol=1e-12, max_iter=5,
                         anderson=1, poisson_max_iter=100)
    info = L.sq_scf_info()
    assert lib.sq_scf(None, None, None, 1.0, 0.0, 1.0, C.byref(sp), None, None, None,
                      C.byref(info), None) == L.SQ_ERR_ARG
    assert b"NULL" in lib.sq_last_error()
    assert lib.sq_destroy(None) == L.SQ_OK


def test_binding_raises_with_message(lib):
    with pytest.raises(L.SQError) as e:
        L.sq_setup(_params(order=0), None, None, None, 512)
    assert e.value.status == L.SQ_ERR_ARG
    assert "order" in str(e.value)


def test_package_has_no_fallback_path():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2011_13517_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "sq_oracle" not in txt, f


def _struct_fields(name):
    src = open(os.path.join(ROOT, "include", "sq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + ";", src).group(1)
    return [m.group(2) for m in
            re.finditer(r"\b(int32_t|int64_t|double|const [a-z0-9_]+ \*)\s*([A-Za-z_0-9]+)", body)]


@pytest.mark.parametrize("name,cls", [("sq_params", L.sq_params), ("sq_info", L.sq_info),
                                      ("sq_projectors", L.sq_projectors)])
def test_binding_struct_layout_matches_header(name, cls):
    """The ctypes structures list the header's fields in the header's order."""
    assert _struct_fields(name) == [f[0] for f in cls._fields_]


@pytest.mark.parametrize("sup_off", [[0, 100, 50], [0, 3, 2], [0, 5, 4], [1, 2, 3], [0, -1, 2]])
def test_malformed_support_offsets_rejected(lib, sup_off):
    """A projector CSR whose offsets run backwards, past nnz = sup_off[-1] or do
    not start at 0 is refused with SQ_ERR_ARG before any table is read (the
    support arrays below hold only nnz rows, so a read past them would be out of
    bounds)."""
    off = np.asarray(sup_off, np.int64)
    nnz = max(int(off[-1]), 0)
    idx = np.zeros(nnz, np.int64)
    chi = np.zeros((nnz, 4))
    c = np.ones((2, 4))
    pr = L.sq_projectors(n_atoms=2, n_proj=4, sup_off=off.ctypes.data, sup_idx=idx.ctypes.data,
                         chi=chi.ctypes.data, dchi=None, c=c.ctypes.data)
    ctx = C.c_void_p()
    st = lib.sq_setup(C.byref(_params()), C.byref(pr), None, None, 512, C.byref(ctx))
    assert st == L.SQ_ERR_ARG
    assert ctx.value is None
    assert b"sup_off" in lib.sq_last_error()
