"""The C-ABI library loads on the CPU and exports what include/erf.h declares.

No compute call is made here (no GPU): only host-side entry points and the
argument checks that run before any HIP call.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2412_04395_amd import erf
from paper_2412_04395_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    syms = set()
    for name in os.listdir(os.path.join(ROOT, "include")):
        if name.endswith(".h"):
            text = open(os.path.join(ROOT, "include", name)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            syms |= set(re.findall(r"\b(erf_[a-z0-9_]+)\s*\(", text))
    return syms


def test_library_exports_every_declared_symbol():
    L = erf.load()
    syms = _declared_symbols()
    assert len(syms) >= 10
    for s in sorted(syms):
        assert hasattr(L, s), s
    assert set(erf.EXPORTS) == syms


@pytest.mark.parametrize("kind", ["uniform", "stretched", "deep"])
def test_host_base_state_equals_oracle_bitwise(kind):
    # the library's host Newton iteration takes the same steps as the oracle's,
    # so both sides build identical initial states around identical base states
    if kind == "uniform":
        cfg = W.cbl()
    elif kind == "stretched":
        cfg = W.deep()
    else:
        cfg = W.bubble2d()
    th0 = W.theta_sounding(cfg)
    a = erf.base_state_host(cfg.dz, th0, cfg.p_surface, cfg.grav)
    b = oracle.base_state(cfg.dz, th0, cfg.p_surface, cfg.grav)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_noalloc_batch_limit_matches_the_header():
    import re
    text = open(os.path.join(ROOT, "include", "erf_mlp.h")).read()
    m = re.search(r"#define ERF_MLP_NOALLOC_MAX_BATCH (\d+)", text)
    assert m and int(m.group(1)) == erf.MLP_NOALLOC_MAX_BATCH


def test_host_moist_base_state_equals_oracle_bitwise():
    # with the deep workload's vapour sounding the Newton steps are again the
    # oracle's; with qv0 = 0 the moist iteration is the dry one bit for bit
    cfg = W.deep()
    th0, qv0 = W.theta_sounding(cfg), W.qv_sounding(cfg)
    a = erf.base_state_host(cfg.dz, th0, cfg.p_surface, cfg.grav, qv0=qv0)
    b = oracle.base_state(cfg.dz, th0, cfg.p_surface, cfg.grav, qv0=qv0)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    z = erf.base_state_host(cfg.dz, th0, cfg.p_surface, cfg.grav, qv0=np.zeros(cfg.nz))
    d = erf.base_state_host(cfg.dz, th0, cfg.p_surface, cfg.grav)
    for x, y in zip(z, d):
        assert np.array_equal(x, y)
    assert not np.array_equal(a[0], d[0])
    with pytest.raises(erf.ErfError):
        erf.base_state_host(cfg.dz, th0, cfg.p_surface, cfg.grav, qv0=-qv0)


def test_create_checks_the_moist_flag():
    cfg = W.small(n_scalars=3, moist=1)
    L = erf.load()
    st, h = _create(cfg)
    if st == erf.ERF_OK:  # created (a GPU is present): release it
        L.erf_destroy(h)
    assert _create(W.small(n_scalars=2, moist=1))[0] == erf.ERF_E_ARG
    assert _create(W.small(n_scalars=3, moist=2))[0] == erf.ERF_E_ARG


def _create(cfg, **kw):
    L = erf.load()
    dz = np.ascontiguousarray(cfg.dz, dtype=np.float64)
    g = erf.Grid(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, dz.ctypes.data_as(C.POINTER(C.c_double)))
    for k, v in kw.items():
        setattr(g, k, v)
    p = erf.params_from_config(cfg)
    h = C.c_void_p()
    return L.erf_create(C.byref(g), C.byref(p), None, C.byref(h)), h


def test_create_rejects_bad_arguments_before_touching_the_gpu():
    cfg = W.small()
    assert _create(cfg, nz=1)[0] == erf.ERF_E_SHAPE
    assert _create(cfg, nx=0)[0] == erf.ERF_E_SHAPE
    assert _create(cfg.replace(n_substeps=3))[0] == erf.ERF_E_ARG
    assert _create(cfg.replace(adv_order_h=7))[0] == erf.ERF_E_ARG
    assert _create(cfg.replace(dz=np.r_[cfg.dz[:-1], -1.0]))[0] == erf.ERF_E_ARG
    assert _create(cfg.replace(n_scalars=9))[0] == erf.ERF_E_ARG
    assert _create(cfg.replace(n_scalars=1, sgs=1))[0] == erf.ERF_E_UNSUPPORTED
    assert _create(cfg.replace(dt=0.0))[0] == erf.ERF_E_ARG
    assert _create(cfg.replace(sgs=4))[0] == erf.ERF_E_ARG
    # the Deardorff closure needs rho e as its one scalar, dry, compressible
    assert _create(cfg.replace(sgs=3))[0] == erf.ERF_E_UNSUPPORTED
    assert _create(cfg.replace(sgs=3, n_scalars=2))[0] == erf.ERF_E_UNSUPPORTED
    assert _create(cfg.replace(sgs=3, n_scalars=3, moist=1))[0] == erf.ERF_E_UNSUPPORTED
    assert _create(cfg.replace(sgs=3, n_scalars=1, alpha_m=1.0))[0] == erf.ERF_E_UNSUPPORTED
    # the roughness length lies between 0 and half the lowest cell
    assert _create(cfg.replace(most_z0=-0.1))[0] == erf.ERF_E_ARG
    assert _create(cfg.replace(most_z0=0.5 * cfg.dz[0]))[0] == erf.ERF_E_ARG
    assert _create(cfg.replace(sgs=2, nu_m=1e-3))[0] == erf.ERF_E_UNSUPPORTED
    assert _create(cfg.replace(sgs=2, n_scalars=1))[0] == erf.ERF_E_UNSUPPORTED
    L = erf.load()
    assert L.erf_create(None, None, None, None) == erf.ERF_E_ARG
    assert L.erf_rk3_step(None, None) == erf.ERF_E_ARG
    assert L.erf_mlp_set_weights(None, None, None) == erf.ERF_E_ARG
    assert L.erf_mlp_forward(None, None, 0, None) == erf.ERF_E_ARG
    assert L.erf_mlp_train_step(None, None, None, 1, 1e-3, None) == erf.ERF_E_ARG
    assert L.erf_box_filter(None, None, 2, 0.0, 1.0, None, None) == erf.ERF_E_ARG


def test_create_checks_the_anelastic_restrictions():
    cfg = W.small(nx=32, ny=16, anelastic=1)
    L = erf.load()
    st, h = _create(cfg)
    if st == erf.ERF_OK:  # created (a GPU is present): release it
        L.erf_destroy(h)
    # the transforms need powers of two up to 2048
    assert _create(cfg, nx=37)[0] == erf.ERF_E_SHAPE
    assert _create(cfg, ny=24)[0] == erf.ERF_E_SHAPE
    assert _create(cfg, nx=4096)[0] == erf.ERF_E_SHAPE
    assert _create(cfg.replace(prec="fp32"))[0] == erf.ERF_E_UNSUPPORTED
    assert _create(cfg.replace(sgs=2))[0] == erf.ERF_E_UNSUPPORTED
    assert _create(cfg.replace(n_scalars=3, moist=1))[0] == erf.ERF_E_UNSUPPORTED
    assert _create(cfg.replace(anelastic=2))[0] == erf.ERF_E_ARG
    out = erf.FieldLayout()
    dz = np.ascontiguousarray(cfg.dz, dtype=np.float64)
    g = erf.Grid(37, cfg.ny, cfg.nz, cfg.dx, cfg.dy, dz.ctypes.data_as(C.POINTER(C.c_double)))
    assert L.erf_layout(C.byref(g), C.byref(erf.params_from_config(cfg)), 0, C.byref(out)) == erf.ERF_E_SHAPE
    # the anelastic calls refuse a missing context
    assert L.erf_ssprk2_step(None, None) == erf.ERF_E_ARG
    assert L.erf_project(None, None, 1.0) == erf.ERF_E_ARG
    assert L.erf_anelastic_pressure(None, None, 0) == erf.ERF_E_ARG


def test_product_path_has_no_oracle_dependency():
    # the product package never imports the oracle
    pkg = os.path.join(ROOT, "paper_2412_04395_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "erf_oracle" not in text, f


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_layout_matches_the_state_conventions(prec):
    """erf_layout restates the conventions of include/erf.h: x fastest, nz + 1
    z-faces for rho w, n_scalars components of rho q, 8- or 4-byte elements,
    and in FP32 storage rho and rho*theta held as perturbations."""
    cfg = W.small(nx=13, ny=7, nz=5, dz=W.uniform_dz(5, 100.0), n_scalars=3, prec=prec)
    eb = 8 if prec == "fp64" else 4
    for f in erf.FIELDS:
        lay = erf.layout(cfg, f)
        nz = cfg.nz + 1 if f == "rw" else cfg.nz
        comps = 3 if f == "rq" else 1
        assert (lay["nx"], lay["ny"], lay["nz"], lay["components"]) == (13, 7, nz, comps), f
        assert (lay["stride_y"], lay["stride_z"], lay["stride_c"]) == (13, 13 * 7, 13 * 7 * nz), f
        assert lay["count"] == 13 * 7 * nz * comps and lay["bytes"] == lay["count"] * eb, f
        assert lay["elem_bytes"] == eb
        assert lay["perturbation"] == (1 if prec == "fp32" and f in ("rho", "rt") else 0), f
    # no scalars: an empty rho q
    lay = erf.layout(W.small(prec=prec), "rq")
    assert lay["components"] == 0 and lay["count"] == 0 and lay["bytes"] == 0


def test_layout_rejects_what_create_rejects():
    L = erf.load()
    cfg = W.small()
    out = erf.FieldLayout()

    def call(nz=None, field=0, **prm):
        c = W.small(**prm) if prm else cfg
        dz = np.ascontiguousarray(c.dz if nz is None else np.full(nz, 100.0), dtype=np.float64)
        g = erf.Grid(c.nx, c.ny, len(dz), c.dx, c.dy, dz.ctypes.data_as(C.POINTER(C.c_double)))
        return L.erf_layout(C.byref(g), C.byref(erf.params_from_config(c)), field, C.byref(out))

    assert call() == erf.ERF_OK
    assert call(field=6) == erf.ERF_E_ARG
    assert call(field=-1) == erf.ERF_E_ARG
    assert call(nz=1) == erf.ERF_E_SHAPE
    assert call(nz=257) == erf.ERF_E_SHAPE
    assert call(n_scalars=9) == erf.ERF_E_ARG
    p = erf.params_from_config(cfg)
    p.precision = 7
    dz = np.ascontiguousarray(cfg.dz, dtype=np.float64)
    g = erf.Grid(cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, dz.ctypes.data_as(C.POINTER(C.c_double)))
    assert L.erf_layout(C.byref(g), C.byref(p), 0, C.byref(out)) == erf.ERF_E_ARG
    assert L.erf_layout(None, C.byref(p), 0, C.byref(out)) == erf.ERF_E_ARG
    assert L.erf_layout(C.byref(g), C.byref(erf.params_from_config(cfg)), 0, None) == erf.ERF_E_ARG
