"""The Deardorff TKE closure (Sec. 2.3, coefficients of Moeng 1984) and the
Monin-Obukhov surface layer (Sec. 3.8) of the HIP path against the FP64
oracle, through the C-ABI (include/erf.h: ERF_SGS_DEARDORFF, most_z0).

The source of rho e is compared through erf_scalar_advance, which adds it
(times dts) after erf_slow_rhs computed it: one call of each on both sides.
Tolerances as for the compressible path: 1e-13 of each field's scale for one
call in FP64, 1e-12 after a few RK3 steps, 1e-5 for the FP32 storage on
FP32-representable inputs.  Exact property: a state without TKE keeps none
(no production without eddy viscosity), bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2412_04395_amd import workloads as W

pytestmark = pytest.mark.gpu

CALL_TOL = 1e-13
STEPS_TOL = 1e-12
TOL32 = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cfg(**kw):
    """A small boundary layer: 5th/3rd-order advection, Deardorff closure,
    surface layer over z0 = 0.1 m with a surface heat flux, geostrophic wind."""
    base = dict(name="cbl_small", nx=40, ny=21, nz=17, dx=20.0, dy=20.0, dz=W.stretched_dz(17, 10.0, 40.0, 400.0),
                dt=0.25, n_substeps=8, adv_order_h=5, adv_order_v=3, sgs=3, n_scalars=1, scalar_scheme=1,
                most_z0=0.1, surf_heat_flux=0.15, f_cor=1e-4, Ug=6.0, Vg=-1.0, seed=51)
    base.update(kw)
    return W.small(**base)


def _sides(cfg):
    from paper_2412_04395_amd import erf
    cfg64 = cfg.replace(prec="fp64")
    th0 = 300.0 + 0.004 * np.maximum(cfg64.z_centres() - 150.0, 0.0)
    o = oracle.Oracle(cfg64)
    b = o.init_base_state(th0, cfg64.p_surface)
    s = erf.Solver(cfg)
    bs = s.init_base_state(th0)
    assert np.array_equal(b["rho0"], bs["rho0"])
    return o, s, th0, b


def _state(cfg, b, th0, seed, e0=0.2):
    """winds with noise, warm noise near the ground at constant pressure, TKE
    varying in space (some cells without)"""
    nz, ny, nx = cfg.nz, cfg.ny, cfg.nx
    shp = (nz, ny, nx)
    z = cfg.z_centres()[:, None, None]
    dth = np.where(z < 150.0, W.uniform_noise(seed, shp, 0.3), 0.0)
    Th = (b["rho0"] * th0)[:, None, None] * np.ones(shp)
    rho = Th / (th0[:, None, None] + dth)
    S = {"rho": rho, "rt": Th,
         "ru": rho * (6.0 + W.uniform_noise(seed + 1, shp, 1.0)),
         "rv": rho * (-1.0 + W.uniform_noise(seed + 2, shp, 1.0)),
         "rw": W.uniform_noise(seed + 3, (nz + 1, ny, nx), 0.3),
         "rq": (rho * np.maximum(e0 * (1.0 + W.uniform_noise(seed + 4, shp, 1.2)), 0.0))[None]}
    S["rw"][0] = S["rw"][-1] = 0.0
    return {k: np.ascontiguousarray(v) for k, v in S.items()}


def _round32(S, b):
    rho0 = b["rho0"][:, None, None]
    T0 = (b["rho0"] * b["theta0"])[:, None, None]
    out = {"rho": rho0 + (S["rho"] - rho0).astype(np.float32).astype(np.float64),
           "rt": T0 + (S["rt"] - T0).astype(np.float32).astype(np.float64)}
    for f in ("ru", "rv", "rw", "rq"):
        out[f] = S[f].astype(np.float32).astype(np.float64)
    return {k: np.ascontiguousarray(v) for k, v in out.items()}


def _errs(got, ref, b, fields):
    rho0 = b["rho0"][:, None, None]
    T0 = (b["rho0"] * b["theta0"])[:, None, None]
    out = {}
    for f in fields:
        g, r = got[f], ref[f]
        if f == "rho":
            g, r = g - rho0, r - rho0
        if f == "rt":
            g, r = g - T0, r - T0
        out[f] = float(np.max(np.abs(g - r)) / max(np.max(np.abs(r)), 1e-300))
    return out


@pytest.mark.parametrize("case", ["tke_most", "tke_slip", "smag_most", "tke_stable", "tke_tall"])
def test_slow_rhs_and_tke_source_match_oracle(case):
    # tke_tall: 40 levels, two chunks of the z-marching FP64 tendency kernel
    kw = {"tke_most": {}, "tke_slip": dict(most_z0=0.0), "smag_most": dict(sgs=1, n_scalars=0),
          "tke_stable": dict(surf_heat_flux=-0.02),
          "tke_tall": dict(nx=20, ny=9, nz=40, dz=W.stretched_dz(40, 10.0, 40.0, 1000.0))}[case]
    cfg = _cfg(**kw)
    o, s, th0, b = _sides(cfg)
    S = _state(cfg, b, th0, 100, e0=0.2 if case != "tke_stable" else 2e-3)
    if not cfg.n_scalars:
        S["rq"] = np.zeros((0,) + S["rho"].shape)
    R = o.slow_rhs(S)
    Sg = s.to_device(S)
    got = s.to_numpy(s.slow_rhs(Sg))
    e = _errs(got, R, b, ("rt", "ru", "rv", "rw"))
    if cfg.n_scalars:
        # the source through the scalar update, with zero fluxes
        dts = 0.5
        F = (np.zeros_like(S["ru"]), np.zeros_like(S["rv"]), np.zeros_like(S["rw"]))
        ref_q = o.scalar_advance(S, S, F, dts, R["rq"])
        import torch
        flux = {f: torch.zeros_like(Sg[f]) for f in ("ru", "rv", "rw")}
        got_q = s.scalar_advance(Sg, Sg, flux, dts).cpu().numpy()
        src_ref = ref_q - S["rq"]
        e["tke_src"] = float(np.max(np.abs((got_q - S["rq"]) - src_ref)) / np.max(np.abs(src_ref)))
    _say(f"slow rhs {case}:", {k: f"{v:.2e}" for k, v in e.items()})
    for k, v in e.items():
        assert v <= CALL_TOL, (k, v)
    if case == "tke_stable":
        assert np.any(R["rq"] != 0.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rk3_steps_with_tke_and_surface_layer_match_oracle(prec):
    cfg = _cfg(prec=prec)
    o, s, th0, b = _sides(cfg)
    S = _state(cfg, b, th0, 200)
    if prec == "fp32":
        S = _round32(S, b)
    Sg = s.from_full(S)
    for _ in range(3):
        o.rk3_step(S)
        s.rk3_step(Sg)
    got = s.to_full(Sg)
    e = _errs(got, S, b, ("rho", "rt", "ru", "rv", "rw", "rq"))
    _say(f"rk3 x3 tke+most {prec}:", {k: f"{v:.2e}" for k, v in e.items()})
    tol = STEPS_TOL if prec == "fp64" else TOL32
    for k, v in e.items():
        assert v <= tol, (k, v)
    assert np.min(got["rq"]) >= 0.0


def test_no_tke_stays_no_tke():
    cfg = _cfg()
    o, s, th0, b = _sides(cfg)
    S = _state(cfg, b, th0, 300, e0=0.0)
    assert np.all(S["rq"] == 0.0)
    Sg = s.to_device(S)
    for _ in range(3):
        s.rk3_step(Sg)
    got = s.to_numpy(Sg)
    assert np.all(got["rq"] == 0.0)
