"""Kessler warm-rain microphysics (include/erf.h: erf_kessler, and erf_rk3_step
with the microphysics switch) against the FP64 oracle, through the C-ABI.

One call: both sides apply the same microphysics step to the same state;
their arithmetic differs only in the rounding of exp, pow and sqrt (~1 ulp)
and in re-associated products, amplified by six Newton steps and the
division by small saturation deficits: the increments agree to 1e-11 of
their scale in FP64.  FP32 storage rounds the stored fields (6e-8 of each
field's scale): 1e-5 of the field's scale.  Precipitation is compared as
accumulated rain per column.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2412_04395_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 1e-5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cfg(**kw):
    base = dict(name="deep_small", nx=40, ny=13, nz=24, n_scalars=3, scalar_scheme=1, adv_order_h=3,
                adv_order_v=3, dt=2.0, n_substeps=8, moist=1, microphysics=1, dx=250.0, dy=250.0,
                dz=W.stretched_dz(24, 50.0, 500.0, 8000.0), seed=71)
    base.update(kw)
    return W.small(**base)


def _sides(cfg):
    from paper_2412_04395_amd import erf
    cfg64 = cfg.replace(prec="fp64")
    th0, qv0 = W.theta_sounding(cfg64), W.qv_sounding(cfg64)
    o = oracle.Oracle(cfg64)
    b = o.init_base_state(th0, cfg64.p_surface, qv0)
    s = erf.Solver(cfg)
    bs = s.init_base_state(th0, qv0=qv0)
    assert np.array_equal(b["rho0"], bs["rho0"])
    return o, s, th0, b


def _wet_state(cfg, o, b, th0, seed):
    """Supersaturated layers, cloud above the autoconversion threshold, rain
    aloft and near the ground in subsaturated air: every process active."""
    S = o.zeros_state()
    shp = S["rho"].shape
    S["rho"][:] = b["rho0"][:, None, None] * (1.0 + W.uniform_noise(seed, shp, 2e-3))
    S["rt"][:] = S["rho"] * (th0[:, None, None] + W.uniform_noise(seed + 1, shp, 0.5))
    z = cfg.z_centres()[:, None, None]
    u = 0.5 * (1.0 + W.uniform_noise(seed + 2, shp, 1.0))
    T0 = (th0 * b["pi0"])[:, None, None]
    qvs0 = np.vectorize(oracle.qvsat)(T0, b["p0"][:, None, None])
    S["rq"][0] = S["rho"] * qvs0 * (0.8 + 0.4 * u)
    S["rq"][1] = S["rho"] * 3e-3 * u * (z > 800.0)
    S["rq"][2] = S["rho"] * 2e-3 * (1.0 - u) * ((z > 2000.0) | (z < 300.0))
    S["ru"][:] = 5.0 * S["rho"]
    return {k: np.ascontiguousarray(v) for k, v in S.items()}


def _round32(S, b):
    rho0 = b["rho0"][:, None, None]
    T0 = (b["rho0"] * b["theta0"])[:, None, None]
    out = {"rho": rho0 + (S["rho"] - rho0).astype(np.float32).astype(np.float64),
           "rt": T0 + (S["rt"] - T0).astype(np.float32).astype(np.float64)}
    for f in ("ru", "rv", "rw", "rq"):
        out[f] = S[f].astype(np.float32).astype(np.float64)
    return {k: np.ascontiguousarray(v) for k, v in out.items()}


def _inc_err(got, ref, start):
    d = np.max(np.abs((got - start) - (ref - start)))
    m = np.max(np.abs(ref - start))
    return d / m if m > 0 else d


@pytest.mark.parametrize("dt", [2.0, 40.0])
def test_kessler_call_matches_oracle_fp64(dt):
    """dt = 40 s sub-steps the rain's fall (Courant number above 0.8)."""
    import torch
    cfg = _cfg()
    o, s, th0, b = _sides(cfg)
    S0 = _wet_state(cfg, o, b, th0, 100)
    ref = {k: v.copy() for k, v in S0.items()}
    o.kessler(ref, dt)
    Sg = s.to_device(S0)
    pg = torch.zeros((cfg.ny, cfg.nx), dtype=torch.float64, device="cuda")
    s.kessler(Sg, dt, pg)
    got = s.to_numpy(Sg)
    e = {"rt": _inc_err(got["rt"], ref["rt"], S0["rt"])}
    for q in range(3):
        e[f"rq{q}"] = _inc_err(got["rq"][q], ref["rq"][q], S0["rq"][q])
    e["precip"] = float(np.max(np.abs(pg.cpu().numpy() - o.precip)) / np.max(np.abs(o.precip)))
    _say(f"kessler fp64 dt {dt}:", {k: f"{v:.2e}" for k, v in e.items()})
    assert np.max(o.precip) > 0 and np.max(np.abs(ref["rq"][1] - S0["rq"][1])) > 0
    for k, v in e.items():
        assert v <= TOL64, (k, v)
    assert np.array_equal(got["rho"], S0["rho"])


def test_kessler_call_matches_oracle_fp32():
    cfg = _cfg(prec="fp32", seed=73)
    o, s, th0, b = _sides(cfg)
    S0 = _round32(_wet_state(cfg, o, b, th0, 200), b)
    ref = {k: v.copy() for k, v in S0.items()}
    o.kessler(ref, 2.0)
    Sg = s.from_full(S0)
    s.kessler(Sg, 2.0)
    got = s.to_full(Sg)
    T0 = (b["rho0"] * b["theta0"])[:, None, None]
    e = {"rt": float(np.max(np.abs(got["rt"] - ref["rt"])) / np.max(np.abs(ref["rt"] - T0)))}
    for q in range(3):
        e[f"rq{q}"] = float(np.max(np.abs(got["rq"][q] - ref["rq"][q])) / np.max(np.abs(ref["rq"][q])))
    prec = s.precipitation()
    e["precip"] = float(np.max(np.abs(prec - o.precip)) / np.max(np.abs(o.precip)))
    _say("kessler fp32:", {k: f"{v:.2e}" for k, v in e.items()})
    for k, v in e.items():
        assert v <= TOL32, (k, v)


def test_rk3_with_microphysics_matches_oracle():
    cfg = _cfg(nx=24, ny=10, seed=75)
    o, s, th0, b = _sides(cfg)
    S = _wet_state(cfg, o, b, th0, 300)
    Sg = s.to_device(S)
    for _ in range(3):
        o.rk3_step(S)
        s.rk3_step(Sg)
    got = s.to_numpy(Sg)
    rho0 = b["rho0"][:, None, None]
    T0 = (b["rho0"] * b["theta0"])[:, None, None]
    e = {"rho": float(np.max(np.abs(got["rho"] - S["rho"])) / np.max(np.abs(S["rho"] - rho0))),
         "rt": float(np.max(np.abs(got["rt"] - S["rt"])) / np.max(np.abs(S["rt"] - T0)))}
    mom = max(np.max(np.abs(S[f])) for f in ("ru", "rv", "rw"))
    for f in ("ru", "rv", "rw"):
        e[f] = float(np.max(np.abs(got[f] - S[f])) / mom)
    for q in range(3):
        e[f"rq{q}"] = float(np.max(np.abs(got["rq"][q] - S["rq"][q])) / np.max(np.abs(S["rq"][q])))
    prec = s.precipitation(reset=True)
    e["precip"] = float(np.max(np.abs(prec - o.precip)) / np.max(np.abs(o.precip)))
    _say("rk3 + kessler x3:", {k: f"{v:.2e}" for k, v in e.items()})
    for k, v in e.items():
        assert v <= TOL64, (k, v)
    assert np.max(s.precipitation()) == 0.0  # reset
    # total water with the fallen rain: the GPU's own budget
    d0 = o.diagnostics(S)
    dg = s.diagnostics(Sg)
    assert abs(sum(dg["scalar_mass"]) / sum(d0["scalar_mass"]) - 1) < 1e-13
