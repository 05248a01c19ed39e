"""Pins of the oracle's Kessler warm-rain microphysics (Sec. 2.4; the scheme of
Kessler 1969 in the form of Klemp & Wilhelmson 1978) to what physics and
mathematics fix: tabulated saturation vapour pressures, the fixed points and
bounds of the saturation adjustment, conservation of total water with the
rain that reaches the ground, the latent-heat balance of every cell, the
thresholds of autoconversion and evaporation, and the sedimentation's flux
form."""
import numpy as np
import pytest

import oracle
from paper_2412_04395_amd import workloads as W

L_V = 2.5e6


def test_saturation_pressure_matches_tables():
    # e_s over water at 0, 10, 20, 30 C from standard psychrometric tables [Pa]
    assert oracle.esat(273.15) == 611.2
    for tc, table in ((10.0, 1228.0), (20.0, 2339.0), (30.0, 4246.0)):
        e = oracle.esat(273.15 + tc)
        assert abs(e / table - 1.0) < 2e-3, (tc, e)
    # Clausius-Clapeyron: d ln e_s / dT = L / (R_v T^2) within the fit's few per cent
    R_v = oracle.const("R_v")
    for T in (275.0, 285.0, 295.0, 305.0):
        h = 1e-3
        slope = (np.log(oracle.esat(T + h)) - np.log(oracle.esat(T - h))) / (2 * h)
        assert abs(slope / (L_V / (R_v * T * T)) - 1.0) < 0.03, T
    # q_vs = eps e / (p - e), eps = R_d / R_v
    eps = oracle.const("R_d") / R_v
    assert oracle.qvsat(293.15, 1e5) == pytest.approx(eps * oracle.esat(293.15) / (1e5 - oracle.esat(293.15)),
                                                       rel=1e-15)


@pytest.mark.parametrize("T,p", [(290.0, 9.0e4), (275.0, 7.0e4), (300.0, 1.0e5)])
def test_adjustment_reaches_saturation_and_conserves(T, p):
    cp = oracle.const("c_p")
    qvs = oracle.qvsat(T, p)
    # supersaturated: condenses until the warmed parcel is exactly saturated
    qv = 1.2 * qvs
    d = oracle.sat_adjust(T, p, qv, 0.0)
    assert d > 0
    assert abs((qv - d) / oracle.qvsat(T + L_V * d / cp, p) - 1.0) < 1e-13
    # exactly saturated with cloud: a fixed point
    assert abs(oracle.sat_adjust(T, p, qvs, 1e-3)) <= 1e-15 * qvs
    # subsaturated, no cloud: nothing happens
    assert oracle.sat_adjust(T, p, 0.8 * qvs, 0.0) == 0.0
    # subsaturated with little cloud: all of it evaporates, the air stays subsaturated
    qc = 1e-5
    d = oracle.sat_adjust(T, p, 0.8 * qvs, qc)
    assert d == -qc
    assert 0.8 * qvs + qc < oracle.qvsat(T - L_V * qc / cp, p)
    # subsaturated with plenty of cloud: evaporates exactly to saturation
    d = oracle.sat_adjust(T, p, 0.98 * qvs, 5e-3)
    assert -5e-3 < d < 0
    assert abs((0.98 * qvs - d) / oracle.qvsat(T + L_V * d / cp, p) - 1.0) < 1e-13


def _moist_cfg(**kw):
    base = dict(name="deep_small", nx=6, ny=5, nz=24, n_scalars=3, scalar_scheme=1, adv_order_h=3,
                adv_order_v=3, dt=2.0, n_substeps=8, moist=1, microphysics=1, dx=250.0, dy=250.0,
                dz=W.stretched_dz(24, 50.0, 500.0, 8000.0), seed=61)
    base.update(kw)
    return W.small(**base)


def _state(cfg, seed, qc_amp=3e-3, qr_amp=2e-3, rh=1.1, rain_base=3000.0):
    """A column set around the moist base state with supersaturated layers,
    cloud above the autoconversion threshold and rain in the upper levels."""
    o = oracle.Oracle(cfg)
    th0, qv0 = W.theta_sounding(cfg), W.qv_sounding(cfg)
    b = o.init_base_state(th0, cfg.p_surface, qv0)
    S = o.zeros_state()
    shp = S["rho"].shape
    S["rho"][:] = b["rho0"][:, None, None] * (1.0 + W.uniform_noise(seed, shp, 2e-3))
    S["rt"][:] = S["rho"] * (th0[:, None, None] + W.uniform_noise(seed + 1, shp, 0.5))
    z = cfg.z_centres()[:, None, None]
    u = 0.5 * (1.0 + W.uniform_noise(seed + 2, shp, 1.0))
    # q_v: rh x saturation at the base state's temperature and pressure
    T0 = (th0 * b["pi0"])[:, None, None]
    qvs0 = np.vectorize(oracle.qvsat)(T0, b["p0"][:, None, None])
    S["rq"][0] = S["rho"] * rh * qvs0 * (0.9 + 0.2 * u)
    S["rq"][1] = S["rho"] * qc_amp * u * (z > 1000.0)
    S["rq"][2] = S["rho"] * qr_amp * u * (z > rain_base)
    return o, b, S


def _exner(S):
    Rd, cp, P00, Rv = (oracle.const(n) for n in ("R_d", "c_p", "P00", "R_v"))
    qv = S["rq"][0] / S["rho"]
    return (Rd * S["rt"] * (1.0 + Rv / Rd * qv) / P00) ** (Rd / (cp - Rd))


def _saturate(S):
    """q_v = q_vs(T, p) where T and p depend on q_v through the moist EOS:
    fixed-point iteration (the dependence is weak; converged to rounding)."""
    P00, cp, Rd = oracle.const("P00"), oracle.const("c_p"), oracle.const("R_d")
    for _ in range(8):
        pi = _exner(S)
        p = P00 * pi ** (cp / Rd)
        T = S["rt"] / S["rho"] * pi
        S["rq"][0] = S["rho"] * np.vectorize(oracle.qvsat)(T, p)


def test_total_water_with_precipitation_is_conserved():
    cfg = _moist_cfg()
    o, b, S = _state(cfg, 5, rain_base=100.0)
    vol = cfg.dx * cfg.dy * np.asarray(cfg.dz)[:, None, None]
    w0 = np.sum(S["rq"][:3].sum(axis=0) * vol)
    for _ in range(6):
        o.kessler(S, 10.0)
    w1 = np.sum(S["rq"][:3].sum(axis=0) * vol)
    fallen = np.sum(o.precip) * cfg.dx * cfg.dy
    assert fallen > 0, "rain must reach the ground"
    assert abs((w1 + fallen) / w0 - 1.0) < 1e-14
    for s in range(3):
        assert np.min(S["rq"][s]) >= 0.0, s


def test_every_cell_balances_latent_heat():
    # pressure held during the step: c_p pi (theta_new - theta) = -L (q_v,new - q_v)
    cfg = _moist_cfg()
    o, b, S = _state(cfg, 9)
    pi = _exner(S)
    th_old, qv_old = S["rt"] / S["rho"], S["rq"][0] / S["rho"]
    o.kessler(S, 8.0)
    th_new, qv_new = S["rt"] / S["rho"], S["rq"][0] / S["rho"]
    cp = oracle.const("c_p")
    lhs = cp * pi * (th_new - th_old)
    rhs = -L_V * (qv_new - qv_old)
    assert np.max(np.abs(qv_new - qv_old)) > 1e-5  # phase changes happened
    assert np.max(np.abs(lhs - rhs)) <= 1e-9 * np.max(np.abs(rhs)) + 1e-12


def test_cloud_below_threshold_makes_no_rain_and_saturated_air_keeps_its_rain():
    cfg = _moist_cfg(nz=10, dz=W.uniform_dz(10, 100.0))
    o, b, S = _state(cfg, 13, qc_amp=9e-4, qr_amp=0.0, rh=1.0)
    # saturated everywhere, cloud below the 1e-3 threshold, no rain
    _saturate(S)
    o.kessler(S, 5.0)
    assert np.max(S["rq"][2]) == 0.0
    assert np.max(o.precip) == 0.0


def test_rain_evaporates_only_up_to_saturation():
    cfg = _moist_cfg(nz=12, dz=W.uniform_dz(12, 100.0))
    o, b, S = _state(cfg, 17, qc_amp=0.0, qr_amp=3e-3, rh=0.5)
    S["rq"][2] = S["rho"] * 3e-3  # rain everywhere, in dry air, no cloud
    qv_old = S["rq"][0] / S["rho"]
    pi = _exner(S)
    o.kessler(S, 300.0)  # long enough to saturate the lowest cells
    p = oracle.const("P00") * pi ** (oracle.const("c_p") / oracle.const("R_d"))
    T = S["rt"] / S["rho"] * pi
    qv = S["rq"][0] / S["rho"]
    qvs = np.vectorize(oracle.qvsat)(T, p)
    assert np.all(qv > qv_old)
    assert np.all(qv <= qvs * (1 + 1e-12))
    assert np.max(S["rq"][1]) == 0.0  # evaporating rain makes no cloud


def test_dry_state_is_unchanged_bitwise():
    cfg = _moist_cfg(nz=8, dz=W.uniform_dz(8, 100.0))
    o, b, S = _state(cfg, 21, qc_amp=0.0, qr_amp=0.0, rh=0.0)
    S0 = {k: v.copy() for k, v in S.items()}
    o.kessler(S, 10.0)
    for f in ("rho", "rt", "rq"):
        assert np.array_equal(S[f], S0[f]), f


def test_sedimentation_is_flux_form_with_a_plausible_fall_speed():
    # one wet cell high in a saturated column without cloud: the rain leaves
    # the cell downward only, mass is conserved, and the mass centroid moves
    # down by the mass-weighted fall speed times dt (flux form, upwind)
    cfg = _moist_cfg(nx=1, ny=1, nz=40, dz=W.uniform_dz(40, 50.0))
    o, b, S = _state(cfg, 25, qc_amp=0.0, qr_amp=0.0, rh=1.0)
    _saturate(S)
    k0 = 30
    S["rq"][2][k0] = 1e-3  # 1 g/m^3 of rain water
    z = cfg.z_centres()
    m0 = S["rq"][2][:, 0, 0].copy()
    dt = 1.0
    o.kessler(S, dt)
    m1 = S["rq"][2][:, 0, 0]
    assert np.sum(m1) == pytest.approx(np.sum(m0), rel=1e-14)
    assert np.all(m1[k0 + 1:] == 0.0) and m1[k0 - 1] > 0
    drop = (np.sum(z * m0) - np.sum(z * m1)) / np.sum(m0) / dt  # centroid speed
    assert 4.0 < drop < 8.0, drop  # 1 g/m^3 of rain falls at about 5-6 m/s
    V = m0[k0] and (m0[k0] - m1[k0]) / dt * 50.0 / m0[k0]  # flux out / mass = V / dz
    assert V == pytest.approx(drop, rel=1e-7)  # the centroid difference cancels ~4 digits


def test_rk3_step_with_microphysics_conserves_water_and_rains():
    cfg = _moist_cfg(nx=8, ny=6, nz=20, dz=W.stretched_dz(20, 50.0, 400.0, 6000.0))
    o, b, S = _state(cfg, 31, rain_base=50.0)
    vol = cfg.dx * cfg.dy * np.asarray(cfg.dz)[:, None, None]
    w0 = np.sum(S["rq"][:3].sum(axis=0) * vol)
    for _ in range(3):
        o.rk3_step(S)
    w1 = np.sum(S["rq"][:3].sum(axis=0) * vol) + np.sum(o.precip) * cfg.dx * cfg.dy
    assert abs(w1 / w0 - 1.0) < 1e-13
    assert np.sum(o.precip) > 0
