"""Terrain-following coordinates (Sec. 3.4, App. A, App. B, App. C) of the HIP
path against the FP64 oracle, through the C-ABI (include/erf.h:
erf_set_terrain, erf_init_base_state_columns).

Tolerances as for the flat compressible path: 1e-13 of each field's scale for
one call, 1e-12 after a few RK3 steps.  The geometry and the per-column base
state are host arithmetic in the same order on both sides and must agree bit
for bit.  At the size of the benchmark's terrain workload (256 x 256 x 128,
too large for the oracle in a test) the checks are properties that hold at any
size: a resting atmosphere stays at rest bit for bit, and mass and sum rho
theta dV are conserved to roundoff.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2412_04395_amd import workloads as W

pytestmark = pytest.mark.gpu

CALL_TOL = 1e-13
STEPS_TOL = 1e-12
TH_S, N_BV, P_SEA = 300.0, 0.01, 1.0e5


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cfg(**kw):
    base = dict(name="terrain_small", nx=40, ny=21, nz=17, dx=200.0, dy=200.0,
                dz=W.stretched_dz(17, 40.0, 400.0, 4000.0), dt=1.0, n_substeps=6, adv_order_h=3,
                adv_order_v=3, f_cor=1e-4, Ug=10.0, Vg=2.0, seed=13)
    base.update(kw)
    return W.small(**base)


def _inputs(cfg, h, Hc, zc):
    th0 = W.stratified_theta(zc, TH_S, N_BV, cfg.grav)
    ps = W.stratified_ground_pressure(W.cell_mean_nodes(h), TH_S, N_BV, P_SEA, cfg.grav)
    return th0, ps


def _sides(cfg, h, beta):
    from paper_2412_04395_amd import erf
    o = oracle.Oracle(cfg)
    o.set_terrain(h, beta)
    Hc, zc = o.terrain_heights()
    s = erf.Solver(cfg)
    s.set_terrain(h, beta)
    Hg, zg = s.terrain_heights()
    assert np.array_equal(Hc, Hg) and np.array_equal(zc, zg)
    th0, ps = _inputs(cfg, h, Hc, zc)
    b = o.init_base_state_columns(th0, ps)
    bs = s.init_base_state_columns(th0, ps)
    for f in ("rho0", "p0", "pi0"):
        assert np.array_equal(b[f], bs[f]), f
    return o, s, b, Hc


def _flow(b, seed, U=10.0, V=2.0):
    shp = b["rho0"].shape
    nz, ny, nx = shp
    rho = b["rho0"] * (1.0 + W.uniform_noise(seed, shp, 1e-3))
    S = {"rho": rho, "rt": b["rho0"] * b["theta0"] * (1.0 + W.uniform_noise(seed + 1, shp, 1e-3)),
         "ru": rho * (U + W.uniform_noise(seed + 2, shp, 1.0)),
         "rv": rho * (V + W.uniform_noise(seed + 3, shp, 1.0)),
         "rw": W.uniform_noise(seed + 4, (nz + 1, ny, nx), 0.3), "rq": np.zeros((0, nz, ny, nx))}
    S["rw"][0] = S["rw"][-1] = 0.0
    return {k: np.ascontiguousarray(v) for k, v in S.items()}


def _errs(got, ref, b, fields):
    out = {}
    for f in fields:
        g, r = got[f], ref[f]
        if f == "rho":
            g, r = g - b["rho0"], r - b["rho0"]
        if f == "rt":
            T0 = b["rho0"] * b["theta0"]
            g, r = g - T0, r - T0
        out[f] = float(np.max(np.abs(g - r)) / max(np.max(np.abs(r)), 1e-300))
    return out


CASES = {
    "btf_o3": dict(beta=1.0, kw={}),
    "sullivan_o5": dict(beta=3.0, kw=dict(adv_order_h=5, adv_order_v=3)),
    "btf_o6_ragged": dict(beta=1.0, kw=dict(nx=70, ny=9, nz=20, dz=W.stretched_dz(20, 30.0, 400.0, 4000.0),
                                            adv_order_h=6, adv_order_v=4)),
    "ridge_o2": dict(beta=3.0, kw=dict(adv_order_h=2, adv_order_v=2), ridge=True),
    "heated_o3": dict(beta=1.0, kw=dict(surf_heat_flux=0.2)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_slow_rhs_and_substeps_match_oracle(case):
    spec = CASES[case]
    cfg = _cfg(**spec["kw"])
    h = W.agnesi_nodes(cfg, 400.0, 1000.0, ridge=spec.get("ridge", False))
    o, s, b, Hc = _sides(cfg, h, spec["beta"])
    S = _flow(b, 100)
    R = o.slow_rhs(S)
    Sg = s.to_device(S)
    Rg = s.slow_rhs(Sg)
    e = _errs(s.to_numpy(Rg), R, b, ("rho", "rt", "ru", "rv", "rw"))
    _say(f"terrain slow rhs {case}:", {k: f"{v:.2e}" for k, v in e.items()})
    for k, v in e.items():
        assert v <= CALL_TOL, (k, v)
    # one stage of substeps from S'' = S_n - S_t with the oracle's tendencies
    Sn = _flow(b, 200)
    out, _ = o.acoustic_substeps(Sn, S, R, 3, cfg.dt / cfg.n_substeps)
    outg, _ = s.acoustic_substeps(s.to_device(Sn), Sg, s.to_device(R), 3, cfg.dt / cfg.n_substeps, sums=False)
    e = _errs(s.to_numpy(outg), out, b, ("rho", "rt", "ru", "rv", "rw"))
    _say(f"terrain substeps {case}:", {k: f"{v:.2e}" for k, v in e.items()})
    for k, v in e.items():
        assert v <= CALL_TOL, (k, v)


def test_rk3_steps_and_diagnostics_match_oracle():
    cfg = _cfg()
    h = W.agnesi_nodes(cfg, 400.0, 1000.0)
    o, s, b, Hc = _sides(cfg, h, 3.0)
    S = _flow(b, 300)
    Sg = s.to_device(S)
    for _ in range(3):
        o.rk3_step(S)
        s.rk3_step(Sg)
    got = s.to_numpy(Sg)
    e = _errs(got, S, b, ("rho", "rt", "ru", "rv", "rw"))
    _say("terrain rk3 x3:", {k: f"{v:.2e}" for k, v in e.items()})
    for k, v in e.items():
        assert v <= STEPS_TOL, (k, v)
    d_o, d_g = o.diagnostics(S), s.diagnostics(Sg)
    for k in ("mass", "theta_mass", "energy"):
        assert d_g[k] == pytest.approx(d_o[k], rel=1e-12), k


def test_single_level_column():
    # nz = 2: the one interior face's tridiagonal row and one-sided vertical
    # differences everywhere
    cfg = _cfg(nz=2, dz=np.array([300.0, 500.0]))
    h = W.agnesi_nodes(cfg, 100.0, 800.0)
    o, s, b, Hc = _sides(cfg, h, 1.0)
    S = _flow(b, 400)
    Sg = s.to_device(S)
    for _ in range(2):
        o.rk3_step(S)
        s.rk3_step(Sg)
    e = _errs(s.to_numpy(Sg), S, b, ("rho", "rt", "ru", "rv", "rw"))
    _say("terrain nz=2 rk3 x2:", {k: f"{v:.2e}" for k, v in e.items()})
    for k, v in e.items():
        assert v <= STEPS_TOL, (k, v)


def test_refusals():
    from paper_2412_04395_amd import erf
    cfg = _cfg()
    h = W.agnesi_nodes(cfg, 400.0, 1000.0)
    for kw in (dict(sgs=1), dict(moist=1, n_scalars=3), dict(prec="fp32"), dict(nu_m=1.0)):
        s = erf.Solver(cfg.replace(**kw))
        with pytest.raises(RuntimeError):
            s.set_terrain(h, 1.0)
    s = erf.Solver(cfg)
    with pytest.raises(RuntimeError):
        s.set_terrain(np.full((cfg.ny, cfg.nx), 5000.0), 1.0)  # above the lid
    s.set_terrain(h, 1.0)
    with pytest.raises(RuntimeError):
        s.init_base_state(np.full(cfg.nz, 300.0))
    # the closure's inputs and the box filter follow the flat grid's axes
    Hc, zc = s.terrain_heights()
    th0, ps = _inputs(cfg, h, Hc, zc)
    b = s.init_base_state_columns(th0, ps)
    Sg = s.to_device(_flow(b, 700))
    with pytest.raises(RuntimeError):
        s.mlp_features(Sg)
    with pytest.raises(RuntimeError):
        s.box_filter(Sg, 1)


def test_benchmark_size_rest_and_conservation():
    from paper_2412_04395_amd import erf
    cfg = W.terrain_hill()
    h = W.agnesi_nodes(cfg, 400.0, 2000.0)
    s = erf.Solver(cfg)
    s.set_terrain(h, 1.0)
    Hc, zc = s.terrain_heights()
    th0, ps = _inputs(cfg, h, Hc, zc)
    b = s.init_base_state_columns(th0, ps)
    shp = b["rho0"].shape
    rest = {"rho": b["rho0"], "rt": b["rho0"] * b["theta0"], "ru": np.zeros(shp), "rv": np.zeros(shp),
            "rw": np.zeros((shp[0] + 1,) + shp[1:]), "rq": np.zeros((0,) + shp)}
    Sg = s.to_device(rest)
    s0 = {k: v.clone() for k, v in Sg.items()}
    s.rk3_step(Sg)
    for f in ("rho", "rt", "ru", "rv", "rw"):
        assert bool((Sg[f] == s0[f]).all()), f
    # a wind over the hill: mass and sum rho theta dV are conserved
    S = {"rho": b["rho0"], "rt": b["rho0"] * b["theta0"], "ru": b["rho0"] * 10.0, "rv": np.zeros(shp),
         "rw": np.zeros((shp[0] + 1,) + shp[1:]), "rq": np.zeros((0,) + shp)}
    Sg = s.to_device({k: np.ascontiguousarray(v) for k, v in S.items()})
    d0 = s.diagnostics(Sg)
    for _ in range(3):
        s.rk3_step(Sg)
    d1 = s.diagnostics(Sg)
    _say("terrain 256x256x128 mass, theta-mass drift:", d1["mass"] / d0["mass"] - 1.0,
         d1["theta_mass"] / d0["theta_mass"] - 1.0, "max w", d1["max_w"])
    assert abs(d1["mass"] / d0["mass"] - 1.0) < 1e-13
    assert abs(d1["theta_mass"] / d0["theta_mass"] - 1.0) < 1e-13
    assert 0.0 < d1["max_w"] < 20.0


def test_witch_of_agnesi_mountain_wave_300_steps():
    # the 2-D ridge case of the oracle's linear-theory pin (Sec. 4.3), 6000 s:
    # the GPU's w equals the oracle's to roundoff after 300 RK3 steps, and
    # meets the same bounds against the linear hydrostatic solution
    from paper_2412_04395_amd import erf
    cfg = _cfg(nx=128, ny=1, nz=60, dx=2000.0, dy=2000.0, dz=W.uniform_dz(60, 500.0), dt=20.0, n_substeps=6,
               f_cor=0.0, Ug=0.0, Vg=0.0, steps=300)
    a, hm, U = 10000.0, 10.0, 10.0
    h = W.agnesi_nodes(cfg, hm, a, ridge=True)
    o, s, b, Hc = _sides(cfg, h, 1.0)
    shp = b["rho0"].shape
    S = {"rho": b["rho0"].copy(), "rt": b["rho0"] * b["theta0"], "ru": b["rho0"] * U, "rv": np.zeros(shp),
         "rw": np.zeros((shp[0] + 1,) + shp[1:]), "rq": np.zeros((0,) + shp)}
    S = {k: np.ascontiguousarray(v) for k, v in S.items()}
    Sg = s.to_device(S)
    for _ in range(cfg.steps):
        o.rk3_step(S)
        s.rk3_step(Sg)
    got = s.to_numpy(Sg)
    e = _errs(got, S, b, ("rho", "rt", "ru", "rw"))
    _say("agnesi 300 steps gpu vs oracle:", {k: f"{v:.2e}" for k, v in e.items()})
    for k, v in e.items():
        assert v <= 1e-10, (k, v)
    rho = got["rho"][:, 0, :]
    wf = got["rw"][1:-1, 0, :] / (0.5 * (rho[1:] + rho[:-1]))
    w = np.zeros_like(rho)
    w[1:-1] = 0.5 * (wf[:-1] + wf[1:])
    _, zc = s.terrain_heights()
    z = zc[:, 0, :]
    x = (np.arange(cfg.nx) + 0.5) * cfg.dx - 0.5 * cfg.nx * cfg.dx
    X = np.broadcast_to(x, z.shape)
    l = N_BV / U
    den = X * X + a * a
    deta = hm * a * (-np.sin(l * z) * den - 2.0 * X * (a * np.cos(l * z) - X * np.sin(l * z))) / den ** 2
    wlin = U * deta * np.sqrt(b["rho0"][0, 0, :] / b["rho0"][:, 0, :])
    m = (z[:, 0] > 300.0) & (z[:, 0] < 2000.0)
    corr = float(np.sum(w[m] * wlin[m]) / np.sqrt(np.sum(w[m] ** 2) * np.sum(wlin[m] ** 2)))
    _say("agnesi lowest 2 km: correlation with the linear solution", corr)
    assert corr > 0.97


@pytest.mark.parametrize("scheme", [0, 1])
def test_scalars_over_terrain_match_oracle(scheme):
    # stage-averaged fluxes (rho Omega vertically) and one scalar update per
    # call; three RK3 steps with two scalars; a uniform mixing ratio stays
    # uniform on the GPU (interpolant of the run's order, and WENO5)
    cfg = _cfg(n_scalars=2, scalar_scheme=scheme, adv_order_h=5, adv_order_v=3)
    h = W.agnesi_nodes(cfg, 400.0, 1000.0)
    o, s, b, Hc = _sides(cfg, h, 3.0)
    S = _flow(b, 500)
    shp = b["rho0"].shape
    S["rq"] = np.ascontiguousarray(np.stack([0.01 * S["rho"], S["rho"] * (1.0 + W.uniform_noise(501, shp, 0.5))]))
    R = o.slow_rhs(S)
    Sn = _flow(b, 600)
    Sn["rq"] = S["rq"].copy()
    dtau = cfg.dt / cfg.n_substeps
    out, F = o.acoustic_substeps(Sn, S, R, 3, dtau)
    Sg, Sng = s.to_device(S), s.to_device(Sn)
    outg, Fg = s.acoustic_substeps(Sng, Sg, s.to_device(R), 3, dtau)
    Fg = s.to_numpy(Fg)
    for name, ref, got in (("Fu", F[0], Fg["ru"]), ("Fv", F[1], Fg["rv"]), ("Fw", F[2], Fg["rw"])):
        e = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        _say(f"terrain flux {name} scheme {scheme}: {e:.2e}")
        assert e <= CALL_TOL, (name, e)
    dts = cfg.dt / 2.0
    ref_q = o.scalar_advance(Sn, S, F, dts)
    import torch
    flux = {f: torch.from_numpy(np.ascontiguousarray(x)).to(s.device, s.dtype) for f, x in zip(("ru", "rv", "rw"), F)}
    got_q = s.scalar_advance(Sng, Sg, flux, dts).cpu().numpy()
    e = float(np.max(np.abs(got_q - ref_q)) / np.max(np.abs(ref_q)))
    _say(f"terrain scalar advance scheme {scheme}: {e:.2e}")
    assert e <= CALL_TOL
    Sg = s.to_device(S)
    for _ in range(3):
        o.rk3_step(S)
        s.rk3_step(Sg)
    got = s.to_numpy(Sg)
    e = _errs(got, S, b, ("rho", "rt", "ru", "rv", "rw", "rq"))
    _say(f"terrain rk3 x3 with scalars scheme {scheme}:", {k: f"{v:.2e}" for k, v in e.items()})
    for k, v in e.items():
        assert v <= STEPS_TOL, (k, v)
    assert np.max(np.abs(got["rq"][0] / got["rho"] / 0.01 - 1.0)) < 1e-13
