"""Pins of the oracle's terrain-following coordinates (Sec. 3.4, App. A, App. B,
App. C) to what the geometry and the equations fix, independently of its own
formulas:

* flat terrain (h = 0) reproduces the flat oracle bit for bit (every metric
  factor is exactly 1 or 0);
* the physical cell heights of a column add up to the distance from its ground
  to the flat lid, for basic (beta = 1) and Sullivan (beta = 3) smoothing;
* the per-column hydrostatic base state matches the analytic constant-N
  atmosphere at each cell's physical height (the columns stand on different
  ground);
* a perturbation pressure that depends on height only has no horizontal
  gradient (the discrete cancellation the App. B metrics are chosen for): the
  metric correction removes the terrain-following difference exactly;
* a resting base state over a hill stays at rest, bit for bit;
* a uniform free stream over smooth terrain without gravity: the mass tendency
  is the truncation error of the discrete metric identity d(h_zeta)/dxi =
  d(h_xi)/dzeta and falls by 4 when the horizontal spacing halves, in the slow
  right-hand side and in the substeps (a wrong sign or placement of the metric
  part of Omega leaves an error that does not converge);
* mass and sum rho theta dV are conserved over RK3 steps over a hill;
* a uniform theta stays uniform (the theta and mass fluxes agree, with
  Omega and h_zeta, in the right-hand side and in the substeps).
"""
import numpy as np
import pytest

import oracle
from paper_2412_04395_amd import workloads as W

TH_S, N_BV, P_SEA = 300.0, 0.01, 1.0e5


def _cfg(**kw):
    base = dict(name="terrain_small", nx=24, ny=12, nz=12, dx=200.0, dy=200.0,
                dz=W.stretched_dz(12, 60.0, 500.0, 3000.0), dt=1.0, n_substeps=6, adv_order_h=3,
                adv_order_v=3, seed=11)
    base.update(kw)
    return W.small(**base)


def _hill(cfg, h_m=300.0, a=800.0):
    return W.agnesi_nodes(cfg, h_m, a)


def _terrain_oracle(cfg, h, beta=1.0, N=N_BV):
    o = oracle.Oracle(cfg)
    o.set_terrain(h, beta)
    Hc, zc = o.terrain_heights()
    hb = W.cell_mean_nodes(h)
    th0 = W.stratified_theta(zc, TH_S, N, cfg.grav) if cfg.grav > 0 else np.full(zc.shape, TH_S)
    ps = W.stratified_ground_pressure(hb, TH_S, N, P_SEA, cfg.grav)
    b = o.init_base_state_columns(th0, ps)
    return o, b, Hc, zc


def _rest(b):
    S = {"rho": b["rho0"].copy(), "rt": b["rho0"] * b["theta0"]}
    nz, ny, nx = S["rho"].shape
    S["ru"] = np.zeros((nz, ny, nx))
    S["rv"] = np.zeros((nz, ny, nx))
    S["rw"] = np.zeros((nz + 1, ny, nx))
    S["rq"] = np.zeros((0, nz, ny, nx))
    return {k: np.ascontiguousarray(v) for k, v in S.items()}


def _flow(cfg, b, seed, U=10.0, V=3.0):
    """the base state with a wind and small noise in every field"""
    S = _rest(b)
    shp = S["rho"].shape
    S["rho"] = S["rho"] * (1.0 + W.uniform_noise(seed, shp, 1e-3))
    S["rt"] = S["rt"] * (1.0 + W.uniform_noise(seed + 1, shp, 1e-3))
    S["ru"] = S["rho"] * (U + W.uniform_noise(seed + 2, shp, 1.0))
    S["rv"] = S["rho"] * (V + W.uniform_noise(seed + 3, shp, 1.0))
    rw = W.uniform_noise(seed + 4, S["rw"].shape, 0.3)
    rw[0] = rw[-1] = 0.0
    S["rw"] = rw
    return {k: np.ascontiguousarray(v) for k, v in S.items()}


def test_flat_terrain_reproduces_the_flat_path_bit_for_bit():
    cfg = _cfg(adv_order_h=5, f_cor=1e-4, Ug=5.0, Vg=1.0)
    zc1 = cfg.z_centres()
    th1 = W.stratified_theta(zc1, TH_S, N_BV, cfg.grav)
    flat = oracle.Oracle(cfg)
    bf = flat.init_base_state(th1, P_SEA)
    ter = oracle.Oracle(cfg)
    ter.set_terrain(np.zeros((cfg.ny, cfg.nx)), 3.0)
    Hc, zc = ter.terrain_heights()
    assert np.array_equal(Hc, np.broadcast_to(np.asarray(cfg.dz)[:, None, None], Hc.shape))
    assert np.allclose(zc, np.broadcast_to(zc1[:, None, None], zc.shape), rtol=1e-15, atol=1e-12)
    shp = (cfg.nz, cfg.ny, cfg.nx)
    bt = ter.init_base_state_columns(np.broadcast_to(th1[:, None, None], shp), np.full(shp[1:], P_SEA))
    for f in ("rho0", "p0", "pi0"):
        assert np.array_equal(bt[f], np.broadcast_to(bf[f][:, None, None], shp)), f
    S = _flow(cfg, bt, 5)
    R1, R2 = flat.slow_rhs(S), ter.slow_rhs(S)
    for f in ("rho", "rt", "ru", "rv", "rw"):
        assert np.array_equal(R1[f], R2[f]), f
    Sn = _flow(cfg, bt, 9)
    o1, F1 = flat.acoustic_substeps(Sn, S, R1, 3, 0.2)
    o2, F2 = ter.acoustic_substeps(Sn, S, R1, 3, 0.2)
    for f in ("rho", "rt", "ru", "rv", "rw"):
        assert np.array_equal(o1[f], o2[f]), f
    A, B = {k: v.copy() for k, v in S.items()}, {k: v.copy() for k, v in S.items()}
    for _ in range(2):
        flat.rk3_step(A)
        ter.rk3_step(B)
    for f in ("rho", "rt", "ru", "rv", "rw"):
        assert np.array_equal(A[f], B[f]), f
    d1, d2 = flat.diagnostics(A), ter.diagnostics(B)
    for k in ("mass", "theta_mass", "energy", "max_w"):
        assert d1[k] == d2[k], k


@pytest.mark.parametrize("beta", [1.0, 3.0])
def test_column_heights_span_ground_to_lid(beta):
    cfg = _cfg()
    h = _hill(cfg, 600.0, 600.0)
    o = oracle.Oracle(cfg)
    o.set_terrain(h, beta)
    Hc, zc = o.terrain_heights()
    zt = float(np.sum(cfg.dz))
    hb = W.cell_mean_nodes(h)
    assert np.all(Hc > 0.0)
    assert np.allclose(Hc.sum(axis=0), zt - hb, rtol=0, atol=1e-10 * zt)
    assert np.all(np.diff(zc, axis=0) > 0.0)
    # centres lie inside their cells: the ground plus the heights below plus half
    below = np.cumsum(Hc, axis=0) - Hc
    assert np.allclose(zc, hb[None] + below + 0.5 * Hc, rtol=0, atol=1e-9 * zt)
    # the lid is flat and basic smoothing shrinks every cell of a column alike
    if beta == 1.0:
        assert np.allclose(Hc / np.asarray(cfg.dz)[:, None, None], (1.0 - hb / zt)[None], rtol=1e-13)


def _base_error(nz, N):
    cfg = _cfg(nz=nz, dz=W.stretched_dz(nz, 720.0 / nz, 6000.0 / nz, 3000.0))
    h = _hill(cfg, 400.0, 600.0)
    o, b, Hc, zc = _terrain_oracle(cfg, h, 3.0, N)
    exact = W.stratified_ground_pressure(zc, TH_S, N, P_SEA, cfg.grav)
    return float(np.max(np.abs(b["p0"] / exact - 1.0))), b


@pytest.mark.parametrize("N", [0.0, N_BV])
def test_column_base_states_follow_the_analytic_atmosphere(N):
    # the trapezoidal hydrostatics is second order: halving every cell height
    # divides the departure from the analytic column by about 4
    e1, b = _base_error(12, N)
    e2, _ = _base_error(24, N)
    assert e1 < 5e-5 and e1 / e2 > 3.5, (e1, e2)
    # with the columns' own heights left out (flat dz), the hill columns would
    # miss by the weight of the displaced air: about g rho0 h / p ~ 4e-2
    assert np.max(np.abs(b["p0"][:, 0, 0] - b["p0"][:, 6, 12])) > 1e3


@pytest.mark.parametrize("beta", [1.0, 3.0])
def test_pressure_depending_on_height_only_has_no_horizontal_gradient(beta):
    cfg = _cfg()
    h = _hill(cfg, 400.0, 700.0)
    o, b, Hc, zc = _terrain_oracle(cfg, h, beta)
    c = -0.02  # Pa/m
    p_target = b["p0"] + c * zc
    Rd, P00, gam = oracle.const("R_d"), oracle.const("P00"), oracle.const("gamma")
    S = _rest(b)
    S["rt"] = np.ascontiguousarray((P00 / Rd) * (p_target / P00) ** (1.0 / gam))
    R = o.slow_rhs(S)
    # the plain difference along the terrain-following level is of size c h_xi
    pp = c * zc
    raw = np.max(np.abs(pp - np.roll(pp, 1, axis=2))) / cfg.dx
    assert raw > 1e-3
    for f in ("ru", "rv"):
        assert np.max(np.abs(R[f])) <= 1e-8 * raw, (f, np.max(np.abs(R[f])), raw)


def test_rest_state_over_a_hill_stays_at_rest():
    cfg = _cfg()
    o, b, Hc, zc = _terrain_oracle(cfg, _hill(cfg), 1.0)
    S = _rest(b)
    R = o.slow_rhs(S)
    for f in ("rho", "rt", "ru", "rv", "rw"):
        assert np.all(R[f] == 0.0), f
    S0 = {k: v.copy() for k, v in S.items()}
    for _ in range(2):
        o.rk3_step(S)
    for f in ("rho", "rt", "ru", "rv", "rw"):
        assert np.array_equal(S[f], S0[f]), f


def _free_stream(nx, ny, substeps):
    # smooth periodic terrain without gravity: a uniform state with a uniform
    # horizontal wind.  The wind blows through the sloping ground (Omega = 0
    # there), so the lowest cells carry that flux; the cells above them see
    # only the truncation error of the metric identity.
    cfg = _cfg(nx=nx, ny=ny, dx=4800.0 / nx, dy=2400.0 / ny, grav=0.0)
    h = W.sinusoid_nodes(cfg, 300.0, 1, 1)
    o, b, Hc, zc = _terrain_oracle(cfg, h, 1.0, 0.0)
    S = _rest(b)
    scale = float(np.max(b["rho0"])) * 10.0 * 300.0 * np.pi / 4800.0 / 3000.0
    if not substeps:
        S["ru"] = np.ascontiguousarray(b["rho0"] * 10.0)
        S["rv"] = np.ascontiguousarray(b["rho0"] * 5.0)
        return float(np.max(np.abs(o.slow_rhs(S)["rho"][1:]))), scale
    Sn = {k: v.copy() for k, v in S.items()}
    Sn["ru"] = np.ascontiguousarray(b["rho0"] * 10.0)
    Sn["rv"] = np.ascontiguousarray(b["rho0"] * 5.0)
    R = {k: np.zeros_like(v) for k, v in S.items()}
    # a short substep: the implicit coupling (dtau^2) stays far below the
    # explicit divergence, so the ground cells' flux does not reach above
    dtau = 1e-4
    out, _ = o.acoustic_substeps(Sn, S, R, 1, dtau)
    return float(np.max(np.abs(out["rho"] - S["rho"])[1:])) / dtau, scale


def test_free_stream_error_converges_at_second_order():
    e1, scale = _free_stream(24, 12, False)
    e2, _ = _free_stream(48, 24, False)
    assert e2 > 0.0 and e1 / e2 > 3.5, (e1, e2)
    # each metric term alone is of size rho U dh/dx / z_t
    assert e1 < 0.1 * scale, (e1, scale)
    # the substeps' continuity (h_zeta-weighted U'', V'' and Omega'' of the new
    # horizontal momenta) gives the same residual as the right-hand side's
    s1, _ = _free_stream(24, 12, True)
    s2, _ = _free_stream(48, 24, True)
    assert abs(s1 / e1 - 1.0) < 1e-6 and abs(s2 / e2 - 1.0) < 1e-6, (s1, e1, s2, e2)


def test_mass_and_theta_mass_are_conserved_over_a_hill():
    cfg = _cfg()
    o, b, Hc, zc = _terrain_oracle(cfg, _hill(cfg), 3.0)
    S = _flow(cfg, b, 21)
    d0 = o.diagnostics(S)
    for _ in range(3):
        o.rk3_step(S)
    d1 = o.diagnostics(S)
    assert abs(d1["mass"] / d0["mass"] - 1.0) < 1e-14
    assert abs(d1["theta_mass"] / d0["theta_mass"] - 1.0) < 1e-14
    assert np.all(np.isfinite(S["rw"])) and d1["max_w"] > 0.0
    # the mass sum weighs every cell by its physical volume
    vol = cfg.dx * cfg.dy * Hc
    S2 = _flow(cfg, b, 21)
    assert o.diagnostics(S2)["mass"] == pytest.approx(float(np.sum(S2["rho"] * vol)), rel=1e-14)


def test_uniform_theta_stays_uniform_over_a_hill():
    cfg = _cfg()
    o, b, Hc, zc = _terrain_oracle(cfg, _hill(cfg), 1.0)
    S = _flow(cfg, b, 31)
    S["rt"] = np.ascontiguousarray(305.0 * S["rho"])
    R = o.slow_rhs(S)
    assert np.max(np.abs(R["rt"] - 305.0 * R["rho"])) <= 1e-12 * 305.0 * np.max(np.abs(R["rho"]))
    for _ in range(2):
        o.rk3_step(S)
    th = S["rt"] / S["rho"]
    assert np.max(np.abs(th / 305.0 - 1.0)) < 1e-13


def _agnesi_wave(o, cfg, a, hm, U, N):
    """Run the flow over a 2-D Witch of Agnesi ridge and return the simulated
    and the linear w at the cell centres, with the centres' heights."""
    h = W.agnesi_nodes(cfg, hm, a, ridge=True)
    o.set_terrain(h, 1.0)
    Hc, zc = o.terrain_heights()
    th0 = W.stratified_theta(zc, TH_S, N, cfg.grav)
    ps = W.stratified_ground_pressure(W.cell_mean_nodes(h), TH_S, N, P_SEA, cfg.grav)
    b = o.init_base_state_columns(th0, ps)
    S = _rest(b)
    S["ru"] = np.ascontiguousarray(b["rho0"] * U)
    for _ in range(cfg.steps):
        o.rk3_step(S)
    rho = S["rho"][:, 0, :]
    wf = S["rw"][1:-1, 0, :] / (0.5 * (rho[1:] + rho[:-1]))
    w = np.zeros_like(rho)
    w[1:-1] = 0.5 * (wf[:-1] + wf[1:])
    z = zc[:, 0, :]
    x = (np.arange(cfg.nx) + 0.5) * cfg.dx - 0.5 * cfg.nx * cfg.dx
    X = np.broadcast_to(x, z.shape)
    # linear hydrostatic flow over the ridge (Queney 1948; Smith 1980): the
    # streamlines are displaced by eta = h_m a (a cos(lz) - x sin(lz)) /
    # (x^2 + a^2), l = N/U, so w = U d(eta)/dx; in a compressible atmosphere
    # the amplitude grows as (rho0(ground)/rho0(z))^(1/2)
    l = N / U
    den = X * X + a * a
    deta = hm * a * (-np.sin(l * z) * den - 2.0 * X * (a * np.cos(l * z) - X * np.sin(l * z))) / den ** 2
    wlin = U * deta * np.sqrt(b["rho0"][0, 0, :] / b["rho0"][:, 0, :])
    return w, wlin, z


def test_witch_of_agnesi_mountain_wave_matches_linear_theory():
    # Sec. 4.3: flow over a Witch of Agnesi ridge against the linear solution.
    # Here a 10 m ridge of 10 km half-width (linear, hydrostatic: N a / U = 10)
    # in a 256 km periodic domain under a 30 km lid, after 6000 s: the
    # vertically propagating waves (group speed about U^2/(N a) = 1 m/s) have
    # not yet come back from the lid into the lowest 4 km.  The bounds allow
    # for 5 cells per half-width, the hydrostatic and small-amplitude
    # approximations of the linear solution and the flow still settling; a
    # wrong sign of the metric part of Omega gives a correlation of 0.25 and
    # twice the amplitude.
    cfg = _cfg(nx=128, ny=1, nz=60, dx=2000.0, dy=2000.0, dz=W.uniform_dz(60, 500.0), dt=20.0, n_substeps=6,
               steps=300)
    w, wlin, z = _agnesi_wave(oracle.Oracle(cfg), cfg, 10000.0, 10.0, 10.0, N_BV)
    for zlo, zhi, cmin, emax in ((300.0, 2000.0, 0.97, 0.25), (2000.0, 4000.0, 0.9, 0.45)):
        m = (z[:, 0] > zlo) & (z[:, 0] < zhi)
        ws, wl = w[m], wlin[m]
        corr = float(np.sum(ws * wl) / np.sqrt(np.sum(ws * ws) * np.sum(wl * wl)))
        err = float(np.linalg.norm(ws - wl) / np.linalg.norm(wl))
        assert corr > cmin and err < emax, (zlo, zhi, corr, err)
        assert abs(np.abs(ws).max() / np.abs(wl).max() - 1.0) < 0.2, (zlo, zhi)


@pytest.mark.parametrize("scheme", [0, 1])
def test_scalars_over_a_hill_keep_a_uniform_mixing_ratio_and_their_mass(scheme):
    # the scalars' stage-averaged fluxes are the substeps' own (rho Omega with
    # the beta weights vertically, h_zeta-weighted horizontally), so a uniform
    # mixing ratio stays uniform as the density changes, and sum rho q dV is
    # conserved (interpolant of the run's order, and WENO5)
    cfg = _cfg(n_scalars=2, scalar_scheme=scheme)
    o, b, Hc, zc = _terrain_oracle(cfg, _hill(cfg), 3.0)
    S = _flow(cfg, b, 41)
    S["rq"] = np.ascontiguousarray(np.stack([0.01 * S["rho"], S["rho"] * (1.0 + W.uniform_noise(43, S["rho"].shape, 0.5))]))
    vol = cfg.dx * cfg.dy * Hc
    m0 = float(np.sum(S["rq"][1] * vol))
    for _ in range(3):
        o.rk3_step(S)
    q = S["rq"][0] / S["rho"]
    assert np.max(np.abs(q / 0.01 - 1.0)) < 1e-13
    assert abs(float(np.sum(S["rq"][1] * vol)) / m0 - 1.0) < 1e-14
    d = o.diagnostics(S)
    assert d["scalar_mass"][1] == pytest.approx(float(np.sum(S["rq"][1] * vol)), rel=1e-14)


def test_scalars_on_flat_terrain_reproduce_the_flat_path():
    cfg = _cfg(n_scalars=1, scalar_scheme=1)
    flat = oracle.Oracle(cfg)
    zc1 = cfg.z_centres()
    th1 = W.stratified_theta(zc1, TH_S, N_BV, cfg.grav)
    bf = flat.init_base_state(th1, P_SEA)
    ter = oracle.Oracle(cfg)
    ter.set_terrain(np.zeros((cfg.ny, cfg.nx)), 1.0)
    shp = (cfg.nz, cfg.ny, cfg.nx)
    bt = ter.init_base_state_columns(np.broadcast_to(th1[:, None, None], shp), np.full(shp[1:], P_SEA))
    S = _flow(cfg, bt, 51)
    S["rq"] = np.ascontiguousarray((S["rho"] * (1.0 + W.uniform_noise(53, shp, 0.5)))[None])
    A, B = {k: v.copy() for k, v in S.items()}, {k: v.copy() for k, v in S.items()}
    for _ in range(2):
        flat.rk3_step(A)
        ter.rk3_step(B)
    for f in ("rho", "rt", "ru", "rv", "rw", "rq"):
        assert np.array_equal(A[f], B[f]), f


def test_surface_heat_flux_over_terrain_heats_the_ground_cells_by_the_flux_times_the_area():
    # a resting atmosphere over a hill with a prescribed kinematic surface heat
    # flux (per unit horizontal area): only the lowest cells gain rho theta,
    # each by rho Q_s dx dy per unit time in total (its tendency times its
    # physical volume), whatever the slope under it
    Qs = 0.2
    cfg = _cfg(surf_heat_flux=Qs)
    o, b, Hc, zc = _terrain_oracle(cfg, _hill(cfg, 500.0, 600.0), 3.0)
    S = _rest(b)
    R = o.slow_rhs(S)
    vol = cfg.dx * cfg.dy * Hc
    assert np.all(R["rt"][1:] == 0.0)
    assert np.allclose(R["rt"][0] * vol[0], S["rho"][0] * Qs * cfg.dx * cfg.dy, rtol=1e-14, atol=0)
    for f in ("rho", "ru", "rv", "rw"):
        assert np.all(R[f] == 0.0), f
