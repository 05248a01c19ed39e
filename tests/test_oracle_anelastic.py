"""Pins of the oracle's anelastic mode (Sec. 2.2: the constraint
div(rho0 u) = 0, buoyancy g rho0 (theta - theta0)/theta0; Sec. 3.2: SSP-RK2 with
a projection after each stage) to what mathematics fixes: the Poisson solve
against a dense least-squares solve of an independently assembled operator,
removal of pure gradients, a divergence-free result and idempotence, the
amplification factor of a two-stage second-order Runge-Kutta scheme on an
inertial oscillation, a resting atmosphere staying at rest, the buoyancy's
closed form and sign, and conservation of rho theta and the scalars."""
import numpy as np
import pytest

import oracle
from paper_2412_04395_amd import workloads as W


def _cfg(**kw):
    base = dict(name="rest", nx=8, ny=4, nz=7, dx=100.0, dy=80.0, dz=W.stretched_dz(7, 50.0, 200.0, 900.0),
                dt=2.0, n_substeps=2, anelastic=1, adv_order_h=3, adv_order_v=3, seed=11)
    base.update(kw)
    return W.small(**base)


def _oracle(cfg):
    o = oracle.Oracle(cfg)
    th0 = 300.0 + 0.004 * cfg.z_centres()
    b = o.init_base_state(th0, 1e5)
    return o, b, th0


def _div(cfg, U, V, Wf):
    """finite-volume divergence written with numpy rolls"""
    dz = np.asarray(cfg.dz)[:, None, None]
    return ((np.roll(U, -1, axis=2) - U) / cfg.dx + (np.roll(V, -1, axis=1) - V) / cfg.dy
            + (Wf[1:] - Wf[:-1]) / dz)


def _grad(cfg, chi):
    """face gradient of a centred field; zero on the lids"""
    dz = np.asarray(cfg.dz)
    U = (chi - np.roll(chi, 1, axis=2)) / cfg.dx
    V = (chi - np.roll(chi, 1, axis=1)) / cfg.dy
    Wf = np.zeros((cfg.nz + 1, cfg.ny, cfg.nx))
    Wf[1:-1] = (chi[1:] - chi[:-1]) / (0.5 * (dz[1:] + dz[:-1]))[:, None, None]
    return U, V, Wf


def _random_faces(cfg, seed):
    shp = (cfg.nz, cfg.ny, cfg.nx)
    U = W.uniform_noise(seed, shp, 3.0)
    V = W.uniform_noise(seed + 1, shp, 2.0)
    Wf = W.uniform_noise(seed + 2, (cfg.nz + 1, cfg.ny, cfg.nx), 1.0)
    Wf[0] = Wf[-1] = 0.0
    return U, V, Wf


def _laplacian_matrix(cfg):
    """L = div grad assembled point by point: periodic second differences in
    x and y, flux form in z with no flux through the lids"""
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    dz = np.asarray(cfg.dz)
    n = nx * ny * nz
    ix = lambda i, j, k: (k * ny + j) * nx + i  # noqa: E731
    L = np.zeros((n, n))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = ix(i, j, k)
                for nb in ((i + 1) % nx, (i - 1) % nx):
                    L[c, ix(nb, j, k)] += 1.0 / cfg.dx ** 2
                    L[c, c] -= 1.0 / cfg.dx ** 2
                for nb in ((j + 1) % ny, (j - 1) % ny):
                    L[c, ix(i, nb, k)] += 1.0 / cfg.dy ** 2
                    L[c, c] -= 1.0 / cfg.dy ** 2
                for kk in (k - 1, k + 1):
                    if 0 <= kk < nz:
                        w = 1.0 / (dz[k] * 0.5 * (dz[k] + dz[kk]))
                        L[c, ix(i, j, kk)] += w
                        L[c, c] -= w
    return L


@pytest.mark.parametrize("shape", [(8, 4, 7), (5, 3, 6), (1, 1, 5), (6, 1, 4)])
def test_poisson_matches_dense_least_squares(shape):
    nx, ny, nz = shape
    cfg = _cfg(nx=nx, ny=ny, nz=nz, dz=W.stretched_dz(nz, 40.0, 200.0, 700.0))
    o, _, _ = _oracle(cfg)
    D = _div(cfg, *_random_faces(cfg, 3))
    assert np.allclose(o.divergence(*_random_faces(cfg, 3)), D, rtol=0, atol=1e-15 * np.abs(D).max())
    phi = o.poisson(D)
    L = _laplacian_matrix(cfg)
    ref = np.linalg.lstsq(L, D.ravel(), rcond=None)[0].reshape(D.shape)
    ref -= ref[0].mean()  # the oracle's gauge: zero horizontal mean in the lowest cell
    assert np.abs(phi[0].mean()) <= 1e-13 * np.abs(phi).max()
    assert np.max(np.abs(phi - ref)) <= 1e-11 * np.max(np.abs(ref))
    # and it solves the system
    assert np.max(np.abs(L @ phi.ravel() - D.ravel())) <= 1e-11 * np.max(np.abs(D))


def test_projection_removes_a_pure_gradient():
    cfg = _cfg(nx=16, ny=8, nz=9, dz=W.stretched_dz(9, 30.0, 300.0, 1500.0))
    o, _, _ = _oracle(cfg)
    chi = W.uniform_noise(21, (cfg.nz, cfg.ny, cfg.nx), 50.0)
    U, V, Wf = _grad(cfg, chi)
    S = {"ru": U.copy(), "rv": V.copy(), "rw": Wf.copy()}
    pp = np.zeros_like(chi)
    o.project(S, 2.0, pp)
    scale = max(np.abs(U).max(), np.abs(V).max(), np.abs(Wf).max())
    for f in ("ru", "rv", "rw"):
        assert np.max(np.abs(S[f])) <= 1e-12 * scale, f
    # psi = phi / dt with phi = chi up to a constant
    d = pp * 2.0 - chi
    assert np.max(np.abs(d - d.mean())) <= 1e-11 * np.abs(chi).max()


def test_projection_is_divergence_free_idempotent_and_keeps_level_means():
    cfg = _cfg(nx=16, ny=8, nz=9, dz=W.stretched_dz(9, 30.0, 300.0, 1500.0))
    o, _, _ = _oracle(cfg)
    U, V, Wf = _random_faces(cfg, 31)
    S = {"ru": U.copy(), "rv": V.copy(), "rw": Wf.copy()}
    o.project(S, 1.0)
    D0, D1 = _div(cfg, U, V, Wf), _div(cfg, S["ru"], S["rv"], S["rw"])
    assert np.max(np.abs(D1)) <= 1e-12 * np.max(np.abs(D0))
    assert np.all(S["rw"][0] == 0.0) and np.all(S["rw"][-1] == 0.0)
    # the correction is a gradient: horizontal means per level are unchanged
    assert np.max(np.abs(S["ru"].mean(axis=(1, 2)) - U.mean(axis=(1, 2)))) <= 1e-13 * np.abs(U).max()
    assert np.max(np.abs(S["rv"].mean(axis=(1, 2)) - V.mean(axis=(1, 2)))) <= 1e-13 * np.abs(V).max()
    S2 = {k: v.copy() for k, v in S.items()}
    o.project(S2, 1.0)
    for f in ("ru", "rv", "rw"):
        assert np.max(np.abs(S2[f] - S[f])) <= 1e-12 * np.abs(U).max(), f


def _rest_state(cfg, o, b, th0, u=0.0, v=0.0):
    S = o.zeros_state()
    S["rho"][:] = b["rho0"][:, None, None]
    S["rt"][:] = (b["rho0"] * th0)[:, None, None]
    S["ru"][:] = b["rho0"][:, None, None] * u
    S["rv"][:] = b["rho0"][:, None, None] * v
    return S


def test_ssprk2_amplification_on_an_inertial_oscillation():
    # uniform wind, f-plane Coriolis only: d(u + i v)/dt = -i f (u + i v); a
    # two-stage second-order Runge-Kutta step multiplies by 1 + z + z^2/2,
    # z = -i f dt (neither stage's pressure nor advection acts on a uniform flow)
    f, dt = 1e-3, 60.0
    cfg = _cfg(f_cor=f, dt=dt)
    o, b, th0 = _oracle(cfg)
    S = _rest_state(cfg, o, b, th0, u=3.0, v=-2.0)
    z = -1j * f * dt
    amp = 1.0 + z + 0.5 * z * z
    w0 = (S["ru"] + 1j * S["rv"]) / b["rho0"][:, None, None]
    for n in range(1, 6):
        o.ssprk2_step(S)
        w = (S["ru"] + 1j * S["rv"]) / b["rho0"][:, None, None]
        assert np.max(np.abs(w - w0 * amp ** n)) <= 1e-13 * np.abs(w0).max(), n
    # |amp| > 1: the scheme's known slight growth on oscillations
    assert abs(amp) > 1.0


def test_resting_atmosphere_stays_at_rest():
    cfg = _cfg(sgs=1, Cs=0.2)
    o, b, th0 = _oracle(cfg)
    S = _rest_state(cfg, o, b, th0)
    for _ in range(5):
        o.ssprk2_step(S)
    for f in ("ru", "rv", "rw"):
        assert np.max(np.abs(S[f])) <= 1e-12, f
    assert np.max(np.abs(o.p_anel)) <= 1e-9


def test_buoyancy_closed_form_and_sign():
    # at rest with zero pressure perturbation, one warm cell: R_W on the two
    # faces of that cell is g rho0 theta'/theta0 / 2, upward
    cfg = _cfg()
    o, b, th0 = _oracle(cfg)
    S = _rest_state(cfg, o, b, th0)
    k, j, i, dth = 3, 2, 5, 0.5
    S["rt"][k, j, i] = b["rho0"][k] * (th0[k] + dth)
    R = o.slow_rhs(S)
    expect = cfg.grav * 0.5 * b["rho0"][k] * ((th0[k] + dth) - th0[k]) / th0[k]
    assert R["rw"][k, j, i] == pytest.approx(expect, rel=1e-12) and expect > 0
    assert R["rw"][k + 1, j, i] == pytest.approx(expect, rel=1e-12)
    mask = np.ones_like(R["rw"], dtype=bool)
    mask[k, j, i] = mask[k + 1, j, i] = False
    assert np.max(np.abs(R["rw"][mask])) <= 1e-12 * expect


def test_rho_theta_and_scalars_are_conserved():
    cfg = _cfg(nx=16, ny=8, nz=10, dz=W.uniform_dz(10, 100.0), n_scalars=2, scalar_scheme=1, dt=5.0)
    o, b, th0 = _oracle(cfg)
    S = _rest_state(cfg, o, b, th0, u=2.0, v=1.0)
    shp = S["rt"].shape
    S["rt"] += b["rho0"][:, None, None] * W.uniform_noise(5, shp, 0.5)
    S["rq"][0] = b["rho0"][:, None, None] * (1e-2 + W.uniform_noise(6, shp, 1e-3))
    S["rq"][1] = b["rho0"][:, None, None] * np.maximum(W.uniform_noise(7, shp, 1e-3), 0.0)
    vol = cfg.dx * cfg.dy * np.asarray(cfg.dz)[:, None, None]
    t0 = np.sum(S["rt"] * vol)
    q0 = [np.sum(S["rq"][s] * vol) for s in range(2)]
    for _ in range(4):
        o.ssprk2_step(S)
    assert abs(np.sum(S["rt"] * vol) / t0 - 1.0) < 1e-14
    for s in range(2):
        assert abs(np.sum(S["rq"][s] * vol) / q0[s] - 1.0) < 1e-13, s
    assert np.max(np.abs(S["rw"])) > 1e-6  # buoyancy drove motion
    # the end state satisfies the constraint
    D = _div(cfg, S["ru"], S["rv"], S["rw"])
    assert np.max(np.abs(D)) <= 1e-12 * np.max(np.abs(S["ru"])) / cfg.dx
