"""Seeded synthetic workloads: grids, run parameters and initial conditions.

This module is the only code shared by the oracle side and the HIP side.  It
holds input descriptions and input generators and none of the method's
arithmetic: the hydrostatic base state is computed by each side and passed in.

Noise is counter-based: SplitMix64 (Steele, Lea & Flood 2014) applied to
``(seed << 32) | linear_cell_index`` gives 64 random bits; the top 53 bits make
a uniform u in [0, 1) and the perturbation is ``a * (2u - 1)``.  The same cell
therefore gets the same value whatever the order of generation.

The workloads stand in for the paper's: a dry warm bubble (Sec. 4.1.2), a
convective boundary layer LES like the scaling case of Sec. 5.2 (5th-order
upwind, Smagorinsky), an 80-level deep-atmosphere case with three advected
moisture tracers like the squall-line timing case of Sec. 5.2, and a density
current (Sec. 4.1.1) used for validation.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# gas constant and heat capacity used only to write soundings (inputs)
_RD, _CP, _P00 = 287.0, 1004.5, 1.0e5


@dataclasses.dataclass
class Config:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: np.ndarray
    dt: float
    n_substeps: int
    steps: int = 1
    beta_s: float = 0.1
    beta_d: float = 0.1
    adv_order_h: int = 2
    adv_order_v: int = 2
    scalar_scheme: int = 0  # 0: momentum interpolants, 1: WENO5-JS
    n_scalars: int = 0
    sgs: int = 0  # 0 none, 1 Smagorinsky, 2 learned closure, 3 Deardorff TKE (scalar 0 is rho e)
    Cs: float = 0.1
    Pr_t: float = 1.0 / 3.0
    nu_m: float = 0.0
    alpha_m: float = 0.0
    f_cor: float = 0.0
    Ug: float = 0.0
    Vg: float = 0.0
    surf_heat_flux: float = 0.0
    grav: float = 9.81
    prec: str = "fp64"  # "fp64" or "fp32" (FP32 bulk, FP64 column solve and sums)
    moist: int = 0  # 1: scalars 0, 1, 2 are rho q_v, rho q_c, rho q_r and enter the dynamics
    microphysics: int = 0  # 1: Kessler warm rain after every RK3 step (needs moist)
    anelastic: int = 0  # 1: anelastic equation set, SSP-RK2 with projections (dry, FP64)
    most_z0: float = 0.0  # > 0: Monin-Obukhov surface layer with this roughness length [m]
    p_surface: float = 1.0e5
    seed: int = 1

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)

    def z_centres(self) -> np.ndarray:
        dz = np.asarray(self.dz, dtype=np.float64)
        return np.cumsum(dz) - 0.5 * dz

    def z_faces(self) -> np.ndarray:
        dz = np.asarray(self.dz, dtype=np.float64)
        return np.concatenate([[0.0], np.cumsum(dz)])


# ---------------------------------------------------------------------------
# counter-based noise
# ---------------------------------------------------------------------------
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function of the 64-bit counter x (numpy uint64)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_noise(seed: int, shape, amplitude: float) -> np.ndarray:
    """a*(2u-1) for every cell of ``shape`` (x fastest), counter = seed<<32 | index."""
    n = int(np.prod(shape))
    ctr = (np.uint64(seed) << np.uint64(32)) | np.arange(n, dtype=np.uint64)
    u = (splitmix64(ctr) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return (amplitude * (2.0 * u - 1.0)).reshape(shape)


# ---------------------------------------------------------------------------
# vertical grids and soundings
# ---------------------------------------------------------------------------
def uniform_dz(nz: int, dz: float) -> np.ndarray:
    return np.full(nz, float(dz))


def stretched_dz(nz: int, dz0: float, dzmax: float, ztop: float) -> np.ndarray:
    """dz_k = min(dz0 r^k, dzmax) with r chosen by bisection so that sum = ztop."""
    def total(r):
        return float(np.minimum(dz0 * r ** np.arange(nz), dzmax).sum())
    lo, hi = 1.0, 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) < ztop:
            lo = mid
        else:
            hi = mid
    dz = np.minimum(dz0 * (0.5 * (lo + hi)) ** np.arange(nz), dzmax)
    return dz * (ztop / dz.sum())


def theta_sounding(cfg: Config) -> np.ndarray:
    """Base-state potential temperature at cell centres for each workload."""
    z = cfg.z_centres()
    kind = cfg.name.split("@")[0]
    if kind.startswith("cbl") or kind.startswith("mlp") or kind.startswith("ens"):
        return np.where(z < 1000.0, 300.0, 300.0 + 3.0e-3 * (z - 1000.0))
    if kind.startswith("deep"):
        th_tr, z_tr, T_tr = 343.0, 12000.0, 213.0
        below = 300.0 + (th_tr - 300.0) * (z / z_tr) ** 1.25
        above = th_tr * np.exp(cfg.grav * (z - z_tr) / (_CP * T_tr))
        return np.where(z <= z_tr, below, above)
    if kind.startswith("isothermal"):
        # theta of an isothermal atmosphere at T = 300 K: theta = T (P00/p)^kappa,
        # p = p_s exp(-g z / (R_d T)) (an input profile, not a base state)
        T = 300.0
        return T * np.exp(cfg.grav * z / (_CP * T))
    return np.full(cfg.nz, 300.0)


def relative_humidity(z: np.ndarray) -> np.ndarray:
    """Relative humidity of the deep-atmosphere sounding: 0.9 up to 1.5 km,
    decaying as a 5/4 power to 0.25 at 12 km, 0.25 above."""
    frac = np.clip((z - 1500.0) / 10500.0, 0.0, 1.0)
    return np.where(z < 1500.0, 0.9, np.where(z < 12000.0, 0.9 - 0.65 * frac ** 1.25, 0.25))


def qv_sounding(cfg: Config) -> np.ndarray:
    """Base-state water vapour mixing ratio q_v0 at cell centres (an input of
    the moist base state).  The relative humidity is converted with the
    saturation pressure of Bolton (1980), e_s = 611.2 exp(17.67 (T - 273.15)
    / (T - 29.65)) Pa, q_vs = 0.622 e_s / (p - e_s), at the temperature and
    pressure of a simple dry estimate of the sounding: the Exner function
    integrated upward as d pi / dz = -g / (c_p theta) from the surface
    pressure.  Only the profile is defined here; each side builds its own
    hydrostatic base state from theta0 and this q_v0."""
    z = cfg.z_centres()
    th = theta_sounding(cfg)
    pis = (cfg.p_surface / _P00) ** (_RD / _CP)
    dz = np.asarray(cfg.dz, dtype=np.float64)
    pi = np.empty(cfg.nz)
    pi[0] = pis - cfg.grav * 0.5 * dz[0] / (_CP * th[0])
    for k in range(1, cfg.nz):
        pi[k] = pi[k - 1] - cfg.grav * 0.5 * (dz[k - 1] + dz[k]) / (_CP * 0.5 * (th[k - 1] + th[k]))
    T = th * pi
    p = _P00 * pi ** (_CP / _RD)
    es = 611.2 * np.exp(17.67 * (T - 273.15) / (T - 29.65))
    return relative_humidity(z) * 0.622 * es / (p - es)


def qv0_of(cfg: Config):
    """The base-state vapour of a moist workload (qv_sounding), None for a dry one."""
    return qv_sounding(cfg) if cfg.moist else None


# ---------------------------------------------------------------------------
# initial states.  Perturbations of theta are applied at constant pressure:
# rho*theta keeps its base value and rho = Theta0 / (theta0 + dtheta).
# ---------------------------------------------------------------------------
def _centres_xy(cfg: Config):
    x = (np.arange(cfg.nx) + 0.5) * cfg.dx
    y = (np.arange(cfg.ny) + 0.5) * cfg.dy
    return x, y


def _face_mean_x(f: np.ndarray) -> np.ndarray:
    return 0.5 * (np.roll(f, 1, axis=-1) + f)


def _face_mean_y(f: np.ndarray) -> np.ndarray:
    return 0.5 * (np.roll(f, 1, axis=-2) + f)


def state_from_theta(cfg: Config, rho0: np.ndarray, theta0: np.ndarray, dtheta: np.ndarray,
                     u0: float = 0.0, v0: float = 0.0) -> dict:
    nz, ny, nx = cfg.nz, cfg.ny, cfg.nx
    Theta0 = (rho0 * theta0)[:, None, None] * np.ones((nz, ny, nx))
    th = theta0[:, None, None] + dtheta
    rho = Theta0 / th
    if getattr(cfg, "anelastic", 0):
        # the anelastic state: density rho0, the same potential temperature
        rho = rho0[:, None, None] * np.ones((nz, ny, nx))
        Theta0 = rho * th
    S = {
        "rho": np.ascontiguousarray(rho),
        "rt": np.ascontiguousarray(Theta0),
        "ru": np.ascontiguousarray(_face_mean_x(rho) * u0),
        "rv": np.ascontiguousarray(_face_mean_y(rho) * v0),
        "rw": np.zeros((nz + 1, ny, nx)),
        "rq": np.zeros((cfg.n_scalars, nz, ny, nx)),
    }
    return S


def initial_state(cfg: Config, rho0: np.ndarray, theta0: np.ndarray, p0: Optional[np.ndarray] = None,
                  pi0: Optional[np.ndarray] = None, qv0: Optional[np.ndarray] = None) -> dict:
    """Seeded initial state of workload ``cfg`` around the given base state
    (qv0: the base-state vapour of a moist workload)."""
    nz, ny, nx = cfg.nz, cfg.ny, cfg.nx
    x, y = _centres_xy(cfg)
    z = cfg.z_centres()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    kind = cfg.name.split("@")[0]
    dth = np.zeros((nz, ny, nx))
    u0 = v0 = 0.0
    if kind.startswith("bubble"):
        # warm bubble: 2 cos^2(pi r / 2), r < 1 (Sec. 4.1.2), centred mid-domain
        xc, zc, rr = 0.5 * nx * cfg.dx, 2000.0, 2000.0
        r = np.sqrt(((X - xc) / rr) ** 2 + ((Z - zc) / rr) ** 2)
        dth = np.where(r < 1.0, 2.0 * np.cos(0.5 * np.pi * r) ** 2, 0.0)
        dth = dth + uniform_noise(cfg.seed, (nz, ny, nx), 0.01)
    elif kind.startswith("density_current"):
        # cold bubble of Sec. 4.1.1 (temperature decrement -15 K), mirrored
        # about x = 0 in a periodic domain of twice the paper's half width
        xc, zc, xr, zr = 0.5 * nx * cfg.dx, 3000.0, 4000.0, 2000.0
        L = np.sqrt(((X - xc) / xr) ** 2 + ((Z - zc) / zr) ** 2)
        dT = np.where(L < 1.0, -15.0 * (np.cos(np.pi * L) + 1.0) / 2.0, 0.0)
        if pi0 is None:
            raise ValueError("density current needs the base-state Exner function")
        dth = dT / pi0[:, None, None]
    elif kind.startswith("cbl") or kind.startswith("mlp") or kind.startswith("ens"):
        dth = np.where(Z < 400.0, uniform_noise(cfg.seed, (nz, ny, nx), 0.1), 0.0)
        u0, v0 = cfg.Ug, cfg.Vg
    elif kind.startswith("deep"):
        xc = 0.5 * nx * cfg.dx
        dxl = np.abs(X - xc)
        taper = np.where(dxl <= 10000.0, 1.0,
                         np.where(dxl <= 12000.0, np.cos(0.5 * np.pi * (dxl - 10000.0) / 2000.0) ** 2, 0.0))
        dth = np.where(Z < 2000.0, -5.0 * (1.0 - Z / 2000.0), 0.0) * taper
        dth = dth + uniform_noise(cfg.seed, (nz, ny, nx), 0.1)
    elif kind.startswith("isothermal"):
        pass
    elif kind.startswith("rest"):
        pass
    else:
        raise ValueError(f"unknown workload {cfg.name}")
    S = state_from_theta(cfg, rho0, theta0, dth, u0, v0)
    if cfg.n_scalars > 0:
        S["rq"] = scalar_layers(cfg, S["rho"], rho0, theta0, p0, pi0, qv0)
    if cfg.sgs == 3:
        # the Deardorff closure's rho e: a seed of 0.1 m^2/s^2 below 400 m
        S["rq"][0] = S["rho"] * np.where(Z < 400.0, 0.1, 0.0)
    return S


def scalar_layers(cfg: Config, rho: np.ndarray, rho0, theta0, p0, pi0, qv0=None) -> np.ndarray:
    """rho*q for the advected tracers: q_v the base-state profile qv0 of a
    moist workload, else from the relative-humidity profile (Bolton 1980
    saturation pressure at the given base state); q_c and q_r smooth layers;
    each with a seeded 5 % relative perturbation."""
    nz, ny, nx = cfg.nz, cfg.ny, cfg.nx
    z = cfg.z_centres()
    q = np.zeros((cfg.n_scalars, nz, ny, nx))
    if cfg.moist:
        if qv0 is None:
            raise ValueError("a moist workload needs the base-state vapour qv0")
        qv = np.asarray(qv0, dtype=np.float64)
    elif p0 is not None and pi0 is not None:
        T = theta0 * pi0
        es = 611.2 * np.exp(17.67 * (T - 273.15) / (T - 29.65))
        qvs = 0.622 * es / (p0 - es)
        qv = relative_humidity(z) * qvs
    else:
        qv = 0.01 * np.exp(-z / 3000.0)
    qc = 1e-4 * np.exp(-((z - 3000.0) / 1000.0) ** 2)
    qr = 1e-5 * np.exp(-((z - 1500.0) / 500.0) ** 2)
    prof = [qv, qc, qr]
    noise = uniform_noise(cfg.seed + 1000, (nz, ny, nx), 1.0)
    for s in range(cfg.n_scalars):
        base = prof[s % 3][:, None, None]
        q[s] = rho * base * (1.0 + 0.05 * noise)
    return np.ascontiguousarray(q)


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------
def bubble2d(**kw) -> Config:
    """Dry 2-D x-z warm bubble, FP64: 64x1x64 at 125 m, 2nd order, no SGS,
    dt = 1 s, 6 substeps, 100 steps."""
    c = Config(name="bubble2d", nx=64, ny=1, nz=64, dx=125.0, dy=125.0, dz=uniform_dz(64, 125.0),
               dt=1.0, n_substeps=6, steps=100, adv_order_h=2, adv_order_v=2, seed=1)
    return c.replace(**kw)


def cbl(n_substeps: int = 6, **kw) -> Config:
    """3-D dry convective boundary layer LES: 256x256x128, 20 m x 20 m x 10 m,
    5th-order upwind, Smagorinsky Cs = 0.1, geostrophic wind 10 m/s,
    surface heat flux 0.2 K m/s, dt = 0.5 s."""
    c = Config(name="cbl", nx=256, ny=256, nz=128, dx=20.0, dy=20.0, dz=uniform_dz(128, 10.0),
               dt=0.5, n_substeps=n_substeps, steps=20, adv_order_h=5, adv_order_v=5, sgs=1,
               Cs=0.1, Pr_t=1.0 / 3.0, f_cor=1.0e-4, Ug=10.0, Vg=0.0, surf_heat_flux=0.2, seed=2)
    return c.replace(**kw)


def cbl_tke(**kw) -> Config:
    """The boundary layer of cbl() with the Deardorff TKE closure (rho e as
    its one scalar, 5th-order upwind like momentum) and a Monin-Obukhov
    surface layer over z0 = 0.1 m, as the paper's ABL cases (Sec. 4.2), with
    the stable 14 substeps."""
    c = cbl(n_substeps=14, name="cbl_tke", sgs=3, n_scalars=1, scalar_scheme=0, most_z0=0.1)
    return c.replace(**kw)


def les_mlp(**kw) -> Config:
    """Coarse LES with the learned subgrid closure: 128x128x64 cells at 40 m
    (5.12 x 5.12 x 2.56 km), the boundary-layer physics of cbl() with the
    closure in place of Smagorinsky (which stays as its fallback), FP32
    storage, dt = 0.4 s with 8 substeps (horizontal acoustic Courant number
    c dtau / dx = 0.43)."""
    c = Config(name="mlp_les", nx=128, ny=128, nz=64, dx=40.0, dy=40.0, dz=uniform_dz(64, 40.0),
               dt=0.4, n_substeps=8, steps=20, adv_order_h=5, adv_order_v=5, sgs=2,
               Cs=0.1, Pr_t=1.0 / 3.0, f_cor=1.0e-4, Ug=10.0, Vg=0.0, surf_heat_flux=0.2, prec="fp32", seed=41)
    return c.replace(**kw)


def les_fine(**kw) -> Config:
    """Fine LES that the learned closure is trained on: the boundary-layer
    physics of cbl() at 10 m, 256x256x128 cells (2.56 x 2.56 x 1.28 km), FP64,
    Smagorinsky, dt = 0.1 s with 8 substeps (c dtau / dx = 0.43).  Its 4x box
    filter lives on the 40 m grid of les_mlp()."""
    c = Config(name="mlp_fine", nx=256, ny=256, nz=128, dx=10.0, dy=10.0, dz=uniform_dz(128, 10.0),
               dt=0.1, n_substeps=8, steps=20, adv_order_h=5, adv_order_v=5, sgs=1,
               Cs=0.1, Pr_t=1.0 / 3.0, f_cor=1.0e-4, Ug=10.0, Vg=0.0, surf_heat_flux=0.2, seed=41)
    return c.replace(**kw)


def ensemble(sizes=((96, 96, 64), (128, 128, 64), (192, 192, 96)), per_size: int = 16, **kw) -> list:
    """Ensemble of boundary-layer LES members at 40 m: per_size members of each
    size (default 16 each of 96x96x64, 128x128x64 and 192x192x96, 82,837,504
    cells), FP32 storage, 5th-order upwind, dt = 0.4 s with 8 substeps.  Member
    m has seed 5000 + m and a surface heat flux drawn uniformly from
    [0.05, 0.3] K m/s (seed 5999); odd members use the learned closure, even
    members Smagorinsky."""
    n = per_size * len(sizes)
    qs = 0.175 + uniform_noise(5999, (n,), 0.125)
    out = []
    for m in range(n):
        nx, ny, nz = sizes[m // per_size]
        c = les_mlp(name=f"ens_{m}", nx=nx, ny=ny, nz=nz, dz=uniform_dz(nz, 40.0), seed=5000 + m,
                    surf_heat_flux=float(qs[m]), sgs=2 if m % 2 else 1)
        out.append(c.replace(**kw))
    return out


def deep(**kw) -> Config:
    """80-level moist deep atmosphere, stretched dz 50-500 m to 20 km, 250 m
    horizontal, q_v, q_c, q_r by WENO5 and in the dynamics (moist EOS,
    buoyancy and acoustic coefficients; no phase change), 3rd-order momentum,
    dt = 2 s, 8 substeps."""
    nz = kw.pop("nz", 80)
    c = Config(name="deep", nx=512, ny=512, nz=nz, dx=250.0, dy=250.0,
               dz=stretched_dz(nz, 50.0, 500.0, 20000.0), dt=2.0, n_substeps=8, steps=20,
               adv_order_h=3, adv_order_v=3, scalar_scheme=1, n_scalars=3, prec="fp32", seed=3, moist=1)
    return c.replace(**kw)


def density_current(dx: float = 100.0, **kw) -> Config:
    """Straka density current (Sec. 4.1.1) at 100 m, mirrored to a periodic
    51.2 km x 6.4 km domain; nu = alpha = 75 m^2/s, 3rd-order advection."""
    nx, nz = int(round(51200.0 / dx)), int(round(6400.0 / dx))
    c = Config(name="density_current", nx=nx, ny=1, nz=nz, dx=dx, dy=dx, dz=uniform_dz(nz, dx),
               dt=dx / 100.0, n_substeps=6, steps=int(round(900.0 / (dx / 100.0))), adv_order_h=3,
               adv_order_v=3, nu_m=75.0, alpha_m=75.0)
    return c.replace(**kw)


def small(name: str = "bubble_small", **kw) -> Config:
    """A small case for parity tests: several tiles and a ragged tail."""
    base = dict(name=name, nx=37, ny=21, nz=19, dx=125.0, dy=100.0, dz=uniform_dz(19, 100.0),
                dt=1.0, n_substeps=6, steps=3, adv_order_h=5, adv_order_v=3, seed=7)
    if "nz" in kw and "dz" not in kw:
        kw["dz"] = uniform_dz(kw["nz"], 100.0)
    base.update(kw)
    return Config(**base)


# ---- terrain-following coordinates (Sec. 3.4, Sec. 4.3) --------------------
def agnesi_nodes(cfg: Config, h_m: float, a: float, ridge: bool = False) -> np.ndarray:
    """Terrain heights h[ny][nx] at the nodes (node (i, j) at x = i dx, y = j dy,
    the low corner of cell (i, j)) of a Witch of Agnesi hill of height h_m and
    half-width a centred in the periodic domain: h_m / (1 + r^2 / a^2), with r
    the distance to the centre (ridge: the x distance only, a 2-D ridge along y)."""
    x = np.arange(cfg.nx) * cfg.dx - 0.5 * cfg.nx * cfg.dx
    y = np.arange(cfg.ny) * cfg.dy - 0.5 * cfg.ny * cfg.dy
    X, Y = np.meshgrid(x, y)
    r2 = X * X if ridge else X * X + Y * Y
    return np.ascontiguousarray(h_m / (1.0 + r2 / (a * a)))


def sinusoid_nodes(cfg: Config, amp: float, mx: int = 1, my: int = 0) -> np.ndarray:
    """Periodic terrain amp (1 + sin(2 pi mx x / Lx) sin... ) / 2 >= 0 at the nodes:
    amp (1 + sin(2 pi mx x / Lx + 2 pi my y / Ly)) / 2."""
    x = np.arange(cfg.nx) / cfg.nx
    y = np.arange(cfg.ny) / cfg.ny
    X, Y = np.meshgrid(x, y)
    return np.ascontiguousarray(0.5 * amp * (1.0 + np.sin(2.0 * np.pi * (mx * X + my * Y))))


def stratified_theta(z: np.ndarray, theta_s: float, N: float, grav: float) -> np.ndarray:
    """Potential temperature of constant buoyancy frequency N at heights z."""
    return theta_s * np.exp(N * N * z / grav)


def stratified_ground_pressure(h: np.ndarray, theta_s: float, N: float, p_sea: float, grav: float) -> np.ndarray:
    """Pressure at height h of the hydrostatic, constant-N atmosphere with
    p = p_sea at z = 0 (the Exner function falls by g/(c_p theta) per metre;
    N = 0: constant theta): the ground pressure of a column standing on h."""
    pi_s = (p_sea / _P00) ** (_RD / _CP)
    if N == 0.0:
        pi = pi_s - grav * h / (_CP * theta_s)
    else:
        pi = pi_s - grav * grav / (_CP * theta_s * N * N) * (1.0 - np.exp(-N * N * h / grav))
    return _P00 * pi ** (_CP / _RD)


def cell_mean_nodes(h: np.ndarray) -> np.ndarray:
    """The mean of the four corner nodes of every cell (periodic), (ny, nx)."""
    return 0.25 * (h + np.roll(h, -1, 1) + np.roll(h, -1, 0) + np.roll(np.roll(h, -1, 0), -1, 1))


def terrain_hill(**kw) -> Config:
    """Flow over a Witch of Agnesi hill like the terrain case of Sec. 4.3, in 3-D
    and periodic: 256 x 256 x 128 cells of 200 m, levels stretched from 40 m to a
    20 km lid, 10 m/s across a 400 m hill of 2 km half-width in a constant-N
    (0.01 1/s) atmosphere; inviscid, 3rd-order advection."""
    base = dict(name="terrain", nx=256, ny=256, nz=128, dx=200.0, dy=200.0,
                dz=stretched_dz(128, 40.0, 400.0, 20000.0), dt=1.0, n_substeps=6, steps=10,
                adv_order_h=3, adv_order_v=3, seed=91)
    base.update(kw)
    return Config(**base)


CONFIGS = {
    "bubble2d": bubble2d,
    "cbl": cbl,
    "deep": deep,
    "les_mlp": les_mlp,
    "les_fine": les_fine,
    "density_current": density_current,
}
